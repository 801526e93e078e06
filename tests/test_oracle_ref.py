"""Pins of the oracle against brute force, an external LP solver in two
independent formulations, special cases with closed forms, and strong
duality (Section 3: the dual optimum equals the DCOPF optimum)."""
import numpy as np
import pytest

from oracle import dual as D
from oracle import ref
from paper_2406_13191_amd import synth


def _tiny_network(seed, nb=6, nl=8, ng=3, qp=False, limit_scale=0.7):
    """A tiny random instance for brute force (connected, binding lines)."""
    rng = np.random.default_rng(seed)
    fb = [int(rng.integers(0, i)) for i in range(1, nb)]
    tb = list(range(1, nb))
    pairs = {(min(a, b), max(a, b)) for a, b in zip(fb, tb)}
    while len(fb) < nl:
        a, b = (int(v) for v in rng.integers(0, nb, 2))
        if a != b and (min(a, b), max(a, b)) not in pairs:
            pairs.add((min(a, b), max(a, b)))
            fb.append(a)
            tb.append(b)
    net = synth.Network(nb, np.array(fb), np.array(tb), rng.uniform(5, 20, nl), 0)
    H = synth.ptdf(net)
    gen_bus = rng.choice(nb, ng, replace=False).astype(np.int32)
    c = rng.uniform(10, 50, ng)
    q = rng.uniform(0.01, 0.1, ng) if qp else np.zeros(ng)
    p_max = rng.uniform(50, 150, ng)
    d = rng.uniform(0, 40, nb)
    d *= 0.6 * p_max.sum() / d.sum()
    # limits: a fraction of the flows of an even dispatch
    p0 = p_max * d.sum() / p_max.sum()
    inj = -d.copy()
    np.add.at(inj, gen_bus, p0)
    F0 = np.abs(H @ inj)
    f_max = np.maximum(limit_scale * F0, 1.0) * rng.uniform(1.0, 2.0, nl)
    prob = synth.Problem(H=H, gen_bus=gen_bus, c=c, q=q, p_min=np.zeros(ng), p_max=p_max,
                         d=d, f_max=f_max, slack=0, net=net)
    return net, prob


def _feasible_tiny(seed, **kw):
    for k in range(50):
        net, p = _tiny_network(seed * 100 + k, **kw)
        if ref.opt_btheta(net, p)["opt"] is not None:
            return net, p
    raise RuntimeError("no feasible tiny instance")


@pytest.mark.parametrize("seed", range(6))
def test_lp_three_references_agree(seed):
    net, p = _feasible_tiny(seed)
    K = D.canonical(p)
    v, _ = ref.lp_vertex_enum(K)
    o1 = ref.opt_ptdf(p)
    o2 = ref.opt_btheta(net, p)
    assert abs(v - o1["opt"]) <= 1e-9 * abs(v)
    assert abs(v - o2["opt"]) <= 1e-9 * abs(v)
    # strong duality: the dual function at HiGHS's multipliers equals OPT
    g = D.dual_value(K, o1["lam"], o1["mu"]).g
    assert abs(g - v) <= 1e-8 * abs(v)


def test_tiny30_vertex_enumeration():
    # The 5 limited lines plus the box leave C(22, 5) = 26,334 vertex candidates;
    # the other lines (1e4 MW) are inert since |F| <= sum |H| |injection| < 1e4.
    net, p = synth.make_network("tiny30", 1)
    K = D.canonical(p)
    inj_abs = p.d.sum() + p.p_max.sum()
    assert np.abs(p.H).max() * inj_abs < 1e4
    inert = [l for l in range(p.n_line) if p.f_max[l] >= 1e4]
    v, _ = ref.lp_vertex_enum(K, drop_lines=inert)
    o = ref.opt_ptdf(p)
    assert abs(v - o["opt"]) <= 1e-9 * abs(v)
    assert abs(D.dual_value(K, o["lam"], o["mu"]).g - v) <= 1e-8 * abs(v)


@pytest.mark.parametrize("seed", range(4))
def test_qp_kkt_enumeration_vs_certificate(seed):
    net, p = _feasible_tiny(seed, nb=5, nl=6, ng=3, qp=True)
    K = D.canonical(p)
    v, x = ref.qp_kkt_enum(K)
    cert = ref.qp_certificate(K, maxiter=5000)
    assert cert["lb"] <= v + 1e-9 * abs(v)
    assert cert["ub"] >= v - 1e-9 * abs(v)
    assert abs(cert["lb"] - v) <= 1e-7 * abs(v)


@pytest.mark.parametrize("qp", [False, True])
def test_economic_dispatch_special_case(qp):
    # No binding line: DCOPF is economic dispatch; mu* = 0 and lambda* is the
    # marginal price, and the dual value there equals the optimum exactly.
    net, p = synth.make_network("geo300q" if qp else "geo300", 7)
    p = p.replace(f_max=np.full(p.n_line, 1e7))
    K = D.canonical(p)
    cost, pd, price = ref.econ_dispatch(p.c, p.q, p.p_min, p.p_max, p.d.sum())
    g = D.dual_value(K, price, np.zeros(2 * p.n_line)).g
    assert abs(g - cost) <= 1e-9 * abs(cost)
    if not qp:
        assert abs(ref.opt_btheta(net, p)["opt"] - cost) <= 1e-9 * abs(cost)


def test_two_bus_congestion_closed_form():
    # bus 0 (slack): cheap unit c0; bus 1: expensive unit c1 and load D > f.
    # OPT = c0 f + c1 (D - f); lambda* = c0 (slack price), mu+* = c1 - c0.
    net = synth.Network(2, np.array([0]), np.array([1]), np.array([10.0]), 0)
    H = synth.ptdf(net)
    np.testing.assert_allclose(H, [[0.0, -1.0]])
    c0, c1, Dl, f = 20.0, 35.0, 100.0, 60.0
    p = synth.Problem(H=H, gen_bus=np.array([0, 1], np.int32), c=np.array([c0, c1]),
                      q=np.zeros(2), p_min=np.zeros(2), p_max=np.array([200.0, 200.0]),
                      d=np.array([0.0, Dl]), f_max=np.array([f]), slack=0, net=net)
    K = D.canonical(p)
    opt = c0 * f + c1 * (Dl - f)
    assert abs(ref.opt_ptdf(p)["opt"] - opt) < 1e-9 * opt
    g = D.dual_value(K, c0, np.array([c1 - c0, 0.0])).g
    assert abs(g - opt) < 1e-9 * opt
    # any other multipliers give less
    assert D.dual_value(K, c0 + 1, np.array([c1 - c0, 0.0])).g < opt
    assert D.dual_value(K, c0, np.array([c1 - c0 + 1, 0.0])).g < opt
