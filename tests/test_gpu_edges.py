"""Edge cases of the HIP paths against the FP64 oracle or a closed form:
columns carrying more units than a wavefront has lanes (the strided unit
loop) and a column block with more units than the batched unit pass
evaluates at once, a batch of one instance (padded to a full tile) against the
single-instance path, the congestion-free case where DCOPF is economic
dispatch (lambda* by bisection, mu stays 0), a two-bus batch with a
single panel column, and a panel too large for the last-level cache (the
passes' nontemporal-load variants)."""
import numpy as np
import pytest

from oracle import dual as D
from paper_2406_13191_amd import synth

pytestmark = pytest.mark.gpu


def _abi():
    from paper_2406_13191_amd import _abi
    return _abi


def crowded_columns(counts=((17, 150), (40, 30), (123, 20))):
    """The 300-bus network with QP units crowded on a few buses (default: 200
    units on three buses, 150, 30 and 20)."""
    _, p = synth.make_network("geo300", 7)
    rng = np.random.default_rng(11)
    gen_bus = np.array([b for b, n in counts for _ in range(n)], np.int32)
    pmax = rng.uniform(10.0, 60.0, gen_bus.size)
    return p.replace(gen_bus=gen_bus, c=rng.uniform(10.0, 60.0, gen_bus.size),
                     q=rng.uniform(0.005, 0.05, gen_bus.size), p_min=np.zeros(gen_bus.size),
                     p_max=pmax)


@pytest.mark.parametrize("precision,rtol", [("fp64", 1e-9), ("fp32", 1e-5)])
@pytest.mark.usefixtures("both_schemes")
def test_units_beyond_a_wavefront_per_column(precision, rtol):
    p = crowded_columns()
    K = D.canonical(p)
    n = 200
    o = D.ascent(K, n, alpha=1e-4, rho=0.99)
    with _abi().DualSolver(p, rule="gdm", alpha=1e-4, rho=0.99, precision=precision) as s:
        assert s.info()["n_cols"] == 3
        s.step(n)
        g = s.gammas(0, n)
        b = s.bound()
    rel = np.abs(g - o.gammas) / np.maximum(np.abs(o.gammas), 1.0)
    print(f"{precision}: worst relative gamma deviation {rel.max():.2e}", flush=True)
    assert rel.max() <= rtol
    assert b == pytest.approx(D.dual_value(K, o.state.lam, o.state.mu).g, rel=max(rtol, 1e-9))


def test_units_beyond_a_wavefront_batched():
    A = _abi()
    p = crowded_columns()
    B = 3
    rng = np.random.default_rng(12)
    Dm = np.tile(p.d, (B, 1)) * rng.uniform(0.9, 1.1, (B, 1))
    Cc = np.tile(p.c, (B, 1)) * rng.uniform(0.95, 1.05, (B, p.n_gen))
    Q = np.tile(p.q, (B, 1))
    net = A.BatchNetwork(p, Dm, Cc, Q, alpha=1e-4, rho=0.99)
    with A.BatchSolver([net]) as b:
        b.step(150)
        g = b.gammas(0, 150)
    for i in range(B):
        o = D.ascent(D.canonical(p.replace(d=Dm[i], c=Cc[i], q=Q[i])), 150, alpha=1e-4, rho=0.99)
        rel = np.abs(g[:, i] - o.gammas) / np.maximum(np.abs(o.gammas), 1.0)
        assert rel.max() <= 1e-4


def test_units_beyond_a_chunk_batched():
    # 1000 units in one column block: the batched unit pass evaluates them in
    # chunks of 768, and the second column's 300 units straddle the boundary
    A = _abi()
    p = crowded_columns(((17, 500), (40, 300), (123, 150), (200, 50)))
    # enough generation for the load: the 1000 units share the same total
    # capacity scaled to the network's load
    p = p.replace(p_max=p.p_max * (1.6 * p.d.sum() / p.p_max.sum()))
    B = 2
    rng = np.random.default_rng(13)
    Dm = np.tile(p.d, (B, 1)) * rng.uniform(0.9, 1.1, (B, 1))
    Cc = np.tile(p.c, (B, 1)) * rng.uniform(0.95, 1.05, (B, p.n_gen))
    Q = np.tile(p.q, (B, 1))
    net = A.BatchNetwork(p, Dm, Cc, Q, alpha=1e-4, rho=0.99)
    with A.BatchSolver([net]) as b:
        b.step(150)
        g = b.gammas(0, 150)
        lam, mu_p, mu_m = b.get_multipliers(0)
    for i in range(B):
        o = D.ascent(D.canonical(p.replace(d=Dm[i], c=Cc[i], q=Q[i])), 150, alpha=1e-4, rho=0.99)
        rel = np.abs(g[:, i] - o.gammas) / np.maximum(np.abs(o.gammas), 1.0)
        print(f"instance {i}: worst relative gamma deviation {rel.max():.2e}", flush=True)
        assert rel.max() <= 1e-4
        assert abs(lam[i] - o.state.lam) <= 1e-4 * max(abs(o.state.lam), 1.0)


@pytest.mark.usefixtures("both_schemes")
def test_batch_of_one_tracks_single_path():
    A = _abi()
    _, p = synth.make_network("geo300q", 7)
    r = synth.STEP_RULES["geo300q"]
    net = A.BatchNetwork(p, p.d[None, :], p.c[None, :], p.q[None, :], alpha=r["alpha"],
                         rho=r["rho"])
    with A.BatchSolver([net]) as b:
        b.step(300)
        gb = b.gammas(0, 300)[:, 0]
    with A.DualSolver(p, rule="gdm", alpha=r["alpha"], rho=r["rho"], precision="fp64") as s:
        s.step(300)
        gs = s.gammas(0, 300)
    rel = np.abs(gb - gs) / np.maximum(np.abs(gs), 1.0)
    print(f"batch of one vs single path: worst relative deviation {rel.max():.2e}", flush=True)
    assert rel.max() <= 1e-4


@pytest.mark.usefixtures("both_schemes")
def test_congestion_free_is_economic_dispatch():
    # limits far above any flow: no line can bind, mu stays exactly 0, and the
    # dual optimum is the economic dispatch price lambda*, found by bisection
    # on sum_g clip((lambda - c_g) / (2 q_g), p_min, p_max) = 1^T d
    _, p = synth.make_network("tiny30", 1)
    rng = np.random.default_rng(13)
    p = p.replace(q=rng.uniform(0.01, 0.05, p.n_gen), f_max=np.full(p.n_line, 1e5))
    Dl = float(np.sum(p.d))

    def supply(lam):
        return float(np.sum(np.clip((lam - p.c) / (2 * p.q), p.p_min, p.p_max)))
    lo, hi = 0.0, 1e4
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if supply(mid) < Dl else (lo, mid)
    lam_star = 0.5 * (lo + hi)
    x = np.clip((lam_star - p.c) / (2 * p.q), p.p_min, p.p_max)
    opt = float(p.c @ x + p.q @ (x * x))
    with _abi().DualSolver(p, rule="gdm", alpha=1e-3, rho=0.9, precision="fp64") as s:
        s.step(3000)
        b, lam, mp, mm = s.bound(want_multipliers=True)
    assert np.all(mp == 0.0) and np.all(mm == 0.0)
    assert lam == pytest.approx(lam_star, rel=1e-6)
    assert b <= opt * (1 + 1e-12)
    assert b == pytest.approx(opt, rel=1e-9)


def test_two_bus_batch_single_column():
    A = _abi()
    net2 = synth.Network(2, np.array([0]), np.array([1]), np.array([10.0]), 0)
    H = synth.ptdf(net2)
    p = synth.Problem(H=H, gen_bus=np.array([0, 0], np.int32), c=np.array([30.0, 45.0]),
                      q=np.zeros(2), p_min=np.zeros(2), p_max=np.array([40.0, 200.0]),
                      d=np.array([0.0, 50.0]), f_max=np.array([80.0]), slack=0)
    Dm = np.array([[0.0, 50.0], [0.0, 70.0]])
    Cc = np.array([[30.0, 45.0], [31.0, 44.0]])
    net = A.BatchNetwork(p, Dm, Cc, None, alpha=1e-3, rho=0.9)
    with A.BatchSolver([net]) as b:
        b.step(100)
        g = b.gammas(0, 100)
        vals = b.bound()
    # merit order (the line, carrying the load behind it, never binds):
    # 40 MW of the cheaper unit, the rest from the other one
    opt = [40.0 * 30.0 + 10.0 * 45.0, 40.0 * 31.0 + 30.0 * 44.0]
    for i in range(2):
        K = D.canonical(p.replace(d=Dm[i], c=Cc[i]))
        o = D.ascent(K, 100, alpha=1e-3, rho=0.9)
        np.testing.assert_allclose(g[:, i], o.gammas, rtol=1e-6, atol=1e-6)
        assert vals[i] <= opt[i] * (1 + 1e-12)        # weak duality


@pytest.mark.usefixtures("both_schemes")
def test_panel_beyond_the_last_level_cache():
    # the FP64 all-bus panel of the 4600-bus network: its two orientations
    # (436 MB) exceed the 256 MiB last-level cache, so the two-pass scheme
    # streams both with nontemporal loads; the read-once scheme reads one
    # orientation (217 MB, plain loads) and 9 chunks per lane per row
    _, p = synth.make_network("bus4600", 4600)
    nl, nb = p.H.shape
    assert 2 * nl * nb * 8 > 256 * 2 ** 20
    r = synth.STEP_RULES["bus4600"]
    K = D.canonical(p)
    n = 30
    o = D.ascent(K, n, alpha=r["alpha"], rho=r["rho"])
    with _abi().DualSolver(p, rule="gdm", alpha=r["alpha"], rho=r["rho"], precision="fp64",
                           panel="allbus") as s:
        s.step(n)
        g = s.gammas(0, n)
        b = s.bound()
    rel = np.abs(g - o.gammas) / np.maximum(np.abs(o.gammas), 1.0)
    print(f"all-bus FP64 panel: worst relative gamma deviation {rel.max():.2e}", flush=True)
    assert rel.max() <= 1e-9
    assert b == pytest.approx(D.dual_value(K, o.state.lam, o.state.mu).g, rel=1e-9)


@pytest.mark.parametrize("name,precision,rtol", [("geo300q", "fp32", 1e-6),
                                                  ("geo300", "fp64", 1e-10),
                                                  ("bus2000", "fp64", 1e-10)])
def test_schemes_agree(name, precision, rtol):
    """Two-pass and read-once iterations: the same trajectory (FP64: to
    rounding; FP32 compared on a QP, whose inner minimiser is continuous, as
    the two schemes sum P^T v in different orders), and each scheme is
    bitwise reproducible."""
    A = _abi()
    p = synth.make_problem(name, 7) if name.startswith("geo") else synth.config_problem(name)
    r = synth.STEP_RULES[name]
    kw = dict(rule="gdm", alpha=r["alpha"], rho=r["rho"], precision=precision)
    g = {}
    for scheme in ("two_pass", "read_once", "read_once"):
        with A.DualSolver(p, scheme=scheme, graph_iters=20, **kw) as s:
            s.step(60)
            g.setdefault(scheme, []).append(s.gammas(0, 60))
    np.testing.assert_array_equal(g["read_once"][0], g["read_once"][1])
    np.testing.assert_allclose(g["read_once"][0], g["two_pass"][0], rtol=rtol, atol=rtol)


def test_read_once_nontemporal_panel_and_width_limit():
    """The FP32 all-bus panel of the 10,000-bus network (508 MB, beyond the
    last-level cache: nontemporal loads, 10 chunks per lane and wavefront)
    on the read-once scheme: one step from a random state matches the FP64
    oracle's step (every unit is quadratic, so the inner minimiser is
    continuous) to 1e-5 (floor 1e-3 max c).  The FP64 all-bus panel (10,000
    columns) is wider than read-once rows allow, which create rejects when
    that scheme is asked for."""
    A = _abi()
    _, p = synth.make_network("bus10000", 10000)
    r = synth.STEP_RULES["bus10000"]
    K = D.canonical(p)
    assert np.all(K.M > 0)
    nl = K.n_line
    rng = np.random.default_rng(5)
    st = D.AscentState.cold(nl)
    st.t = 9
    st.lam = float(rng.uniform(10, 60))
    st.mu = rng.exponential(2.0, 2 * nl) * (rng.random(2 * nl) < 0.2)
    st.v_mu = rng.normal(0, 0.2, 2 * nl)
    st.v_lam = float(rng.normal(0, 1))
    st1 = D.gdm_update(st, D.dual_value(K, st.lam, st.mu), r["alpha"], r["rho"])
    buf = np.concatenate([[st.t, st.lam, st.v_lam, 0.0, 0.0], st.mu[:nl], st.mu[nl:],
                          st.v_mu[:nl], st.v_mu[nl:], np.zeros(2 * nl)])
    with A.DualSolver(p, rule="gdm", alpha=r["alpha"], rho=r["rho"], precision="fp32",
                      panel="allbus", scheme="read_once") as s:
        assert s.info()["n_cols"] == p.n_bus
        s.set_state(buf)
        s.step(1)
        got = s.split_state(s.get_state())
    floor = 1e-3 * K.c.max()
    scale = max(np.abs(st1.mu).max(), floor)
    err = max(np.abs(got["mu_p"] - st1.mu[:nl]).max(), np.abs(got["mu_m"] - st1.mu[nl:]).max())
    print(f"read-once FP32 all-bus 10,000-bus panel: one-step mu error / scale "
          f"{err / scale:.2e}", flush=True)
    assert err <= 1e-5 * scale
    assert abs(got["lam"] - st1.lam) <= 1e-5 * max(abs(st1.lam), floor)
    with pytest.raises(A.DcopfError) as e:
        A.DualSolver(p, rule="gdm", alpha=r["alpha"], rho=r["rho"], precision="fp64",
                     panel="allbus", scheme="read_once")
    assert e.value.status == -1 and "too wide" in str(e.value)
