"""Parity of the single-instance HIP path with the FP64 oracle.

One step from an identical state (every rule, both precisions, both panel
modes), the exact FP64 bound at full sizes, full FP64 trajectories, FP32
trajectories of the continuous (QP) map, determinism, checkpoint / resume,
graph vs direct launches, the solve loop, and edge shapes.
"""
import math
import sys

import numpy as np
import pytest

from oracle import dual as D
from oracle import ref
from paper_2406_13191_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("both_schemes")]

U32 = 2.0 ** -24


def _abi():
    from paper_2406_13191_amd import _abi
    return _abi


_PROBS = {}


def prob(name, seed=None):
    key = (name, seed)
    if key not in _PROBS:
        print(f"[gen] {name} seed={seed}", flush=True)
        _PROBS[key] = synth.config_problem(name) if seed is None else synth.make_problem(name, seed)
    return _PROBS[key]


def to_buf(st: D.AscentState, rule: str, nl: int):
    vel_l = st.v_lam if rule == "gdm" else st.m_lam
    vel = st.v_mu if rule == "gdm" else st.m_mu
    return np.concatenate([[st.t, st.lam, vel_l, st.s_lam, 0.0], st.mu[:nl], st.mu[nl:],
                           vel[:nl], vel[nl:], st.s_mu[:nl], st.s_mu[nl:]])


def rand_state(K, rng, rule, scale):
    nl = K.n_line
    st = D.AscentState.cold(nl)
    st.lam = float(rng.uniform(10, 60))
    st.mu = rng.exponential(scale, 2 * nl) * (rng.random(2 * nl) < 0.2)
    st.v_lam = float(rng.normal(0, 1))
    st.v_mu = rng.normal(0, scale * 0.1, 2 * nl)
    st.m_lam = st.v_lam
    st.m_mu = st.v_mu.copy()
    st.s_lam = float(rng.uniform(1, 100))
    st.s_mu = rng.uniform(0, 1e4, 2 * nl)
    st.t = int(rng.integers(0, 50))
    return st


def fp32_col_bound(K, mu, n):
    """Error bound of the FP32 product w = P^T v per generator: each lane
    accumulates ~n/64 terms in sequence, then a 6-level butterfly, plus the
    FP32 rounding of v and of P (first order)."""
    nl = K.n_line
    v = np.abs(mu[:nl] - mu[nl:])
    HC = np.abs(K.C[:nl])
    return (n / 64 + 10) * U32 * (HC.T @ v)


def near_tie_free(K, st, tau):
    ev = D.dual_value(K, st.lam, st.mu)
    lin = K.M == 0
    return np.all(np.abs(ev.a[lin]) > tau[lin])


UPDATES = {
    "gdm": lambda st, ev, r: D.gdm_update(st, ev, r["alpha"], r["rho"]),
    "gdm_literal": lambda st, ev, r: D.gdm_update(st, ev, r["alpha"], r["rho"], literal=True),
    "adam": lambda st, ev, r: D.adam_update(st, ev, 0.05, 0.9, 0.99, 1e-8),
    "adagrad": lambda st, ev, r: D.adagrad_update(st, ev, 0.5, 1e-8),
}


def solver_for(p, rule_key, precision, panel="genbus", name=None, **extra):
    r = synth.STEP_RULES[name]
    rule = "gdm" if rule_key.startswith("gdm") else rule_key
    kw = dict(rule=rule, alpha=r["alpha"], rho=r["rho"], literal=rule_key == "gdm_literal",
              precision=precision, panel=panel)
    if rule == "adam":
        kw.update(alpha=0.05, beta1=0.9, beta2=0.99, eps=1e-8)
    if rule == "adagrad":
        kw.update(alpha=0.5, eps=1e-8)
    kw.update(extra)
    return _abi().DualSolver(p, **kw)


def compare_state(s, st_ref, rule, nl, rtol, atol_mu):
    got = s.split_state(s.get_state())
    mu_ref_p, mu_ref_m = st_ref.mu[:nl], st_ref.mu[nl:]
    scale = max(np.abs(st_ref.mu).max(), 1.0)
    np.testing.assert_allclose(got["mu_p"], mu_ref_p, rtol=rtol, atol=atol_mu * scale)
    np.testing.assert_allclose(got["mu_m"], mu_ref_m, rtol=rtol, atol=atol_mu * scale)
    assert got["lam"] == pytest.approx(st_ref.lam, rel=rtol, abs=atol_mu)
    vel = st_ref.v_mu if rule == "gdm" else st_ref.m_mu
    np.testing.assert_allclose(np.concatenate([got["v_p"], got["v_m"]]), vel, rtol=rtol,
                               atol=atol_mu * max(np.abs(vel).max(), 1.0))
    assert got["k"] == st_ref.t


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["tiny30", "geo300", "geo300q", "bus2000"])
@pytest.mark.parametrize("rule_key", ["gdm", "gdm_literal", "adam", "adagrad"])
@pytest.mark.parametrize("panel", ["genbus", "allbus"])
def test_one_step_fp64(name, rule_key, panel):
    p = prob(name, 7) if name.startswith("geo") else prob(name)
    K = D.canonical(p)
    rng = np.random.default_rng(11)
    rule = "gdm" if rule_key.startswith("gdm") else rule_key
    tau = np.full(K.c.size, 1e-9 * K.c.max())
    for _ in range(20):
        st = rand_state(K, rng, rule, 5.0)
        if near_tie_free(K, st, tau):
            break
    ev = D.dual_value(K, st.lam, st.mu)
    st1 = UPDATES[rule_key](st, ev, synth.STEP_RULES[name])
    with solver_for(p, rule_key, "fp64", panel, name=name) as s:
        s.set_state(to_buf(st, rule, K.n_line))
        s.step(1)
        compare_state(s, st1, rule, K.n_line, rtol=1e-10, atol_mu=1e-11)
        got = s.split_state(s.get_state())
        g = s.gammas(st.t, 1)[0]
        nl = K.n_line
        mu_err = max(np.abs(got["mu_p"] - st1.mu[:nl]).max(), np.abs(got["mu_m"] - st1.mu[nl:]).max())
        print(f"fp64 {name} {rule_key} {panel}: mu err / max mu "
              f"{mu_err / max(np.abs(st1.mu).max(), 1e-300):.1e}, lambda rel err "
              f"{abs(got['lam'] - st1.lam) / max(abs(st1.lam), 1e-300):.1e}, gamma rel err "
              f"{abs(g - ev.g) / abs(ev.g):.1e}", flush=True)
        assert g == pytest.approx(ev.g, rel=1e-12)


@pytest.mark.parametrize("name", ["geo300", "geo300q", "bus2000", "bus4600", "bus10000"])
@pytest.mark.parametrize("rule_key", ["gdm", "adam"])
def test_one_step_fp32(name, rule_key):
    """FP32 products: multipliers within 1e-5 relative of the oracle (floor
    1e-3 max c), and within the derived FP32 product error bound."""
    p = prob(name, 7) if name.startswith("geo") else prob(name)
    K = D.canonical(p)
    rng = np.random.default_rng(5)
    rule = rule_key
    for _ in range(30):
        st = rand_state(K, rng, rule, 2.0)
        tau = 2 * fp32_col_bound(K, st.mu, K.n_line)
        if near_tie_free(K, st, tau):
            break
    else:
        pytest.fail("no state without near ties")
    ev = D.dual_value(K, st.lam, st.mu)
    st1 = UPDATES[rule_key](st, ev, synth.STEP_RULES[name])
    with solver_for(p, rule_key, "fp32", name=name) as s:
        s.set_state(to_buf(st, rule, K.n_line))
        s.step(1)
        got = s.split_state(s.get_state())
    nl = K.n_line
    floor = 1e-3 * K.c.max()
    tol_a17 = 1e-5 * max(np.abs(st1.mu).max(), floor)
    err = max(np.abs(got["mu_p"] - st1.mu[:nl]).max(), np.abs(got["mu_m"] - st1.mu[nl:]).max())
    lam_err = abs(got["lam"] - st1.lam)
    print(f"fp32 {name} {rule_key}: mu err / scale {err / max(np.abs(st1.mu).max(), floor):.1e}, "
          f"lambda err / scale {lam_err / max(abs(st1.lam), floor):.1e}", flush=True)
    assert err <= tol_a17, (err, tol_a17)
    assert lam_err <= 1e-5 * max(abs(st1.lam), floor)
    if rule_key == "gdm":
        # line residual error: FP32 F = P x with ~n_cols/64 sequential terms
        x = ev.x
        HC = np.abs(K.C[:nl])
        n_cols = len(np.unique(p.gen_bus))
        # a QP unit's p* = clip(-r / 2q) moves by up to |dw| / 2q with the
        # FP32 error dw of its reduced cost; a linear unit does not move
        # (no near ties)
        dw = fp32_col_bound(K, st.mu, K.n_line)
        dp = np.where(K.M > 0, dw / (2 * np.where(K.M > 0, K.M, 1.0)), 0.0)
        f_err = ((n_cols / 64 + 10) * U32 * (HC @ np.abs(x)) + HC @ dp
                 + 1e-9 * np.abs(p.f_max))
        a = synth.STEP_RULES[name]["alpha"]
        assert np.all(np.abs(got["mu_p"] - st1.mu[:nl]) <= a * f_err + 1e-12 * np.abs(st1.mu[:nl]))


@pytest.mark.parametrize("name", ["tiny30", "geo300", "geo300q", "bus2000", "bus4600", "bus10000"])
def test_exact_bound_matches_oracle(name):
    """The exact FP64 bound at a given iterate equals the oracle's dual value
    to 1e-7 relative (FP64 throughout: expect ~1e-13)."""
    p = prob(name, 7) if name.startswith("geo") else prob(name)
    K = D.canonical(p)
    rng = np.random.default_rng(3)
    st = rand_state(K, rng, "gdm", 3.0)
    g_ref = D.dual_value(K, st.lam, st.mu).g
    for prec in ("fp32", "fp64"):
        if name == "bus10000" and prec == "fp64":
            continue
        with solver_for(p, "gdm", prec, name=name) as s:
            s.set_state(to_buf(st, "gdm", K.n_line))
            v, lam, mp, mm = s.bound(want_multipliers=True)
        print(f"exact bound {name} ({prec} loop): rel err {abs(v - g_ref) / abs(g_ref):.1e}",
              flush=True)
        assert abs(v - g_ref) <= 1e-7 * abs(g_ref), (v, g_ref)
        assert abs(v - g_ref) <= 1e-11 * abs(g_ref)
        np.testing.assert_array_equal(mp, st.mu[:K.n_line])


def test_trajectory_fp64_tiny30():
    """C1 (30 buses, FP64 products, 5000 iterations): the whole monitor
    trajectory and the final multipliers match the oracle."""
    p = prob("tiny30")
    K = D.canonical(p)
    r = synth.STEP_RULES["tiny30"]
    ref_res = D.ascent(K, 5000, alpha=r["alpha"], rho=r["rho"])
    with solver_for(p, "gdm", "fp64", name="tiny30", graph_iters=50) as s:
        s.step(5000)
        gam = s.gammas(0, 5000)
        got = s.split_state(s.get_state())
    rel = np.abs(gam - ref_res.gammas) / np.maximum(np.abs(ref_res.gammas), 1.0)
    first_bad = int(np.argmax(rel > 1e-9)) if np.any(rel > 1e-9) else None
    print("max rel gamma diff", rel.max(), "first divergence", first_bad, flush=True)
    assert first_bad is None
    nl = K.n_line
    np.testing.assert_allclose(got["mu_p"], ref_res.state.mu[:nl], rtol=1e-8, atol=1e-8)
    np.testing.assert_allclose(got["mu_m"], ref_res.state.mu[nl:], rtol=1e-8, atol=1e-8)
    assert got["lam"] == pytest.approx(ref_res.state.lam, rel=1e-9)


@pytest.mark.parametrize("rule", ["adam", "adagrad"])
def test_trajectory_fp64_adaptive_rules(rule):
    p = prob("tiny30")
    K = D.canonical(p)
    kw = dict(alpha=0.05, beta1=0.9, beta2=0.99) if rule == "adam" else dict(alpha=0.5)
    ref_res = D.ascent(K, 1000, rule=rule, eps=1e-8, **kw)
    with _abi().DualSolver(p, rule=rule, precision="fp64", eps=1e-8, **kw) as s:
        s.step(1000)
        gam = s.gammas(0, 1000)
    np.testing.assert_allclose(gam, ref_res.gammas, rtol=1e-9)


def test_trajectory_fp32_qp():
    """The QP inner minimiser is continuous, so FP32-product trajectories stay
    close to the FP64 oracle over many iterations (here 300, geo300q)."""
    p = prob("geo300q", 7)
    K = D.canonical(p)
    r = synth.STEP_RULES["geo300q"]
    ref_res = D.ascent(K, 300, alpha=r["alpha"], rho=r["rho"])
    with solver_for(p, "gdm", "fp32", name="geo300q") as s:
        s.step(300)
        gam = s.gammas(0, 300)
        got = s.split_state(s.get_state())
    nl = K.n_line
    rel = np.abs(gam - ref_res.gammas) / np.maximum(np.abs(ref_res.gammas), 1.0)
    print("max rel gamma diff (fp32 qp)", rel.max(), flush=True)
    assert rel.max() <= 1e-6
    scale = max(np.abs(ref_res.state.mu).max(), 1e-3 * K.c.max())
    err = max(np.abs(got["mu_p"] - ref_res.state.mu[:nl]).max(),
              np.abs(got["mu_m"] - ref_res.state.mu[nl:]).max())
    print("mu err / scale", err / scale, flush=True)
    assert err <= 1e-5 * scale


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_deterministic_graph_and_resume(precision):
    p = prob("geo300", 7)
    kw = dict(rule="gdm", alpha=3e-4, rho=0.99, precision=precision)
    A = _abi()
    with A.DualSolver(p, **kw) as s1, A.DualSolver(p, graph_iters=16, **kw) as s2:
        s1.step(200)
        s2.step(200)
        a, b = s1.get_state(), s2.get_state()
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(s1.gammas(0, 200), s2.gammas(0, 200))
        s1.step(150)
        full = s1.get_state()
    with A.DualSolver(p, **kw) as s3:
        s3.set_state(a)
        s3.step(150)
        np.testing.assert_array_equal(s3.get_state(), full)


@pytest.mark.parametrize("name,precision,rtol", [("geo300q", "fp32", 1e-6),
                                                  ("geo300", "fp64", 1e-10)])
def test_panel_modes_agree(name, precision, rtol):
    """Generator-bus panel vs the full PTDF: the same dual values.  FP32 is
    compared on the QP, whose inner minimiser is continuous (on an LP the two
    panels' different FP32 rounding can flip a bang-bang unit and the
    trajectories part legitimately); FP64 on the LP."""
    p = prob(name, 7)
    A = _abi()
    r = synth.STEP_RULES[name]
    kw = dict(rule="gdm", alpha=r["alpha"], rho=r["rho"], precision=precision)
    with A.DualSolver(p, panel="genbus", **kw) as s1, A.DualSolver(p, panel="allbus", **kw) as s2:
        assert s2.info()["n_cols"] == p.n_bus
        s1.step(50)
        s2.step(50)
        g1, g2 = s1.gammas(0, 50), s2.gammas(0, 50)
        np.testing.assert_allclose(g1, g2, rtol=rtol, atol=rtol)
        assert s1.bound() == pytest.approx(s2.bound(), rel=rtol)


def test_solve_reaches_gap_tiny30():
    net, p = synth.make_network("tiny30", 1)
    opt = ref.opt_btheta(net, p)["opt"]
    with solver_for(p, "gdm", "fp64", name="tiny30", graph_iters=50) as s:
        r = s.solve(opt=opt, gap_tol=1e-3, max_iters=5000, check_every=100)
    assert r["status"] == 1
    assert r["bound"] <= opt * (1 + 1e-12)
    assert r["gap"] <= 1e-3
    assert r["iter_of_bound"] % 100 == 0


def test_stop_rule_and_best():
    p = prob("tiny30")
    with solver_for(p, "gdm", "fp64", name="tiny30") as s:
        r = s.solve(dgamma_tol=1e12, max_iters=1000, check_every=10)
        assert r["status"] == 2 and r["iters"] == 10
        v, k = s.best()
        assert v == r["bound"] and k == 10


def test_edge_two_bus_single_generator():
    # one generator at the slack, one line, one load: n_cols = 1, ragged tiles
    net = synth.Network(2, np.array([0]), np.array([1]), np.array([10.0]), 0)
    H = synth.ptdf(net)
    p = synth.Problem(H=H, gen_bus=np.array([0], np.int32), c=np.array([30.0]), q=np.zeros(1),
                      p_min=np.zeros(1), p_max=np.array([200.0]), d=np.array([0.0, 50.0]),
                      f_max=np.array([80.0]), slack=0)
    K = D.canonical(p)
    ref_res = D.ascent(K, 200, alpha=1e-3, rho=0.9)
    with _abi().DualSolver(p, rule="gdm", alpha=1e-3, rho=0.9, precision="fp64") as s:
        s.step(200)
        np.testing.assert_allclose(s.gammas(0, 200), ref_res.gammas, rtol=1e-12)
        assert s.bound() <= 30.0 * 50.0 * (1 + 1e-12)


def test_zero_iterations_and_cold_bound():
    p = prob("tiny30")
    K = D.canonical(p)
    with solver_for(p, "gdm", "fp32", name="tiny30") as s:
        s.step(0)
        assert s.bound() == pytest.approx(float(K.c @ K.lo), abs=1e-9)
        assert s.info()["iters"] == 0


def test_time_phases_leaves_iterate_unchanged():
    p = prob("geo300", 7)
    with solver_for(p, "gdm", "fp32", name="geo300") as s:
        s.step(7)
        a = s.get_state()
        ms = s.time_phases(20)
        assert ms[0] > 0 and ms[1] > 0
        np.testing.assert_array_equal(s.get_state(), a)
        s.step(5)
        with solver_for(p, "gdm", "fp32", name="geo300") as s2:
            s2.step(12)
            np.testing.assert_array_equal(s.get_state(), s2.get_state())


# ---------------------------------------------------------------------------
# Step decay (alpha_t = alpha / (1 + decay t), t the state's counter)
# ---------------------------------------------------------------------------
DECAY = 0.02


@pytest.mark.parametrize("rule_key", ["gdm", "gdm_literal", "adam", "adagrad"])
def test_one_step_decay_fp64(rule_key):
    """One step at a random counter t > 0 with step decay, FP64 products:
    the device takes the oracle's step alpha / (1 + decay t)."""
    name = "geo300"
    p = prob(name, 7)
    K = D.canonical(p)
    rng = np.random.default_rng(29)
    rule = "gdm" if rule_key.startswith("gdm") else rule_key
    tau = np.full(K.c.size, 1e-9 * K.c.max())
    for _ in range(20):
        st = rand_state(K, rng, rule, 5.0)
        if near_tie_free(K, st, tau) and st.t > 0:
            break
    ev = D.dual_value(K, st.lam, st.mu)
    r = dict(synth.STEP_RULES[name])
    base_alpha = {"adam": 0.05, "adagrad": 0.5}.get(rule, r["alpha"])
    a_t = D.step_size(base_alpha, DECAY, st.t)
    if rule_key == "gdm":
        st1 = D.gdm_update(st, ev, a_t, r["rho"])
    elif rule_key == "gdm_literal":
        st1 = D.gdm_update(st, ev, a_t, r["rho"], literal=True)
    elif rule == "adam":
        st1 = D.adam_update(st, ev, a_t, 0.9, 0.99, 1e-8)
    else:
        st1 = D.adagrad_update(st, ev, a_t, 1e-8)
    with solver_for(p, rule_key, "fp64", name=name, decay=DECAY) as s:
        s.set_state(to_buf(st, rule, K.n_line))
        s.step(1)
        compare_state(s, st1, rule, K.n_line, rtol=1e-10, atol_mu=1e-11)
        got = s.split_state(s.get_state())
    # the decayed step differs measurably from the undecayed one
    st_nodecay = UPDATES[rule_key](st, ev, r)
    nl = K.n_line
    moved = np.abs(st_nodecay.mu - st.mu).max()
    assert np.abs(got["mu_p"] - st_nodecay.mu[:nl]).max() + \
        np.abs(got["mu_m"] - st_nodecay.mu[nl:]).max() > 1e-3 * moved
    print(f"decay {rule_key}: t = {st.t}, step {a_t:.3e} vs {base_alpha:.3e}", flush=True)


@pytest.mark.parametrize("rule", ["gdm", "adam", "adagrad"])
def test_trajectory_fp64_decay(rule):
    """Whole FP64 trajectories with step decay match the oracle (30-bus
    network, 1000 iterations)."""
    p = prob("tiny30")
    K = D.canonical(p)
    r = synth.STEP_RULES["tiny30"]
    kw = {"gdm": dict(alpha=r["alpha"], rho=r["rho"]),
          "adam": dict(alpha=0.05, beta1=0.9, beta2=0.99),
          "adagrad": dict(alpha=0.5)}[rule]
    ref_res = D.ascent(K, 1000, rule=rule, eps=1e-8, decay=1e-3, **kw)
    with _abi().DualSolver(p, rule=rule, precision="fp64", eps=1e-8, decay=1e-3,
                           graph_iters=50, **kw) as s:
        s.step(1000)
        gam = s.gammas(0, 1000)
        got = s.split_state(s.get_state())
    rel = np.abs(gam - ref_res.gammas) / np.maximum(np.abs(ref_res.gammas), 1.0)
    print(f"decay trajectory {rule}: max rel gamma diff {rel.max():.2e}", flush=True)
    assert rel.max() <= 1e-9
    assert got["k"] == 1000
    assert got["lam"] == pytest.approx(ref_res.state.lam, rel=1e-9)
