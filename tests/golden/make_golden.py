"""Writes the stored expected values under tests/golden/ from the FP64 oracle
(and the seeded input generator) only.  Run: python tests/golden/make_golden.py

c1_tiny30.json: the 30-bus FP64 configuration (41 lines, 6 generators; GDM,
Algorithm 1 heavy-ball reading, alpha = 1e-4, rho = 0.99, 5000 iterations
from lambda = mu = 0): the dual value gamma_k every 100 iterations, the best
bound and its iteration, the final multipliers, and the HiGHS optimum of
the same instance with the resulting gap (Section 3.3, Section 4's gap).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dual as D  # noqa: E402
from oracle import ref  # noqa: E402
from paper_2406_13191_amd import synth  # noqa: E402

N_ITERS, ALPHA, RHO = 5000, 1e-4, 0.99


def c1():
    net, p = synth.make_network("tiny30", 1)
    K = D.canonical(p)
    res = D.ascent(K, N_ITERS, alpha=ALPHA, rho=RHO)
    opt = ref.opt_btheta(net, p)["opt"]
    mu = res.state.mu
    return dict(
        config="tiny30 seed 1: 30 buses, 41 lines, 6 generators, linear costs; GDM "
               f"heavy-ball alpha={ALPHA} rho={RHO}; {N_ITERS} iterations from zero; FP64",
        n_iters=N_ITERS, alpha=ALPHA, rho=RHO,
        gammas_every_100=[float(g) for g in res.gammas[::100]],
        best=res.best, best_iter=res.best_iter,
        final_lambda=float(res.state.lam),
        final_mu_nonzero=[[int(i), float(mu[i])] for i in range(mu.size) if mu[i] != 0.0],
        opt_highs=opt, gap=(opt - res.best) / abs(opt))


if __name__ == "__main__":
    with open(os.path.join(HERE, "c1_tiny30.json"), "w") as f:
        json.dump(c1(), f, indent=1)
        f.write("\n")
    print("written")
