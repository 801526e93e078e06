"""CPU FP64 oracle for the projected dual ascent of DCOPF (arXiv 2406.13191).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The
GPU path never calls, links or imports this package, and this package never
imports the GPU path.  Inputs come from ``paper_2406_13191_amd.synth`` (input
construction only) or are built by the caller.

Modules
  dual   - canonical form (eq. general), the dual function g (eqs. LP dual and
           final QP dual, Section 3), its supergradient, the paper's
           normalised forms (Appendix A1/A2), and the ascent rules (Algorithm 1
           gradient with momentum; Adam and AdaGrad of Section 3.3).
  ref    - references that pin the oracle: vertex enumeration (LP), KKT
           active-set enumeration (QP), economic dispatch, HiGHS optima in the
           PTDF and in the bus-angle (reduced-B) form, a QP certificate.
  mlp    - FP64 reference of the warm-start network (forward/backward, Adam).

Parity status: every function here is pinned by tests/test_oracle_*.py
against closed forms, brute force or an external solver, except the ascent
trajectory itself, which the paper prints no numbers for; it is pinned by
convergence to the HiGHS optimum and by step identities instead.
"""
