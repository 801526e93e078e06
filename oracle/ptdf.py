"""FP64 oracle: the PTDF matrix of a network (Section 2, the PTDF form of
eq. DCOPF).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

With the incidence matrix E (line l: +1 at its from bus, -1 at its to bus)
and Omega = diag(b) of the series susceptances, the line flows of a bus
injection vector x (withdrawn at the slack bus) are F = H_a x with

    H_a[:, keep] = Omega E_r (E_r^T Omega E_r)^{-1},   H_a[:, slack] = 0,

where E_r drops the slack column (keep = every other bus) and
B_r = E_r^T Omega E_r is the reduced susceptance matrix (symmetric positive
definite for a connected network with positive susceptances).
"""
from __future__ import annotations

import numpy as np


def incidence(n_bus, fbus, tbus):
    nl = len(fbus)
    E = np.zeros((nl, n_bus))
    E[np.arange(nl), fbus] = 1.0
    E[np.arange(nl), tbus] = -1.0
    return E


def reduced_b(n_bus, fbus, tbus, b, slack):
    """B_r = E_r^T Omega E_r (dense) and the kept bus indices."""
    E = incidence(n_bus, fbus, tbus)
    keep = np.array([i for i in range(n_bus) if i != slack])
    Er = E[:, keep]
    return Er.T @ (np.asarray(b, float)[:, None] * Er), keep, Er


def ptdf(n_bus, fbus, tbus, b, slack) -> np.ndarray:
    """Dense H_a [n_line, n_bus] by a dense solve with B_r."""
    b = np.asarray(b, float)
    Br, keep, Er = reduced_b(n_bus, fbus, tbus, b, slack)
    # H_r^T = B_r^{-1} (Omega E_r)^T  (B_r symmetric)
    Hr = np.linalg.solve(Br, (b[:, None] * Er).T).T
    H = np.zeros((len(fbus), n_bus))
    H[:, keep] = Hr
    return H


def ptdf_rows(n_bus, fbus, tbus, b, slack, lines) -> np.ndarray:
    """Rows `lines` of H_a: row l = b_l (e_f - e_t)^T B_r^{-1} on the kept
    buses, from one sparse factorisation of B_r (for large networks)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    b = np.asarray(b, float)
    fbus, tbus = np.asarray(fbus), np.asarray(tbus)
    nl = len(fbus)
    rows = np.arange(nl)
    E = sp.csr_matrix((np.concatenate([np.ones(nl), -np.ones(nl)]),
                       (np.concatenate([rows, rows]), np.concatenate([fbus, tbus]))),
                      shape=(nl, n_bus))
    keep = np.array([i for i in range(n_bus) if i != slack])
    Er = E[:, keep].tocsc()
    Br = (Er.T @ sp.diags(b) @ Er).tocsc()
    lu = spla.splu(Br)
    R = np.asarray((Er[lines].multiply(b[lines][:, None])).todense()).T   # [n-1, k]
    Z = lu.solve(R)                        # B_r^{-1} (Omega E_r)^T for those lines
    out = np.zeros((len(lines), n_bus))
    out[:, keep] = Z.T
    return out
