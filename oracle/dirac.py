"""Oracle: the two-dimensional Wilson-Dirac operator of the Schwinger model (test infrastructure).

Paper, Introduction / Schwinger Model subsection: the lattice is
Lambda = {(n_t, n_x)}, 0 <= n_t < N_t, 0 <= n_x < N_x, and

    D[n, m] = (m0 + 2) delta_{n,m}
              - 1/2 sum_mu [ (1 - sigma_mu) U_mu(n) delta_{n+mu, m}
                            + (1 + sigma_mu) U_mu(n - mu)^* delta_{n-mu, m} ]

with sigma_0 = [[0, 1], [1, 0]], sigma_1 = [[0, -i], [i, 0]] and
sigma_3 = i sigma_0 sigma_1 = diag(-1, 1).  Fermion fields are periodic in space and
antiperiodic in time: psi(N_t, x) = -psi(0, x).

Readings (the paper does not fix them):
* mu = 0 is the time direction (the paper writes n = (n_t, n_x) and lists sigma_0 first).
* the antiperiodic sign is -1 on the forward hop out of t = N_t - 1 and on the backward
  hop out of t = 0; the links themselves are periodic.

Indexing: site index n = t * N_x + x, degree of freedom 2 * n + spin.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

SIGMA0 = np.array([[0, 1], [1, 0]], dtype=complex)
SIGMA1 = np.array([[0, -1j], [1j, 0]], dtype=complex)
SIGMA = (SIGMA0, SIGMA1)
SIGMA3 = 1j * SIGMA0 @ SIGMA1          # diag(-1, +1)
EYE2 = np.eye(2, dtype=complex)


def dirac_matrix(U: np.ndarray, m0: float) -> sp.csr_matrix:
    """Sparse D for links U[mu, t, x] (complex) and bare mass m0, built entry by entry.

    Duplicate entries are summed, so lattices with N = 2 in a direction (where the
    forward and the backward neighbour coincide) come out right as well.
    """
    nt, nx = U.shape[1], U.shape[2]
    T, X = np.meshgrid(np.arange(nt), np.arange(nx), indexing="ij")
    site = (T * nx + X).ravel()
    rows, cols, vals = [], [], []
    for a in range(2):
        rows.append(2 * site + a)
        cols.append(2 * site + a)
        vals.append(np.full(site.size, m0 + 2.0, dtype=complex))
    for mu in range(2):
        if mu == 0:
            fwd = (((T + 1) % nt) * nx + X).ravel()
            bwd = (((T - 1) % nt) * nx + X).ravel()
            s_fwd = np.where(T == nt - 1, -1.0, 1.0).ravel()
            s_bwd = np.where(T == 0, -1.0, 1.0).ravel()
            u_bwd = np.conj(U[0][(T - 1) % nt, X]).ravel()
        else:
            fwd = (T * nx + (X + 1) % nx).ravel()
            bwd = (T * nx + (X - 1) % nx).ravel()
            s_fwd = np.ones(site.size)
            s_bwd = np.ones(site.size)
            u_bwd = np.conj(U[1][T, (X - 1) % nx]).ravel()
        u_fwd = U[mu].ravel()
        proj_f = EYE2 - SIGMA[mu]
        proj_b = EYE2 + SIGMA[mu]
        for a in range(2):
            for b in range(2):
                if proj_f[a, b] != 0:
                    rows.append(2 * site + a)
                    cols.append(2 * fwd + b)
                    vals.append(-0.5 * proj_f[a, b] * s_fwd * u_fwd)
                if proj_b[a, b] != 0:
                    rows.append(2 * site + a)
                    cols.append(2 * bwd + b)
                    vals.append(-0.5 * proj_b[a, b] * s_bwd * u_bwd)
    n = 2 * nt * nx
    D = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return D.tocsr()


def sigma3_full(nsites: int) -> sp.csr_matrix:
    """sigma_3 acting on every site: diag(-1, +1, -1, +1, ...)."""
    return sp.diags(np.tile(np.array([-1.0, 1.0]), nsites)).tocsr()


def field_to_vector(psi: np.ndarray) -> np.ndarray:
    """[Nt][Nx][2] complex field -> flat vector with dof 2 * (t * Nx + x) + spin."""
    return np.ascontiguousarray(psi).reshape(-1)


def vector_to_field(v: np.ndarray, nt: int, nx: int) -> np.ndarray:
    return v.reshape(nt, nx, 2)


def dirac_at_sites(U: np.ndarray, m0: float, psi: np.ndarray, ts: np.ndarray,
                   xs: np.ndarray) -> np.ndarray:
    """(D psi)(n) at the sites n = (ts[k], xs[k]) only, from the same definition as
    dirac_matrix, for lattices too large to assemble D: returns [len(ts)][2] complex.

    Each site takes its two forward and two backward neighbours with the spin projectors
    (1 -/+ sigma_mu), the links U_mu(n) and U_mu(n - mu)^*, and the time-boundary sign."""
    nt, nx = U.shape[1], U.shape[2]
    ts = np.asarray(ts)
    xs = np.asarray(xs)
    out = (m0 + 2.0) * psi[ts, xs]
    for mu in range(2):
        if mu == 0:
            tf, xf, tb, xb = (ts + 1) % nt, xs, (ts - 1) % nt, xs
            sf = np.where(ts == nt - 1, -1.0, 1.0)
            sb = np.where(ts == 0, -1.0, 1.0)
        else:
            tf, xf, tb, xb = ts, (xs + 1) % nx, ts, (xs - 1) % nx
            sf = sb = np.ones(ts.shape)
        fwd = (sf * U[mu][ts, xs])[:, None] * psi[tf, xf]
        bwd = (sb * np.conj(U[mu][tb, xb]))[:, None] * psi[tb, xb]
        out = out - 0.5 * (fwd @ (EYE2 - SIGMA[mu]).T + bwd @ (EYE2 + SIGMA[mu]).T)
    return out
