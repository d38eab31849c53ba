"""Oracle: flexible GMRES(m), right-preconditioned (test infrastructure).

The paper uses FGMRES as the outer solver with the multigrid method as preconditioner and
a relative tolerance of 1e-10 (Introduction; Numerical Results).  The paper fixes nothing
else; the reading used here (and by the GPU library):

* restart length m, start x0 = 0 unless given;
* Arnoldi step j: z_j = M v_j, w = D z_j, classical Gram-Schmidt applied twice
  (h = V^H w; w -= V h; h' = V^H w; w -= V h'; h += h'), h_{j+1,j} = ||w||,
  v_{j+1} = w / h_{j+1,j};
* Givens rotation for (a, b) = (H_jj, H_{j+1,j}) after the earlier rotations:
  nu = sqrt(|a|^2 + |b|^2), c = |a| / nu, s = (a / |a|) conj(b) / nu (c = 0, s = 1 if a = 0);
  a rotation maps (x, y) -> (c x + s y, -conj(s) x + c y); g_{j+1} = -conj(s) g_j, g_j = c g_j;
* the cycle ends when |g_{j+1}| <= tol ||b||, when j + 1 = m, on breakdown
  (h_{j+1,j} <= 1e-300 ||b||) or at the iteration cap; then y = R^{-1} g, x += Z y and the
  true residual ||b - D x|| decides convergence (relative to ||b||), else the cycle restarts;
* iterations = Arnoldi steps; history = |g_{j+1}| / ||b|| per step, and the true relative
  residual after each cycle.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla


@dataclass
class SolveInfo:
    iterations: int = 0
    restarts: int = 0
    converged: bool = False
    true_rel_residual: float = np.inf
    history: list = field(default_factory=list)          # (value, is_true_residual)


def givens(a: complex, b: complex):
    if a == 0:
        return 0.0, 1.0 + 0j
    nu = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    c = abs(a) / nu
    s = (a / abs(a)) * np.conj(b) / nu
    return c, s


def fgmres(apply_A, b: np.ndarray, precond, m: int = 20, tol: float = 1e-10,
           max_iters: int = 10000, x0: np.ndarray | None = None):
    """Solve A x = b; returns (x, SolveInfo)."""
    info = SolveInfo()
    x = np.zeros_like(b) if x0 is None else x0.astype(complex).copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0:
        info.converged, info.true_rel_residual = True, 0.0
        return np.zeros_like(b), info
    while True:
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm:
            info.converged, info.true_rel_residual = True, beta / bnorm
            return x, info
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m), dtype=complex)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=complex)
        g = np.zeros(m + 1, dtype=complex)
        g[0] = beta
        k = 0
        for j in range(m):
            z = precond(V[j])
            Z.append(z)
            w = apply_A(z)
            Vm = np.array(V)
            h = Vm.conj() @ w
            w = w - Vm.T @ h
            h2 = Vm.conj() @ w
            w = w - Vm.T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):
                t1 = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                t2 = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j], H[i + 1, j] = t1, t2
            c, s = givens(H[j, j], H[j + 1, j])
            H[j, j] = c * H[j, j] + s * H[j + 1, j]
            H[j + 1, j] = 0.0
            cs[j], sn[j] = c, s
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            info.iterations += 1
            k = j + 1
            info.history.append((abs(g[j + 1]) / bnorm, False))
            if (abs(g[j + 1]) <= tol * bnorm or hn <= 1e-300 * bnorm
                    or info.iterations >= max_iters):
                break
            V.append(w / hn)
        y = sla.solve_triangular(H[:k, :k], g[:k])
        x = x + np.array(Z[:k]).T @ y
        r = b - apply_A(x)
        info.true_rel_residual = np.linalg.norm(r) / bnorm
        info.history.append((info.true_rel_residual, True))
        if info.true_rel_residual <= tol:
            info.converged = True
            return x, info
        if info.iterations >= max_iters:
            return x, info
        info.restarts += 1


def gmres(apply_A, b: np.ndarray, tol: float, max_steps: int):
    """Unpreconditioned GMRES from x0 = 0, one cycle of at most max_steps Arnoldi steps (the
    paper's coarsest-level solver, run there to relative tolerance 0.1; Numerical Results).
    The reading used here (and by the GPU library): the Arnoldi, rotation and stopping rules of
    one FGMRES cycle above with M = I (so z_j = v_j); the cycle stops when |g_{j+1}| <= tol ||b||,
    on breakdown or after max_steps steps, and x = V_k R^{-1} g is returned without a restart or
    a true-residual test.  Returns (x, steps); b = 0 gives x = 0 after no step."""
    n = b.shape[0]
    beta = np.linalg.norm(b)
    if beta == 0:
        return np.zeros_like(b, dtype=complex), 0
    V = np.zeros((max_steps + 1, n), dtype=complex)
    V[0] = b / beta
    R = np.zeros((max_steps, max_steps), dtype=complex)
    cs = np.zeros(max_steps)
    sn = np.zeros(max_steps, dtype=complex)
    g = np.zeros(max_steps + 1, dtype=complex)
    g[0] = beta
    k = 0
    for j in range(max_steps):
        w = apply_A(V[j])
        # classical Gram-Schmidt, applied twice
        h = V[: j + 1].conj() @ w
        w = w - V[: j + 1].T @ h
        h2 = V[: j + 1].conj() @ w
        w = w - V[: j + 1].T @ h2
        h = h + h2
        hn = np.linalg.norm(w)
        col = np.append(h, hn)
        for i in range(j):                       # earlier rotations
            t1 = cs[i] * col[i] + sn[i] * col[i + 1]
            t2 = -np.conj(sn[i]) * col[i] + cs[i] * col[i + 1]
            col[i], col[i + 1] = t1, t2
        c, s = givens(col[j], col[j + 1])
        col[j] = c * col[j] + s * col[j + 1]
        cs[j], sn[j] = c, s
        R[: j + 1, j] = col[: j + 1]
        g[j + 1] = -np.conj(s) * g[j]
        g[j] = c * g[j]
        k = j + 1
        if abs(g[j + 1]) <= tol * beta or hn <= 1e-300 * beta:
            break
        V[j + 1] = w / hn
    y = sla.solve_triangular(R[:k, :k], g[:k])
    return V[:k].T @ y, k

