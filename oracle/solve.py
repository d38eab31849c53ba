"""Oracle: the AM-AMG-preconditioned FGMRES solve of D x = psi end to end (test infrastructure)."""
from __future__ import annotations

import numpy as np

from .amg import SetupParams, setup, vcycle
from .dirac import dirac_matrix
from .fgmres import fgmres


def solve(U: np.ndarray, m0: float, psi: np.ndarray, prm: SetupParams | None = None,
          restart: int = 20, tol: float = 1e-10, max_iters: int = 10000,
          preconditioned: bool = True, levels=None):
    """Solve D x = psi for one field psi[Nt][Nx][2]; returns (x[Nt][Nx][2], info, levels).

    ``preconditioned=False`` runs plain GMRES(restart) with the same Arnoldi/Givens rules.
    A prebuilt hierarchy can be passed in ``levels``.
    """
    nt, nx = U.shape[1], U.shape[2]
    b = np.ascontiguousarray(psi).reshape(-1).astype(complex)
    if preconditioned:
        prm = prm or SetupParams()
        if levels is None:
            levels = setup(U, m0, prm)
        D = levels[0].A

        def precond(v):
            return vcycle(levels, 0, v, prm)
    else:
        D = dirac_matrix(U, m0)

        def precond(v):
            return v.copy()
    x, info = fgmres(lambda v: D @ v, b, precond, m=restart, tol=tol, max_iters=max_iters)
    return x.reshape(nt, nx, 2), info, levels
