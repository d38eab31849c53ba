"""Oracle: critical-mass estimate (test infrastructure).

The paper takes the critical masses of its ensembles from the literature (table of
critical values) and runs at fixed distances |m0 - m_c|.  For the synthetic gauge fields
here m_c is estimated per configuration: D(m0) = D(0) + m0 I, so the smallest real part
of the spectrum of D(m0) is m0 + lambda_min with lambda_min = min Re lambda(D(0)); the
reading used is m_c = -lambda_min, so that m0 = m_c + gap puts the smallest real part of
the spectrum of D(m0) at the gap.  lambda_min is taken from shift-invert Arnoldi around
0 (the k eigenvalues nearest the origin); small lattices are cross-checked by dense eig.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .dirac import dirac_matrix


def critical_mass(U: np.ndarray, k: int = 24, dense: bool = False) -> float:
    D0 = dirac_matrix(U, 0.0)
    if dense:
        vals = np.linalg.eigvals(D0.toarray())
    else:
        vals = spla.eigs(D0.tocsc(), k=min(k, D0.shape[0] - 2), sigma=0.0,
                         return_eigenvectors=False)
    return float(-np.min(vals.real))
