"""Orthogonalisation step of the Arnoldi process (oracle).

Test infrastructure only.  Arnoldi (Sec. 4, Eq. (arnoldi)) builds an
orthonormal basis V of the Krylov space of g_k(U), with H_m = V^dagger g_k(U) V
upper Hessenberg.  Each new filtered vector w is orthogonalised against the
current basis; the oracle does this by classical Gram-Schmidt applied twice
(the second pass removes what rounding left behind):

    h1 = V^H w,  w1 = w - V h1,  h2 = V^H w1,  w2 = w1 - V h2,
    H[:, j] = h1 + h2,  beta = ||w2||,  v_{j+1} = w2 / beta.
"""

from __future__ import annotations

from typing import Tuple

import numpy as np

__all__ = ["cgs2"]


def cgs2(V: np.ndarray, w: np.ndarray) -> Tuple[np.ndarray, float, np.ndarray]:
    """Returns (h[j], beta, v_next) for basis V[d, j] and vector w[d]."""
    h1 = V.conj().T @ w
    w1 = w - V @ h1
    h2 = V.conj().T @ w1
    w2 = w1 - V @ h2
    beta = float(np.linalg.norm(w2))
    v = w2 / beta if beta > 0 else w2
    return h1 + h2, beta, v
