"""Entanglement entropy of eigenstates and Page's value (oracle).

Test infrastructure only.  Sec. 5, Eq. (ee): S_A = -sum_i s_i^2 ln s_i^2, where
s_i are the singular values of the state reshaped as a 2^{L_A} x 2^{L-L_A}
matrix (left block = sites 1..L_A).  Eq. (page): the random pure-state average
for L_A <= L_B, sum_{k=2^{L_B}+1}^{2^L} 1/k - (2^{L_A}-1)/2^{L_B+1}.
"""

from __future__ import annotations

import numpy as np

__all__ = ["entropy", "page"]


def entropy(psi: np.ndarray, L: int, LA: int) -> float:
    """Von Neumann entropy of the left L_A sites of the normalised state psi."""
    M = np.asarray(psi, dtype=np.complex128).reshape(2 ** LA, 2 ** (L - LA))
    s = np.linalg.svd(M, compute_uv=False)
    p = s * s
    p = p[p > 0]
    return float(-(p * np.log(p)).sum())


def page(L: int, LA: int) -> float:
    """Eq. (page), with L_A and L_B swapped when L_A > L_B (S_A = S_B)."""
    LB = L - LA
    if LA > LB:
        LA, LB = LB, LA
    k = np.arange(2 ** LB + 1, 2 ** L + 1, dtype=np.float64)
    return float((1.0 / k).sum() - (2 ** LA - 1) / 2 ** (LB + 1))
