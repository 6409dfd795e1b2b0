"""The geometric-sum spectral filter (oracle).

Test infrastructure only.  Follows Sec. 3 of the paper:

* Eq. (geo): g_k(U) = sum_{m=0..k} exp(-i m phi) U^m.
* Eq. (geo2): closed form [1 - e^{-i(k+1)phi} U^{k+1}] [1 - e^{-i phi} U]^{-1}.
* Eq. (gkmapping): on the unit circle, g_k(e^{i theta}) =
  (1 - e^{i(k+1)(theta-phi)}) / (1 - e^{i(theta-phi)}), equal to k+1 at
  theta = phi and zero at theta - phi = +-2 pi/(k+1).
* Eq. (poly): a general polynomial sum_m a_m U^m.
"""

from __future__ import annotations

import cmath
import math
from typing import Callable, Sequence

import numpy as np

__all__ = [
    "geometric_sum",
    "polynomial",
    "gk_scalar",
    "gk_dirichlet",
    "gk_spectral",
]


def geometric_sum(matvec: Callable[[np.ndarray], np.ndarray], psi: np.ndarray,
                  k: int, phi: float) -> np.ndarray:
    """Eq. (geo) by its definition: accumulate the terms (e^{-i phi} U)^m psi."""
    if k < 0:
        raise ValueError("k must be >= 0")
    rot = cmath.exp(-1j * phi)
    term = np.array(psi, dtype=np.complex128, copy=True)
    acc = term.copy()
    for _ in range(k):
        term = rot * matvec(term)
        acc = acc + term
    return acc


def polynomial(matvec: Callable[[np.ndarray], np.ndarray], psi: np.ndarray,
               coeffs: Sequence[complex]) -> np.ndarray:
    """Eq. (poly) by its definition: sum_m a_m U^m psi."""
    term = np.array(psi, dtype=np.complex128, copy=True)
    acc = coeffs[0] * term
    for a in coeffs[1:]:
        term = matvec(term)
        acc = acc + a * term
    return acc


def gk_scalar(omega, k: int, phi: float):
    """g_k evaluated at complex numbers omega, as the polynomial's sum rewritten
    with the geometric-series identity (Eq. (geo2) / Eq. (gkmapping)).

    Near z = e^{-i phi} omega = 1 the quotient is replaced by the sum itself.
    """
    om = np.asarray(omega, dtype=np.complex128)
    z = om * cmath.exp(-1j * phi)
    out = np.empty_like(z)
    near = np.abs(1.0 - z) < 1e-3
    far = ~near
    out[far] = (1.0 - z[far] ** (k + 1)) / (1.0 - z[far])
    if np.any(near):
        zn = z[near]
        acc = np.zeros_like(zn)
        t = np.ones_like(zn)
        for _ in range(k + 1):
            acc += t
            t = t * zn
        out[near] = acc
    return out


def gk_dirichlet(theta, k: int, phi: float):
    """Eq. (gkmapping) for points e^{i theta} on the unit circle, written as a
    Dirichlet kernel: e^{i k d/2} sin((k+1) d/2) / sin(d/2), d = theta - phi,
    whose limit at d -> 0 is k + 1."""
    d = np.asarray(theta, dtype=np.float64) - phi
    half = 0.5 * d
    s = np.sin(half)
    num = np.sin((k + 1) * half)
    ratio = np.where(np.abs(s) < 1e-300, float(k + 1), num / np.where(s == 0, 1.0, s))
    return np.exp(1j * k * half) * ratio


def gk_spectral(U: np.ndarray, psi: np.ndarray, k: int, phi: float) -> np.ndarray:
    """g_k(U) psi through the eigendecomposition U = V diag(omega) V^{-1}:
    V diag(g_k(omega)) V^{-1} psi (the filter keeps eigenvectors, Sec. 3)."""
    om, V = np.linalg.eig(U)
    c = np.linalg.solve(V, psi)
    return V @ (gk_scalar(om, k, phi) * c)
