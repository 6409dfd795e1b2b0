"""Eigenpairs of U closest to a target on the unit circle (oracle).

Test infrastructure only.  The problem is the paper's Sec. 3 opening: all n_ev
eigenpairs (omega_n, |n>) of U whose eigenvalue lies closest to
z_tgt = e^{i phi}.  The oracle solves it by full diagonalisation (LAPACK zgeev
via numpy, the paper's full-diagonalisation baseline of Sec. 5) and ranks
eigenvalues by arc distance |arg(omega e^{-i phi})|.  Eigenvalues are recovered
as Rayleigh quotients omega_n = <n|U|n> and checked with the residual
r_n = || U|n> - omega_n |n> ||_2 (Sec. 4, Eq. (residual)).
"""

from __future__ import annotations

import cmath
from typing import Callable, Tuple

import numpy as np

__all__ = ["arc_distance", "closest", "full_closest", "rayleigh", "residuals"]


def arc_distance(omega, phi: float) -> np.ndarray:
    """|arg(omega e^{-i phi})| in [0, pi]."""
    return np.abs(np.angle(np.asarray(omega) * cmath.exp(-1j * phi)))


def closest(omega: np.ndarray, nev: int, phi: float) -> np.ndarray:
    """Indices of the nev eigenvalues closest to e^{i phi}, nearest first."""
    dist = arc_distance(omega, phi)
    order = np.argsort(dist, kind="stable")
    return order[:nev]


def full_closest(U: np.ndarray, nev: int, phi: float) -> Tuple[np.ndarray, np.ndarray]:
    """Full diagonalisation, then the nev eigenpairs closest to the target.

    Returns (omega[nev], V[d, nev]) with unit-norm columns, nearest first.
    """
    om, V = np.linalg.eig(U)
    idx = closest(om, nev, phi)
    V = V[:, idx]
    V = V / np.linalg.norm(V, axis=0, keepdims=True)
    return om[idx], V


def rayleigh(matvec: Callable[[np.ndarray], np.ndarray], v: np.ndarray) -> complex:
    """omega = <v|U|v> / <v|v>."""
    return complex(np.vdot(v, matvec(v)) / np.vdot(v, v))


def residuals(matvec: Callable[[np.ndarray], np.ndarray], omega: np.ndarray,
              V: np.ndarray) -> np.ndarray:
    """r_n = || U v_n - omega_n v_n ||_2 for each column v_n of V."""
    return np.array([np.linalg.norm(matvec(V[:, n]) - omega[n] * V[:, n])
                     for n in range(V.shape[1])])
