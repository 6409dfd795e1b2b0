"""Floquet operators U, built densely and applied matrix-free (oracle).

Test infrastructure only (see the package docstring).  No code is shared with
the HIP library.

Basis convention: site i (1-based) is bit ``L - i`` of the basis index, so site
1 is the most significant bit and the leftmost Kronecker factor.  This is the
C-order reshaping of the wave function used by the paper's matrix-vector
product (Eq. (matvec)) and by its entanglement cut (Eq. (ee)).

Kicked Ising chain (the benchmark model; the paper's method applies to any
local Floquet U, Sec. 2 last paragraph):

    U = D K,   K = prod_i exp(-i g X_i),   D = diag(exp(-i E(s))),
    E(s) = sum_i J_i z_i z_{i+1} + h_i z_i,   z_i = 1 - 2 b_i(s),

K acting first; with periodic boundaries the bond (L, 1) is included.

Brickwork random circuit (Sec. 2, Eq. (U), Eq. (unitary)):

    U = U_a U_b,  U_b = u_1 u_{2,3} ... u_{L-2,L-1} u_L,  U_a = u_{1,2} ... u_{L-1,L},

U_b acting first.  Each layer covers every site exactly once, so each layer is
one Kronecker product of its gates in site order.

General local circuit (the method applies to any local U, Sec. 2): gates on
one site or on a nearest-neighbour pair, in the order they act,

    U = G_{n-1} ... G_1 G_0,   G = 1_{2^(i-1)} (x) u (x) 1_{2^(L-i-w+1)},

each embedded by Kronecker products at its first site i (width w).
"""

from __future__ import annotations

import math
from typing import Callable, List, Sequence, Tuple

import numpy as np

__all__ = [
    "site_z",
    "ki_energies",
    "ki_kick",
    "ki_dense",
    "ki_apply",
    "bw_gate_list",
    "bw_dense",
    "bw_apply",
    "circuit_gate_list",
    "circuit_dense",
    "circuit_apply",
    "dense",
    "matvec",
]

DENSE_MAX_L = 13


def site_z(L: int, i: int, s: np.ndarray) -> np.ndarray:
    """z_i = +1 if site i is in state 0, -1 if in state 1 (site i <-> bit L-i)."""
    return 1 - 2 * ((s >> (L - i)) & 1).astype(np.int64)


def ki_energies(L: int, J: Sequence[float], h: Sequence[float], periodic: bool) -> np.ndarray:
    """E(s) for every basis state s in [0, 2^L), by summing over sites."""
    s = np.arange(2 ** L, dtype=np.int64)
    E = np.zeros(2 ** L, dtype=np.float64)
    last_bond = L if periodic else L - 1
    for i in range(1, last_bond + 1):
        j = i + 1 if i < L else 1
        E += J[i - 1] * site_z(L, i, s) * site_z(L, j, s)
    for i in range(1, L + 1):
        E += h[i - 1] * site_z(L, i, s)
    return E


def ki_kick(g: float) -> np.ndarray:
    """exp(-i g X) = cos(g) I - i sin(g) X."""
    c, sn = math.cos(g), math.sin(g)
    return np.array([[c, -1j * sn], [-1j * sn, c]], dtype=np.complex128)


def ki_dense(p) -> np.ndarray:
    """Dense kicked-Ising U = D K from an explicit Kronecker product."""
    L = p.L
    if L > DENSE_MAX_L:
        raise ValueError(f"dense U limited to L <= {DENSE_MAX_L}")
    k1 = ki_kick(p.g)
    K = np.ones((1, 1), dtype=np.complex128)
    for _ in range(L):
        K = np.kron(K, k1)
    phase = np.exp(-1j * ki_energies(L, p.J, p.h, p.periodic))
    return phase[:, None] * K


_ENERGIES = {}


def _ki_energies_kept(L: int, J: Sequence[float], h: Sequence[float], periodic: bool) -> np.ndarray:
    """ki_energies, kept for the last few chains: E(s) of a chain does not
    change between applications, and at L = 20 it costs ~10x the kicks.
    The returned array is shared; callers only read it."""
    key = (L, np.asarray(J, dtype=np.float64).tobytes(), np.asarray(h, dtype=np.float64).tobytes(), bool(periodic))
    E = _ENERGIES.get(key)
    if E is None:
        E = ki_energies(L, J, h, periodic)
        if len(_ENERGIES) >= 4:
            _ENERGIES.clear()
        _ENERGIES[key] = E
    return E


def ki_apply(p, psi: np.ndarray) -> np.ndarray:
    """Matrix-free U psi: one 2x2 kick per site on the reshaped state, then D."""
    L = p.L
    k1 = ki_kick(p.g)
    x = np.asarray(psi, dtype=np.complex128)
    for i in range(1, L + 1):
        x = x.reshape(2 ** (i - 1), 2, 2 ** (L - i))
        x = np.einsum("ab,xbz->xaz", k1, x)
    x = x.reshape(-1)
    return np.exp(-1j * _ki_energies_kept(L, p.J, p.h, p.periodic)) * x


def bw_gate_list(p) -> Tuple[List[Tuple[Tuple[int, ...], np.ndarray]], List[Tuple[Tuple[int, ...], np.ndarray]]]:
    """Unpack the flat gate array into (sites, matrix) per layer."""
    from workloads import brickwork_layout  # input layout only (no arithmetic)

    layer_b, layer_a = brickwork_layout(p.L)
    flat = np.asarray(p.gates, dtype=np.complex128)
    pos = 0
    out_b, out_a = [], []
    for sites, dest in [(s, out_b) for s in layer_b] + [(s, out_a) for s in layer_a]:
        n = 2 ** len(sites)
        dest.append((sites, flat[pos:pos + n * n].reshape(n, n)))
        pos += n * n
    if pos != flat.size:
        raise ValueError("gate array has the wrong length")
    return out_b, out_a


def bw_dense(p) -> np.ndarray:
    """Dense brickwork U = U_a U_b, each layer a Kronecker product in site order."""
    if p.L > DENSE_MAX_L:
        raise ValueError(f"dense U limited to L <= {DENSE_MAX_L}")
    layer_b, layer_a = bw_gate_list(p)
    layers = []
    for layer in (layer_b, layer_a):
        M = np.ones((1, 1), dtype=np.complex128)
        for _, u in layer:
            M = np.kron(M, u)
        layers.append(M)
    Ub, Ua = layers
    return Ua @ Ub


def bw_apply(p, psi: np.ndarray) -> np.ndarray:
    """Matrix-free brickwork U psi: every gate of U_b, then every gate of U_a."""
    L = p.L
    layer_b, layer_a = bw_gate_list(p)
    x = np.asarray(psi, dtype=np.complex128)
    for sites, u in layer_b + layer_a:
        i = sites[0]
        n = len(sites)
        x = x.reshape(2 ** (i - 1), 2 ** n, 2 ** (L - i - n + 1))
        x = np.einsum("ab,xbz->xaz", u, x)
    return x.reshape(-1)


def circuit_gate_list(p) -> List[Tuple[int, int, np.ndarray]]:
    """Unpack a general circuit into (first site, width, matrix) in acting order."""
    flat = np.asarray(p.gates, dtype=np.complex128)
    out = []
    pos = 0
    for i, w in zip(p.sites, p.widths):
        i, w = int(i), int(w)
        if w not in (1, 2) or i < 1 or i + w - 1 > p.L:
            raise ValueError(f"bad gate at site {i}, width {w}")
        n = 2 ** w
        out.append((i, w, flat[pos:pos + n * n].reshape(n, n)))
        pos += n * n
    if pos != flat.size:
        raise ValueError("gate array has the wrong length")
    return out


def circuit_dense(p) -> np.ndarray:
    """Dense U: the product of every embedded gate, the first acting first."""
    L = p.L
    if L > DENSE_MAX_L:
        raise ValueError(f"dense U limited to L <= {DENSE_MAX_L}")
    U = np.eye(2 ** L, dtype=np.complex128)
    for i, w, u in circuit_gate_list(p):
        G = np.kron(np.kron(np.eye(2 ** (i - 1)), u), np.eye(2 ** (L - i - w + 1)))
        U = G @ U
    return U


def circuit_apply(p, psi: np.ndarray) -> np.ndarray:
    """Matrix-free U psi: every gate in acting order."""
    L = p.L
    x = np.asarray(psi, dtype=np.complex128)
    for i, w, u in circuit_gate_list(p):
        x = x.reshape(2 ** (i - 1), 2 ** w, 2 ** (L - i - w + 1))
        x = np.einsum("ab,xbz->xaz", u, x)
    return x.reshape(-1)


def dense(p) -> np.ndarray:
    """Dense U of any model."""
    if hasattr(p, "J"):
        return ki_dense(p)
    if hasattr(p, "sites"):
        return circuit_dense(p)
    return bw_dense(p)


def matvec(p) -> Callable[[np.ndarray], np.ndarray]:
    """Matrix-free U of any model, as a callable."""
    if hasattr(p, "J"):
        return lambda v: ki_apply(p, v)
    if hasattr(p, "sites"):
        return lambda v: circuit_apply(p, v)
    return lambda v: bw_apply(p, v)
