"""Seeded synthetic inputs for the Floquet filter-diagonalisation workloads.

This module only *draws* numbers: model couplings, target phases, Haar-random
gates and start vectors.  It holds none of the method's arithmetic (no U, no
filter, no orthogonalisation), so both the CPU oracle and the HIP path can take
their inputs from it without sharing any computation.

Conventions (shared data layout, not arithmetic):

* Sites are numbered 1..L.  Arrays ``J`` and ``h`` hold ``J[i-1] = J_i`` and
  ``h[i-1] = h_i``.
* Brickwork gates are listed as one flat ``complex128`` array: first the layer
  that acts first on a ket (``U_b``), then the second layer (``U_a``), each
  layer from the left end of the chain to the right.  A two-site gate on sites
  ``(i, i+1)`` is a row-major 4x4 matrix whose local basis index is
  ``2*b_i + b_{i+1}``; a one-site gate is a row-major 2x2 matrix.  The layer
  pattern follows the two-layer brickwork circuit of the paper's model section
  (Eq. (U) and Eq. (unitary)); for odd L the single-site gates sit at the
  other ends (first layer: site 1 alone, second layer: site L alone).
* Random draws come from ``numpy.random.default_rng(seed)`` in a fixed order:
  J[0:L], h[0:L], then phi (only where it is random), then gates.  Start
  vectors come from ``default_rng(seed + 1)``.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "KickedIsingParams",
    "BrickworkParams",
    "CircuitParams",
    "circuit",
    "circuit_from_brickwork",
    "kicked_ising",
    "brickwork",
    "counter_uniform_complex",
    "brickwork_layout",
    "brickwork_cz",
    "haar_unitary",
    "start_vector",
    "random_state",
    "CONFIGS",
    "batched_sizes",
    "config_kicked_ising",
]


@dataclasses.dataclass
class KickedIsingParams:
    L: int
    J: np.ndarray  # (L,) float64, J[i-1] couples sites i and i+1 (site L+1 == site 1 if periodic)
    h: np.ndarray  # (L,) float64, longitudinal field on site i
    g: float       # transverse kick angle
    periodic: bool
    phi: float     # target phase (only used by the filter / eigensolver)


@dataclasses.dataclass
class CircuitParams:
    """A general local Floquet circuit: gates in the order they act (first
    acts first), each on one site or on the nearest-neighbour pair
    (site, site+1); ``gates`` holds their row-major matrices back to back
    (4 or 16 complex128 entries; two-site local index 2*b_i + b_{i+1})."""
    L: int
    sites: np.ndarray   # (G,) int, first site (1-based)
    widths: np.ndarray  # (G,) int, 1 or 2
    gates: np.ndarray   # flat complex128
    phi: float


@dataclasses.dataclass
class BrickworkParams:
    L: int
    gates: np.ndarray  # flat complex128, layer b then layer a (see module docstring)
    phi: float


def kicked_ising(L: int, seed: int, *, J_range=(0.8, 1.2), h_range=(-2.0, 2.0),
                 g: float = 0.9, periodic: bool = True,
                 phi: Optional[float] = 0.0) -> KickedIsingParams:
    """Kicked Ising chain couplings: J_i ~ U[J_range], h_i ~ U[h_range].

    ``phi=None`` draws the target phase uniformly from [0, 2*pi) after J and h.
    """
    if L < 1:
        raise ValueError("L must be >= 1")
    rng = np.random.default_rng(seed)
    J = rng.uniform(J_range[0], J_range[1], size=L)
    h = rng.uniform(h_range[0], h_range[1], size=L)
    if phi is None:
        phi = float(rng.uniform(0.0, 2.0 * math.pi))
    return KickedIsingParams(L=L, J=J.astype(np.float64), h=h.astype(np.float64),
                             g=float(g), periodic=bool(periodic), phi=float(phi))


def haar_unitary(n: int, rng: np.random.Generator) -> np.ndarray:
    """One n x n unitary from the Haar measure (Mezzadri's recipe: QR of a
    complex Ginibre matrix, with the phases of R's diagonal divided out)."""
    z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return (q * (d / np.abs(d))[None, :]).astype(np.complex128)


def brickwork_layout(L: int) -> Tuple[List[Tuple[int, ...]], List[Tuple[int, ...]]]:
    """Sites touched by each gate, per layer, in the flat-array order.

    Returns ``(layer_b, layer_a)``; each entry is a tuple of 1-based sites,
    ``(i,)`` for a one-site gate and ``(i, i+1)`` for a two-site gate.  Each
    layer covers every site exactly once.
    """
    if L < 2:
        raise ValueError("brickwork needs L >= 2")
    if L % 2 == 0:
        layer_b = [(1,)] + [(i, i + 1) for i in range(2, L - 1, 2)] + [(L,)]
        layer_a = [(i, i + 1) for i in range(1, L, 2)]
    else:
        layer_b = [(1,)] + [(i, i + 1) for i in range(2, L, 2)]
        layer_a = [(i, i + 1) for i in range(1, L - 1, 2)] + [(L,)]
    return layer_b, layer_a


def brickwork(L: int, seed: int, *, phi: float = 0.0) -> BrickworkParams:
    """Haar-random brickwork gates for an open chain of L sites."""
    rng = np.random.default_rng(seed)
    layer_b, layer_a = brickwork_layout(L)
    mats = []
    for sites in layer_b + layer_a:
        u = haar_unitary(2 ** len(sites), rng)
        mats.append(u.reshape(-1))
    return BrickworkParams(L=L, gates=np.concatenate(mats).astype(np.complex128), phi=float(phi))


def brickwork_cz(L: int, seed: int, *, phi: float = 0.0) -> BrickworkParams:
    """Another gate set on the same layout: every two-site gate is a
    controlled-Z entangler dressed with Haar-random one-site rotations,
    CZ (r_i x r_{i+1}); the one-site gates are Haar-random."""
    rng = np.random.default_rng(seed)
    layer_b, layer_a = brickwork_layout(L)
    cz = np.diag([1.0, 1.0, 1.0, -1.0]).astype(np.complex128)
    mats = []
    for sites in layer_b + layer_a:
        if len(sites) == 1:
            mats.append(haar_unitary(2, rng))
        else:
            r1, r2 = haar_unitary(2, rng), haar_unitary(2, rng)
            mats.append(cz @ np.kron(r1, r2))
    return brickwork_from_matrices(L, mats, phi)


def circuit(L: int, seed: int, *, depth: int = 3, phi: float = 0.0) -> CircuitParams:
    """A local circuit of ``depth`` layers that is not a brickwork: layer t
    puts Haar-random two-site gates on the bonds (i, i+1) with i = t+1 (mod 3)
    and a Haar-random one-site gate on every site left free; the layers act
    in order t = 0, 1, ...  (gates within a layer listed from site 1 up)."""
    if L < 3:
        raise ValueError("circuit needs L >= 3")
    rng = np.random.default_rng(seed)
    sites, widths, mats = [], [], []
    for t in range(depth):
        covered = set()
        layer = []
        for i in range(1, L):
            if (i - 1) % 3 == t % 3:
                layer.append((i, 2))
                covered.update((i, i + 1))
        for i in range(1, L + 1):
            if i not in covered:
                layer.append((i, 1))
        layer.sort()
        for i, w in layer:
            sites.append(i)
            widths.append(w)
            mats.append(haar_unitary(2 ** w, rng).reshape(-1))
    return CircuitParams(L=L, sites=np.array(sites, dtype=np.int32), widths=np.array(widths, dtype=np.int32),
                         gates=np.concatenate(mats).astype(np.complex128), phi=float(phi))


def circuit_from_brickwork(p: BrickworkParams) -> CircuitParams:
    """The brickwork circuit written as a general gate list (U_b first)."""
    layer_b, layer_a = brickwork_layout(p.L)
    sites = [s[0] for s in layer_b + layer_a]
    widths = [len(s) for s in layer_b + layer_a]
    return CircuitParams(L=p.L, sites=np.array(sites, dtype=np.int32), widths=np.array(widths, dtype=np.int32),
                         gates=np.asarray(p.gates, dtype=np.complex128).copy(), phi=p.phi)


def brickwork_from_matrices(L: int, mats: Sequence[np.ndarray], phi: float = 0.0) -> BrickworkParams:
    """Pack explicit gate matrices (same order as ``brickwork_layout``)."""
    layer_b, layer_a = brickwork_layout(L)
    sites = layer_b + layer_a
    if len(mats) != len(sites):
        raise ValueError(f"expected {len(sites)} gates, got {len(mats)}")
    flat = []
    for s, m in zip(sites, mats):
        m = np.asarray(m, dtype=np.complex128)
        if m.shape != (2 ** len(s), 2 ** len(s)):
            raise ValueError(f"gate on sites {s} must be {2**len(s)}x{2**len(s)}")
        flat.append(m.reshape(-1))
    return BrickworkParams(L=L, gates=np.concatenate(flat), phi=float(phi))


def start_vector(d: int, seed: int) -> np.ndarray:
    """Normalised complex Gaussian vector of length d from default_rng(seed + 1)."""
    rng = np.random.default_rng(seed + 1)
    v = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    return (v / np.linalg.norm(v)).astype(np.complex128)


_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)
_SEED_MUL = np.uint64(0x100000001B3)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea and Flood 2014; constants as in
    Vigna's public reference implementation), elementwise on uint64."""
    x = x + _GOLDEN
    x = (x ^ (x >> np.uint64(30))) * _MIX1
    x = (x ^ (x >> np.uint64(27))) * _MIX2
    return x ^ (x >> np.uint64(31))


def counter_uniform_complex(d: int, seed: int) -> np.ndarray:
    """Counter-based start vector: entry i = (2u - 1) + i(2u' - 1) with u, u'
    the top 53 bits of SplitMix64(seed * 0x100000001B3 + 2i) and of
    SplitMix64(seed * 0x100000001B3 + 2i + 1), scaled to [0, 1).  The library
    draws its seeded start vectors from the same published generator (its own
    implementation), so a test can build start blocks with known relations to
    them.  Not normalised."""
    with np.errstate(over="ignore"):
        base = np.uint64(seed) * _SEED_MUL
        i = np.arange(d, dtype=np.uint64)
        a = _splitmix64(base + np.uint64(2) * i)
        b = _splitmix64(base + np.uint64(2) * i + np.uint64(1))
    scale = 1.0 / 9007199254740992.0
    ua = (a >> np.uint64(11)).astype(np.float64) * scale
    ub = (b >> np.uint64(11)).astype(np.float64) * scale
    return (2.0 * ua - 1.0) + 1j * (2.0 * ub - 1.0)


def random_state(d: int, seed: int, count: int = 1) -> np.ndarray:
    """``count`` independent normalised complex Gaussian vectors, shape (count, d)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((count, d)) + 1j * rng.standard_normal((count, d))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v.astype(np.complex128)


# ---------------------------------------------------------------------------
# The benchmark workloads.  Seeds: workload n uses base seed 1000*n; the
# batched workload's realisation r uses 4000 + r and its sizes come from
# default_rng(40000).
# ---------------------------------------------------------------------------

CONFIGS = {
    "ki_L10": dict(model="kicked_ising", L=10, seed=1000, k=64, nev=20, ncv=60,
                   dtype="c128", phi=0.0, tol=1e-10),
    "ki_L16": dict(model="kicked_ising", L=16, seed=2000, k=200, nev=50, ncv=120,
                   dtype="c128", phi=None, tol=1e-10),
    "ki_L20": dict(model="kicked_ising", L=20, seed=3000, k=400, nev=100, ncv=220,
                   dtype="c64+refine", phi=0.0, tol=1e-10, W=(1.0, 3.0)),
    "ki_batched": dict(model="kicked_ising", L=(12, 16), n_real=256, seed=4000, k=150,
                       nev=20, ncv=60, dtype="c64+refine",
                       phis=(0.0, 0.5 * math.pi, math.pi, 1.5 * math.pi), tol=1e-10),
    "bw_L24": dict(model="brickwork", L=24, seed=5000, k=300, nev=40, ncv=100,
                   dtype="c64+refine", phi=0.0, tol=1e-9),
}


def batched_sizes(n_real: int = 256, lo: int = 12, hi: int = 16) -> np.ndarray:
    """Chain lengths of the batched workload, uniform on {lo..hi}."""
    return np.random.default_rng(40000).integers(lo, hi + 1, size=n_real)


def config_kicked_ising(name: str, *, W: Optional[float] = None, realisation: int = 0,
                        L: Optional[int] = None) -> KickedIsingParams:
    """Couplings of one named kicked-Ising workload."""
    c = CONFIGS[name]
    if name == "ki_batched":
        sizes = batched_sizes(c["n_real"], c["L"][0], c["L"][1])
        LL = int(sizes[realisation]) if L is None else int(L)
        return kicked_ising(LL, c["seed"] + realisation, phi=0.0)
    LL = c["L"] if L is None else int(L)
    if name == "ki_L20":
        w = 1.0 if W is None else float(W)
        return kicked_ising(LL, c["seed"], h_range=(-w, w), phi=c["phi"])
    return kicked_ising(LL, c["seed"], phi=c["phi"])
