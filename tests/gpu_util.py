"""Helpers shared by the GPU tests: building ops from workload parameters and
moving states between NumPy and the device (no arithmetic of the method)."""

import sys

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected without a visible GPU")
    return torch


def to_dev(x, dtype):
    torch = require_gpu()
    t = torch.from_numpy(np.ascontiguousarray(x))
    return t.to(device="cuda", dtype=dtype)


def to_np(t):
    return t.detach().cpu().numpy()


def ki_op(p):
    from paper_2102_05054_amd import kicked_ising
    return kicked_ising(p.L, p.J, p.h, p.g, p.periodic)


def bw_op(p):
    from paper_2102_05054_amd import brickwork
    return brickwork(p.L, p.gates)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def circ_op(p):
    from paper_2102_05054_amd import circuit
    return circuit(p.L, p.sites, p.widths, p.gates)


_ORACLE_MEMO = {}


def _nbytes(x):
    if isinstance(x, tuple):
        return sum(_nbytes(y) for y in x)
    return getattr(x, "nbytes", 0)


def memo(key, make):
    """An expensive oracle result (a dense U, its full diagonalisation), made
    once per test run and shared by the tests that name the same model (at
    most ~4 GiB held; the oldest entries go first)."""
    if key not in _ORACLE_MEMO:
        value = make()
        while _ORACLE_MEMO and sum(_nbytes(v) for v in _ORACLE_MEMO.values()) + _nbytes(value) > 4 << 30:
            del _ORACLE_MEMO[next(iter(_ORACLE_MEMO))]
        _ORACLE_MEMO[key] = value
    return _ORACLE_MEMO[key]


def dense_closest(key, U, nev, phi):
    """The oracle's eig.full_closest(U, nev, phi) with the full
    diagonalisation of U done once per key: every pair from the oracle, then
    its own nearest-first selection."""
    from oracle import eig
    om, V = memo(("eig",) + tuple(key), lambda: eig.full_closest(U, U.shape[0], 0.0))
    idx = eig.closest(om, nev, phi)
    return om[idx], V[:, idx]
