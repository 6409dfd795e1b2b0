"""apply_filter_many_noalloc (the allocation-free block filter) against
apply_filter_many through the C ABI: two calls in a row on the library's one
scratch array, the second with a smaller input, both precisions, and the
argument checks."""

import numpy as np
import pytest

from gpu_util import ki_op, require_gpu, say, to_dev, to_np
from workloads import kicked_ising, random_state

pytestmark = pytest.mark.gpu


def _tol(dt, k):
    return 1e-12 * (k + 1) if dt == "c128" else 2e-7 * (k + 1) + 2e-6


def _elem_err(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_noalloc_matches_apply_filter_many_twice(dt):
    torch = require_gpu()
    tdt = torch.complex128 if dt == "c128" else torch.complex64
    # first call: L = 16, 4 vectors; second call: L = 12, 2 vectors (smaller
    # input, other op, other target) on the same scratch array
    cases = [(16, 4, 30, 0.7), (12, 2, 17, 2.9)]
    for L, n, k, phi in cases:
        say(f"noalloc L={L} n={n} k={k} {dt}")
        p = kicked_ising(L, 1200 + L)
        psi = random_state(2 ** L, 40 + L, n)
        with ki_op(p) as op:
            dpsi = to_dev(psi, tdt)
            ref = to_np(op.apply_filter_many(dpsi, k, phi))
            out = torch.empty_like(dpsi)
            got = to_np(op.apply_filter_many_noalloc(dpsi, k, phi, out))
            torch.cuda.synchronize()
        for j in range(n):
            assert _elem_err(got[j], ref[j]) < _tol(dt, k), (L, j)


def test_noalloc_single_vector_large_state_and_copy():
    # one vector at L = 20 (multi-pass plan) after a small call; k = 0 copies
    torch = require_gpu()
    p = kicked_ising(20, 1300)
    psi = random_state(2 ** 20, 5, 1)
    with ki_op(p) as op:
        dpsi = to_dev(psi, torch.complex128)
        ref = to_np(op.apply_filter(dpsi[0], 9, 1.3))
        out = torch.empty_like(dpsi)
        got = to_np(op.apply_filter_many_noalloc(dpsi, 9, 1.3, out))[0]
        assert _elem_err(got, ref) < _tol("c128", 9)
        cp = to_np(op.apply_filter_many_noalloc(dpsi, 0, 1.3, out))
        assert np.array_equal(cp, psi)


def test_noalloc_complex64_L24_wide_tiles():
    # one complex64 vector at L = 24: the untimed default shape has the 14-bit
    # low-bit tile of the three-layout pass; against the single-vector filter
    torch = require_gpu()
    say("noalloc L=24 c64 one vector")
    p = kicked_ising(24, 1400)
    psi = random_state(2 ** 24, 6, 1)
    with ki_op(p) as op:
        dpsi = to_dev(psi, torch.complex64)
        ref = to_np(op.apply_filter(dpsi[0], 5, 0.4))
        out = torch.empty_like(dpsi)
        got = to_np(op.apply_filter_many_noalloc(dpsi, 5, 0.4, out))[0]
        torch.cuda.synchronize()
    assert _elem_err(got, ref) < _tol("c64", 5)


def test_noalloc_argument_errors():
    torch = require_gpu()
    from paper_2102_05054_amd import FloquetError
    from workloads import brickwork
    from gpu_util import bw_op
    p = kicked_ising(8, 3)
    with ki_op(p) as op:
        x = torch.zeros((65, 2 ** 8), dtype=torch.complex128, device="cuda")
        with pytest.raises(FloquetError):
            op.apply_filter_many_noalloc(x, 3, 0.0, torch.empty_like(x))  # more than 64 vectors
        y = x[:2].contiguous()
        with pytest.raises(FloquetError):
            op.apply_filter_many_noalloc(y, -1, 0.0, torch.empty_like(y))
    q = brickwork(6, 2)
    with bw_op(q) as op:
        z = torch.zeros((2, 2 ** 6), dtype=torch.complex128, device="cuda")
        with pytest.raises(FloquetError):
            op.apply_filter_many_noalloc(z, 3, 0.0, torch.empty_like(z))
