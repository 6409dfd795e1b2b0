"""GPU parity of apply_filter_many (the filter of a block of vectors, one
launch per Horner pass for all of them) against the oracle's geometric sum."""

import numpy as np
import pytest

from gpu_util import bw_op, circ_op, ki_op, rel, require_gpu, say, to_dev, to_np
from oracle import filters, models
from workloads import brickwork, circuit, kicked_ising, random_state

pytestmark = pytest.mark.gpu


def _dt(name):
    torch = require_gpu()
    return torch.complex128 if name == "c128" else torch.complex64


def _tol(dt, k):
    return 1e-12 * (k + 1) if dt == "c128" else 2e-7 * (k + 1) + 2e-6


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("L,n,k,phi", [(4, 3, 7, 0.3), (9, 2, 25, 1.1), (12, 5, 40, 4.0), (16, 4, 12, 0.7),
                                       (20, 2, 3, 5.0)])
def test_filter_many_kicked_ising(dt, L, n, k, phi):
    # single-workgroup shapes (L <= 13) and the multi-pass plan (L = 16, 20)
    say(f"apply_filter_many L={L} n={n} k={k} {dt}")
    p = kicked_ising(L, 700 + L)
    psi = random_state(2 ** L, 31 + L, n)
    ref = np.stack([filters.geometric_sum(lambda v: models.ki_apply(p, v), psi[j], k, phi) for j in range(n)])
    with ki_op(p) as op:
        dpsi = to_dev(psi, _dt(dt))
        dout = op.apply_filter_many(dpsi, k, phi)
        out = to_np(dout)
        # a second call on the same buffers reuses the launch descriptors
        dpsi.copy_(to_dev(psi[::-1].copy(), _dt(dt)))
        out2 = to_np(op.apply_filter_many(dpsi, k, phi, out=dout))
    for j in range(n):
        assert rel(out[j], ref[j]) < _tol(dt, k), j
        assert rel(out2[j], ref[n - 1 - j]) < _tol(dt, k), j


def test_filter_many_copy_single_vector_and_brickwork():
    # k = 0 copies; one vector takes the single-vector path; a small
    # brickwork op takes its one-tile pass with one workgroup per vector
    torch = require_gpu()
    p = kicked_ising(10, 3)
    psi = random_state(2 ** 10, 4, 3)
    with ki_op(p) as op:
        out0 = to_np(op.apply_filter_many(to_dev(psi, torch.complex128), 0, 0.2))
        one = to_np(op.apply_filter_many(to_dev(psi[:1], torch.complex128), 5, 0.2))
        ref1 = to_np(op.apply_filter(to_dev(psi[0], torch.complex128), 5, 0.2))
    assert np.array_equal(out0, psi)
    assert np.array_equal(one[0], ref1)
    q = brickwork(8, 11)
    U = models.dense(q)
    psi = random_state(2 ** 8, 6, 2)
    with bw_op(q) as op:
        out = to_np(op.apply_filter_many(to_dev(psi, torch.complex128), 9, 1.7))
    for j in range(2):
        assert rel(out[j], filters.geometric_sum(lambda v: U @ v, psi[j], 9, 1.7)) < 1e-11


def test_filter_many_argument_errors():
    torch = require_gpu()
    from paper_2102_05054_amd import FloquetError
    from paper_2102_05054_amd._lib import FQ_C128, lib
    p = kicked_ising(6, 1)
    with ki_op(p) as op:
        psi = to_dev(random_state(64, 1, 2), torch.complex128)
        with pytest.raises(FloquetError):
            op.apply_filter_many(psi, -1, 0.0)
        with pytest.raises(FloquetError):
            op.apply_filter_many(psi, 3, float("nan"))
        # overlapping buffers (out shifted by one vector into psi)
        buf = torch.zeros((3, 64), dtype=torch.complex128, device="cuda")
        st = lib().apply_filter_many(op.handle, 3, 0.0, FQ_C128, 2, buf.data_ptr(), buf[1].data_ptr(), None)
        assert st != 0


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("L,n,k", [(10, 64, 5), (14, 16, 3), (18, 3, 1)])
def test_filter_many_many_vectors_and_order_one(dt, L, n, k):
    # many vectors per launch (the single-workgroup form at L = 10, the
    # multi-pass one at L = 14) and k = 1 (the prologue pass and one Horner
    # pass only)
    say(f"apply_filter_many L={L} n={n} k={k} {dt}")
    p = kicked_ising(L, 730 + L)
    psi = random_state(2 ** L, 60 + L, n)
    with ki_op(p) as op:
        out = to_np(op.apply_filter_many(to_dev(psi, _dt(dt)), k, 2.9))
    for j in (0, n // 2, n - 1):
        ref = filters.geometric_sum(lambda v: models.ki_apply(p, v), psi[j], k, 2.9)
        assert rel(out[j], ref) < _tol(dt, k), j


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("L,n,k,phi", [(7, 5, 6, 0.9), (13, 3, 4, 2.2), (14, 4, 5, 0.4), (17, 2, 3, 1.5),
                                       (18, 64, 1, 3.3), (20, 4, 2, 0.8)])
def test_filter_many_brickwork(dt, L, n, k, phi):
    # brickwork: one launch per pass for all vectors, items = (vector, tile);
    # L = 7, 13 one tile per vector (complex128 splits L = 13), L = 14, 17
    # two passes, L = 18 with 64 vectors and L = 20 with 4 (complex64: the
    # persistent pipelined form for the 2^13 / 2^14 tiles)
    say(f"apply_filter_many brickwork L={L} n={n} k={k} {dt}")
    p = brickwork(L, 940 + L)
    psi = random_state(2 ** L, 70 + L, n)
    mv = (lambda v, U=models.dense(p): U @ v) if L <= 10 else (lambda v: models.bw_apply(p, v))
    with bw_op(p) as op:
        dpsi = to_dev(psi, _dt(dt))
        out = to_np(op.apply_filter_many(dpsi, k, phi))
        one = to_np(op.apply_filter(dpsi[n - 1], k, phi))
    assert rel(out[n - 1], one) < (1e-14 if dt == "c128" else 1e-6)
    for j in sorted({0, n // 2, n - 1}):
        ref = filters.geometric_sum(mv, psi[j], k, phi)
        assert rel(out[j], ref) < _tol(dt, k), j


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_filter_many_circuit(dt):
    # a general circuit (gates in any order) through the same multi-vector passes
    L, n, k = 15, 3, 4
    say(f"apply_filter_many circuit L={L} n={n} k={k} {dt}")
    p = circuit(L, 960, depth=4)
    psi = random_state(2 ** L, 80, n)
    with circ_op(p) as op:
        out = to_np(op.apply_filter_many(to_dev(psi, _dt(dt)), k, 0.6))
    for j in range(n):
        ref = filters.geometric_sum(lambda v: models.circuit_apply(p, v), psi[j], k, 0.6)
        assert rel(out[j], ref) < _tol(dt, k), j


def test_filter_many_folded_passes_match_single_vector_filter():
    # four complex128 vectors per launch take the folded passes (K D K x + K psi
    # with K psi precomputed per tile group); the single-vector filter does
    # not: both agree to rounding, and vector 0 matches the oracle
    torch = require_gpu()
    L, n, k, phi = 20, 4, 6, 0.45
    say(f"apply_filter_many folded L={L} n={n} k={k}")
    p = kicked_ising(L, 760)
    psi = random_state(2 ** L, 61, n)
    with ki_op(p) as op:
        dpsi = to_dev(psi, torch.complex128)
        many = to_np(op.apply_filter_many(dpsi, k, phi))
        ones = [to_np(op.apply_filter(dpsi[j], k, phi)) for j in range(n)]
    for j in range(n):
        assert rel(many[j], ones[j]) < 1e-13, j
    ref = filters.geometric_sum(lambda v: models.ki_apply(p, v), psi[0], k, phi)
    assert rel(many[0], ref) < _tol("c128", k)
