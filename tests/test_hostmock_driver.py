"""The Krylov-Schur driver on the CPU, through a host mock of the device layer.

The driver sources (krylov.cpp, block.cpp, dense.cpp) are compiled with g++
against a host stand-in for the HIP runtime and kernels whose operator is a
diagonal unitary with known phases (paper_2102_05054_amd/hostmock).  This
exercises restarts, the mixed-precision hand-over, the block solver,
non-convergence, NaN detection, out-of-memory and invariant subspaces without
a GPU, once under AddressSanitizer + UBSan (a self-test executable) and once
through the C ABI from Python.
"""

import ctypes
import math
import os
import subprocess
from ctypes import POINTER, c_double, c_int, c_longlong, c_void_p

import numpy as np
import pytest

from paper_2102_05054_amd import build as B
from paper_2102_05054_amd._lib import (FQ_C64, FQ_C128, FQ_ENOMEM, FQ_ENUMERIC, FQ_NOT_CONVERGED, FQ_OK,
                                       FqArnoldiOpts, FqArnoldiStats)

_mock = None


def mock():
    global _mock
    if _mock is None:
        if not os.path.exists(B.MOCK_LIB):
            B.build_hostmock(verbose=False)
        m = ctypes.CDLL(B.MOCK_LIB)
        m.fq_mock_create.argtypes = [c_int, POINTER(c_double), POINTER(c_void_p)]
        m.fq_mock_create.restype = c_int
        m.fq_mock_destroy.argtypes = [c_void_p]
        m.fq_mock_set_free_bytes.argtypes = [ctypes.c_ulonglong]
        m.fq_mock_set_nan_at.argtypes = [c_longlong]
        m.arnoldi_eigs.argtypes = [c_void_p, c_int, c_double, POINTER(FqArnoldiOpts), POINTER(c_double), c_void_p,
                                   POINTER(c_double), POINTER(FqArnoldiStats), c_void_p]
        m.arnoldi_eigs.restype = c_int
        m.floquet_last_error.restype = ctypes.c_char_p
        _mock = m
    return _mock


def mock_solve(phases, nev, phi, k, ncv, dtype=FQ_C128, block=1, max_restarts=200, want_vectors=False):
    m = mock()
    L = int(round(math.log2(len(phases))))
    ph = np.ascontiguousarray(phases, dtype=np.float64)
    op = c_void_p()
    assert m.fq_mock_create(L, ph.ctypes.data_as(POINTER(c_double)), ctypes.byref(op)) == FQ_OK
    try:
        o = FqArnoldiOpts(k=k, ncv=ncv, tol=1e-10, max_restarts=max_restarts, filter_dtype=dtype, refine=1, seed=3,
                          v0_dev=None, refine_k=0, poly_coeffs=None, block=block)
        ev = np.zeros(2 * nev)
        res = np.zeros(nev)
        st = FqArnoldiStats()
        vec = np.zeros((nev, len(phases)), dtype=np.complex128) if want_vectors else None
        status = m.arnoldi_eigs(op, nev, phi, ctypes.byref(o), ev.ctypes.data_as(POINTER(c_double)),
                                c_void_p(vec.ctypes.data) if want_vectors else None,
                                res.ctypes.data_as(POINTER(c_double)), ctypes.byref(st), None)
        msg = m.floquet_last_error().decode()
    finally:
        m.fq_mock_destroy(op)
    return status, ev[0::2] + 1j * ev[1::2], res, st.as_dict(), vec, msg


def closest(phases, nev, phi):
    w = np.exp(1j * np.asarray(phases))
    dist = np.abs(np.angle(w * np.exp(-1j * phi)))
    return w[np.argsort(dist, kind="stable")[:nev]]


def test_sanitized_selftest():
    # every scenario of hostmock/selftest.cpp under ASan + UBSan (host code only)
    if not os.path.exists(B.MOCK_SELFTEST):
        B.build_hostmock_selftest(verbose=False)
    r = subprocess.run([B.MOCK_SELFTEST], capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "PASSED: 0 failure(s)" in r.stdout


@pytest.mark.parametrize("dtype", [FQ_C128, FQ_C64])
@pytest.mark.parametrize("block", [1, 2, 4, 8])
def test_mock_pairs_and_vectors(block, dtype):
    rng = np.random.default_rng(5)
    ph = rng.uniform(-np.pi, np.pi, 2 ** 9)
    st, ev, res, stats, vec, msg = mock_solve(ph, 7, 2.2, 40, 40, dtype=dtype, block=block, want_vectors=True)
    assert st == FQ_OK, msg
    assert np.max(np.abs(ev - closest(ph, 7, 2.2))) < 1e-12
    assert res.max() <= 1e-10
    if dtype == FQ_C64:
        assert stats["n_U_apps_c64"] > 0 and stats["t_refine"] >= 0.0
    # U is diagonal: every eigenvector is one basis state
    for n in range(7):
        assert np.max(np.abs(vec[n]) ** 2) > 1 - 1e-10
        s = int(np.argmax(np.abs(vec[n])))
        assert abs(np.exp(1j * ph[s]) - ev[n]) < 1e-12


def test_mock_failure_paths():
    m = mock()
    rng = np.random.default_rng(6)
    ph = rng.uniform(-np.pi, np.pi, 2 ** 8)
    st, ev, res, stats, _, _ = mock_solve(ph, 6, 0.0, 2, 10, max_restarts=0)
    assert st == FQ_NOT_CONVERGED and stats["nconv"] == int((res <= 1e-10).sum())
    m.fq_mock_set_nan_at(3)
    try:
        st, *_, msg = mock_solve(ph, 6, 0.0, 20, 24)
    finally:
        m.fq_mock_set_nan_at(-1)
    assert st == FQ_ENUMERIC and "non-finite" in msg
    m.fq_mock_set_free_bytes(1 << 20)
    try:
        st, *_, msg = mock_solve(rng.uniform(-np.pi, np.pi, 2 ** 12), 10, 0.0, 10, 100)
    finally:
        m.fq_mock_set_free_bytes(64 << 30)
    assert st == FQ_ENOMEM and "free device memory" in msg


def test_mock_invariant_spaces():
    # ncv = d: the last Arnoldi step spans the whole space (exact pairs)
    rng = np.random.default_rng(7)
    ph = rng.uniform(-np.pi, np.pi, 16)
    st, ev, res, _, _, msg = mock_solve(ph, 5, 0.7, 3, 16)
    assert st == FQ_OK, msg
    assert np.max(np.abs(ev - closest(ph, 5, 0.7))) < 1e-12
    # three distinct eigenvalues: invariant at dimension 3 < nev = 4
    ph3 = np.array([0.1, 0.5, 0.9] * 22)[:64]
    st, *_, msg = mock_solve(ph3, 4, 0.0, 5, 20)
    assert st == FQ_ENUMERIC and "invariant" in msg


def test_mock_paper_rule_defaults():
    # k = 0 and ncv = 0 select the paper's rule (Sec. 5, Table "bench" caption)
    rng = np.random.default_rng(8)
    L, nev = 11, 12
    ph = rng.uniform(-np.pi, np.pi, 2 ** L)
    st, ev, res, stats, _, msg = mock_solve(ph, nev, 1.5, 0, 0)
    assert st == FQ_OK, msg
    ncv = int(math.floor(2 ** (L / 2 + 1)))
    k = int(math.floor(0.8 * 2 ** (L + 1) / ncv))
    assert (ncv, k) == (90, 36)
    assert stats["n_U_apps"] - nev == k * stats["n_filter_apps"]
    assert np.max(np.abs(ev - closest(ph, nev, 1.5))) < 1e-12
