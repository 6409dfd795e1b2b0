"""Host-side checks of the C ABI: the library loads, exports every entry point
that include/floquet.h declares, rejects bad arguments without a GPU, and its
small dense Schur step (used by the Krylov-Schur restart) is correct."""

import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT

pytestmark = pytest.mark.filterwarnings("ignore")


def _declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^\s*(?:fq_status|const char\s*\*|long long)\s+(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_core_entry_points():
    names = _declared_functions()
    for n in ["create_floquet_op", "destroy_floquet_op", "apply_U", "apply_filter", "arnoldi_eigs",
              "arnoldi_eigs_batched", "floquet_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2102_05054_amd import _lib
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    bound = {n for n, _, _ in _lib.SIGNATURES}
    assert set(_declared_functions()) <= bound


def test_graph_capture_switch():
    # process-wide switch of the batched solver's graph replay (host only)
    from paper_2102_05054_amd import _lib
    L = _lib.lib()
    assert L.fq_set_graph_capture(2) == _lib.FQ_EINVAL
    assert b"0 or 1" in L.floquet_last_error()
    assert L.fq_set_graph_capture(0) == _lib.FQ_OK
    assert L.fq_set_graph_capture(1) == _lib.FQ_OK


def test_invalid_arguments_are_rejected_on_host():
    from paper_2102_05054_amd import _lib
    L = _lib.lib()
    # NULL op / out pointers are rejected before any device work
    assert L.apply_U(None, 1, None, None, None) == _lib.FQ_EINVAL
    assert L.apply_filter(None, 3, 0.0, 1, None, None, None) == _lib.FQ_EINVAL
    assert b"NULL" in L.floquet_last_error()
    assert L.create_floquet_op(None, None) == _lib.FQ_EINVAL
    assert L.destroy_floquet_op(None) == _lib.FQ_OK
    out = ctypes.c_void_p()
    desc = _lib.FqModelDesc(model=0, L=1, periodic=1)
    assert L.create_floquet_op(ctypes.byref(desc), ctypes.byref(out)) == _lib.FQ_EINVAL
    desc = _lib.FqModelDesc(model=0, L=31, periodic=1)
    assert L.create_floquet_op(ctypes.byref(desc), ctypes.byref(out)) == _lib.FQ_EINVAL
    opts = _lib.FqArnoldiOpts(k=10, ncv=20, tol=1e-10, max_restarts=10)
    assert L.arnoldi_eigs(None, 5, 0.0, ctypes.byref(opts), None, None, None, None, None) == _lib.FQ_EINVAL


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (40, 3), (120, 4), (260, 5)])
def test_host_schur_against_lapack(n, seed):
    from paper_2102_05054_amd import host_schur
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    T, Z, w = host_schur(A)
    scale = np.linalg.norm(A)
    assert np.linalg.norm(Z @ T @ Z.conj().T - A) < 1e-13 * scale * n
    assert np.linalg.norm(Z.conj().T @ Z - np.eye(n)) < 1e-13 * n
    assert np.abs(np.tril(T, -1)).max(initial=0) == 0
    # eigenvalues = LAPACK's, ordered by decreasing modulus
    ref = np.linalg.eigvals(A)
    ref = ref[np.argsort(-np.abs(ref), kind="stable")]
    assert np.allclose(np.abs(w), np.abs(ref), atol=1e-11 * scale)
    for x in w:
        assert np.min(np.abs(ref - x)) < 1e-10 * scale


def test_host_schur_hessenberg_with_clusters():
    # Krylov-Schur matrices: triangular block + a full row (restart), near-equal moduli
    from paper_2102_05054_amd import host_schur
    rng = np.random.default_rng(9)
    n = 60
    ang = np.sort(rng.uniform(-1e-3, 1e-3, n))
    A = np.diag(100 * np.exp(1j * ang)).astype(complex) + np.triu(rng.standard_normal((n, n)), 1) * 0.1
    A[40, :40] = rng.standard_normal(40) * 1e-3
    T, Z, w = host_schur(A)
    assert np.linalg.norm(Z @ T @ Z.conj().T - A) < 1e-12 * np.linalg.norm(A)
    assert np.all(np.diff(np.abs(w)) <= 1e-12 * 100)


@pytest.mark.parametrize("L,nev", [(10, 50), (12, 50), (16, 50), (20, 50), (20, 100)])
def test_paper_parameter_rule(L, nev):
    # Table "bench" caption: n_cv = floor(2^(L/2+1)), k = 0.8 * 2^(L+1) / n_cv
    # (k floored); n_cv > 2 n_ev (Sec. 4).  The table's L = 20 row: n_cv = 2048, k = 819.
    from paper_2102_05054_amd import paper_parameters
    ncv, k = paper_parameters(L, nev)
    expect_ncv = max(int(2 ** (L / 2 + 1)), 2 * nev + 1)
    assert ncv == expect_ncv
    assert k == int(0.8 * 2 ** (L + 1) / ncv)
    if L == 20 and nev == 50:
        assert (ncv, k) == (2048, 819)


@pytest.mark.parametrize("L,nev,expect", [(2, 1, (3, 2)), (4, 8, (15, 1)), (6, 40, (63, 1)), (8, 10, (32, 12))])
def test_paper_parameter_rule_small_chains(L, nev, expect):
    # n_cv is raised to 2 nev + 1 but kept below d = 2^L: a Krylov space of
    # dimension d is the whole space (the last Arnoldi step would break down)
    from paper_2102_05054_amd import paper_parameters
    assert paper_parameters(L, nev) == expect


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (5, 2), (64, 3), (300, 4)])
def test_host_hermitian_eigenvalues_against_lapack(n, seed):
    # the eigenvalue step of entanglement_entropy (Householder + implicit QL)
    from paper_2102_05054_amd import _lib
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = X @ X.conj().T / n  # Hermitian PSD like a reduced density matrix
    a = np.stack([A.real, A.imag], axis=-1).reshape(-1).copy()
    w = np.zeros(n)
    assert _lib.lib().fq_host_eigvalsh(n, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
    assert np.allclose(w, np.linalg.eigvalsh(A), atol=1e-12 * max(1.0, np.abs(A).max()) * n)


def test_host_hermitian_eigenvalues_degenerate_and_diagonal():
    from paper_2102_05054_amd import _lib
    A = np.diag([0.5, 0.25, 0.25, 0.0]).astype(complex)
    a = np.stack([A.real, A.imag], axis=-1).reshape(-1).copy()
    w = np.zeros(4)
    assert _lib.lib().fq_host_eigvalsh(4, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
    assert np.allclose(w, [0.0, 0.25, 0.25, 0.5], atol=1e-15)
