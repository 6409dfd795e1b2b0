"""Python face of the C ABI: the same entry points, taking torch tensors.

PyTorch only supplies device memory (``data_ptr()``) and the current HIP
stream; every computation happens in libfloquet.so.
"""

from __future__ import annotations

import ctypes
from ctypes import POINTER, c_double, c_void_p
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (FQ_BRICKWORK, FQ_C64, FQ_C128, FQ_CIRCUIT, FQ_KICKED_ISING, FQ_NOT_CONVERGED, FQ_OK,
                   FqArnoldiOpts, FqArnoldiStats, FqModelDesc, check, lib)

__all__ = ["FloquetOp", "kicked_ising", "brickwork", "circuit", "arnoldi_eigs_batched", "host_schur",
           "paper_parameters"]


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.complex64:
        return FQ_C64
    if t.dtype == torch.complex128:
        return FQ_C128
    raise TypeError(f"state tensors must be complex64 or complex128, got {t.dtype}")


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


def _dptr(t):
    return c_void_p(t.data_ptr())


def _dbl_array(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    return a, a.ctypes.data_as(POINTER(c_double))


class FloquetOp:
    """Owns one ``floquet_op`` handle (create_floquet_op / destroy_floquet_op)."""

    def __init__(self, desc: FqModelDesc, keep=()):
        self._keep = keep
        h = c_void_p()
        check(lib().create_floquet_op(ctypes.byref(desc), ctypes.byref(h)), "create_floquet_op")
        self.handle = h
        self.L = desc.L
        self.dim = int(lib().floquet_op_dim(h))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            check(lib().destroy_floquet_op(self.handle), "destroy_floquet_op")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- checks ----------------------------------------------------------
    def _check_state(self, t, name):
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
        if not t.is_contiguous() or t.numel() != self.dim:
            raise ValueError(f"{name} must be contiguous with {self.dim} elements")

    # -- entry points ----------------------------------------------------
    def apply_U(self, psi, out=None, stream=None):
        """out = U psi."""
        torch = _torch()
        self._check_state(psi, "psi")
        out = torch.empty_like(psi) if out is None else out
        self._check_state(out, "out")
        if out.dtype != psi.dtype:
            raise TypeError("psi and out must have the same dtype")
        check(lib().apply_U(self.handle, _dtype_code(psi), _dptr(psi), _dptr(out), _stream_ptr(stream)), "apply_U")
        return out

    def apply_filter(self, psi, k: int, phi: float, out=None, stream=None):
        """out = sum_{n=0..k} (e^{-i phi} U)^n psi."""
        torch = _torch()
        self._check_state(psi, "psi")
        out = torch.empty_like(psi) if out is None else out
        self._check_state(out, "out")
        if out.dtype != psi.dtype:
            raise TypeError("psi and out must have the same dtype")
        check(lib().apply_filter(self.handle, int(k), float(phi), _dtype_code(psi), _dptr(psi), _dptr(out),
                                 _stream_ptr(stream)), "apply_filter")
        return out

    def apply_filter_many(self, psi, k: int, phi: float, out=None, stream=None):
        """out[j] = sum_{n=0..k} (e^{-i phi} U)^n psi[j] for the rows of psi (n_vec x d)."""
        torch = _torch()
        if psi.dim() != 2 or psi.shape[1] != self.dim or not psi.is_cuda or not psi.is_contiguous():
            raise ValueError(f"psi must be a contiguous (n_vec, {self.dim}) device tensor")
        out = torch.empty_like(psi) if out is None else out
        if out.shape != psi.shape or out.dtype != psi.dtype or not out.is_cuda or not out.is_contiguous():
            raise ValueError("out must be a contiguous device tensor of psi's shape and dtype")
        check(lib().apply_filter_many(self.handle, int(k), float(phi), _dtype_code(psi), int(psi.shape[0]),
                                      _dptr(psi), _dptr(out), _stream_ptr(stream)), "apply_filter_many")
        return out

    def apply_filter_many_noalloc(self, psi, k: int, phi: float, out, stream=None):
        """apply_filter_many without device allocation (kicked Ising, 1..64 vectors);
        ``out`` must be given (the call allocates nothing)."""
        if psi.dim() != 2 or psi.shape[1] != self.dim or not psi.is_cuda or not psi.is_contiguous():
            raise ValueError(f"psi must be a contiguous (n_vec, {self.dim}) device tensor")
        if out.shape != psi.shape or out.dtype != psi.dtype or not out.is_cuda or not out.is_contiguous():
            raise ValueError("out must be a contiguous device tensor of psi's shape and dtype")
        check(lib().apply_filter_many_noalloc(self.handle, int(k), float(phi), _dtype_code(psi), int(psi.shape[0]),
                                              _dptr(psi), _dptr(out), _stream_ptr(stream)),
              "apply_filter_many_noalloc")
        return out

    def apply_polynomial(self, psi, coeffs: Sequence[complex], out=None, stream=None):
        """out = sum_m coeffs[m] U^m psi."""
        torch = _torch()
        self._check_state(psi, "psi")
        out = torch.empty_like(psi) if out is None else out
        self._check_state(out, "out")
        c = np.asarray(coeffs, dtype=np.complex128)
        flat, ptr = _dbl_array(np.stack([c.real, c.imag], axis=1).reshape(-1))
        check(lib().apply_polynomial(self.handle, len(c) - 1, ptr, _dtype_code(psi), _dptr(psi), _dptr(out),
                                     _stream_ptr(stream)), "apply_polynomial")
        return out

    def arnoldi_eigs(self, nev: int, phi: float, *, k: int = 0, ncv: int = 0, tol: float = 1e-10,
                     max_restarts: int = 200, filter_dtype: str = "c128", refine: bool = True,
                     seed: int = 0, v0=None, want_vectors: bool = True, stream=None,
                     allow_not_converged: bool = False, refine_k: int = 0, poly=None, block: int = 1):
        """Eigenpairs of U closest to e^{i phi}.  Returns (evals, evecs, resid, stats, status).

        ``k = 0`` / ``ncv = 0`` select the paper's rule (fq_paper_parameters: n_cv =
        floor(2^(L/2+1)), k = floor(0.8 * 2^(L+1) / n_cv) for the n_cv used).
        ``poly`` (optional): coefficients a_0..a_k of the filter sum_m a_m U^m used
        instead of the geometric sum (k is then len(poly) - 1).
        ``block`` (1, 2, 4 or 8): vectors filtered per Krylov step (block Krylov-Schur)."""
        torch = _torch()
        pc = None
        if poly is not None:
            c = np.asarray(poly, dtype=np.complex128)
            k = len(c) - 1
            pc, pcp = _dbl_array(np.stack([c.real, c.imag], axis=1).reshape(-1))
        opts = FqArnoldiOpts(k=int(k), ncv=int(ncv), tol=float(tol), max_restarts=int(max_restarts),
                             filter_dtype=FQ_C64 if filter_dtype == "c64" else FQ_C128,
                             refine=1 if refine else 0, seed=int(seed),
                             v0_dev=c_void_p(v0.data_ptr()) if v0 is not None else None, refine_k=int(refine_k),
                             poly_coeffs=pcp if pc is not None else None, block=int(block))
        if v0 is not None:
            self._check_state(v0, "v0")
            if v0.dtype != torch.complex128:
                raise TypeError("v0 must be complex128")
        evals = np.zeros(2 * nev)
        resid = np.zeros(nev)
        stats = FqArnoldiStats()
        evecs = None
        if want_vectors:
            evecs = torch.empty((nev, self.dim), dtype=torch.complex128, device="cuda")
        st = lib().arnoldi_eigs(self.handle, int(nev), float(phi), ctypes.byref(opts),
                                evals.ctypes.data_as(POINTER(c_double)),
                                _dptr(evecs) if evecs is not None else None,
                                resid.ctypes.data_as(POINTER(c_double)), ctypes.byref(stats),
                                _stream_ptr(stream))
        check(st, "arnoldi_eigs", allow=(FQ_OK, FQ_NOT_CONVERGED) if allow_not_converged else (FQ_OK,))
        return evals[0::2] + 1j * evals[1::2], evecs, resid, stats.as_dict(), st

    def entanglement_entropy(self, states, LA: int, stream=None):
        """S_A for each row of ``states`` (n x d complex128 device tensor), cut after site LA."""
        torch = _torch()
        if states.dim() == 1:
            states = states.unsqueeze(0)
        if not states.is_cuda or states.dtype != torch.complex128 or not states.is_contiguous() \
                or states.shape[1] != self.dim:
            raise ValueError(f"states must be a contiguous complex128 device tensor of shape (n, {self.dim})")
        out = np.zeros(states.shape[0])
        check(lib().entanglement_entropy(self.handle, int(LA), _dptr(states), int(states.shape[0]),
                                         out.ctypes.data_as(POINTER(c_double)), _stream_ptr(stream)),
              "entanglement_entropy")
        return out


def kicked_ising(L: int, J, h, g: float, periodic: bool = True) -> FloquetOp:
    """Kicked-Ising U = D K (see include/floquet.h)."""
    Ja, Jp = _dbl_array(J)
    ha, hp = _dbl_array(h)
    if Ja.size != L or ha.size != L:
        raise ValueError("J and h need L entries")
    desc = FqModelDesc(model=FQ_KICKED_ISING, L=int(L), periodic=1 if periodic else 0, J=Jp, h=hp,
                       g=float(g), gates=None, n_gates=0)
    return FloquetOp(desc, keep=(Ja, ha))


def brickwork(L: int, gates) -> FloquetOp:
    """Brickwork U = U_a U_b from the flat complex128 gate array."""
    g = np.ascontiguousarray(np.asarray(gates, dtype=np.complex128))
    flat, ptr = _dbl_array(np.stack([g.real, g.imag], axis=1).reshape(-1))
    desc = FqModelDesc(model=FQ_BRICKWORK, L=int(L), periodic=0, J=None, h=None, g=0.0, gates=ptr,
                       n_gates=int(L) + 1)
    return FloquetOp(desc, keep=(flat,))


def circuit(L: int, sites, widths, gates) -> FloquetOp:
    """General local circuit: gate q acts (in list order) on sites[q] ..
    sites[q] + widths[q] - 1 (1-based, width 1 or 2) with the row-major
    matrices packed back to back in ``gates`` (see include/floquet.h)."""
    sa = np.ascontiguousarray(np.asarray(sites, dtype=np.int32))
    wa = np.ascontiguousarray(np.asarray(widths, dtype=np.int32))
    if sa.size != wa.size or sa.size < 1:
        raise ValueError("sites and widths need one entry per gate")
    g = np.ascontiguousarray(np.asarray(gates, dtype=np.complex128))
    if g.size != int(np.sum(np.where(wa == 1, 4, 16))):
        raise ValueError("gates must hold 4 entries per one-site and 16 per two-site gate")
    flat, ptr = _dbl_array(np.stack([g.real, g.imag], axis=1).reshape(-1))
    desc = FqModelDesc(model=FQ_CIRCUIT, L=int(L), periodic=0, J=None, h=None, g=0.0, gates=ptr,
                       n_gates=int(sa.size), gate_sites=sa.ctypes.data_as(POINTER(ctypes.c_int)),
                       gate_widths=wa.ctypes.data_as(POINTER(ctypes.c_int)))
    return FloquetOp(desc, keep=(flat, sa, wa))


def arnoldi_eigs_batched(ops: Sequence[FloquetOp], phis: Sequence[float], nev: int, *, k=0, ncv: int,
                         tol: float = 1e-10, max_restarts: int = 200, filter_dtype: str = "c128",
                         refine: bool = True, seed: int = 0, want_vectors: bool = False, stream=None,
                         allow_not_converged=False, refine_k: int = 0, poly=None):
    """All (op, phi) problems in one call.

    ``k`` is one filter order for every op or a sequence with one per op;
    ``k = 0`` selects the paper's rule per chain length for the given ncv.
    Returns (evals[n_ops, n_phi, nev], resid, stats, status), plus the
    eigenvectors (list over problems of (nev, d) complex128 device tensors)
    when ``want_vectors``.
    """
    torch = _torch()
    n_ops, n_phi = len(ops), len(phis)
    handles = (c_void_p * n_ops)(*[o.handle for o in ops])
    ph, php = _dbl_array(phis)
    pc = None
    if poly is not None:
        c = np.asarray(poly, dtype=np.complex128)
        k = len(c) - 1
        pc, pcp = _dbl_array(np.stack([c.real, c.imag], axis=1).reshape(-1))
    if np.ndim(k) == 0:
        kk = None
        k0 = int(k)
    else:
        if len(k) != n_ops:
            raise ValueError("k needs one entry per op")
        kk = (ctypes.c_int * n_ops)(*[int(x) for x in k])
        k0 = int(k[0])
    opts = FqArnoldiOpts(k=k0, ncv=int(ncv), tol=float(tol), max_restarts=int(max_restarts),
                         filter_dtype=FQ_C64 if filter_dtype == "c64" else FQ_C128,
                         refine=1 if refine else 0, seed=int(seed), v0_dev=None, refine_k=int(refine_k),
                         poly_coeffs=pcp if pc is not None else None)
    evals = np.zeros(n_ops * n_phi * 2 * nev)
    resid = np.zeros(n_ops * n_phi * nev)
    stats = (FqArnoldiStats * (n_ops * n_phi))()
    vecs = None
    vec_ptrs = None
    if want_vectors:
        vecs = [torch.empty((nev, ops[i].dim), dtype=torch.complex128, device="cuda")
                for i in range(n_ops) for _ in range(n_phi)]
        vec_ptrs = (c_void_p * (n_ops * n_phi))(*[v.data_ptr() for v in vecs])
    st = lib().arnoldi_eigs_batched(handles, n_ops, php, n_phi, int(nev), ctypes.byref(opts), kk,
                                    evals.ctypes.data_as(POINTER(c_double)), vec_ptrs,
                                    resid.ctypes.data_as(POINTER(c_double)), stats, _stream_ptr(stream))
    check(st, "arnoldi_eigs_batched", allow=(FQ_OK, FQ_NOT_CONVERGED) if allow_not_converged else (FQ_OK,))
    ev = (evals[0::2] + 1j * evals[1::2]).reshape(n_ops, n_phi, nev)
    out = (ev, resid.reshape(n_ops, n_phi, nev), [s.as_dict() for s in stats], st)
    if want_vectors:
        out = out + (vecs,)
    return out


def host_schur(A: np.ndarray):
    """Host-only helper: complex Schur form with largest |eigenvalue| first.  Returns (T, Z, w)."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    a = np.ascontiguousarray(A.T).reshape(-1)  # column-major
    ab = np.stack([a.real, a.imag], axis=1).reshape(-1).copy()
    zb = np.zeros(2 * n * n)
    wb = np.zeros(2 * n)
    check(lib().fq_host_schur(n, ab.ctypes.data_as(POINTER(c_double)), zb.ctypes.data_as(POINTER(c_double)),
                              wb.ctypes.data_as(POINTER(c_double))), "fq_host_schur")
    T = (ab[0::2] + 1j * ab[1::2]).reshape(n, n).T
    Z = (zb[0::2] + 1j * zb[1::2]).reshape(n, n).T
    return T, Z, wb[0::2] + 1j * wb[1::2]


def paper_parameters(L: int, nev: int):
    """(ncv, k) from the paper's rule (see fq_paper_parameters in include/floquet.h)."""
    ncv, k = ctypes.c_int(), ctypes.c_int()
    check(lib().fq_paper_parameters(int(L), int(nev), ctypes.byref(ncv), ctypes.byref(k)), "fq_paper_parameters")
    return ncv.value, k.value


def set_graph_capture(on: bool):
    """HIP-graph replay of the lockstep filters of arnoldi_eigs_batched (see
    fq_set_graph_capture in include/floquet.h); on by default."""
    check(lib().fq_set_graph_capture(1 if on else 0), "fq_set_graph_capture")
