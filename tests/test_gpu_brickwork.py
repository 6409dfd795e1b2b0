"""GPU parity of the brickwork U pass (light-cone split into two tile passes),
its Horner filter and the eigensolver, against the oracle."""

import math

import numpy as np
import pytest

from gpu_util import bw_op, rel, require_gpu, say, to_dev, to_np
from oracle import eig, filters, models
from workloads import (brickwork, brickwork_cz, brickwork_from_matrices, brickwork_layout, haar_unitary,
                       random_state)

pytestmark = pytest.mark.gpu

TOL_U = {"c128": 1e-12, "c64": 3e-6}


def _dt(name):
    torch = require_gpu()
    return torch.complex128 if name == "c128" else torch.complex64


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("L", [2, 3, 4, 5, 8, 11, 12, 13])
def test_apply_U_dense_parity(dt, L):
    say(f"bw apply_U dense L={L} {dt}")
    p = brickwork(L, 50 + L)
    U = models.bw_dense(p)
    psi = random_state(2 ** L, 5 + L)[0]
    with bw_op(p) as op:
        out = to_np(op.apply_U(to_dev(psi, _dt(dt))))
    assert rel(out, U @ psi) < TOL_U[dt]


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("L", [14, 15, 18, 24])
def test_apply_U_matrix_free_parity(dt, L):
    say(f"bw apply_U matrix-free L={L} {dt}")
    p = brickwork(L, 60 + L)
    psi = random_state(2 ** L, 3)[0]
    with bw_op(p) as op:
        out = to_np(op.apply_U(to_dev(psi, _dt(dt))))
    assert rel(out, models.bw_apply(p, psi)) < TOL_U[dt]


def _cnot_high_controls_low():
    m = np.eye(4, dtype=complex)
    m[2:, 2:] = [[0, 1], [1, 0]]
    return m


def test_layer_order_hand_example():
    # X on site 1 (first layer), then CNOT with site 1 as control (second
    # layer): |00> -> |10> -> |11>; the other order or local-bit convention gives |10>.
    torch = require_gpu()
    X = np.array([[0, 1], [1, 0]], complex)
    p = brickwork_from_matrices(2, [X, np.eye(2), _cnot_high_controls_low()])
    e = np.zeros(4, complex)
    e[0] = 1
    with bw_op(p) as op:
        out = to_np(op.apply_U(to_dev(e, torch.complex128)))
    assert np.allclose(out, [0, 0, 0, 1], atol=1e-15)


@pytest.mark.parametrize("L", [16, 24])
def test_product_gates_eigenstate(L):
    # Product two-site gates make U a product of one-site unitaries A_i B_i;
    # a product of their eigenvectors is an eigenvector of U with the product
    # of the eigenvalues (any L; no dense U needed).
    torch = require_gpu()
    rng = np.random.default_rng(L)
    layer_b, layer_a = brickwork_layout(L)
    mats, fac = [], {"b": {}, "a": {}}
    for name, layer in (("b", layer_b), ("a", layer_a)):
        for sites in layer:
            if len(sites) == 1:
                u = haar_unitary(2, rng)
                fac[name][sites[0]] = u
                mats.append(u)
            else:
                x, y = haar_unitary(2, rng), haar_unitary(2, rng)
                fac[name][sites[0]], fac[name][sites[1]] = x, y
                mats.append(np.kron(x, y))
    p = brickwork_from_matrices(L, mats)
    v = np.ones(1, complex)
    lam = 1.0 + 0j
    for i in range(1, L + 1):
        w, V = np.linalg.eig(fac["a"][i] @ fac["b"][i])
        v = np.kron(v, V[:, i % 2])
        lam *= w[i % 2]
    with bw_op(p) as op:
        out = to_np(op.apply_U(to_dev(v, torch.complex128)))
    assert np.linalg.norm(out - lam * v) < 1e-12


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("L,k,phi", [(6, 9, 0.3), (12, 30, 2.0), (16, 4, 1.0)])
def test_apply_filter_parity(dt, L, k, phi):
    say(f"bw apply_filter L={L} k={k} {dt}")
    p = brickwork(L, 70 + L)
    psi = random_state(2 ** L, 8)[0]
    mv = (lambda v, U=models.bw_dense(p): U @ v) if L <= 12 else (lambda v: models.bw_apply(p, v))
    ref = filters.geometric_sum(mv, psi, k, phi)
    with bw_op(p) as op:
        out = to_np(op.apply_filter(to_dev(psi, _dt(dt)), k, phi))
    tol = 1e-12 * (k + 1) if dt == "c128" else 2e-7 * (k + 1) + 3e-6
    assert rel(out, ref) < tol


@pytest.mark.timeout(300)
def test_apply_filter_L24_workload_elementwise():
    # the brick-wall filter as the L = 24 benchmark runs it (the workload's
    # seeded Haar circuit, both passes with e^{-i phi} and +psi fused into the
    # second, complex64 through the pipelined tile kernel), element-wise
    # against the oracle's geometric sum (Eq. (geo)); complex128 beside it
    from workloads import CONFIGS
    c = CONFIGS["bw_L24"]
    p = brickwork(c["L"], c["seed"])
    psi = random_state(2 ** c["L"], 12)[0]
    k, phi = 2, 0.7
    ref = filters.geometric_sum(lambda v: models.bw_apply(p, v), psi, k, phi)
    scale = np.max(np.abs(ref))
    with bw_op(p) as op:
        for dt in ("c64", "c128"):
            say(f"bw apply_filter L=24 workload k={k} {dt}")
            out = to_np(op.apply_filter(to_dev(psi, _dt(dt)), k, phi))
            err = float(np.max(np.abs(out - ref)) / scale)
            tol = 1e-12 * (k + 1) if dt == "c128" else 2e-7 * (k + 1) + 3e-6
            assert err < tol, (dt, err)
            del out


def test_apply_polynomial_parity():
    torch = require_gpu()
    p = brickwork(9, 71)
    U = models.bw_dense(p)
    coeffs = np.array([0.5, 1j, -0.25, 0.1 + 0.2j])
    psi = random_state(2 ** 9, 4)[0]
    with bw_op(p) as op:
        out = to_np(op.apply_polynomial(to_dev(psi, torch.complex128), coeffs))
    assert rel(out, filters.polynomial(lambda v: U @ v, psi, list(coeffs))) < 1e-12


@pytest.mark.parametrize("filter_dtype", ["c128", "c64"])
def test_arnoldi_brickwork_L10(filter_dtype):
    say(f"bw arnoldi L=10 {filter_dtype}")
    L, nev, k, ncv = 10, 20, 30, 60
    p = brickwork(L, 1234)
    U = models.bw_dense(p)
    om_ref, V_ref = eig.full_closest(U, nev, 0.0)
    with bw_op(p) as op:
        ev, vecs, res, stats, st = op.arnoldi_eigs(nev, 0.0, k=k, ncv=ncv, tol=1e-10, seed=2,
                                                   filter_dtype=filter_dtype)
        vecs = to_np(vecs)
    assert np.max(np.abs(ev - om_ref)) < 1e-12
    assert res.max() <= 1e-10
    for n in range(nev):
        assert np.linalg.norm(U @ vecs[n] - ev[n] * vecs[n]) < 1e-10


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("L", [7, 10, 16])
def test_other_gate_set_parity(dt, L):
    # controlled-Z entanglers dressed with random one-site rotations: U and the
    # Horner filter against the oracle (dense for L <= 12, matrix-free above)
    say(f"bw CZ gate set L={L} {dt}")
    p = brickwork_cz(L, 300 + L)
    psi = random_state(2 ** L, 12)[0]
    mv = (lambda v, U=models.bw_dense(p): U @ v) if L <= 12 else (lambda v: models.bw_apply(p, v))
    with bw_op(p) as op:
        out_u = to_np(op.apply_U(to_dev(psi, _dt(dt))))
        out_f = to_np(op.apply_filter(to_dev(psi, _dt(dt)), 12, 0.7))
    assert rel(out_u, mv(psi)) < TOL_U[dt]
    tol = 1e-12 * 13 if dt == "c128" else 2e-7 * 13 + 3e-6
    assert rel(out_f, filters.geometric_sum(mv, psi, 12, 0.7)) < tol


def test_other_gate_set_eigenpairs():
    L, nev = 10, 12
    p = brickwork_cz(L, 777)
    U = models.bw_dense(p)
    om_ref, _ = eig.full_closest(U, nev, 1.9)
    with bw_op(p) as op:
        ev, _, res, stats, st = op.arnoldi_eigs(nev, 1.9, k=40, ncv=40, tol=1e-10, seed=3, filter_dtype="c64",
                                                want_vectors=False)
    assert np.max(np.abs(ev - om_ref)) < 1e-12
    assert res.max() <= 1e-10
