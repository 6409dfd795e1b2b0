"""GPU parity of general local Floquet circuits (any order of one- and
two-site gates, split into two blocks along their light cone) against the
oracle's dense and matrix-free U."""

import numpy as np
import pytest

from gpu_util import bw_op, circ_op, memo, rel, require_gpu, say, to_dev, to_np
from oracle import eig, filters, models
from workloads import brickwork, circuit, circuit_from_brickwork, random_state

pytestmark = pytest.mark.gpu

TOL_U = {"c128": 1e-12, "c64": 3e-6}


def _dt(name):
    torch = require_gpu()
    return torch.complex128 if name == "c128" else torch.complex64


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("L,depth", [(3, 2), (6, 3), (11, 4), (12, 3), (13, 3), (16, 3), (18, 5)])
def test_circuit_U_and_filter_parity(dt, L, depth):
    say(f"circuit U/filter L={L} depth={depth} {dt}")
    p = circuit(L, 800 + L, depth=depth)
    psi = random_state(2 ** L, 21)[0]
    if L <= 12:
        U = memo(("circuit", L, 800 + L, depth), lambda: models.circuit_dense(p))
        mv = lambda v: U @ v  # noqa: E731
    else:
        mv = lambda v: models.circuit_apply(p, v)  # noqa: E731
    with circ_op(p) as op:
        out_u = to_np(op.apply_U(to_dev(psi, _dt(dt))))
        out_f = to_np(op.apply_filter(to_dev(psi, _dt(dt)), 9, 0.4))
    assert rel(out_u, mv(psi)) < TOL_U[dt]
    tol = 1e-12 * 10 if dt == "c128" else 2e-7 * 10 + 3e-6
    assert rel(out_f, filters.geometric_sum(mv, psi, 9, 0.4)) < tol


@pytest.mark.parametrize("L", [10, 16])
def test_brickwork_as_circuit_matches_brickwork(L):
    # the brickwork written as a gate list takes the same split and windows
    torch = require_gpu()
    p = brickwork(L, 900 + L)
    psi = random_state(2 ** L, 22)[0]
    with bw_op(p) as a, circ_op(circuit_from_brickwork(p)) as b:
        x = to_dev(psi, torch.complex128)
        ya, yb = to_np(a.apply_filter(x, 5, 1.0)), to_np(b.apply_filter(x, 5, 1.0))
    assert np.max(np.abs(ya - yb)) < 1e-14


def test_circuit_eigenpairs():
    L, nev = 10, 10
    p = circuit(L, 555, depth=3)
    U = models.circuit_dense(p)
    om_ref, _ = eig.full_closest(U, nev, 0.8)
    with circ_op(p) as op:
        ev, vecs, res, stats, st = op.arnoldi_eigs(nev, 0.8, k=40, ncv=36, tol=1e-10, seed=5, filter_dtype="c64")
        vecs = to_np(vecs)
    assert np.max(np.abs(ev - om_ref)) < 1e-12
    assert res.max() <= 1e-10
    for n in range(nev):
        assert np.linalg.norm(U @ vecs[n] - ev[n] * vecs[n]) < 1e-10


def test_circuit_too_deep_for_two_blocks():
    # a deep circuit at L = 20 has a light cone wider than two tiles: EINVAL
    require_gpu()
    from paper_2102_05054_amd import FloquetError
    p = circuit(20, 77, depth=12)
    with pytest.raises(FloquetError):
        circ_op(p)


def test_circuit_bad_description():
    require_gpu()
    from paper_2102_05054_amd import FloquetError, circuit as mk
    u = np.eye(4, dtype=np.complex128).reshape(-1)
    with pytest.raises(FloquetError):
        mk(4, [4], [2], u)  # pair (4, 5) outside the chain
    with pytest.raises(FloquetError):
        mk(4, [1], [3], np.eye(8, dtype=np.complex128).reshape(-1)[:16])  # width 3


def test_circuit_complex64_only_when_complex128_tiles_are_too_small():
    # depth 3 at L = 24: the light cone fits 14-bit complex64 tiles but not
    # 13-bit complex128 ones; complex64 works, complex128 calls fail cleanly
    torch = require_gpu()
    from paper_2102_05054_amd import FloquetError
    L = 24
    p = circuit(L, 2424, depth=3)
    psi = random_state(2 ** L, 23)[0]
    with circ_op(p) as op:
        out = to_np(op.apply_U(to_dev(psi, torch.complex64)))
        with pytest.raises(FloquetError):
            op.apply_U(to_dev(psi, torch.complex128))
    assert rel(out, models.circuit_apply(p, psi)) < TOL_U["c64"]


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("L,depth", [(14, 1), (14, 2), (16, 1), (17, 2)])
def test_shallow_circuits_few_windows(dt, L, depth):
    # shallow circuits give passes of one to three windows, so the first and
    # last window fused with the tile's load and store coincide or touch
    say(f"shallow circuit L={L} depth={depth} {dt}")
    p = circuit(L, 870 + L + depth, depth=depth)
    psi = random_state(2 ** L, 23, 3)
    mv = lambda v: models.circuit_apply(p, v)  # noqa: E731
    with circ_op(p) as op:
        out_u = to_np(op.apply_U(to_dev(psi[0], _dt(dt))))
        out_m = to_np(op.apply_filter_many(to_dev(psi, _dt(dt)), 5, 2.1))
    assert rel(out_u, mv(psi[0])) < TOL_U[dt]
    tol = 1e-12 * 6 if dt == "c128" else 2e-7 * 6 + 3e-6
    for j in range(3):
        assert rel(out_m[j], filters.geometric_sum(mv, psi[j], 5, 2.1)) < tol, j
