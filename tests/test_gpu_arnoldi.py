"""GPU parity of the eigensolver against full diagonalisation (oracle)."""

import math

import numpy as np
import pytest

from gpu_util import ki_op, rel, require_gpu, say, to_dev, to_np
from oracle import eig, models
from workloads import CONFIGS, config_kicked_ising, kicked_ising

pytestmark = pytest.mark.gpu


def _match(evals, om_ref, tol):
    for x in evals:
        assert np.min(np.abs(om_ref - x)) < tol, (x, np.min(np.abs(om_ref - x)))


@pytest.mark.parametrize("filter_dtype", ["c128", "c64"])
def test_ki_L10_workload(filter_dtype):
    # Kicked Ising L = 10, k = 64, nev = 20, ncv = 60, phi = 0, against zgeev.
    c = CONFIGS["ki_L10"]
    say(f"arnoldi ki_L10 {filter_dtype}")
    p = config_kicked_ising("ki_L10")
    U = models.ki_dense(p)
    om_ref, V_ref = eig.full_closest(U, c["nev"], c["phi"])
    with ki_op(p) as op:
        ev, vecs, res, stats, st = op.arnoldi_eigs(c["nev"], c["phi"], k=c["k"], ncv=c["ncv"], tol=1e-10,
                                                   filter_dtype=filter_dtype, seed=1)
        vecs = to_np(vecs)
    say(stats)
    assert np.max(np.abs(ev - om_ref)) < 1e-12
    assert res.max() <= 1e-10
    for n in range(c["nev"]):
        assert abs(abs(np.vdot(V_ref[:, n], vecs[n])) - 1) < 1e-10
        # residual recomputed by the oracle
        assert np.linalg.norm(U @ vecs[n] - ev[n] * vecs[n]) < 1e-10


@pytest.mark.parametrize("L,phi,nev,k,ncv", [(8, 2.0, 6, 20, 20), (12, 4.1, 10, 60, 40)])
def test_random_targets(L, phi, nev, k, ncv):
    say(f"arnoldi L={L} phi={phi}")
    p = kicked_ising(L, 900 + L)
    U = models.ki_dense(p)
    om_ref, _ = eig.full_closest(U, nev, phi)
    with ki_op(p) as op:
        ev, _, res, stats, st = op.arnoldi_eigs(nev, phi, k=k, ncv=ncv, tol=1e-10, seed=3, want_vectors=False)
    assert np.max(np.abs(ev - om_ref)) < 1e-12
    assert res.max() <= 1e-10


def test_not_converged_reports_partial():
    p = kicked_ising(10, 5)
    with ki_op(p) as op:
        ev, _, res, stats, st = op.arnoldi_eigs(20, 0.0, k=4, ncv=24, tol=1e-10, max_restarts=0, seed=1,
                                                want_vectors=False, allow_not_converged=True)
    assert st == 1
    assert stats["nconv"] == int((res <= 1e-10).sum())


def test_refinement_filter_order():
    # a separate (lower) filter order for the FP64 refinement still meets the
    # FP64 targets; the U-application count reflects both orders
    p = kicked_ising(10, 77)
    U = models.ki_dense(p)
    om_ref, _ = eig.full_closest(U, 8, 0.7)
    with ki_op(p) as op:
        ev, _, res, st, status = op.arnoldi_eigs(8, 0.7, k=40, ncv=24, tol=1e-10, filter_dtype="c64", seed=4,
                                                 want_vectors=False, refine_k=20)
    assert np.max(np.abs(ev - om_ref)) < 1e-12
    assert res.max() <= 1e-10
    assert st["n_U_apps_c64"] % 40 == 0
    # FP64 part: refinement filter applications of order 20 plus nev = 8 U per Ritz check
    assert st["n_U_apps"] > st["n_U_apps_c64"]
