"""GPU parity of the entanglement entropy of states and eigenstates (Sec. 5,
Eq. (ee)) against the oracle, and of brickwork eigenstates against Page's
value (Eq. (page))."""

import math

import numpy as np
import pytest

from gpu_util import bw_op, require_gpu, say, to_dev, to_np
from oracle import entanglement
from workloads import brickwork, random_state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L", [6, 10, 13])
def test_random_states_parity(L):
    torch = require_gpu()
    say(f"entropy random states L={L}")
    states = random_state(2 ** L, 100 + L, count=4)
    p = brickwork(L, 1)
    with bw_op(p) as op:
        X = to_dev(states, torch.complex128)
        for LA in sorted({1, L // 2, L - 1, max(1, L // 3)}):
            got = op.entanglement_entropy(X, LA)
            ref = [entanglement.entropy(v, L, LA) for v in states]
            assert np.allclose(got, ref, atol=1e-10), (LA, got, ref)


def test_hand_states():
    torch = require_gpu()
    L = 6
    prod = np.zeros(2 ** L, complex)
    prod[9] = 1
    bell = np.zeros(2 ** L, complex)
    bell[0] = bell[0b001100] = 1 / math.sqrt(2)
    with bw_op(brickwork(L, 2)) as op:
        S = op.entanglement_entropy(to_dev(np.stack([prod, bell]), torch.complex128), 3)
    assert abs(S[0]) < 1e-12
    assert abs(S[1] - math.log(2)) < 1e-12


def test_brickwork_eigenstates_follow_page():
    # Eigenstates of the ergodic brickwork circuit are infinite-temperature
    # states: their cut entropy sits at Page's random-state value (Sec. 5).
    torch = require_gpu()
    L, nev = 12, 20
    p = brickwork(L, 4242)
    with bw_op(p) as op:
        ev, vecs, res, st, s = op.arnoldi_eigs(nev, 0.0, k=51, ncv=102, tol=1e-10, seed=3)
        assert res.max() < 1e-10
        for LA in (3, 6):
            S = op.entanglement_entropy(vecs, LA)
            ref = [entanglement.entropy(v, L, LA) for v in to_np(vecs)]
            assert np.allclose(S, ref, atol=1e-10)
            page = entanglement.page(L, LA)
            say(f"L={L} LA={LA}: mean S {S.mean():.4f} +- {S.std():.4f}, Page {page:.4f}")
            assert abs(S.mean() - page) < 0.05


@pytest.mark.timeout(300)
@pytest.mark.parametrize("L", [16, 18])
def test_circuit_workload_eigenstates_follow_page(L):
    # The brickwork circuit workload's solve (nev = 40, ncv = 100, complex64
    # filter + FP64 refinement, k by the paper's rule for this ncv) at sizes
    # the oracle can check pair by pair: every residual recomputed with the
    # oracle's matrix-free U, and the half-chain entropy of the eigenstates at
    # Page's random-state value (Sec. 5, Eq. (page)).
    from oracle import models
    require_gpu()
    p = brickwork(L, 5000 + L)
    nev, ncv = 40, 100
    with bw_op(p) as op:
        ev, vecs, res, st, s = op.arnoldi_eigs(nev, 0.0, k=0, ncv=ncv, tol=1e-9, filter_dtype="c64", block=4, seed=2)
        say(f"circuit workload L={L}: {st}")
        assert s == 0 and res.max() <= 1e-9
        S = op.entanglement_entropy(vecs, L // 2)
        v = to_np(vecs)
    r = [np.linalg.norm(models.bw_apply(p, v[n]) - ev[n] * v[n]) for n in range(nev)]
    assert max(r) <= 1e-9
    assert np.max(np.abs(np.abs(ev) - 1.0)) <= 1e-9
    ref = [entanglement.entropy(v[n], L, L // 2) for n in range(0, nev, 8)]
    assert np.allclose(S[0::8], ref, atol=1e-10)
    page = entanglement.page(L, L // 2)
    say(f"L={L} LA={L // 2}: mean S {S.mean():.4f} +- {S.std():.4f}, Page {page:.4f}")
    assert abs(S.mean() - page) < 0.05
