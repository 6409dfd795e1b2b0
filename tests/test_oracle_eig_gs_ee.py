"""Pins of the oracle's eigen-selection, Gram-Schmidt and entanglement code."""

import cmath
import math

import numpy as np
import pytest

from conftest import load_golden
from oracle import eig, entanglement, filters, gram_schmidt, models
from workloads import KickedIsingParams, brickwork, kicked_ising, random_state


def test_closest_hand_example():
    om = np.exp(1j * np.array([3.0, 0.1, -0.05, 1.0, -2.0, 0.2]))
    assert list(eig.closest(om, 3, 0.0)) == [2, 1, 5]
    # target pi: arc distances |3 - pi| = 0.14, |-2 + pi|... (-2 -> 2pi - 2 - pi = 1.14)
    assert list(eig.closest(om, 2, math.pi)) == [0, 4]


def test_full_closest_on_diagonal_unitary():
    # g = 0: U = diag(e^{-iE}); the closest eigenvalues are the basis-state phases.
    p = KickedIsingParams(L=3, J=np.array([1.0, 2, 3]), h=np.array([0.1, 0.2, 0.3]), g=0.0,
                          periodic=True, phi=0.0)
    om, V = eig.full_closest(models.ki_dense(p), 2, 0.0)
    # E = 0.2 (s=2) and -0.2 (s=5) are the two smallest |E| mod 2pi of the hand table.
    got = sorted(int(np.argmax(np.abs(V[:, n]))) for n in range(2))
    assert got == [2, 5]
    assert np.allclose(sorted(np.angle(om)), [-0.2, 0.2], atol=1e-14)


@pytest.mark.parametrize("which,L", [("ki", 10), ("bw", 10)])
def test_full_diag_residuals_at_paper_level(which, L):
    # Table "bench": zgeev residuals at L = 10 are ~1.9e-14; ours must be of that order.
    rows = {int(r[0]): r for r in load_golden("paper_table_bench.txt")}
    p = kicked_ising(L, 21) if which == "ki" else brickwork(L, 21)
    U = models.dense(p)
    om, V = eig.full_closest(U, 50, 0.0)
    res = eig.residuals(lambda v: U @ v, om, V)
    assert res.max() < 10 * rows[L][2]
    assert np.allclose(np.abs(om), 1.0, atol=1e-12)
    rq = np.array([eig.rayleigh(lambda v: U @ v, V[:, n]) for n in range(5)])
    assert np.allclose(rq, om[:5], atol=1e-12)


def test_residual_and_rayleigh_of_a_mixed_vector_hand_example():
    # Eq. (residual) on a vector that is NOT an eigenvector: U = diag(1, i),
    # v = (cos a, sin a).  By hand: U v - 1 v = (0, (i - 1) sin a), so
    # r = sqrt(2) sin a; the Rayleigh quotient is cos^2 a + i sin^2 a, and
    # U v - omega v = sin a cos a (1 - i) (-sin a, cos a), norm sqrt(2) sin a cos a.
    a = 0.1
    U = np.diag([1.0, 1j])
    v = np.array([math.cos(a), math.sin(a)], dtype=complex)
    mv = lambda x: U @ x  # noqa: E731
    r1 = eig.residuals(mv, np.array([1.0 + 0j]), v[:, None])
    assert abs(r1[0] - math.sqrt(2) * math.sin(a)) < 1e-15
    om = eig.rayleigh(mv, v)
    assert abs(om - (math.cos(a) ** 2 + 1j * math.sin(a) ** 2)) < 1e-15
    r2 = eig.residuals(mv, np.array([om]), v[:, None])
    assert abs(r2[0] - math.sqrt(2) * math.sin(a) * math.cos(a)) < 1e-15
    # one column per vector, in order; an exact eigenvector has residual 0
    V = np.stack([v, np.array([0.0, 1.0 + 0j])], axis=1)
    r3 = eig.residuals(mv, np.array([1.0 + 0j, 1j]), V)
    assert abs(r3[0] - math.sqrt(2) * math.sin(a)) < 1e-15 and r3[1] == 0.0


def test_filtered_eigenvalues_follow_closed_form():
    # Eigenvectors of U are eigenvectors of g_k(U) with eigenvalue g_k(omega) (Sec. 4).
    p = kicked_ising(7, 31)
    U = models.dense(p)
    om, V = eig.full_closest(U, 6, 0.4)
    for n in range(6):
        gv = filters.geometric_sum(lambda v: U @ v, V[:, n], 25, 0.4)
        lam = filters.gk_scalar(np.array([om[n]]), 25, 0.4)[0]
        assert np.linalg.norm(gv - lam * V[:, n]) < 1e-10 * abs(lam)


@pytest.mark.parametrize("d,j", [(64, 1), (200, 7), (1024, 30)])
def test_cgs2_invariants(d, j):
    rng = np.random.default_rng(d + j)
    A = rng.standard_normal((d, j)) + 1j * rng.standard_normal((d, j))
    V, _ = np.linalg.qr(A)
    w = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    h, beta, v = gram_schmidt.cgs2(V, w)
    assert np.linalg.norm(V.conj().T @ v) < 1e-13
    assert abs(np.linalg.norm(v) - 1) < 1e-14
    assert np.allclose(V @ h + beta * v, w, atol=1e-12)
    # Hand case: w already in span(V) leaves nothing (beta ~ 0).
    h2, beta2, _ = gram_schmidt.cgs2(V, V @ np.arange(1, j + 1))
    assert beta2 < 1e-12 and np.allclose(h2, np.arange(1, j + 1), atol=1e-12)


def test_entropy_hand_states():
    L = 6
    prod = np.zeros(2 ** L, complex)
    prod[5] = 1
    assert entanglement.entropy(prod, L, 3) == pytest.approx(0.0, abs=1e-14)
    # Bell pair between sites 3 and 4 (across the cut L_A = 3), rest in |0>:
    bell = np.zeros(2 ** L, complex)
    bell[0] = bell[0b001100] = 1 / math.sqrt(2)
    assert entanglement.entropy(bell, L, 3) == pytest.approx(math.log(2))
    assert entanglement.entropy(bell, L, 2) == pytest.approx(0.0, abs=1e-14)


def test_page_values():
    # Two qubits: Page's average is 1/3 nat (sum_{k=3}^{4} 1/k - 1/4).
    assert entanglement.page(2, 1) == pytest.approx(1 / 3)
    # Symmetry S_A = S_B, and with H_N = ln N + gamma + 1/(2N) + O(N^-2) the sum
    # gives ln m - m/(2n) + 1/(2mn) + O(n^-2) for m = 2^{L_A} <= n = 2^{L_B}.
    assert entanglement.page(10, 7) == pytest.approx(entanglement.page(10, 3))
    m, n = 2.0 ** 4, 2.0 ** 12
    assert entanglement.page(16, 4) == pytest.approx(math.log(m) - m / (2 * n) + 1 / (2 * m * n), abs=2e-8)


def test_random_states_follow_page():
    # Haar-random states sit at Page's value with small spread (Sec. 5).
    L = 10
    states = random_state(2 ** L, 12345, count=20)
    for LA in (3, 5):
        s = np.array([entanglement.entropy(v, L, LA) for v in states])
        # within four standard errors of the sample mean
        assert abs(s.mean() - entanglement.page(L, LA)) < 4 * s.std() / math.sqrt(len(s))
