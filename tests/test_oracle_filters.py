"""Pins of the oracle's geometric-sum filter: closed forms of the paper
(Eq. (geo2), Eq. (gkmapping)), special cases and the spectral form."""

import cmath
import math

import numpy as np
import pytest

from oracle import filters, models
from workloads import brickwork, kicked_ising


@pytest.mark.parametrize("k,phi", [(0, 0.0), (1, 0.3), (7, 2.0), (30, -1.1)])
def test_gk_scalar_matches_dirichlet_on_circle(k, phi):
    theta = np.linspace(-math.pi, math.pi, 1001)
    a = filters.gk_scalar(np.exp(1j * theta), k, phi)
    b = filters.gk_dirichlet(theta, k, phi)
    assert np.allclose(a, b, atol=1e-10 * (k + 1))


@pytest.mark.parametrize("k", [1, 5, 30, 400])
def test_gk_peak_and_first_zeros(k):
    # Sec. 3 after Eq. (gkmapping): value k+1 at the target, zero at +-2pi/(k+1).
    phi = 0.7
    assert filters.gk_dirichlet(phi, k, phi) == pytest.approx(k + 1)
    assert filters.gk_scalar(np.array([cmath.exp(1j * phi)]), k, phi)[0] == pytest.approx(k + 1)
    for sgn in (1, -1):
        th = phi + sgn * 2 * math.pi / (k + 1)
        assert abs(filters.gk_dirichlet(th, k, phi)) < 1e-9 * (k + 1)
        assert abs(filters.gk_scalar(np.array([cmath.exp(1j * th)]), k, phi)[0]) < 1e-9 * (k + 1)


def test_gk_scalar_small_hand_values():
    # k = 1: g_1(w) = 1 + e^{-i phi} w; k = 2 at w = -1, phi = 0: 1 - 1 + 1 = 1.
    w = np.array([0.3 + 0.4j])
    assert filters.gk_scalar(w, 1, 0.5)[0] == pytest.approx(1 + cmath.exp(-0.5j) * w[0])
    assert filters.gk_scalar(np.array([-1 + 0j]), 2, 0.0)[0] == pytest.approx(1.0)


def test_geometric_sum_k0_is_identity():
    p = kicked_ising(5, 1)
    psi = np.random.default_rng(0).standard_normal(32) + 0j
    assert np.array_equal(filters.geometric_sum(lambda v: models.ki_apply(p, v), psi, 0, 1.0), psi)


@pytest.mark.parametrize("which,L,k,phi", [("ki", 6, 9, 0.4), ("bw", 6, 13, 2.5), ("ki", 8, 64, 0.0)])
def test_geometric_sum_closed_form_identity(which, L, k, phi):
    # Eq. (geo2) as a matrix identity: (1 - e^{-i phi} U) g_k(U) psi
    #   = (1 - e^{-i (k+1) phi} U^{k+1}) psi.
    p = kicked_ising(L, 4) if which == "ki" else brickwork(L, 4)
    U = models.dense(p)
    psi = np.random.default_rng(1).standard_normal(2 ** L) + 1j * np.random.default_rng(2).standard_normal(2 ** L)
    g = filters.geometric_sum(lambda v: U @ v, psi, k, phi)
    lhs = g - cmath.exp(-1j * phi) * (U @ g)
    rhs = psi - cmath.exp(-1j * (k + 1) * phi) * (np.linalg.matrix_power(U, k + 1) @ psi)
    assert np.allclose(lhs, rhs, atol=1e-11 * (k + 1))


@pytest.mark.parametrize("L,k,phi", [(6, 20, 0.0), (8, 64, 1.3)])
def test_geometric_sum_matches_spectral_form(L, k, phi):
    # The filter keeps eigenvectors and maps omega -> g_k(omega) (Sec. 3).
    p = kicked_ising(L, 8)
    U = models.dense(p)
    psi = np.random.default_rng(3).standard_normal(2 ** L) + 0j
    a = filters.geometric_sum(lambda v: U @ v, psi, k, phi)
    b = filters.gk_spectral(U, psi, k, phi)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-11


def test_filter_phase_shift_equivalence():
    # g_k(U; phi) = g_k(e^{-i phi} U; 0).
    p = kicked_ising(5, 9)
    U = models.dense(p)
    psi = np.random.default_rng(4).standard_normal(32) + 0j
    phi = 0.9
    a = filters.geometric_sum(lambda v: U @ v, psi, 11, phi)
    b = filters.geometric_sum(lambda v: cmath.exp(-1j * phi) * (U @ v), psi, 11, 0.0)
    assert np.allclose(a, b, atol=1e-12)


def test_polynomial_reduces_to_geometric_sum():
    p = kicked_ising(5, 10)
    mv = lambda v: models.ki_apply(p, v)  # noqa: E731
    psi = np.random.default_rng(5).standard_normal(32) + 0j
    phi, k = 0.3, 6
    coeffs = [cmath.exp(-1j * m * phi) for m in range(k + 1)]
    assert np.allclose(filters.polynomial(mv, psi, coeffs), filters.geometric_sum(mv, psi, k, phi), atol=1e-12)
