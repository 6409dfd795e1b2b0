"""Pins of the oracle's Floquet operators against facts that do not come from
the oracle itself: hand-derived worked examples, closed-form spectra of special
cases, unitarity, and agreement of two independent constructions."""

import cmath
import math
from collections import Counter

import numpy as np
import pytest

from conftest import load_golden
from oracle import models
from workloads import (CircuitParams, circuit, circuit_from_brickwork, KickedIsingParams, brickwork, brickwork_from_matrices,
                       kicked_ising)


def _ki(L, J, h, g, periodic=True):
    return KickedIsingParams(L=L, J=np.asarray(J, float), h=np.asarray(h, float), g=g,
                             periodic=periodic, phi=0.0)


def _match_spectra(a, b, tol):
    """Greedy nearest matching of two eigenvalue multisets."""
    a = list(np.asarray(a, complex))
    b = list(np.asarray(b, complex))
    assert len(a) == len(b)
    for x in a:
        j = int(np.argmin([abs(x - y) for y in b]))
        assert abs(x - b[j]) < tol, (x, b[j])
        b.pop(j)


def test_ki_energies_hand_example():
    # tests/golden/ki_L3_energies.txt: L=3, J=(1,2,3), h=(0.1,0.2,0.3), by hand.
    rows = load_golden("ki_L3_energies.txt")
    Ep = models.ki_energies(3, [1, 2, 3], [0.1, 0.2, 0.3], True)
    Eo = models.ki_energies(3, [1, 2, 3], [0.1, 0.2, 0.3], False)
    Ez = models.ki_energies(3, [1, 2, 3], [0, 0, 0], True)
    for s, ep, eo, ez in rows:
        s = int(s)
        assert Ep[s] == pytest.approx(ep, abs=1e-13)
        assert Eo[s] == pytest.approx(eo, abs=1e-13)
        assert Ez[s] == pytest.approx(ez, abs=1e-13)


def test_ki_g0_is_diagonal_phase():
    # g = 0: K = I, so U = diag(exp(-i E(s))) with the hand-derived energies.
    rows = load_golden("ki_L3_energies.txt")
    U = models.ki_dense(_ki(3, [1, 2, 3], [0.1, 0.2, 0.3], 0.0))
    expect = np.array([cmath.exp(-1j * r[1]) for r in rows])
    assert np.allclose(U, np.diag(expect), atol=1e-14)


def test_ki_kick_sign_and_order_hand_example():
    # L = 2, open, J_1 = 0.5, h = (0.3, -0.2), g = 0.4.  K first, then D:
    # K|00> = (c|0> - i s|1>) (x) (c|0> - i s|1>) = c^2|00> - ics|01> - ics|10> - s^2|11>
    # E(00) = 0.6, E(01) = 0.0, E(10) = -1.0, E(11) = 0.4 (by hand).
    c, s = math.cos(0.4), math.sin(0.4)
    E = [0.6, 0.0, -1.0, 0.4]
    expect = np.array([c * c, -1j * c * s, -1j * c * s, -s * s]) * np.exp(-1j * np.array(E))
    p = _ki(2, [0.5, 0.0], [0.3, -0.2], 0.4, periodic=False)
    e0 = np.zeros(4, complex)
    e0[0] = 1
    assert np.allclose(models.ki_dense(p) @ e0, expect, atol=1e-14)
    assert np.allclose(models.ki_apply(p, e0), expect, atol=1e-14)


@pytest.mark.parametrize("L", [3, 6, 7])
def test_ki_free_kick_spectrum(L):
    # J = h = 0: U = exp(-i g X)^{(x)L}; eigenvalues exp(-i g (L - 2m)) with
    # multiplicity binomial(L, m).
    g = 0.37
    U = models.ki_dense(_ki(L, np.zeros(L), np.zeros(L), g))
    expect = [cmath.exp(-1j * g * (L - 2 * m)) for m in range(L + 1) for _ in range(math.comb(L, m))]
    _match_spectra(np.linalg.eigvals(U), expect, 1e-10)


def test_ki_g_half_pi_spectrum_hand_example():
    # g = pi/2: K = (-i)^L X^{(x)L} pairs s with its complement s'; on that pair
    # U has eigenvalues +-(-i)^L exp(-i (E(s)+E(s'))/2) = +-(-i)^L exp(-i E_zz(s)).
    # L = 3 periodic: E_zz in {6, -4, 0, -2} for the pairs (0,7),(1,6),(2,5),(3,4).
    p = _ki(3, [1, 2, 3], [0.1, 0.2, 0.3], math.pi / 2)
    pref = (-1j) ** 3
    expect = [sgn * pref * cmath.exp(-1j * e) for e in (6, -4, 0, -2) for sgn in (1, -1)]
    _match_spectra(np.linalg.eigvals(models.ki_dense(p)), expect, 1e-12)


@pytest.mark.parametrize("L,periodic", [(5, True), (8, True), (9, False)])
def test_ki_dense_unitary_and_matches_matrix_free(L, periodic):
    p = kicked_ising(L, 11 + L, periodic=periodic)
    U = models.ki_dense(p)
    assert np.linalg.norm(U.conj().T @ U - np.eye(2 ** L)) < 1e-12
    rng = np.random.default_rng(5)
    psi = rng.standard_normal(2 ** L) + 1j * rng.standard_normal(2 ** L)
    assert np.allclose(U @ psi, models.ki_apply(p, psi), atol=1e-12)


def _cnot_high_controls_low():
    m = np.eye(4, dtype=complex)
    m[2:, 2:] = [[0, 1], [1, 0]]
    return m


def _cnot_low_controls_high():
    m = np.zeros((4, 4), complex)
    m[0, 0] = m[2, 2] = 1
    m[3, 1] = m[1, 3] = 1
    return m


X = np.array([[0, 1], [1, 0]], complex)
I2 = np.eye(2, dtype=complex)
I4 = np.eye(4, dtype=complex)


@pytest.mark.parametrize("L,mats,start,expect", [
    # L = 2: layer b = [u_1, u_2], layer a = [u_12].  X on site 1 first, then
    # CNOT with site 1 as control: |00> -> |10> -> |11> (index 3).  The reversed
    # layer order or the other local-bit convention would give index 2.
    (2, [X, I2, _cnot_high_controls_low()], 0, 3),
    # L = 3: layer b = [u_1, u_23], layer a = [u_12, u_3]: |000> -> |100> -> |110> (6).
    (3, [X, I4, _cnot_high_controls_low(), I2], 0, 6),
    # L = 4: layer b = [u_1, u_23, u_4], layer a = [u_12, u_34]:
    # X on site 4, then CNOT controlled by site 4 onto site 3: |0000> -> |0001> -> |0011>.
    (4, [I2, I4, X, I4, _cnot_low_controls_high()], 0, 3),
])
def test_bw_layer_order_and_local_index_hand_examples(L, mats, start, expect):
    p = brickwork_from_matrices(L, mats)
    e = np.zeros(2 ** L, complex)
    e[start] = 1
    out_dense = models.bw_dense(p) @ e
    out_mf = models.bw_apply(p, e)
    target = np.zeros(2 ** L, complex)
    target[expect] = 1
    assert np.allclose(out_dense, target, atol=1e-14)
    assert np.allclose(out_mf, target, atol=1e-14)


@pytest.mark.parametrize("L", [4, 5])
def test_bw_product_gates_spectrum(L):
    # Two-site gates u_{i,i+1} = a (x) b make each layer a product of one-site
    # unitaries; U = U_a U_b is then prod over sites of (A_i B_i) and its
    # eigenvalues are all products of one eigenvalue of each A_i B_i.
    from workloads import brickwork_layout, haar_unitary
    rng = np.random.default_rng(3)
    layer_b, layer_a = brickwork_layout(L)
    mats, site_factor = [], {"b": {}, "a": {}}
    for name, layer in (("b", layer_b), ("a", layer_a)):
        for sites in layer:
            if len(sites) == 1:
                u = haar_unitary(2, rng)
                site_factor[name][sites[0]] = u
                mats.append(u)
            else:
                a, b = haar_unitary(2, rng), haar_unitary(2, rng)
                site_factor[name][sites[0]] = a
                site_factor[name][sites[1]] = b
                mats.append(np.kron(a, b))
    p = brickwork_from_matrices(L, mats)
    per_site = [np.linalg.eigvals(site_factor["a"][i] @ site_factor["b"][i]) for i in range(1, L + 1)]
    expect = [1.0 + 0j]
    for ev in per_site:
        expect = [x * y for x in expect for y in ev]
    _match_spectra(np.linalg.eigvals(models.bw_dense(p)), expect, 1e-10)


@pytest.mark.parametrize("L", [2, 6, 7, 10])
def test_bw_dense_unitary_and_matches_matrix_free(L):
    p = brickwork(L, 77 + L)
    U = models.bw_dense(p)
    assert np.linalg.norm(U.conj().T @ U - np.eye(2 ** L)) < 1e-11
    rng = np.random.default_rng(6)
    psi = rng.standard_normal(2 ** L) + 1j * rng.standard_normal(2 ** L)
    assert np.allclose(U @ psi, models.bw_apply(p, psi), atol=1e-12)


def test_bw_layer_swap_keeps_spectrum():
    # U_a U_b and U_b U_a are similar (conjugate by U_a), so the spectrum does
    # not depend on which layer acts first; the order only moves eigenvectors.
    L = 6
    p = brickwork(L, 99)
    lb, la = models.bw_gate_list(p)

    def layer(lst):
        M = np.ones((1, 1), complex)
        for _, u in lst:
            M = np.kron(M, u)
        return M

    Ua, Ub = layer(la), layer(lb)
    _match_spectra(np.linalg.eigvals(Ua @ Ub), np.linalg.eigvals(Ub @ Ua), 1e-10)
    assert np.allclose(models.bw_dense(p), Ua @ Ub, atol=1e-13)


# ---------------------------------------------------------------------------
# General local circuits
# ---------------------------------------------------------------------------

def _circ(L, gates):
    """CircuitParams from a list of (site, matrix) in acting order."""
    sites = [s for s, _ in gates]
    widths = [1 if np.asarray(m).shape == (2, 2) else 2 for _, m in gates]
    flat = np.concatenate([np.asarray(m, dtype=np.complex128).reshape(-1) for _, m in gates])
    return CircuitParams(L=L, sites=np.array(sites), widths=np.array(widths), gates=flat, phi=0.0)


X2 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128)


@pytest.mark.parametrize("gates,expect", [
    # X on site 1 (the most significant bit) then CNOT controlled by site 1: |00> -> |10> -> |11>
    ([(1, X2), (1, CNOT)], 3),
    # the same gates in the other order: |00> -> |00> -> |10>
    ([(1, CNOT), (1, X2)], 2),
    # X on site 2 then CNOT (control site 1 is 0): |00> -> |01>
    ([(2, X2), (1, CNOT)], 1),
])
def test_circuit_order_hand_examples(gates, expect):
    p = _circ(2, gates)
    psi = np.zeros(4, dtype=np.complex128)
    psi[0] = 1
    for out in (models.circuit_dense(p) @ psi, models.circuit_apply(p, psi)):
        assert np.argmax(np.abs(out)) == expect and abs(abs(out[expect]) - 1) < 1e-15


@pytest.mark.parametrize("L", [5, 8])
def test_circuit_of_brickwork_layout_is_brickwork(L):
    # the brickwork written as a general gate list gives the same U exactly
    p = brickwork(L, 600 + L)
    Ub = models.bw_dense(p)
    Uc = models.circuit_dense(circuit_from_brickwork(p))
    assert np.max(np.abs(Ub - Uc)) < 1e-13


@pytest.mark.parametrize("L", [4, 7])
def test_circuit_unitary_and_matrix_free(L):
    p = circuit(L, 700 + L, depth=3)
    U = models.circuit_dense(p)
    assert np.max(np.abs(U.conj().T @ U - np.eye(2 ** L))) < 1e-12
    psi = np.random.default_rng(1).standard_normal(2 ** L) + 0j
    assert np.max(np.abs(U @ psi - models.circuit_apply(p, psi))) < 1e-12


def test_circuit_layers_commute_when_disjoint():
    # gates on disjoint sites commute: swapping them inside the list keeps U
    rng = np.random.default_rng(5)
    a = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))[0]
    b = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))[0]
    U1 = models.circuit_dense(_circ(5, [(1, a), (3, b)]))
    U2 = models.circuit_dense(_circ(5, [(3, b), (1, a)]))
    assert np.max(np.abs(U1 - U2)) < 1e-14
