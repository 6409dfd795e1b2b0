"""GPU parity of the kicked-Ising U pass and the Horner filter against the
oracle (dense Kronecker U for L <= 12, the oracle's matrix-free U above)."""

import cmath
import math

import numpy as np
import pytest

from gpu_util import ki_op, memo, rel, require_gpu, say, to_dev, to_np
from oracle import filters, models
from workloads import KickedIsingParams, kicked_ising, random_state

pytestmark = pytest.mark.gpu

# complex128: rounding of O(L) butterflies + phase; complex64: ~sqrt(L) * 2^-24 per U.
TOL_U = {"c128": 1e-12, "c64": 3e-6}


def _dt(name):
    torch = require_gpu()
    return torch.complex128 if name == "c128" else torch.complex64


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("L,g,periodic", [
    (2, 0.9, True), (3, 0.9, False), (5, 1.3, True), (6, 0.9, True), (7, 0.4, False),
    (8, 1.3, True), (10, 0.9, True), (11, 0.9, True), (12, 1.4, False), (12, 0.9, True),
])
def test_apply_U_dense_parity(dt, L, g, periodic):
    say(f"apply_U dense L={L} g={g} periodic={periodic} {dt}")
    p = kicked_ising(L, 100 + L, g=g, periodic=periodic)
    U = models.ki_dense(p)
    psi = random_state(2 ** L, 7 + L)[0]
    with ki_op(p) as op:
        out = to_np(op.apply_U(to_dev(psi, _dt(dt))))
    assert rel(out, U @ psi) < TOL_U[dt]


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("L", [13, 14, 16, 20])
def test_apply_U_matrix_free_parity(dt, L):
    say(f"apply_U matrix-free L={L} {dt}")
    p = kicked_ising(L, 200 + L)
    psi = random_state(2 ** L, 9)[0]
    with ki_op(p) as op:
        out = to_np(op.apply_U(to_dev(psi, _dt(dt))))
    assert rel(out, models.ki_apply(p, psi)) < TOL_U[dt]


def test_apply_U_in_place_and_norm():
    torch = require_gpu()
    p = kicked_ising(16, 5)
    psi = random_state(2 ** 16, 3)[0]
    with ki_op(p) as op:
        x = to_dev(psi, torch.complex128)
        op.apply_U(x, out=x)
        out = to_np(x)
    assert rel(out, models.ki_apply(p, psi)) < 1e-12
    assert abs(np.linalg.norm(out) - 1) < 1e-12


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("L,g", [(22, 0.9), (25, 0.9)])
def test_apply_U_large_special_cases(dt, L, g):
    # Sampled outputs at large L from closed forms: g = 0 gives out = e^{-iE(s)} psi(s);
    # g = pi/2 gives out(s') = (-i)^L e^{-iE(s')} psi(s) with s' the complement of s.
    torch = require_gpu()
    say(f"apply_U special cases L={L} {dt}")
    rng = np.random.default_rng(L)
    d = 2 ** L
    psi = (rng.standard_normal(d) + 1j * rng.standard_normal(d)) / math.sqrt(2 * d)
    idx = rng.integers(0, d, size=200)
    tol = TOL_U[dt] * 10
    bound = tol * np.abs(psi).max() * 10
    for gg in (0.0, math.pi / 2):
        p = kicked_ising(L, 300 + L, g=gg)
        with ki_op(p) as op:
            out = to_np(op.apply_U(to_dev(psi, _dt(dt))))
        for s in idx:
            E = 0.0
            sp = s if gg == 0.0 else (d - 1) ^ s
            z = [1 - 2 * ((sp >> (L - i)) & 1) for i in range(1, L + 1)]
            E = sum(p.J[i] * z[i] * z[(i + 1) % L] for i in range(L)) + sum(p.h[i] * z[i] for i in range(L))
            pref = 1.0 if gg == 0.0 else (-1j) ** L
            expect = pref * cmath.exp(-1j * E) * psi[s]
            assert abs(out[sp] - expect) < bound


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_apply_filter_L25_special_cases(dt):
    # the filter on the three-tile-group schedule of L = 25, sampled against
    # closed forms (Eq. (geo) with U from the two special points):
    #   g = 0:    U psi(s) = e^{-iE(s)} psi(s), so the filter is the geometric
    #             sum of z e^{-iE(s)}, z = e^{-i phi}, times psi(s);
    #   g = pi/2: U psi(t) = c e^{-iE(t)} psi(t'), c = (-i)^L, t' the
    #             complement of t, so with k = 2 the filter at t is
    #             psi(t) + z c e^{-iE(t)} psi(t') + z^2 c^2 e^{-iE(t)} e^{-iE(t')} psi(t)
    L, k, phi = 25, 2, 0.7
    d = 2 ** L

    def draw():
        rng = np.random.default_rng(2500)
        v = (rng.standard_normal(d) + 1j * rng.standard_normal(d)) / math.sqrt(2 * d)
        return v, rng.integers(0, d, size=200)
    psi, idx = memo(("psi", L, 2500), draw)
    z = cmath.exp(-1j * phi)
    c = (-1j) ** L
    for gg in (0.0, math.pi / 2):
        say(f"apply_filter L=25 special case g={gg:.4f} {dt}")
        p = kicked_ising(L, 320, g=gg)
        E = memo(("ki-E", L, 320, gg), lambda: models.ki_energies(L, p.J, p.h, p.periodic))
        with ki_op(p) as op:
            out = to_np(op.apply_filter(to_dev(psi, _dt(dt)), k, phi))
        scale = np.max(np.abs(out))
        for t in idx:
            tc = (d - 1) ^ int(t)
            if gg == 0.0:
                w = z * cmath.exp(-1j * E[t])
                expect = (1 + w + w * w) * psi[t]
            else:
                expect = (psi[t] + z * c * cmath.exp(-1j * E[t]) * psi[tc]
                          + z * z * c * c * cmath.exp(-1j * (E[t] + E[tc])) * psi[t])
            tol = 1e-12 * (k + 1) if dt == "c128" else 2e-7 * (k + 1) + 2e-6
            assert abs(out[t] - expect) < tol * scale, (gg, int(t), abs(out[t] - expect) / scale)
        del out


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("L,k,phi", [(4, 3, 0.3), (6, 0, 1.0), (6, 1, 2.0), (10, 64, 0.0), (11, 17, 4.0),
                                     (12, 40, 1.1)])
def test_apply_filter_dense_parity(dt, L, k, phi):
    say(f"apply_filter dense L={L} k={k} phi={phi} {dt}")
    p = kicked_ising(L, 400 + L)
    U = models.ki_dense(p)
    psi = random_state(2 ** L, 11)[0]
    ref = filters.geometric_sum(lambda v: U @ v, psi, k, phi)
    with ki_op(p) as op:
        out = to_np(op.apply_filter(to_dev(psi, _dt(dt)), k, phi))
    tol = 1e-12 * (k + 1) if dt == "c128" else 2e-7 * (k + 1) + 2e-6
    assert rel(out, ref) < tol


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("L,k,phi", [(16, 20, 0.7), (20, 3, 5.0)])
def test_apply_filter_matrix_free_parity(dt, L, k, phi):
    say(f"apply_filter matrix-free L={L} k={k} {dt}")
    p = kicked_ising(L, 500 + L)
    psi = random_state(2 ** L, 13)[0]
    ref = filters.geometric_sum(lambda v: models.ki_apply(p, v), psi, k, phi)
    with ki_op(p) as op:
        out = to_np(op.apply_filter(to_dev(psi, _dt(dt)), k, phi))
    tol = 1e-12 * (k + 1) if dt == "c128" else 2e-7 * (k + 1) + 2e-6
    assert rel(out, ref) < tol


def _maxrel(out, ref):
    return float(np.max(np.abs(out - ref)) / np.max(np.abs(ref)))


@pytest.mark.timeout(300)
@pytest.mark.parametrize("L,g", [(21, 0.9), (22, 0.9), (23, 0.9), (24, 0.9), (22, 1.4)])
def test_apply_filter_large_states_elementwise(L, g):
    # the single-vector passes of large states (three register layouts for
    # 16-amplitude tiles, 14-bit low tiles for complex64 at L = 24; g = 1.4
    # takes the swapped kick form and the two-layout pass), element-wise
    # against the oracle's matrix-free U: the filter (Eq. (geo)), a
    # polynomial with coefficients (Eq. (poly)) and U itself (the phase pass
    # without psi); at L = 24 also two vectors per launch
    say(f"apply_filter large state L={L} g={g}")
    p = kicked_ising(L, 550 + L, g=g)
    psi = random_state(2 ** L, 17)[0]
    k, phi = 2, 2.1  # the prologue kick pass and two Horner passes
    powers = []

    def matvec(v):
        r = models.ki_apply(p, v)
        powers.append(r)
        return r

    ref = filters.geometric_sum(matvec, psi, k, phi)
    rot = np.exp(-1j * phi)
    u1, u2 = powers[0], powers[1] / rot  # U psi and U^2 psi
    coeffs = np.array([0.3 - 0.2j, -1.1 + 0.4j, 0.7 + 0.9j])
    ref_poly = coeffs[0] * psi + coeffs[1] * u1 + coeffs[2] * u2
    with ki_op(p) as op:
        for dt in ("c128", "c64"):
            tol = 1e-12 * (k + 1) if dt == "c128" else 2e-7 * (k + 1) + 2e-6
            x = to_dev(psi, _dt(dt))
            err = _maxrel(to_np(op.apply_filter(x, k, phi)), ref)
            assert err < tol, ("filter", dt, err)
            err = _maxrel(to_np(op.apply_polynomial(x, coeffs)), ref_poly)
            assert err < tol, ("polynomial", dt, err)
            err = _maxrel(to_np(op.apply_U(x)), u1)
            assert err < TOL_U[dt], ("U", dt, err)
            if L == 24:
                torch = require_gpu()
                xx = torch.stack([x, x]).contiguous()
                del x
                out2 = to_np(op.apply_filter_many(xx, k, phi))
                del xx
                for j in range(2):
                    err = _maxrel(out2[j], ref)
                    assert err < tol, ("filter_many", dt, j, err)
                del out2


@pytest.mark.parametrize("L", [8, 12])
def test_apply_polynomial_parity(L):
    torch = require_gpu()
    p = kicked_ising(L, 600 + L)
    U = models.ki_dense(p)
    rng = np.random.default_rng(L)
    coeffs = rng.standard_normal(9) + 1j * rng.standard_normal(9)
    psi = random_state(2 ** L, 17)[0]
    ref = filters.polynomial(lambda v: U @ v, psi, list(coeffs))
    with ki_op(p) as op:
        out = to_np(op.apply_polynomial(to_dev(psi, torch.complex128), coeffs))
        out0 = to_np(op.apply_polynomial(to_dev(psi, torch.complex128), coeffs[:1]))
    assert rel(out, ref) < 1e-11
    assert rel(out0, coeffs[0] * psi) < 1e-15


def test_filter_eigenvector_closed_form():
    # g_k(U) v = g_k(omega) v for an eigenvector (Eq. (gkmapping)).
    torch = require_gpu()
    from oracle import eig
    p = kicked_ising(10, 77)
    U = models.ki_dense(p)
    om, V = eig.full_closest(U, 3, 0.5)
    with ki_op(p) as op:
        for n in range(3):
            out = to_np(op.apply_filter(to_dev(V[:, n], torch.complex128), 50, 0.5))
            lam = filters.gk_scalar(np.array([om[n]]), 50, 0.5)[0]
            assert np.linalg.norm(out - lam * V[:, n]) < 1e-10 * abs(lam)


def test_determinism_bitwise():
    torch = require_gpu()
    p = kicked_ising(18, 3)
    psi = to_dev(random_state(2 ** 18, 1)[0], torch.complex64)
    with ki_op(p) as op:
        a = to_np(op.apply_filter(psi, 30, 0.2))
        b = to_np(op.apply_filter(psi, 30, 0.2))
    assert np.array_equal(a, b)
