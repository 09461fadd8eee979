"""Pins of the oracle's pointwise pieces: log-mean, two-point flux, face flux.

Paper: averages, log-mean and jump and the momentum flux with the gravity
term rho_hat [[phi]] / 2, rho_hat = {{b}} {{rho}}_log / b^- (Sec. 4.1);
the partner's gravity term is -G b^-/b^+ (Sec. 4.1); the flux is the
entropy-conservative two-point flux of the balance law (Sec. 3).  Entropy
variables are taken here as the complex-step gradient of
eta = -rho s/(gamma - 1), written in this file from its definition, so that
the entropy-conservation pin does not rely on the oracle's own formula.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle as O

G = 1.4
EPS = np.finfo(float).eps


def _state(rng, phi, T=None):
    rho = rng.uniform(0.05, 1.5)
    u = rng.uniform(-60, 60, 3)
    T = rng.uniform(200, 320) if T is None else T
    p = rho * 287.0 * T
    E = p / (G - 1) + 0.5 * rho * (u @ u) + rho * phi
    return np.array([rho, *(rho * u), E])


def _pressure(q, phi):
    return (G - 1) * (q[4] - 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0] - q[0] * phi)


def _eta(q, phi):
    p = _pressure(q, phi)
    s = np.log(p) - G * np.log(q[0])
    return -q[0] * s / (G - 1)


def _v_complex_step(q, phi):
    v = np.zeros(5)
    h = 1e-30
    for i in range(5):
        qc = q.astype(complex)
        qc[i] += 1j * h * max(1.0, abs(q[i]))
        v[i] = _eta(qc, phi).imag / (h * max(1.0, abs(q[i])))
    return v


def _physical_flux(r, q, phi):
    # Euler flux of the conservative equations (Eq:euler), total energy incl. rho phi
    p = _pressure(q, phi)
    u = q[1:4] / q[0]
    f = np.zeros(5)
    f[0] = q[1 + r]
    f[1:4] = q[1:4] * u[r]
    f[1 + r] += p
    f[4] = (q[4] + p) * u[r]
    return f


def test_logmean_vs_mpmath():
    """Series branch: within a few ulp.  Log branch ([[a]]/(ln b - ln a) with
    per-node logarithms, Sec. 4.1): the rounding of ln a and ln b is
    amplified by 1/|ln(b/a)|, so the error bound is
    (|ln a| + |ln b| + 1) 2^-52 / |ln(b/a)| relative, plus a few ulp."""
    mpmath.mp.dps = 50
    rng = np.random.default_rng(0)
    for k in range(600):
        a = rng.uniform(0.01, 100.0) if k % 3 else rng.uniform(0.5, 2.0)
        if k % 2:
            ratio = 1.0 + rng.choice([-1, 1]) * 10.0 ** rng.uniform(-9, 0)
        else:
            ratio = 10.0 ** rng.uniform(-3, 3)
        b = a * ratio
        exact = (mpmath.mpf(b) - mpmath.mpf(a)) / (mpmath.log(b) - mpmath.log(a))
        got = O.logmean(a, b)
        ulp = np.spacing(float(exact))
        f = (b - a) / (b + a)
        if f * f < 1e-4:
            bound = 4 * ulp
        else:
            dl = abs(math.log(b / a))
            bound = 4 * ulp + float(exact) * (abs(math.log(a)) + abs(math.log(b)) + 1) * EPS / dl
        assert abs(got - float(exact)) <= bound, (a, b, got, float(exact))
    # nondimensional values near 1 (the scale the states are stored at):
    # within 32 ulp everywhere
    worst = 0.0
    for k in range(400):
        a = rng.uniform(0.8, 1.25)
        b = a * (1.0 + rng.choice([-1, 1]) * 10.0 ** rng.uniform(-9, -0.5))
        exact = (mpmath.mpf(b) - mpmath.mpf(a)) / (mpmath.log(b) - mpmath.log(a))
        worst = max(worst, abs(O.logmean(a, b) - float(exact)) / np.spacing(float(exact)))
    assert worst <= 32, worst


def test_logmean_properties():
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, b = rng.uniform(0.01, 10.0, 2)
        assert O.logmean(a, b) == O.logmean(b, a)           # bitwise symmetric
        assert O.logmean(a, a) == a                           # consistent
        lam = rng.uniform(0.1, 10.0)                          # 1-homogeneous
        assert abs(O.logmean(lam * a, lam * b) - lam * O.logmean(a, b)) < 1e-13 * lam * max(a, b)
        c = a * (1 + 1e-6)                                    # series branch: exact 2^k scaling
        k2 = 2.0 ** rng.integers(-5, 6)
        assert O.logmean(k2 * a, k2 * c) == k2 * O.logmean(a, c)
        lo, hi = min(a, b), max(a, b)
        assert math.sqrt(a * b) * (1 - 1e-14) <= O.logmean(a, b) <= 0.5 * (a + b) * (1 + 1e-14)
        assert lo <= O.logmean(a, b) <= hi


@pytest.mark.parametrize("r", [0, 1, 2])
def test_two_point_flux_consistency(r):
    rng = np.random.default_rng(10 + r)
    for _ in range(50):
        phi = rng.uniform(0, 3e5)
        q = _state(rng, phi)
        F = O.two_point_flux(r, q, q, phi, phi, G)
        f = _physical_flux(r, q, phi)
        assert np.allclose(F, f, rtol=1e-13, atol=1e-12 * np.abs(f).max())
        # the oracle's own physical flux agrees too
        assert np.allclose(O.euler_flux(r, q, phi, G), f, rtol=1e-14, atol=1e-13 * np.abs(f).max())


@pytest.mark.parametrize("r", [0, 1, 2])
def test_two_point_flux_symmetry_and_gravity_partner(r):
    rng = np.random.default_rng(20 + r)
    for _ in range(100):
        pa, pb = rng.uniform(0, 3e5, 2)
        qa, qb = _state(rng, pa), _state(rng, pb)
        Fab = O.two_point_flux(r, qa, qb, pa, pb, G)
        Fba = O.two_point_flux(r, qb, qa, pb, pa, G)
        # mass, energy and transverse momentum are symmetric
        for v in [0, 4] + [1 + c for c in range(3) if c != r]:
            assert abs(Fab[v] - Fba[v]) <= 1e-14 * max(1.0, abs(Fab[v])), v
        # normal momentum: symmetric part + gravity; G_ba = -G_ab b_a/b_b
        pra, prb = _pressure(qa, pa), _pressure(qb, pb)
        ba, bb = qa[0] / (2 * pra), qb[0] / (2 * prb)
        Fz = O.two_point_flux(r, qa, qb, 0.0, 0.0, G)  # same pair without geopotential jump
        # recompute each side's pressures consistently with its own phi
        Sab = O.two_point_flux(r, qa, qb, pa, pb, G)
        # gravity part of Fab by subtracting the symmetric average of the two orders
        # (the symmetric part S is the same in both orders)
        Gab_plus_S = Fab[1 + r]
        Gba_plus_S = Fba[1 + r]
        # S + G_ab and S - G_ab b_a / b_b  =>  G_ab (1 + b_a/b_b) = difference
        Gab = (Gab_plus_S - Gba_plus_S) / (1.0 + ba / bb)
        rho_ln = O.logmean(qa[0], qb[0])
        expect = 0.5 * (0.5 * (ba + bb) * rho_ln / ba) * (pb - pa)
        assert abs(Gab - expect) <= 1e-9 * max(1.0, abs(Fab[1 + r])), (Gab, expect)
        del Fz, Sab


@pytest.mark.parametrize("r", [0, 1, 2])
def test_entropy_conservation_condition(r):
    """v_a . F(a,b) - v_b . F(b,a) = -(psi_b - psi_a), psi = rho u_r: the
    two-point condition that makes the flux-differencing volume term
    entropy conservative for the balance law with the gravity term."""
    rng = np.random.default_rng(30 + r)
    for _ in range(100):
        pa = rng.uniform(0, 3e5)
        pb = pa + rng.uniform(-3e3, 3e3)
        qa, qb = _state(rng, pa), _state(rng, pb)
        if rng.uniform() < 0.5:  # near-equal states exercise the series branch
            qb = qa * (1 + rng.uniform(-1e-4, 1e-4, 5))
        va, vb = _v_complex_step(qa, pa), _v_complex_step(qb, pb)
        Fab = O.two_point_flux(r, qa, qb, pa, pb, G)
        Fba = O.two_point_flux(r, qb, qa, pb, pa, G)
        lhs = va @ Fab - vb @ Fba
        rhs = -(qb[1 + r] - qa[1 + r])
        scale = np.abs(va * Fab).sum() + np.abs(vb * Fba).sum()
        assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)


def test_entropy_variables_match_complex_step():
    rng = np.random.default_rng(40)
    for _ in range(50):
        phi = rng.uniform(0, 3e5)
        q = _state(rng, phi)
        assert np.allclose(O.entropy_vars(q, phi, G), _v_complex_step(q, phi), rtol=1e-12,
                           atol=1e-14)
        assert abs(O.entropy_density(q, phi, G) - _eta(q, phi)) <= 1e-13 * abs(_eta(q, phi))


def test_isothermal_well_balanced_pair_identity():
    # T constant, rho ~ exp(-phi/(R T)), u = 0  =>  {{p}} + G_ab = p_a
    T = 250.0
    rng = np.random.default_rng(50)
    for _ in range(100):
        za, zb = rng.uniform(0, 3e4, 2)
        pa_, pb_ = 9.81 * za, 9.81 * zb
        rho_a = math.exp(-pa_ / (287.0 * T))
        rho_b = math.exp(-pb_ / (287.0 * T))
        qa = np.array([rho_a, 0, 0, 0, rho_a * 287.0 * T / (G - 1) + rho_a * pa_])
        qb = np.array([rho_b, 0, 0, 0, rho_b * 287.0 * T / (G - 1) + rho_b * pb_])
        F = O.two_point_flux(2, qa, qb, pa_, pb_, G)
        p_a = rho_a * 287.0 * T
        assert abs(F[3] - p_a) <= 1e-12 * p_a
        assert F[0] == 0.0 and F[4] == 0.0


@pytest.mark.parametrize("r", [0, 1, 2])
def test_surface_flux(r):
    rng = np.random.default_rng(60 + r)
    for _ in range(50):
        phi = rng.uniform(0, 3e5)
        q = _state(rng, phi)
        f = _physical_flux(r, q, phi)
        for s in (-1, 1):
            for surf in (O.SURF_RUSANOV, O.SURF_EC):
                Fn = O.surface_flux(r, s, q, q, phi, phi, G, surf)
                assert np.allclose(Fn, s * f, rtol=1e-13, atol=1e-12 * np.abs(f).max())
        # Rusanov adds -lambda/2 [[q]], lambda = max(|u.n| + c)
        qp = _state(rng, phi)
        Fr = O.surface_flux(r, 1, q, qp, phi, phi, G, O.SURF_RUSANOV)
        Fe = O.surface_flux(r, 1, q, qp, phi, phi, G, O.SURF_EC)
        c = lambda qq: math.sqrt(G * _pressure(qq, phi) / qq[0])
        lam = max(abs(q[1 + r] / q[0]) + c(q), abs(qp[1 + r] / qp[0]) + c(qp))
        assert np.allclose(Fr - Fe, -0.5 * lam * (qp - q), rtol=1e-11,
                           atol=1e-9 * np.abs(Fe).max())
        # dissipation is entropy dissipative: [[v]] . (F_rus - F_ec) <= 0
        dv = _v_complex_step(qp, phi) - _v_complex_step(q, phi)
        assert dv @ (Fr - Fe) <= 1e-12 * np.abs(dv * (Fr - Fe)).sum()


def _jacobian_complex_step(r, q, phi):
    # d f_r / dq of the test's own physical flux, exact to roundoff
    A = np.zeros((5, 5))
    h = 1e-30
    for k in range(5):
        qc = q.astype(complex)
        step = h * max(1.0, abs(q[k]))
        qc[k] += 1j * step
        A[:, k] = _physical_flux_c(r, qc, phi).imag / step
    return A


def _physical_flux_c(r, q, phi):
    p = (G - 1) * (q[4] - 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0] - q[0] * phi)
    u = q[1:4] / q[0]
    f = np.zeros(5, dtype=complex)
    f[0] = q[1 + r]
    f[1:4] = q[1:4] * u[r]
    f[1 + r] += p
    f[4] = (q[4] + p) * u[r]
    return f


def _matrix_diss(r, s, qm, qp, phi):
    """D of F* = s f_r(q-, q+) - D/2 for the matrix-dissipation face flux."""
    Fm = O.surface_flux(r, s, qm, qp, phi, phi, G, O.SURF_MATRIX)
    Fe = O.surface_flux(r, s, qm, qp, phi, phi, G, O.SURF_EC)
    return -2.0 * (Fm - Fe)


@pytest.mark.parametrize("r", [0, 1, 2])
def test_matrix_dissipation_vanishes_at_equal_states(r):
    rng = np.random.default_rng(70 + r)
    for _ in range(50):
        phi = rng.uniform(0, 3e5)
        q = _state(rng, phi)
        for s in (-1, 1):
            Fm = O.surface_flux(r, s, q, q, phi, phi, G, O.SURF_MATRIX)
            assert np.array_equal(Fm, O.surface_flux(r, s, q, q, phi, phi, G, O.SURF_EC))


@pytest.mark.parametrize("r", [0, 1, 2])
def test_matrix_dissipation_small_jump_is_roe_matrix(r):
    # For a small jump D -> |A| [[q]] with |A| = V |Lambda| V^-1 the modulus of
    # the normal flux Jacobian (eigen-decomposition by numpy of the
    # complex-step Jacobian of the physical flux, gravity included): pins the
    # eigenvectors, eigenvalues, scaling and averages to first order.
    rng = np.random.default_rng(80 + r)
    for _ in range(30):
        phi = rng.uniform(0, 3e5)
        q = _state(rng, phi)
        dq = _state(rng, phi) - q
        eps = 1e-6
        qp = q + eps * dq
        qbar = 0.5 * (q + qp)
        lam, V = np.linalg.eig(_jacobian_complex_step(r, qbar, phi))
        absA = (V @ np.diag(np.abs(lam)) @ np.linalg.inv(V)).real
        want = absA @ (qp - q)
        for s in (-1, 1):
            D = _matrix_diss(r, s, q, qp, phi)
            scale = np.abs(absA) @ np.abs(qp - q)
            assert np.all(np.abs(D - want) <= 1e-5 * scale), (D, want)


@pytest.mark.parametrize("r", [0, 1, 2])
def test_matrix_dissipation_is_entropy_stable_and_antisymmetric(r):
    rng = np.random.default_rng(90 + r)
    for _ in range(200):
        phi = rng.uniform(0, 3e5)
        qm, qp = _state(rng, phi), _state(rng, phi)
        dv = _v_complex_step(qp, phi) - _v_complex_step(qm, phi)
        D = _matrix_diss(r, 1, qm, qp, phi)
        # [[v]] . D >= 0: the face only removes entropy
        assert dv @ D >= -1e-12 * np.abs(dv * D).sum()
        assert dv @ D > 0.0
        # independent of the normal's sign; the neighbour sees -F*
        assert np.allclose(_matrix_diss(r, -1, qm, qp, phi), D, rtol=1e-12,
                           atol=1e-12 * np.abs(D).max())
        Fa = O.surface_flux(r, 1, qm, qp, phi, phi, G, O.SURF_MATRIX)
        Fb = O.surface_flux(r, -1, qp, qm, phi, phi, G, O.SURF_MATRIX)
        assert np.allclose(Fa, -Fb, rtol=1e-12, atol=1e-12 * np.abs(Fa).max())


@pytest.mark.parametrize("r", [0, 1, 2])
def test_matrix_dissipation_keeps_a_stationary_contact(r):
    # rho jumps, p and the velocity are equal on both sides and u.n = 0: the
    # Roe-type dissipation vanishes (Rusanov's does not); this fixes the
    # log-mean enthalpy average h_hat, with which the acoustic projections
    # reduce to [[ln p]] = 0
    rng = np.random.default_rng(100 + r)
    for _ in range(50):
        phi = rng.uniform(0, 3e5)
        p = rng.uniform(3e3, 1e5)
        u = rng.uniform(-40, 40, 3)
        u[r] = 0.0
        ra, rb = rng.uniform(0.05, 1.5, 2)
        mk = lambda rho: np.array([rho, *(rho * u), p / (G - 1) + 0.5 * rho * (u @ u) + rho * phi])
        qm, qp = mk(ra), mk(rb)
        D = _matrix_diss(r, 1, qm, qp, phi)
        Dr = -2.0 * (O.surface_flux(r, 1, qm, qp, phi, phi, G, O.SURF_RUSANOV)
                     - O.surface_flux(r, 1, qm, qp, phi, phi, G, O.SURF_EC))
        assert np.all(np.abs(D) <= 1e-11 * np.abs(Dr).max()), (D, Dr)
