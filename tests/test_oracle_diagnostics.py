"""Pins of the oracle's integral diagnostics (oracle_entropy out[0..2]).

out[0] = sum_K int eta, out[1] = sum_K int rho, out[2] = sum_K int E with the
LGL quadrature; the paper tracks the mass and total-energy integrals
(Sec. 5.2).  A drift of these integrals is blind to a wrong Jacobian or a
wrong quadrature weight (both scale the start and the end alike), so each
integral is checked here against a value fixed by mathematics alone:
  - closed-form integrals of polynomials of degree <= 2N-1 per direction,
    which LGL quadrature integrates exactly (different degree and box length
    in each direction, so a weight taken from the wrong direction fails);
  - a state of constant rho, u and p under gravity (E carries rho g z), whose
    entropy density is constant: int eta = eta V, and int E has a closed
    form because z enters linearly;
  - on the warped (curved) box, which the warp maps onto itself: the volume
    integral converges to the box volume, and constant densities give
    ratios that do not depend on J at all.
Each planted mistake at the end (a J off by a factor, a weight of another
direction, a missing geopotential in eta) fails one of these checks.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2605_16684_amd import workloads as W

G = 1.4
LO = (100.0, -250.0, 0.0)
HI = (1100.0, 550.0, 1200.0)


def _mesh(N, K, grav=9.81, warp=None, periodic=(1, 1, 0)):
    return O.Mesh(N, K, LO, HI, periodic, gamma=G, gas_R=287.0, grav=grav, warp=warp)


def _poly_state(m, deg, amp_r=0.3, amp_e=0.1):
    """rho = 1 + amp_r s_x^a s_y^b s_z^c, m = 0, E = 2.5e5 (1 + amp_e s_x^c s_y^a s_z^b),
    s = (x - lo)/L, with exact integrals V (1 + amp/((a+1)(b+1)(c+1)))."""
    a, b, c = deg
    xyz = m.coords()
    s = [(xyz[:, d] - LO[d]) / (HI[d] - LO[d]) for d in range(3)]
    q = np.zeros(m.shape)
    q[:, 0] = 1.0 + amp_r * s[0] ** a * s[1] ** b * s[2] ** c
    q[:, 4] = 2.5e5 * (1.0 + amp_e * s[0] ** c * s[1] ** a * s[2] ** b)
    V = np.prod([HI[d] - LO[d] for d in range(3)])
    mono = 1.0 / ((a + 1) * (b + 1) * (c + 1))
    return q, V * (1.0 + amp_r * mono), 2.5e5 * V * (1.0 + amp_e * mono)


def _uniform_state(m, rho=1.1, u=(3.0, -2.0, 1.5), p=9.0e4, grav=9.81):
    """Constant rho, u and p; E = p/(gamma-1) + rho|u|^2/2 + rho g z at the nodes."""
    xyz = m.coords()
    q = np.zeros(m.shape)
    q[:, 0] = rho
    for d in range(3):
        q[:, 1 + d] = rho * u[d]
    ke = 0.5 * rho * sum(c * c for c in u)
    q[:, 4] = p / (G - 1) + ke + rho * grav * xyz[:, 2]
    s = math.log(p) - G * math.log(rho)
    eta = -rho * s / (G - 1)
    return q, eta, p / (G - 1) + ke


@pytest.mark.parametrize("N,deg", [(3, (5, 2, 0)), (4, (1, 7, 3)), (5, (9, 0, 4))])
def test_polynomial_integrals_are_exact(N, deg):
    m = _mesh(N, (3, 2, 2))
    q, int_rho, int_E = _poly_state(m, deg)
    out = m.entropy(q)
    assert abs(out[1] / int_rho - 1.0) < 1e-14, out[1] / int_rho - 1.0
    assert abs(out[2] / int_E - 1.0) < 1e-14, out[2] / int_E - 1.0


def test_polynomial_one_degree_too_high_is_not_exact():
    # the exactness above is a property of degree <= 2N-1 (LGL), which the
    # same check detects when it is violated: a guard that the pin is sharp
    m = _mesh(3, (1, 1, 1))
    q, int_rho, _ = _poly_state(m, (7, 0, 0))
    out = m.entropy(q)
    assert abs(out[1] / int_rho - 1.0) > 1e-6


@pytest.mark.parametrize("N,K", [(3, (2, 2, 3)), (6, (1, 2, 1))])
def test_uniform_state_entropy_and_energy_integrals(N, K):
    m = _mesh(N, K)
    q, eta, e_int = _uniform_state(m)
    out = m.entropy(q)
    V = np.prod([HI[d] - LO[d] for d in range(3)])
    zbar = 0.5 * (LO[2] + HI[2])
    assert abs(out[0] / (eta * V) - 1.0) < 1e-14, out[0] / (eta * V) - 1.0
    assert abs(out[1] / (1.1 * V) - 1.0) < 1e-14
    assert abs(out[2] / ((e_int + 1.1 * 9.81 * zbar) * V) - 1.0) < 1e-14


def test_uniform_state_on_warped_box():
    # the warp maps the box onto itself: int 1 dV converges spectrally to the
    # box volume; constant eta and rho give out[0]/out[1] = eta/rho whatever J is,
    # provided eta uses the geopotential of the warped nodes
    V = np.prod([HI[d] - LO[d] for d in range(3)])
    errs = {}
    for N in (3, 5, 7):
        m = _mesh(N, (3, 2, 3), warp=(0.04, 0.03, 0.05))
        q, eta, _ = _uniform_state(m)
        out = m.entropy(q)
        errs[N] = abs(out[1] / (1.1 * V) - 1.0)
        assert abs((out[0] / out[1]) / (eta / 1.1) - 1.0) < 1e-13
    # measured 2.7e-5, 5.0e-8, 1.5e-11: spectral decay (a J scaled by a constant
    # factor or with a wrong sign would miss by O(1))
    assert errs[3] < 1e-4 and errs[5] < 1e-6 and errs[7] < 1e-9, errs
    assert errs[7] < errs[5] / 100 < errs[3] / 1e4, errs


def test_planted_mistakes_fail_the_pins():
    """Each plausible mistake in the quadrature of oracle_entropy, restated in
    numpy on the oracle's own nodes, misses one of the closed forms above."""
    N = 3
    m = _mesh(N, (3, 2, 2))
    xi, w, _, _ = m.tables()
    h = [(HI[d] - LO[d]) / m.K[d] for d in range(3)]
    Nq = N + 1
    ii = np.arange(m.Np)
    i, j, k = ii % Nq, (ii // Nq) % Nq, ii // (Nq * Nq)
    J = h[0] * h[1] * h[2] / 8.0
    q, int_rho, _ = _poly_state(m, (5, 2, 0))

    def integral(wq):
        return (q[:, 0] * wq[None, :]).sum()

    good = integral(J * w[i] * w[j] * w[k])
    assert abs(good / int_rho - 1) < 1e-14
    assert abs(integral(J * w[i] * w[i] * w[k]) / int_rho - 1) > 1e-6    # weight of another direction
    assert abs(integral(J * 2 * w[i] * w[j] * w[k]) / int_rho - 1) > 1e-6  # J = h^3/4
    qu, eta, _ = _uniform_state(m)
    p_wrong = (G - 1) * (qu[:, 4] - 0.5 * (qu[:, 1:4] ** 2).sum(axis=1) / qu[:, 0])  # no rho phi
    eta_wrong = -qu[:, 0] * (np.log(p_wrong) - G * np.log(qu[:, 0])) / (G - 1)
    V = np.prod([HI[d] - LO[d] for d in range(3)])
    assert abs((eta_wrong * J * w[i] * w[j] * w[k]).sum() / (eta * V) - 1) > 1e-6
