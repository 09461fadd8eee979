"""Pins of the oracle's LGL tables and LSRK(5,4) coefficients.

The paper's elements carry (N+1)^3 LGL nodes with collocated LGL
quadrature and apply the 1-D LGL derivative matrix along tensor lines
(Sec. 3); time stepping is the Carpenter-Kennedy LSRK(5,4) scheme (Sec. 3).
"""
import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _expr(s):
    return float(eval(s, {"__builtins__": {}}, {"sqrt": math.sqrt}))


def _golden_lgl():
    rows = {}
    with open(os.path.join(GOLD, "lgl_closed_forms.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            N, i, x, w = line.split()
            rows.setdefault(int(N), []).append((int(i), _expr(x), _expr(w)))
    return rows


@pytest.mark.parametrize("N", [3, 4])
def test_lgl_closed_forms(N):
    x, w, _ = O.lgl(N)
    for i, xg, wg in _golden_lgl()[N]:
        assert abs(x[i] - xg) <= 2e-16
        assert abs(w[i] - wg) <= 4e-16


@pytest.mark.parametrize("N", [2, 3, 4, 5, 7, 10, 15])
def test_lgl_nodes_against_mpmath(N):
    # independent route: high-precision roots of (1 - x^2) P_N'(x)
    mpmath.mp.dps = 30
    x, w, _ = O.lgl(N)
    for i in range(1, N):
        r = mpmath.findroot(lambda t: mpmath.diff(lambda s: mpmath.legendre(N, s), t), x[i])
        assert abs(float(r) - x[i]) <= 2.5e-16
        wi = 2 / (N * (N + 1) * mpmath.legendre(N, r) ** 2)
        assert abs(float(wi) - w[i]) <= 4e-16 * max(1.0, float(wi))


@pytest.mark.parametrize("N", range(1, 16))
def test_lgl_quadrature_exactness(N):
    # LGL quadrature with N+1 points is exact for degree <= 2N - 1
    x, w, _ = O.lgl(N)
    assert abs(w.sum() - 2.0) < 1e-14
    for m in range(0, 2 * N):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.dot(w, x ** m) - exact) < 5e-14
    # and not exact at degree 2N (distinguishes Lobatto from Gauss points)
    m = 2 * N
    assert abs(np.dot(w, x ** m) - 2.0 / (m + 1)) > 1e-10


@pytest.mark.parametrize("N", range(1, 16))
def test_derivative_matrix(N):
    x, w, D = O.lgl(N)
    # exact on polynomials of degree <= N
    for m in range(0, N + 1):
        dm = m * x ** (m - 1) if m > 0 else np.zeros_like(x)
        assert np.max(np.abs(D @ x ** m - dm)) < 2e-12 * max(1, N * N)
    # barycentric construction (independent formula)
    lam = np.array([1.0 / np.prod([x[j] - x[k] for k in range(N + 1) if k != j])
                    for j in range(N + 1)])
    Db = np.zeros((N + 1, N + 1))
    for i in range(N + 1):
        for j in range(N + 1):
            if i != j:
                Db[i, j] = lam[j] / lam[i] / (x[i] - x[j])
        Db[i, i] = -Db[i].sum()
    assert np.max(np.abs(D - Db)) < 1e-12 * N * N
    # summation by parts: W D + D^T W = B = diag(-1, 0, ..., 0, 1)
    W = np.diag(w)
    B = np.zeros((N + 1, N + 1))
    B[0, 0], B[N, N] = -1.0, 1.0
    assert np.max(np.abs(W @ D + D.T @ W - B)) < 1e-13 * N


def test_skew_operator_row_sums():
    m = O.Mesh(4, (1, 1, 1), (0, 0, 0), (1, 1, 1), (1, 1, 1), grav=0.0)
    xi, w, D, S = m.tables()
    # S = Q - Q^T with Q = W D; rows sum to -B_aa
    assert np.max(np.abs(S + S.T)) == 0.0
    rs = S.sum(axis=1)
    assert abs(rs[0] - 1.0) < 1e-14 and abs(rs[-1] + 1.0) < 1e-14
    assert np.max(np.abs(rs[1:-1])) < 1e-14


def _golden_stability():
    out = {}
    with open(os.path.join(GOLD, "lsrk54_stability.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, c = line.split()
            out[int(k)] = float(Fraction(c))
    return out


def test_lsrk_stability_polynomial():
    # one step of y' = lambda y with lambda = a + i b, as a real 2x2 system,
    # through the oracle's own stepping routine
    coef = _golden_stability()
    rng = np.random.default_rng(3)
    for _ in range(20):
        a, b = rng.uniform(-2.0, 0.5), rng.uniform(-2.5, 2.5)
        M = np.array([[a, -b], [b, a]])
        y = O.lsrk_linear(M, [1.0, 0.0], 1.0, 1)
        z = complex(a, b)
        Rz = sum(c * z ** k for k, c in coef.items())
        assert abs(complex(y[0], y[1]) - Rz) < 1e-14 * max(1.0, abs(Rz))


def test_lsrk_order_conditions_polynomial_exactness():
    # a fourth-order scheme integrates y' = m t^(m-1) exactly for m <= 4
    for mpow in range(1, 5):
        y = O.lsrk_poly(mpow, 0.3, 0.3 ** mpow, 0.17, 7)
        exact = (0.3 + 7 * 0.17) ** mpow
        assert abs(y - exact) < 1e-13 * max(1.0, exact), mpow
    y = O.lsrk_poly(5, 0.3, 0.3 ** 5, 0.17, 7)
    assert abs(y - (0.3 + 7 * 0.17) ** 5) > 1e-9


def test_lsrk_convergence_order():
    # y' = -y + sin(t) style linear test: observed order 4 on y' = M y
    M = np.array([[-0.3, -1.0], [1.0, -0.3]])
    T = 2.0
    ev, V = np.linalg.eig(M)
    exact = (V @ np.diag(np.exp(ev * T)) @ np.linalg.inv(V) @ np.array([1.0, 0.5])).real
    errs = []
    for n in (10, 20, 40):
        y = O.lsrk_linear(M, [1.0, 0.5], T / n, n)
        errs.append(np.linalg.norm(y - exact))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 3.8
