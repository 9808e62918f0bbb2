"""Pins of the oracle's basis (eq. param) and Step-1 QP (Alg. 1, eq. over_2).

The basis is pinned by identities of polynomials of degree <= 10 (it must
reproduce every such polynomial and its derivatives exactly), not by its own
formula. The Step-1 solve is pinned by closed-form special cases, by exact
satisfaction of the boundary conditions, by a hand-computed cost, and by
first-order optimality along every feasible direction.
"""
from math import comb

import numpy as np
import pytest


def monomial_coeffs(m, n=10):
    """Bernstein coefficients of tau^m: tau^m = sum_i C(i,m)/C(n,m) B_i,n."""
    return np.array([comb(i, m) / comb(n, m) if i >= m else 0.0 for i in range(n + 1)])


def poly_coeffs(a, t_f, n=10):
    """Coefficients of sum_m a_m t^m with t = t_f tau."""
    c = np.zeros(n + 1)
    for m, am in enumerate(a):
        c += am * t_f ** m * monomial_coeffs(m, n)
    return c


@pytest.mark.parametrize("T", [2, 7, 50, 100, 128])
def test_basis_partition_and_endpoints(orc, T):
    W, Wd, Wdd = orc.basis(T, 5.0)
    assert np.allclose(W.sum(1), 1.0, atol=1e-14)
    assert np.allclose(Wd.sum(1), 0.0, atol=1e-12)
    assert np.allclose(Wdd.sum(1), 0.0, atol=1e-11)
    assert np.allclose(W[0], np.eye(11)[0]) and np.allclose(W[-1], np.eye(11)[10])


@pytest.mark.parametrize("m", range(11))
def test_basis_reproduces_monomials(orc, m):
    T, t_f = 37, 5.0
    W, Wd, Wdd = orc.basis(T, t_f)
    t = np.linspace(0.0, t_f, T)
    c = poly_coeffs([0] * m + [1.0], t_f)
    f = t ** m
    fd = m * t ** (m - 1) if m >= 1 else 0 * t
    fdd = m * (m - 1) * t ** (m - 2) if m >= 2 else 0 * t
    scale = max(1.0, t_f ** m)
    assert np.allclose(W @ c, f, atol=1e-12 * scale)
    assert np.allclose(Wd @ c, fd, atol=1e-11 * scale)
    assert np.allclose(Wdd @ c, fdd, atol=1e-10 * scale)


def _scene(orc, ego, M=0):
    return orc.Scene(np.asarray(ego, float), np.zeros((M, 4)))


def test_step1_exact_constant_velocity(orc):
    """v_d = vx0 on every segment, ax0 = 0: x(t) = x0 + vx0 t has zero
    velocity-tracking and smoothness cost, so it is the exact minimiser;
    y_d = y0 with vy0 = ay0 = 0 gives y(t) = y0."""
    par = orc.default_params(T=100)
    ego = [3.0, 3.5, 17.0, 0.0, 0.0, 0.0]
    p = np.array([3.5] * 4 + [17.0] * 4)
    xi = orc.step1(par, _scene(orc, ego), p)[0]
    W, _, _ = orc.basis(par.T, par.t_f)
    t = np.linspace(0, par.t_f, par.T)
    assert np.abs(W @ xi[:11] - (3.0 + 17.0 * t)).max() < 1e-10
    assert np.abs(W @ xi[11:] - 3.5).max() < 1e-12
    assert orc.lower_cost(par, p, xi) < 1e-18 * 1e6


def test_step1_boundary_conditions(orc):
    par = orc.default_params(T=50)
    rng = np.random.default_rng(0)
    W, Wd, Wdd = orc.basis(par.T, par.t_f)
    for _ in range(5):
        ego = np.array([rng.uniform(-5, 5), rng.uniform(-3, 3), rng.uniform(5, 25),
                        rng.uniform(-1, 1), rng.uniform(-2, 2), rng.uniform(-1, 1)])
        p = np.concatenate([rng.uniform(-4, 4, 4), rng.uniform(5, 25, 4)])
        xi = orc.step1(par, _scene(orc, ego), p)[0]
        cx, cy = xi[:11], xi[11:]
        got = [W[0] @ cx, Wd[0] @ cx, Wdd[0] @ cx, W[0] @ cy, Wd[0] @ cy, Wdd[0] @ cy, Wd[-1] @ cy]
        want = [ego[0], ego[2], ego[4], ego[1], ego[3], ego[5], 0.0]
        assert np.allclose(got, want, atol=1e-9)


def test_lower_cost_hand_computed(orc):
    """x(t) = A0 + A1 t + A2 t^2, y(t) = B0 + B1 t have xddot = 2 A2,
    xdot = A1 + 2 A2 t, yddot = 0, ydot = B1, so each term of eq. cost is a
    number written out below; the segment of t_k is floor(4k/T)."""
    T = 12
    par = orc.default_params(T=T, k_p=0.7, k_v=1.3, w_s=0.5, w_l=2.0, w_v=3.0)
    A0, A1, A2, B0, B1 = 1.0, 10.0, 0.4, -1.0, 0.25
    xi = np.concatenate([poly_coeffs([A0, A1, A2], par.t_f), poly_coeffs([B0, B1], par.t_f)])
    p = np.array([0.5, -1.5, 2.0, 3.0, 11.0, 12.0, 9.0, 14.0])
    J = 0.0
    for k in range(T):
        t = par.t_f * k / (T - 1)
        s = (4 * k) // T
        x_d, x_dd = A1 + 2 * A2 * t, 2 * A2
        y, y_d, y_dd = B0 + B1 * t, B1, 0.0
        J += par.w_s * (x_dd ** 2 + y_dd ** 2)
        J += par.w_l * (y_dd + par.k_p * (y - p[s]) + par.k_v * y_d) ** 2
        J += par.w_v * (x_dd + par.k_p * (x_d - p[4 + s])) ** 2
    assert abs(orc.lower_cost(par, p, xi) - J) < 1e-9 * J


def test_step1_optimal_along_feasible_directions(orc):
    """First-order optimality: the cost gradient is orthogonal to every
    direction d with A_eq d = 0 (central differences of the exact quadratic),
    and the cost does not decrease along any of them."""
    par = orc.default_params(T=40)
    W, Wd, Wdd = orc.basis(par.T, par.t_f)
    Z = np.zeros(11)
    A = np.array([np.r_[W[0], Z], np.r_[Wd[0], Z], np.r_[Wdd[0], Z],
                  np.r_[Z, W[0]], np.r_[Z, Wd[0]], np.r_[Z, Wdd[0]], np.r_[Z, Wd[-1]]])
    _, _, Vt = np.linalg.svd(A)
    Nul = Vt[7:]  # 15 feasible directions
    rng = np.random.default_rng(3)
    ego = [0.0, 0.0, 14.0, 0.3, 0.5, -0.2]
    for _ in range(3):
        p = np.concatenate([rng.uniform(-4, 4, 4), rng.uniform(5, 25, 4)])
        xi = orc.step1(par, _scene(orc, ego), p)[0]
        J0 = orc.lower_cost(par, p, xi)
        for d in Nul:
            eps = 1e-3
            Jp = orc.lower_cost(par, p, xi + eps * d)
            Jm = orc.lower_cost(par, p, xi - eps * d)
            grad = (Jp - Jm) / (2 * eps)
            curv = (Jp + Jm - 2 * J0) / eps ** 2
            assert abs(grad) < 1e-6 * max(1.0, J0)
            assert curv > 0 and Jp >= J0 - 1e-9 and Jm >= J0 - 1e-9


def test_step1_is_affine_in_p(orc):
    """The minimiser of a QP whose linear term is linear in p is affine in p."""
    par = orc.default_params(T=30)
    sc = _scene(orc, [0, 0, 12, 0, 0, 0])
    rng = np.random.default_rng(4)
    p1, p2 = rng.uniform(0, 20, 8), rng.uniform(0, 20, 8)
    a = 0.3
    x1, x2, x3 = orc.step1(par, sc, np.stack([p1, p2, a * p1 + (1 - a) * p2]))
    assert np.allclose(x3, a * x1 + (1 - a) * x2, atol=1e-9)
