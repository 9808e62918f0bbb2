"""Pins of the oracle's projection (Alg. 2) and target pass.

No passage of the paper prints iterate values. Every step of each iteration
is pinned in test_oracle_alg2_steps.py; here, what is pinned of the whole:
  * the closed-form (alpha, d) of step split_alpha_o against a brute-force
    grid minimisation, and the clips of steps clip_d_o .. clip_d_a on
    hand-computed cases;
  * the exact fixed point xi^k = xi_bar when no constraint is active;
  * invariances the method has (mirror in y, shift in x, sample order);
  * convergence: with many iterations the residual of a feasible scene
    vanishes, and each xi-update satisfies the equality constraints.
"""
import numpy as np
import pytest


def const_xi(X, Y):
    """Bernstein coefficients of the constant trajectory (X, Y)."""
    return np.r_[np.full(11, X), np.full(11, Y)]


def line_xi(x0, vx, y0, vy, t_f):
    """Coefficients of x = x0 + vx t, y = y0 + vy t (degree elevation of a line)."""
    i = np.arange(11) / 10.0
    return np.r_[x0 + vx * t_f * i, y0 + vy * t_f * i]


def test_obstacle_target_matches_grid_minimiser(orc):
    """Step split_alpha_o: for each neighbour, the minimiser over (alpha, d)
    of |(dx, dy) - (a d cos alpha, b d sin alpha)|, then d clipped to >= 1."""
    T = 3
    par = orc.default_params(T=T, M=1)
    a, b = par.ell_a, par.ell_b
    al = np.linspace(-np.pi, np.pi, 1441)[:-1]
    dd = np.linspace(0.0, 4.0, 801)
    AL, DD = np.meshgrid(al, dd, indexing="ij")
    rng = np.random.default_rng(5)
    for _ in range(12):
        dx, dy = rng.uniform(-7, 7), rng.uniform(-3, 3)
        obs = np.array([[10.0, 1.0, 0.0, 0.0]])
        xi = const_xi(10.0 + dx, 1.0 + dy)
        h, s, da = orc.targets(par, orc.Scene([10 + dx, 1 + dy, 0, 0, 0, 0], obs), xi, np.zeros(T))
        err = (dx - a * DD * np.cos(AL)) ** 2 + (dy - b * DD * np.sin(AL)) ** 2
        i, j = np.unravel_index(np.argmin(err), err.shape)
        d = max(1.0, DD[i, j])
        want = (10.0 + a * d * np.cos(AL[i, j]), 1.0 + b * d * np.sin(AL[i, j]))
        rows = (1 + 2) * T
        got = (h[0], h[rows + 0])
        assert np.allclose(got, want, atol=2e-2), (dx, dy, got, want)


def test_obstacle_target_outside_is_identity_and_centre(orc):
    T = 2
    par = orc.default_params(T=T, M=2)
    obs = np.array([[0.0, 0.0, 0.0, 0.0], [30.0, 0.0, 0.0, 0.0]])
    xi = const_xi(30.0, 0.0)  # exactly at the centre of the second neighbour
    h, _, _ = orc.targets(par, orc.Scene([30, 0, 0, 0, 0, 0], obs), xi, np.zeros(T))
    rows = (2 + 2) * T
    # first neighbour is far: target equals the trajectory point
    assert np.allclose([h[0], h[rows]], [30.0, 0.0], atol=1e-12)
    # centre: atan2(0, 0) = 0 and d = 1: target is (x_o + a, y_o)
    assert np.allclose([h[T], h[rows + T]], [30.0 + par.ell_a, 0.0], atol=1e-12)


def test_velocity_acceleration_clips_hand_cases(orc):
    T = 5
    par = orc.default_params(T=T, M=0, v_max=30.0, a_max=8.0, kappa_max=0.2)
    rows = 2 * T
    sc = orc.Scene([0, 0, 0, 0, 0, 0], np.zeros((0, 4)))
    # straight line above the speed limit: d_v = v_max, heading kept; a = 0
    h, _, da = orc.targets(par, sc, line_xi(0, 36.0, 0, 0, par.t_f), np.zeros(T))
    assert np.allclose(h[0:T], 30.0) and np.allclose(h[rows:rows + T], 0.0)
    assert np.allclose(h[T:2 * T], 0.0) and np.allclose(da, 0.0)
    # diagonal line below the limit: unchanged velocity
    h, _, _ = orc.targets(par, sc, line_xi(0, 12.0, 0, 5.0, par.t_f), np.zeros(T))
    assert np.allclose(h[0:T], 12.0) and np.allclose(h[rows:rows + T], 5.0)


@pytest.mark.parametrize("V,A,da0", [(10.0, 12.0, 5.0), (2.0, 3.0, 8.0), (1.0, 0.5, 3.0)])
def test_curvature_coupled_clips_on_parabola(orc, V, A, da0):
    """Parabola x = V t, y = A t^2/2: v = (V, A t), acc = (0, A) and
    |sin(alpha_a - alpha_v)| = V/|v|. The curvature bound turns into the
    lower speed bound sqrt(d_a_prev |sin| / kappa_max) and the upper
    acceleration bound d_v^2 kappa_max / |sin| (steps clip_d_v, clip_d_a);
    the middle case makes the speed bound active."""
    T = 5
    par = orc.default_params(T=T, M=0, v_max=30.0, a_max=8.0, kappa_max=0.2)
    rows = 2 * T
    sc = orc.Scene([0, 0, 0, 0, 0, 0], np.zeros((0, 4)))
    i = np.arange(11)
    c_y = 0.5 * A * par.t_f ** 2 * i * (i - 1) / 90.0  # A/2 t^2 in Bernstein form
    xi = np.r_[V * par.t_f * i / 10.0, c_y]
    h, _, da = orc.targets(par, sc, xi, np.full(T, da0))
    t = np.linspace(0, par.t_f, T)
    active = 0
    for k in range(T):
        v = np.hypot(V, A * t[k])
        sn = V / v
        vmin = np.sqrt(da0 * sn / 0.2)
        active += vmin > v
        d_v = min(max(v, vmin), 30.0)
        amax = min(8.0, d_v ** 2 * 0.2 / sn)
        d_a = min(A, amax)
        assert np.isclose(da[k], d_a, rtol=1e-12)
        assert np.isclose(np.hypot(h[k], h[rows + k]), d_v, rtol=1e-12)
        assert np.isclose(h[T + k], 0.0, atol=1e-12) and np.isclose(h[rows + T + k], d_a, rtol=1e-12)
    if V == 2.0:
        assert active > 0


def test_centripetal_bound_on_curved_road(orc):
    """Step clip_d_v with road curvature: cos(alpha_v) = 1 on a line along
    x, so the speed is capped at sqrt(c_max / |kappa|)."""
    T = 4
    par = orc.default_params(T=T, M=0, v_max=30.0, c_max=4.0)
    sc = orc.Scene([0, 0, 0, 0, 0, 0], np.zeros((0, 4)), kappa_road=0.01)
    h, _, _ = orc.targets(par, sc, line_xi(0, 25.0, 0, 0, par.t_f), np.zeros(T))
    assert np.allclose(h[0:T], 20.0, rtol=1e-12)
    # along y the centripetal bound does not bind (cos alpha_v = 0)
    h, _, _ = orc.targets(par, sc, line_xi(0, 0.0, 0, 25.0, par.t_f), np.zeros(T))
    assert np.allclose(h[2 * T:3 * T], 25.0, rtol=1e-12)


def test_lane_slack(orc):
    T = 4
    par = orc.default_params(T=T, M=0, y_lb=-7.0, y_ub=7.0)
    sc = orc.Scene([0, 0, 0, 0, 0, 0], np.zeros((0, 4)))
    for Y, s_up, s_lo in [(0.0, 7.0, 7.0), (8.0, 0.0, 15.0), (-9.0, 16.0, 0.0)]:
        _, s, _ = orc.targets(par, sc, const_xi(0.0, Y), np.zeros(T))
        assert np.allclose(s[:T], s_up) and np.allclose(s[T:], s_lo)


def far_scene(orc, M=3):
    obs = np.array([[400.0 + 50 * i, 3.5, 15.0, 0.0] for i in range(M)])
    return orc.Scene(np.array([0, 0, 15.0, 0, 0, 0]), obs)


@pytest.mark.parametrize("rho", [1.0, 2.5, 0.3])
def test_inactive_constraints_fixed_point(orc, rho):
    par = orc.default_params(T=60, M=3, K=15, rho=rho)
    sc = far_scene(orc)
    p = np.array([[0.5, 1.0, 1.0, 0.5, 15, 16, 17, 17.5], [0, 0, 0, 0, 15, 15, 15, 15]])
    xb = orc.step1(par, sc, p)
    xs, it = orc.project(par, sc, xb, return_iterates=True)
    r, _ = orc.residual_cost(par, sc, xb)
    assert np.all(r == 0.0)
    assert np.abs(it - xb[:, None, :]).max() < 1e-8


def _random_scene(orc, rng, M):
    obs = np.column_stack([rng.uniform(-10, 80, M), rng.choice([-3.5, 0, 3.5], M),
                           rng.uniform(8, 20, M), np.zeros(M)])
    return np.array([0, 0, 14.0, 0, 0, 0]), obs


def test_mirror_and_shift_invariance(orc):
    par = orc.default_params(T=50, M=4, K=10)
    rng = np.random.default_rng(6)
    ego, obs = _random_scene(orc, rng, 4)
    p = orc.sample(par, 11, 0, 16, True)
    xb = orc.step1(par, orc.Scene(ego, obs), p)
    xs = orc.project(par, orc.Scene(ego, obs), xb)
    # mirror y -> -y (lane bounds are symmetric)
    egom, obsm, pm = ego.copy(), obs.copy(), p.copy()
    egom[[1, 3, 5]] *= -1
    obsm[:, [1, 3]] *= -1
    pm[:, :4] *= -1
    scm = orc.Scene(egom, obsm)
    xsm = orc.project(par, scm, orc.step1(par, scm, pm))
    assert np.abs(xsm[:, :11] - xs[:, :11]).max() < 1e-8
    assert np.abs(xsm[:, 11:] + xs[:, 11:]).max() < 1e-8
    # shift x by D
    D = 123.25
    egos, obss = ego.copy(), obs.copy()
    egos[0] += D
    obss[:, 0] += D
    scs = orc.Scene(egos, obss)
    xss = orc.project(par, scs, orc.step1(par, scs, p))
    assert np.abs(xss[:, :11] - (xs[:, :11] + D)).max() < 1e-8
    assert np.abs(xss[:, 11:] - xs[:, 11:]).max() < 1e-8


def test_sample_order_invariance(orc):
    par = orc.default_params(T=40, M=3, K=8)
    rng = np.random.default_rng(8)
    ego, obs = _random_scene(orc, rng, 3)
    sc = orc.Scene(ego, obs)
    p = orc.sample(par, 3, 0, 10, True)
    xs = orc.project(par, sc, orc.step1(par, sc, p))
    perm = rng.permutation(10)
    xs2 = orc.project(par, sc, orc.step1(par, sc, p[perm]))
    assert np.array_equal(xs2, xs[perm])


def test_iterates_keep_equalities_and_converge(orc):
    par = orc.default_params(T=60, M=3, K=300)
    ego = np.array([0, 0, 14.0, 0, 0, 0])
    obs = np.array([[20.0, 0.0, 8.0, 0.0], [35.0, 3.5, 9.0, 0.0], [30.0, -3.5, 10.0, 0.0]])
    sc = orc.Scene(ego, obs)
    p = orc.sample(par, 5, 0, 12, True)
    xb = orc.step1(par, sc, p)
    xs, it = orc.project(par, sc, xb, return_iterates=True)
    W, Wd, Wdd = orc.basis(par.T, par.t_f)
    # A_eq xi^k = b for every iterate
    for k in (1, 50, 300):
        X = it[:, k]
        assert np.allclose(X[:, :11] @ W[0], ego[0], atol=1e-8)
        assert np.allclose(X[:, :11] @ Wd[0], ego[2], atol=1e-8)
        assert np.allclose(X[:, 11:] @ Wd[-1], 0.0, atol=1e-8)
    r0, _ = orc.residual_cost(par, sc, xb)
    r1, _ = orc.residual_cost(par, sc, xs)
    assert r0.sum() > 1.0            # the scene has active constraints
    assert r1.sum() < 0.02 * r0.sum()
