"""Pins of the oracle's road profile (Table ineq_list: the centripetal row's
kappa(x(t)) and the lane limits y_lb(x(t)), y_ub(x(t)) as functions of the
ego's position along the road): reduction to the constant road, hand-computed
residual rows and target-pass values on linear profiles, clamping beyond the
knots, and invariance under a shift along the road."""
import numpy as np


def line_xi(x0, vx, y0, vy, t_f):
    i = np.arange(11) / 10.0
    return np.r_[x0 + vx * t_f * i, y0 + vy * t_f * i]


def scene(orc, ego, obs=None, **road):
    return orc.Scene(np.asarray(ego, float), np.zeros((0, 4)) if obs is None else np.asarray(obs, float), **road)


def test_constant_profile_equals_constant_road(orc):
    """A profile whose knots all hold (kappa, y_lb, y_ub) gives exactly the
    results of the constant road with that curvature and those limits."""
    par = orc.default_params(T=60, M=3, K=10, y_lb=-5.0, y_ub=6.0)
    ego = [0.0, 0.5, 18.0, 0.2, 0.3, -0.1]
    obs = [[20.0, 0.0, 12.0, 0.0], [45.0, 3.5, 15.0, 0.0], [-10.0, -3.5, 22.0, 0.0]]
    const = scene(orc, ego, obs, kappa_road=0.015)
    prof = scene(orc, ego, obs, road=np.tile([0.015, -5.0, 6.0], (7, 1)), road_x0=-50.0, road_dx=40.0)
    p = orc.sample(par, 3, 0, 40, True)
    xb_c = orc.step1(par, const, p)
    xs_c = orc.project(par, const, xb_c)
    xs_p = orc.project(par, prof, orc.step1(par, prof, p))
    assert np.array_equal(xs_c, xs_p)
    assert all(np.array_equal(a, b) for a, b in zip(orc.residual_cost(par, const, xs_c),
                                                     orc.residual_cost(par, prof, xs_p)))
    one = scene(orc, ego, obs, road=np.array([[0.015, -5.0, 6.0]]))
    assert np.array_equal(orc.project(par, one, xb_c), xs_c)


def test_residual_on_linear_profile(orc):
    """Straight line x = x0 + V t at lateral Y on a road with kappa(x) =
    k0 + k1 (x - X0) and y_ub(x) = u0 + u1 (x - X0) (two knots, linear):
    the centripetal row sums max(0, V^2 |kappa(x_k)| - c_max), the lane row
    max(0, Y - y_ub(x_k))."""
    T = 40
    par = orc.default_params(T=T, M=0, c_max=4.0, v_max=40.0)
    X0, dx, k0, k1, u0, u1 = 10.0, 150.0, 0.005, 1e-4, 3.0, -0.01
    road = np.array([[k0, -7.0, u0], [k0 + k1 * dx, -7.0, u0 + u1 * dx]])
    V, Y = 20.0, 2.5
    sc = scene(orc, [0, Y, V, 0, 0, 0], road=road, road_x0=X0, road_dx=dx)
    r, cu = orc.residual_cost(par, sc, line_xi(0.0, V, Y, 0.0, par.t_f))
    want = 0.0
    for k in range(T):
        x = V * par.t_f * k / (T - 1)
        u = min(max((x - X0) / dx, 0.0), 1.0)
        kap = k0 + k1 * dx * u
        yub = u0 + u1 * dx * u
        want += max(0.0, V * V * abs(kap) - 4.0) + max(0.0, Y - yub)
    assert abs(r[0] - want) < 1e-9 * max(1.0, want)
    assert want > 1.0  # both rows active somewhere


def test_targets_follow_the_profile(orc):
    """On a straight line at speed V the centripetal clip gives the velocity
    target magnitude min(V, sqrt(c_max / |kappa(x_k)|)) at each instant, and
    the lane slack is max(0, y_ub(x_k) - Y) on the upper rows."""
    T = 30
    par = orc.default_params(T=T, M=0, c_max=4.0, v_max=40.0)
    X0, dx = 0.0, 100.0
    road = np.array([[0.0, -7.0, 4.0], [0.03, -7.0, 1.0]])
    V, Y = 18.0, 2.0
    sc = scene(orc, [0, Y, V, 0, 0, 0], road=road, road_x0=X0, road_dx=dx)
    xi = line_xi(0.0, V, Y, 0.0, par.t_f)
    h, s, _ = orc.targets(par, sc, xi, np.zeros(T))
    for k in range(T):
        x = V * par.t_f * k / (T - 1)
        u = min(max(x / dx, 0.0), 1.0)
        kap = 0.03 * u
        vmax = V if kap == 0 else min(V, np.sqrt(4.0 / kap))
        assert abs(h[0 * T + k] - vmax) < 1e-9  # x row of the velocity target (M = 0)
        yub = 4.0 - 3.0 * u
        assert abs(s[k] - max(0.0, yub - Y)) < 1e-9


def test_profile_is_constant_beyond_its_knots(orc):
    """Before the first knot and after the last the end values hold."""
    T = 20
    par = orc.default_params(T=T, M=0, c_max=4.0, v_max=40.0)
    road = np.array([[0.02, -7.0, 7.0], [0.0, -7.0, 7.0], [0.05, -7.0, 7.0]])
    V = 20.0
    # trajectory entirely before the first knot: kappa = 0.02 at every instant
    sc = scene(orc, [0, 0, V, 0, 0, 0], road=road, road_x0=500.0, road_dx=10.0)
    r, _ = orc.residual_cost(par, sc, line_xi(0.0, V, 0.0, 0.0, par.t_f))
    assert abs(r[0] - T * (V * V * 0.02 - 4.0)) < 1e-9
    # entirely beyond the last knot: kappa = 0.05
    sc2 = scene(orc, [0, 0, V, 0, 0, 0], road=road, road_x0=-500.0, road_dx=10.0)
    r2, _ = orc.residual_cost(par, sc2, line_xi(0.0, V, 0.0, 0.0, par.t_f))
    assert abs(r2[0] - T * (V * V * 0.05 - 4.0)) < 1e-9


def test_projection_shift_invariance_with_road(orc):
    """Shifting ego, neighbours and the road profile by D along x shifts the
    projected trajectories by D."""
    par = orc.default_params(T=50, M=2, K=8, c_max=4.0)
    road = np.array([[0.0, -6.0, 7.0], [0.02, -5.0, 5.0], [0.01, -7.0, 6.0]])
    ego = np.array([0.0, 1.0, 17.0, 0.0, 0.0, 0.0])
    obs = np.array([[30.0, 0.0, 10.0, 0.0], [60.0, 3.5, 12.0, 0.0]])
    D = 64.0
    p = orc.sample(orc.default_params(T=50, M=2), 7, 0, 24, True)
    a = scene(orc, ego, obs, road=road, road_x0=20.0, road_dx=35.0)
    e2, o2 = ego.copy(), obs.copy()
    e2[0] += D
    o2[:, 0] += D
    b = scene(orc, e2, o2, road=road, road_x0=20.0 + D, road_dx=35.0)
    xa = orc.project(par, a, orc.step1(par, a, p))
    xb = orc.project(par, b, orc.step1(par, b, p))
    assert np.allclose(xb[:, :11] - D, xa[:, :11], atol=1e-7)
    assert np.allclose(xb[:, 11:], xa[:, 11:], atol=1e-7)
