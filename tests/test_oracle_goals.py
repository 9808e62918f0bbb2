"""Pins of the oracle's goal-position behavioural inputs (p = [x_f - x0, y_f],
eq. behaviour_param with the final boundary of eq. final_boundary, as in the
Batch-MPC baseline of Sec. V-A) and of the fixed-grid initial sampler
(MPC-Grid of Sec. V-A): closed-form special cases, exact boundary
conditions, first-order optimality, the cost with no set-point terms, the
projection's invariants, sampler moments, and the grid's closed form."""
import numpy as np
import pytest


def goal_par(orc, **over):
    kw = dict(behaviour=1)
    kw.update(over)
    return orc.default_params(**kw)


def scene(orc, ego, obs=None):
    return orc.Scene(np.asarray(ego, float), np.zeros((0, 4)) if obs is None else np.asarray(obs, float))


def goals(*rows):
    p = np.zeros((len(rows), 8))
    for i, (dx, yf) in enumerate(rows):
        p[i, 0], p[i, 1] = dx, yf
    return p


def test_goal_step1_exact_constant_velocity(orc):
    """Goal x_f = x0 + vx0 t_f, y_f = y0 with ax0 = vy0 = ay0 = 0: the
    straight line at constant speed meets every boundary condition with zero
    acceleration, so it is the exact minimiser of the smoothness cost."""
    par = goal_par(orc, T=100, M=0)
    ego = [3.0, 3.5, 17.0, 0.0, 0.0, 0.0]
    xi = orc.step1(par, scene(orc, ego), goals((17.0 * par.t_f, 3.5)))[0]
    W, _, _ = orc.basis(par.T, par.t_f)
    t = np.linspace(0, par.t_f, par.T)
    assert np.abs(W @ xi[:11] - (3.0 + 17.0 * t)).max() < 1e-9
    assert np.abs(W @ xi[11:] - 3.5).max() < 1e-11


def test_goal_step1_boundary_conditions(orc):
    par = goal_par(orc, T=50, M=0)
    rng = np.random.default_rng(0)
    W, Wd, Wdd = orc.basis(par.T, par.t_f)
    for _ in range(5):
        ego = np.array([rng.uniform(-5, 5), rng.uniform(-3, 3), rng.uniform(5, 25),
                        rng.uniform(-1, 1), rng.uniform(-2, 2), rng.uniform(-1, 1)])
        dx, yf = rng.uniform(20, 120), rng.uniform(-4, 4)
        xi = orc.step1(par, scene(orc, ego), goals((dx, yf)))[0]
        cx, cy = xi[:11], xi[11:]
        got = [W[0] @ cx, Wd[0] @ cx, Wdd[0] @ cx, W[0] @ cy, Wd[0] @ cy, Wdd[0] @ cy, Wd[-1] @ cy,
               W[-1] @ cx, W[-1] @ cy]
        want = [ego[0], ego[2], ego[4], ego[1], ego[3], ego[5], 0.0, ego[0] + dx, yf]
        assert np.allclose(got, want, atol=1e-9)


def test_goal_cost_has_no_set_point_terms(orc):
    """With goal positions the lower-level cost is the smoothness term alone:
    x = A0 + A1 t + A2 t^2, y = B0 + B1 t give T w_s (2 A2)^2 whatever p."""
    T = 12
    par = goal_par(orc, T=T, w_s=0.5, w_l=2.0, w_v=3.0)
    i = np.arange(11) / 10.0
    tf = par.t_f
    A0, A1, A2, B0, B1 = 1.0, 10.0, 0.4, -1.0, 0.25
    cx = A0 + A1 * tf * i + A2 * tf ** 2 * i * (np.arange(11) - 1) / 9.0
    cy = B0 + B1 * tf * i
    xi = np.r_[cx, cy]
    for p in (goals((50.0, 1.0))[0], goals((80.0, -3.5))[0]):
        assert abs(orc.lower_cost(par, p, xi) - T * 0.5 * (2 * A2) ** 2) < 1e-9


def test_goal_step1_optimal_along_feasible_directions(orc):
    par = goal_par(orc, T=40, M=0)
    W, Wd, Wdd = orc.basis(par.T, par.t_f)
    Z = np.zeros(11)
    A = np.array([np.r_[W[0], Z], np.r_[Wd[0], Z], np.r_[Wdd[0], Z],
                  np.r_[Z, W[0]], np.r_[Z, Wd[0]], np.r_[Z, Wdd[0]], np.r_[Z, Wd[-1]],
                  np.r_[W[-1], Z], np.r_[Z, W[-1]]])
    _, _, Vt = np.linalg.svd(A)
    Nul = Vt[9:]  # 13 feasible directions
    ego = [0.0, 0.0, 14.0, 0.3, 0.5, -0.2]
    for p in goals((60.0, 2.0), (95.0, -3.0)):
        xi = orc.step1(par, scene(orc, ego), p[None])[0]
        J0 = orc.lower_cost(par, p, xi)
        for d in Nul:
            eps = 1e-3
            Jp, Jm = orc.lower_cost(par, p, xi + eps * d), orc.lower_cost(par, p, xi - eps * d)
            assert abs((Jp - Jm) / (2 * eps)) < 1e-6 * max(1.0, J0)
            assert (Jp + Jm - 2 * J0) / eps ** 2 > 0


def test_goal_projection_keeps_the_boundary_rows(orc):
    """Every xi-update of Alg. 2 satisfies A_eq xi = b, including the goal
    rows; with no active constraint xi_bar is a fixed point."""
    par = goal_par(orc, T=60, M=3, K=8)
    W, Wd, Wdd = orc.basis(par.T, par.t_f)
    ego = [0.0, 0.0, 15.0, 0.0, 0.0, 0.0]
    obs = [[12.0, 0.0, 10.0, 0.0], [30.0, 3.5, 12.0, 0.0], [-15.0, -3.5, 20.0, 0.0]]
    p = goals((60.0, 3.5), (90.0, 0.0), (40.0, -3.5))
    sc = scene(orc, ego, obs)
    xb = orc.step1(par, sc, p)
    _, it = orc.project(par, sc, xb, return_iterates=True, p=p)
    for j in range(3):
        for k in range(par.K + 1):
            cx, cy = it[j, k, :11], it[j, k, 11:]
            rows = [W[0] @ cx, Wd[0] @ cx, Wdd[0] @ cx, W[0] @ cy, Wd[0] @ cy, Wdd[0] @ cy, Wd[-1] @ cy,
                    W[-1] @ cx, W[-1] @ cy]
            assert np.allclose(rows, [0, 15, 0, 0, 0, 0, 0, p[j, 0], p[j, 1]], atol=1e-8)
    far = scene(orc, ego, [[900.0, 0.0, 15.0, 0.0]])
    par1 = goal_par(orc, T=60, M=1, K=6)
    pq = goals((75.0, 0.0))
    xb1 = orc.step1(par1, far, pq)
    assert np.allclose(orc.project(par1, far, xb1, p=pq), xb1, atol=1e-12)
    with pytest.raises(ValueError):
        orc.project(par1, far, xb1)


def test_goal_sampler_moments(orc):
    """Structured goal draws have the moments initial_moments states; Gaussian
    goal draws have mean mu and covariance L L^T in the two goal inputs and
    are exactly zero in the others."""
    par = goal_par(orc)
    mu, S = orc.initial_moments(par)
    assert np.all(mu[2:] == 0) and np.all(S[2:] == 0) and np.all(S[:, 2:] == 0)
    N = 40000
    p = orc.sample(par, 12345, 0, N, True)
    assert np.all(p[:, 2:] == 0)
    assert np.all((p[:, 0] > par.t_f * par.vd_lo) & (p[:, 0] <= par.t_f * par.vd_hi))
    m = p[:, :2].mean(axis=0)
    C = np.cov(p[:, :2].T)
    se = np.sqrt(np.diag(S)[:2] / N)
    assert np.all(np.abs(m - mu[:2]) < 5 * se)
    assert np.allclose(np.diag(C), np.diag(S)[:2], rtol=0.03)
    assert abs(C[0, 1]) < 0.03 * np.sqrt(S[0, 0] * S[1, 1])
    mu2 = np.r_[70.0, 1.5, np.zeros(6)]
    L = np.zeros((8, 8))
    L[:2, :2] = [[6.0, 0.0], [0.8, 0.5]]
    L[2:, 2:] = np.eye(6)  # must be ignored
    q = orc.sample(par, 999, 3, N, False, mu2, L)
    assert np.all(q[:, 2:] == 0)
    assert np.allclose(q[:, :2].mean(axis=0), mu2[:2], atol=5 * 6.0 / np.sqrt(N))
    assert np.allclose(np.cov(q[:, :2].T), L[:2, :2] @ L[:2, :2].T, rtol=0.03, atol=0.01)


@pytest.mark.parametrize("behaviour", [0, 1])
@pytest.mark.parametrize("N", [3, 64, 100])
def test_grid_sampler_closed_form(orc, behaviour, N):
    """Grid point j: lane centre j mod 3 and the midpoint of velocity bin
    floor(j/3) of ceil(N/3) equal bins of (vd_lo, vd_hi]; independent of the
    seed and the iteration. The velocities of a full set of bins have the
    discrete-uniform variance range^2 (1 - 1/nb^2) / 12."""
    par = orc.default_params(behaviour=behaviour, sampler=1)
    p = orc.sample(par, 1, 0, N, True)
    assert np.array_equal(p, orc.sample(par, 77, 4, N, True))
    nb = -(-N // 3)
    width = (par.vd_hi - par.vd_lo) / nb
    lanes = np.array(list(par.lane_c))
    for j in range(N):
        v = par.vd_lo + width * (j // 3 + 0.5)
        if behaviour:
            assert np.allclose(p[j], np.r_[par.t_f * v, lanes[j % 3], np.zeros(6)], rtol=0, atol=1e-12)
        else:
            assert np.allclose(p[j], np.r_[np.full(4, lanes[j % 3]), np.full(4, v)], rtol=0, atol=1e-12)
    if N % 3 == 0:
        vs = p[:, 0] / par.t_f if behaviour else p[:, 4]
        rng2 = (par.vd_hi - par.vd_lo) ** 2
        assert np.isclose(vs.mean(), 0.5 * (par.vd_lo + par.vd_hi))
        assert np.isclose(vs.var(), rng2 * (1 - 1 / nb ** 2) / 12)


def test_goal_plan_and_grid_plan(orc):
    """Alg. 1 with goal positions keeps the unused inputs at zero in mu and
    Sigma and returns a trajectory that meets its goal; MPC-Grid (one
    iteration from the grid) returns the best grid point, the same for any
    seed."""
    par = goal_par(orc, T=50, M=4, K=10, L=3)
    ego = np.array([0.0, 0.0, 14.0, 0.0, 0.0, 0.0])
    obs = np.array([[25.0, 0.0, 9.0, 0.0], [-15.0, 3.5, 18.0, 0.0], [40.0, -3.5, 11.0, 0.0],
                    [8.0, 3.5, 13.0, 0.0]])
    sc = orc.Scene(ego, obs)
    res = orc.plan(par, sc, 5, 64)
    W, _, _ = orc.basis(par.T, par.t_f)
    assert np.all(res.mu[2:] == 0) and np.all(res.Sigma[2:] == 0) and np.all(res.Sigma[:, 2:] == 0)
    assert abs(W[-1] @ res.xi_best[:11] - (ego[0] + res.p_best[0])) < 1e-8
    assert abs(W[-1] @ res.xi_best[11:] - res.p_best[1]) < 1e-8
    for behaviour in (0, 1):
        pg = orc.default_params(T=50, M=4, K=10, L=1, sampler=1, behaviour=behaviour)
        a, b = orc.plan(pg, sc, 5, 60), orc.plan(pg, sc, 99, 60)
        assert a.best_index == b.best_index and np.array_equal(a.xi_best, b.xi_best)
        grid = orc.sample(pg, 0, 0, 60, True)
        assert np.array_equal(a.p_best, grid[a.best_index])
