"""GPU parity of the goal-position behavioural inputs (PLAN_BEHAV_GOALS: p =
[x_f - x0, y_f], eq. final_boundary, cost c_s alone) and of the fixed-grid
initial sampler (PLAN_SAMPLER_GRID; with one upper iteration the MPC-Grid
baseline) against the FP64 oracle: the lower level teacher-forced on the
oracle's samples in both precisions, Alg. 1 one iteration at a time, and the
closed loop in goal mode."""
import numpy as np
import pytest

from paper_2212_02224_amd import workload
from parity_common import Spread, check_positions
from test_parity_plan import run_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pl():
    import paper_2212_02224_amd as pl
    pl.load()
    return pl


def pos_err(orc, T, t_f, xa, xb):
    W, _, _ = orc.basis(T, t_f)
    dx = (xa[:, :11] - xb[:, :11]) @ W.T
    dy = (xa[:, 11:] - xb[:, 11:]) @ W.T
    return np.sqrt(dx ** 2 + dy ** 2).max(axis=1)


@pytest.mark.parametrize("precision,tol", [(0, 1e-4), (1, 1e-3), (2, 1e-4)])
@pytest.mark.parametrize("N,T,M,structured", [(256, 100, 10, True), (37, 50, 4, True), (64, 100, 20, False),
                                              (9, 128, 3, True)])
def test_goal_lower_parity(orc, pl, precision, tol, N, T, M, structured):
    K = 15
    par = orc.default_params(T=T, M=M, K=K, behaviour=1)
    s = workload.scene(8, N + T + M, M)
    sc = orc.Scene(s.ego, s.obstacles)
    if structured:
        p = orc.sample(par, s.seed, 0, N, True)
    else:
        mu = np.r_[60.0, 1.0, np.zeros(6)]
        Lc = np.zeros((8, 8))
        Lc[:2, :2] = [[15.0, 0.0], [0.5, 1.5]]
        p = orc.sample(par, s.seed, 2, N, False, mu, Lc)
    print(f"[goal parity] precision {precision} N={N} T={T} M={M} structured={structured}", flush=True)
    xb_o = orc.step1(par, sc, p)
    xs_o = orc.project(par, sc, xb_o, p=p)
    r_o, c_o = orc.residual_cost(par, sc, xs_o)
    cfg = pl.plan_config_init(T_set=[T], M_set=[M], proj_iters=K, max_N=max(N, 16), max_requests=1,
                              precision=precision, behaviour=pl.PLAN_BEHAV_GOALS)
    h = pl.plan_create(cfg)
    req = pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed)
    xb_g, xs_g, r_g, c_g = pl.plan_lower_solve(h, req, p)
    e_bar = pos_err(orc, T, par.t_f, xb_g, xb_o)
    e_star = pos_err(orc, T, par.t_f, xs_g, xs_o)
    sp = Spread(orc, par, sc, xb_o, xs_o, p=p)
    print(f"   xi_bar err {e_bar.max():.2e}", flush=True)
    check_positions("xi*", e_star, sp, tol)
    assert e_bar.max() <= 1e-4
    r_scale = 10.0 if precision == 1 else 1.0
    assert np.all(np.abs(r_g - r_o) <= sp.r_bar(r_scale * (1e-3 + 1e-4 * np.abs(r_o))))
    assert np.all(np.abs(c_g - c_o) <= sp.cu_bar(r_scale * 1e-4 * np.abs(c_o) + 1e-4))
    # the goal rows: x(t_f) = x0 + p0, y(t_f) = p1, ydot(t_f) = 0 (coefficients c10, c9 = c10)
    assert np.all(np.abs(xs_g[:, 10] - (s.ego[0] + p[:, 0])) <= 1e-4 * (1 + np.abs(p[:, 0])))
    assert np.all(np.abs(xs_g[:, 21] - p[:, 1]) <= 1e-5) and np.array_equal(xs_g[:, 20], xs_g[:, 21])


@pytest.mark.parametrize("cfgid,scene_idx", [(1, 0), (2, 0)])
def test_goal_plan_parity_per_iteration(orc, pl, cfgid, scene_idx):
    run_config(orc, pl, cfgid, scene_idx, behaviour=1)


def test_goal_plan_parity_fp16_split(orc, pl):
    run_config(orc, pl, 1, 1, precision=1, tol_scale=10.0, pos_tol=1e-3, behaviour=1)


@pytest.mark.parametrize("behaviour", [0, 1])
@pytest.mark.parametrize("cfgid", [1, 2])
def test_grid_plan_parity(orc, pl, behaviour, cfgid):
    """MPC-Grid: one upper iteration from the fixed grid (samples, residuals,
    elite sets, update and returned sample checked as in the plan parity)."""
    run_config(orc, pl, cfgid, 2, behaviour=behaviour, sampler=1, L=1)


def test_grid_plan_does_not_depend_on_the_seed(pl):
    cfg = pl.plan_config_init(T_set=[100], M_set=[10], proj_iters=20, upper_iters=1, max_N=1000, max_requests=2,
                              sampler=pl.PLAN_SAMPLER_GRID)
    h = pl.plan_create(cfg)
    s = workload.scene(2, 4, 10)
    a, b = pl.plan_solve_batch(h, [pl.Request(N=1000, T=100, ego=s.ego, obstacles=s.obstacles, seed=seed)
                                   for seed in (1, 2)])
    assert a.status == b.status == 0 and a.best_index == b.best_index
    assert np.array_equal(a.xi_best, b.xi_best) and np.array_equal(a.p_best, b.p_best)


def test_goal_closed_loop_equals_single_plans(orc, pl):
    """The receding-horizon loop with goal positions: each cycle's plan is
    the single plan of that cycle's state, and the goal slots of mu stay
    the only nonzero ones."""
    kw = dict(T_set=[50, 100], M_set=[4, 10], proj_iters=10, upper_iters=3, max_N=256, max_requests=2,
              behaviour=pl.PLAN_BEHAV_GOALS)
    h = pl.plan_create(pl.plan_config_init(**kw))
    reqs = []
    for i, (N, T, M) in enumerate([(128, 100, 10), (64, 50, 4)]):
        s = workload.scene(8, 500 + i, M)
        reqs.append(pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, session_id=40 + i))
    cycles = 3
    _, log = pl.plan_mpc_run(h, reqs, cycles, 5, init=pl.PLAN_MPC_WARM)
    assert np.all(log["status"] == 0)
    assert np.all(log["mu"][:, :, 2:] == 0)
    ref = pl.plan_create(pl.plan_config_init(**kw))
    for e, r in enumerate(reqs):
        par = orc.default_params(T=r.T, M=r.M)
        for c in range(cycles):
            obs = (np.asarray(r.obstacles, float) if c == 0
                   else orc.advance(par, np.zeros(22), r.obstacles, c - 1, 5)[1])
            extra = dict(mu0=log["mu"][e, c - 1], sigma0=log["sigma"][e, c - 1]) if c else {}
            q = pl.Request(N=r.N, T=r.T, ego=log["ego"][e, c], obstacles=obs, seed=r.seed + c, **extra)
            one = pl.plan_solve_batch(ref, [q])[0]
            assert one.status == 0 and np.array_equal(one.xi_best, log["xi"][e, c]), (e, c)
