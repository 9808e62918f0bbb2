"""GPU parity of the road profile (the centripetal row's curvature kappa(x)
and the lane limits y_lb(x), y_ub(x) of Table ineq_list, evaluated at each
iterate's position along the road) against the FP64 oracle: the lower level
teacher-forced on the oracle's samples in both precisions, Alg. 1 one
iteration at a time, the closed loop on a curved road; and, on the GPU
alone, a one-knot profile against the constant road it describes and batches
that mix requests with and without a profile."""
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


def road_kw(cfgid, idx):
    rp, rx0, rdx = workload.curved_road(cfgid, idx)
    return dict(road=rp, road_x0=rx0, road_dx=rdx)


@pytest.mark.parametrize("precision,tol", [(0, 1e-4), (1, 1e-3), (2, 1e-4)])
@pytest.mark.parametrize("N,T,M,idx,v0", [(256, 100, 10, 0, 18.0), (37, 50, 4, 1, 20.0), (9, 128, 3, 4, 22.0),
                                           (200, 64, 20, 3, 24.0)])
def test_road_lower_parity(orc, pl, precision, tol, N, T, M, idx, v0):
    K = 15
    par = orc.default_params(T=T, M=M, K=K)
    s = workload.scene(6, idx, M)
    s.ego[2] = v0  # faster than the scenes' default, so that the bend's centripetal row binds
    rk = road_kw(6, idx)
    sc = orc.Scene(s.ego, s.obstacles, **rk)
    p = orc.sample(par, s.seed, 0, N, True)
    print(f"[road parity] precision {precision} N={N} T={T} M={M} road {idx}", flush=True)
    xb_o = orc.step1(par, sc, p)
    xs_o = orc.project(par, sc, xb_o)
    r_o, c_o = orc.residual_cost(par, sc, xs_o)
    # the profile matters: on the straight road many projections end elsewhere
    xs_flat = orc.project(par, orc.Scene(s.ego, s.obstacles), xb_o)
    assert np.mean(pos_err(orc, T, par.t_f, xs_flat, xs_o) > 1e-2) > 0.1
    cfg = pl.plan_config_init(T_set=[T], M_set=[M], proj_iters=K, max_N=max(N, 16), max_requests=1,
                              precision=precision)
    h = pl.plan_create(cfg)
    req = pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, **rk)
    xb_g, xs_g, r_g, c_g = pl.plan_lower_solve(h, req, p)
    e_bar = pos_err(orc, T, par.t_f, xb_g, xb_o)
    e_star = pos_err(orc, T, par.t_f, xs_g, xs_o)
    sp = Spread(orc, par, sc, xb_o, xs_o)
    print(f"   xi_bar err {e_bar.max():.2e}", flush=True)
    check_positions("xi*", e_star, sp, tol)
    assert e_bar.max() <= 1e-4
    r_scale = 10.0 if precision == 1 else 1.0
    assert np.all(np.abs(r_g - r_o) <= sp.r_bar(r_scale * (1e-3 + 1e-4 * np.abs(r_o))))
    assert np.all(np.abs(c_g - c_o) <= sp.cu_bar(r_scale * 1e-4 * np.abs(c_o) + 1e-4))


@pytest.mark.parametrize("cfgid,scene_idx", [(1, 0), (2, 0)])
def test_road_plan_parity_per_iteration(orc, pl, cfgid, scene_idx):
    run_config(orc, pl, cfgid, scene_idx, road=True)


def test_road_plan_parity_fp16_split(orc, pl):
    run_config(orc, pl, 1, 1, precision=1, tol_scale=10.0, pos_tol=1e-3, road=True)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_one_knot_profile_equals_constant_road(pl, precision):
    """A profile of one knot (kappa, y_lb, y_ub) describes the constant road
    with that curvature and the configured lane limits: same plan, bit for
    bit, though it runs in the kernel variant with the profile lookup."""
    cfg = pl.plan_config_init(T_set=[50, 100], M_set=[4, 10], proj_iters=10, upper_iters=3, max_N=512,
                              max_requests=1, precision=precision)
    h = pl.plan_create(cfg)
    for i, (N, T, M, kappa) in enumerate([(256, 100, 10, 0.012), (64, 50, 4, -0.02), (500, 100, 4, 0.0)]):
        s = workload.scene(6, 40 + i, M)
        base = dict(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed)
        a = pl.plan_solve_batch(h, [pl.Request(kappa_road=kappa, **base)])[0]
        b = pl.plan_solve_batch(h, [pl.Request(road=np.array([[kappa, cfg.y_lb, cfg.y_ub]]), road_x0=25.0,
                                               **base)])[0]
        assert a.status == b.status == 0
        assert a.best_index == b.best_index, i
        assert np.array_equal(a.xi_best, b.xi_best) and np.array_equal(a.mu, b.mu), i


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_mixed_road_batch_equals_alone(pl, precision):
    """Requests with and without a profile in one batch and in the served
    mode (separate launches per kernel variant) return what they return
    alone."""
    kw = dict(T_set=[50, 100], M_set=[4, 10, 20], proj_iters=8, upper_iters=3, max_N=1024, max_requests=8,
              precision=precision)
    mix = [(64, 50, 4, True), (300, 100, 10, False), (17, 100, 20, True), (512, 50, 10, False),
           (250, 100, 20, True), (128, 50, 20, True)]
    reqs = []
    for i, (N, T, M, road) in enumerate(mix):
        s = workload.scene(6, 60 + i, M)
        s.ego[2] = 20.0
        rk = road_kw(6, 60 + i) if road else {}
        reqs.append(pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, request_id=i, **rk))
    h1 = pl.plan_create(pl.plan_config_init(**kw))
    alone = [pl.plan_solve_batch(h1, [r])[0] for r in reqs]
    h2 = pl.plan_create(pl.plan_config_init(**kw))
    batch = pl.plan_solve_batch(h2, reqs)
    h3 = pl.plan_create(pl.plan_config_init(**kw))
    tickets = [pl.plan_submit(h3, r) for r in reqs]
    got = {}
    for _ in range(200):
        pl.plan_progress(h3)
        for t in tickets:
            if t not in got:
                r = pl.plan_poll(h3, t)
                if r is not None:
                    got[t] = r
        if len(got) == len(tickets):
            break
    assert len(got) == len(tickets)
    for i, a in enumerate(alone):
        for b in (batch[i], got[tickets[i]]):
            assert a.status == b.status == 0, i
            assert a.best_index == b.best_index and np.array_equal(a.xi_best, b.xi_best), i
            assert np.array_equal(a.mu, b.mu) and np.array_equal(a.sigma, b.sigma), i


def test_road_closed_loop_equals_single_plans(orc, pl):
    """The receding-horizon loop on a curved road: the profile is fixed along
    the road (absolute x), so each cycle's plan is the single plan of that
    cycle's state with the same profile."""
    kw = dict(T_set=[50, 100], M_set=[4, 10], proj_iters=10, upper_iters=3, max_N=256, max_requests=2)
    h = pl.plan_create(pl.plan_config_init(**kw))
    reqs, rks = [], []
    for i, (N, T, M) in enumerate([(128, 100, 10), (64, 50, 4)]):
        s = workload.scene(6, 80 + i, M)
        rk = road_kw(6, 80 + i)
        rks.append(rk)
        reqs.append(pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, session_id=60 + i, **rk))
    cycles = 3
    _, log = pl.plan_mpc_run(h, reqs, cycles, 5, init=pl.PLAN_MPC_WARM)
    assert np.all(log["status"] == 0)
    ref = pl.plan_create(pl.plan_config_init(**kw))
    for e, r in enumerate(reqs):
        par = orc.default_params(T=r.T, M=r.M)
        for c in range(cycles):
            obs = (np.asarray(r.obstacles, float) if c == 0
                   else orc.advance(par, np.zeros(22), r.obstacles, c - 1, 5)[1])
            extra = dict(mu0=log["mu"][e, c - 1], sigma0=log["sigma"][e, c - 1]) if c else {}
            q = pl.Request(N=r.N, T=r.T, ego=log["ego"][e, c], obstacles=obs, seed=r.seed + c, **rks[e], **extra)
            one = pl.plan_solve_batch(ref, [q])[0]
            assert one.status == 0 and np.array_equal(one.xi_best, log["xi"][e, c]), (e, c)


def test_bad_road_profiles_rejected(pl):
    h = pl.plan_create(pl.plan_config_init(T_set=[50], M_set=[4], max_N=64, max_requests=1))
    s = workload.scene(6, 90, 4)
    base = dict(N=64, T=50, ego=s.ego, obstacles=s.obstacles, seed=s.seed)
    good = np.array([[0.01, -7.0, 7.0], [0.02, -7.0, 6.0]])
    for bad in (dict(road=np.tile(good[:1], (pl.PLAN_MAX_ROAD + 1, 1))),
                dict(road=np.array([[0.01, 7.0, 7.0]])),
                dict(road=good, road_dx=0.0),
                dict(road=good, road_dx=-5.0),
                dict(road=np.array([[np.nan, -7.0, 7.0]])),
                dict(road=good, road_x0=np.inf)):
        assert pl.plan_solve_batch(h, [pl.Request(**base, **bad)])[0].status == pl.PLAN_E_INVALID, bad
    assert pl.plan_solve_batch(h, [pl.Request(**base, road=good, road_dx=30.0)])[0].status == 0


def test_served_request_owns_its_road_profile(pl):
    """plan_submit copies the profile: overwriting the caller's array before
    the request is admitted changes nothing."""
    kw = dict(T_set=[100], M_set=[10], proj_iters=8, upper_iters=2, max_N=256, max_requests=2)
    s = workload.scene(6, 95, 10)
    s.ego[2] = 20.0
    rk = road_kw(6, 95)
    alone = pl.plan_solve_batch(pl.plan_create(pl.plan_config_init(**kw)),
                                [pl.Request(N=256, T=100, ego=s.ego, obstacles=s.obstacles, seed=s.seed, **rk)])[0]
    h = pl.plan_create(pl.plan_config_init(**kw))
    road = rk["road"].copy()
    t = pl.plan_submit(h, pl.Request(N=256, T=100, ego=s.ego, obstacles=s.obstacles, seed=s.seed,
                                     road=road, road_x0=rk["road_x0"], road_dx=rk["road_dx"]))
    road[:] = 0.0  # y_lb = y_ub = 0: an invalid profile, if it were read now
    got = None
    for _ in range(10):
        pl.plan_progress(h)
        got = pl.plan_poll(h, t)
        if got is not None:
            break
    assert got is not None and got.status == alone.status == 0
    assert got.best_index == alone.best_index and np.array_equal(got.xi_best, alone.xi_best)
