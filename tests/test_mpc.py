"""GPU checks of the receding-horizon closed loop (plan_mpc_run): the loop
that runs on the device without host round trips equals a host-driven
sequence of single plans bit for bit (same state, neighbours, seed and warm
start per cycle), and its advance step has the properties that define it:
each cycle starts at the previous cycle's returned trajectory evaluated at
the execution instant, and a cycle is flagged as a collision exactly when an
executed instant lies inside a neighbour's ellipse (evaluated here in FP64
with the Bernstein basis of eq. param). The per-iteration parity of each
plan against the oracle is covered by the plan parity tests; the warm start
enters them the same way (a given mu, Sigma at iteration 0). The oracle's
own advance is pinned on the CPU (test_oracle_mpc.py)."""
import numpy as np
import pytest

from paper_2212_02224_amd import workload

pytestmark = pytest.mark.gpu

N_EXEC = 5


@pytest.fixture(scope="module")
def pl():
    import paper_2212_02224_amd as pl
    pl.load()
    return pl


def episodes(pl, mix, base):
    reqs = []
    for i, (N, T, M) in enumerate(mix):
        s = workload.scene(6, base + i, M)
        reqs.append(pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, request_id=i,
                               session_id=1000 + base + i))
    return reqs


def obstacles_at_cycle(orc, par, obs0, c):
    if c == 0:
        return np.asarray(obs0, float).reshape(-1, 4)
    # the neighbours depend only on their first-cycle states and the cycle
    return orc.advance(par, np.zeros(22), obs0, c - 1, N_EXEC)[1]


def check_loop_against_single_plans(orc, pl, precision, init):
    mix = [(64, 50, 4), (200, 100, 10), (17, 100, 20)]
    cycles = 4
    kw = dict(T_set=[50, 100], M_set=[4, 10, 20], proj_iters=10, upper_iters=3, max_N=256, max_requests=4,
              precision=precision)
    h = pl.plan_create(pl.plan_config_init(**kw))
    reqs = episodes(pl, mix, 10 * precision + 20 * init)
    print(f"[mpc] precision {precision} init {init}: {len(reqs)} episodes x {cycles} cycles", flush=True)
    res, log = pl.plan_mpc_run(h, reqs, cycles, N_EXEC, init=init)
    assert np.all(log["status"] == 0)
    ref = pl.plan_create(pl.plan_config_init(**kw))
    for e, r in enumerate(reqs):
        par = orc.default_params(T=r.T, M=r.M)
        assert np.array_equal(log["ego"][e, 0], np.asarray(r.ego, float))
        for c in range(cycles):
            extra = {}
            if c > 0 and init == pl.PLAN_MPC_WARM:
                extra = dict(mu0=log["mu"][e, c - 1], sigma0=log["sigma"][e, c - 1])
            q = pl.Request(N=r.N, T=r.T, ego=log["ego"][e, c], obstacles=obstacles_at_cycle(orc, par, r.obstacles, c),
                           seed=r.seed + c, **extra)
            one = pl.plan_solve_batch(ref, [q])[0]
            assert one.status == 0
            assert np.array_equal(one.xi_best, log["xi"][e, c]), (e, c)
            assert np.array_equal(one.mu, log["mu"][e, c]) and np.array_equal(one.sigma, log["sigma"][e, c]), (e, c)
            assert np.array_equal([one.cost_upper, one.residual], log["cost"][e, c])
        assert np.array_equal(res[e].xi_best, log["xi"][e, -1]) and np.array_equal(res[e].mu, log["mu"][e, -1])
    return reqs, log


@pytest.mark.parametrize("init", [0, 1])
def test_mpc_loop_equals_single_plans_fp32(orc, pl, init):
    check_loop_against_single_plans(orc, pl, 0, init)


@pytest.mark.parametrize("init", [0, 1])
def test_mpc_loop_equals_single_plans_fp16_split(orc, pl, init):
    check_loop_against_single_plans(orc, pl, 1, init)


def check_advance(orc, reqs, log, cycles):
    """The properties of the advance step on the loop's own logs: the state
    of cycle c + 1 is trajectory xi_c at t_{n_exec} (position, velocity,
    acceleration of both axes), and cycle c is flagged iff an executed
    instant t_0..t_{n_exec} lies inside a neighbour's ellipse, the
    neighbours moving at constant velocity from their first-cycle states
    (scene time (c n_exec + k) t_f / (T - 1)). Returns the largest state
    difference."""
    worst = 0.0
    for e, r in enumerate(reqs):
        par = orc.default_params(T=r.T, M=r.M)
        W, Wd, Wdd = orc.basis(r.T, par.t_f)
        obs0 = np.asarray(r.obstacles, float).reshape(-1, 4)
        for c in range(cycles):
            xi = log["xi"][e, c]
            k = N_EXEC
            want = np.array([W[k] @ xi[:11], W[k] @ xi[11:], Wd[k] @ xi[:11], Wd[k] @ xi[11:],
                             Wdd[k] @ xi[:11], Wdd[k] @ xi[11:]])
            d = np.abs(want - log["ego"][e, c + 1])
            worst = max(worst, d.max())
            assert np.all(d <= 1e-9 * (1 + np.abs(want))), (e, c, d)
            hit = False
            for kk in range(N_EXEC + 1):
                x, y = W[kk] @ xi[:11], W[kk] @ xi[11:]
                s = (c * N_EXEC + kk) * par.t_f / (r.T - 1)
                u = (x - (obs0[:, 0] + obs0[:, 2] * s)) / par.ell_a
                v = (y - (obs0[:, 1] + obs0[:, 3] * s)) / par.ell_b
                hit = hit or bool(np.any(u * u + v * v < 1.0))
            assert bool(log["collided"][e, c]) == hit, (e, c)
    return worst


def test_mpc_advance_properties(orc, pl):
    mix = [(128, 100, 10), (64, 50, 4), (96, 100, 20), (32, 50, 10)]
    cycles = 6
    h = pl.plan_create(pl.plan_config_init(T_set=[50, 100], M_set=[4, 10, 20], proj_iters=10, upper_iters=3,
                                           max_N=128, max_requests=4))
    reqs = episodes(pl, mix, 40)
    _, log = pl.plan_mpc_run(h, reqs, cycles, N_EXEC)
    worst = check_advance(orc, reqs, log, cycles)
    print(f"[mpc] advance: largest state difference {worst:.2e}", flush=True)
    # each cycle starts where the previous one ended: x moves forward
    assert np.all(np.diff(log["ego"][:, :, 0], axis=1) > 0)


def test_mpc_collision_is_reported(orc, pl):
    """A neighbour placed on the ego (normalised distance below 1 at t = 0)
    is a collision of the first cycle, and the flags have the advance
    properties."""
    T, M = 50, 4
    h = pl.plan_create(pl.plan_config_init(T_set=[T], M_set=[M], proj_iters=10, upper_iters=2, max_N=64,
                                           max_requests=2))
    s = workload.scene(6, 99, M)
    obs = np.array(s.obstacles, float)
    obs[0] = [s.ego[0] + 1.0, s.ego[1], s.ego[2], 0.0]  # inside the ellipse, same speed
    reqs = [pl.Request(N=64, T=T, ego=s.ego, obstacles=obs, seed=5, session_id=77)]
    _, log = pl.plan_mpc_run(h, reqs, 2, N_EXEC)
    assert log["collided"][0, 0] == 1
    check_advance(orc, reqs, log, 2)


@pytest.mark.parametrize("init", [0, 1])
def test_mpc_episode_results_do_not_depend_on_the_batch(pl, init):
    """An episode's loop alone equals the same episode inside a batch."""
    kw = dict(T_set=[50, 100], M_set=[4, 10, 20], proj_iters=8, upper_iters=3, max_N=512, max_requests=4)
    mix = [(300, 100, 10), (512, 50, 20), (40, 100, 4)]
    reqs = episodes(pl, mix, 60)
    h = pl.plan_create(pl.plan_config_init(**kw))
    _, both = pl.plan_mpc_run(h, reqs, 3, N_EXEC, init=init)
    for e in range(len(reqs)):
        h1 = pl.plan_create(pl.plan_config_init(**kw))
        _, alone = pl.plan_mpc_run(h1, [reqs[e]], 3, N_EXEC, init=init)
        for k in ("ego", "xi", "mu", "collided"):
            assert np.array_equal(alone[k][0], both[k][e]), (e, k)


def test_mpc_rejects_bad_arguments(pl):
    h = pl.plan_create(pl.plan_config_init(T_set=[50], M_set=[4], proj_iters=5, upper_iters=2, max_N=64,
                                           max_requests=2))
    s = workload.scene(6, 5, 4)

    def req(sid, T=50):
        return pl.Request(N=16, T=T, ego=s.ego, obstacles=s.obstacles, seed=1, session_id=sid)

    W = pl.PLAN_MPC_WARM
    for reqs, cycles, n_exec, init in [([req(0)], 2, 5, W), ([req(3), req(3)], 2, 5, 0), ([req(3)], 0, 5, 0),
                                       ([req(3)], 2, 50, 0), ([req(3)], 2, 0, W), ([req(3), req(4), req(5)], 1, 5, 0),
                                       ([req(3, T=60)], 1, 5, 0), ([req(3)], 1, 5, 7)]:
        with pytest.raises(pl.PlanError) as ei:
            pl.plan_mpc_run(h, reqs, cycles, n_exec, init=init)
        assert ei.value.status == pl.PLAN_E_INVALID
    # the handle still works afterwards; without a warm start no session is needed
    res, log = pl.plan_mpc_run(h, [req(0), req(0)], 2, 5, log=("ego", "collided"))
    assert res[0].status == 0 and set(log) == {"ego", "collided"}


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_mpc_full_size(orc, pl, precision):
    """The measured closed-loop configuration at full size: 256 episodes of
    N = 1000, T = 100, M = 10, L = 5, K = 20 (the headline planner), here for
    three cycles. Every cycle succeeds, the advance properties hold for every
    episode and cycle, and sampled episodes equal the same episode run
    alone, bit for bit."""
    c = workload.CONFIGS[2]
    N, T, M, L, K = c["N"], c["T"], c["M"], c["L"], c["K"]
    cycles, n_ep = 3, 256
    kw = dict(T_set=[T], M_set=[M], proj_iters=K, upper_iters=L, max_N=N, precision=precision)
    reqs = []
    for i in range(n_ep):
        s = workload.scene(7, i, M)
        reqs.append(pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, request_id=i,
                               session_id=1 + i))
    print(f"[mpc full size] precision {precision}: {n_ep} episodes x {cycles} cycles, N={N}", flush=True)
    h = pl.plan_create(pl.plan_config_init(max_requests=n_ep, **kw))
    _, log = pl.plan_mpc_run(h, reqs, cycles, N_EXEC)
    assert np.all(log["status"] == 0)
    worst = check_advance(orc, reqs, log, cycles)
    print(f"   advance: largest state difference {worst:.2e}; collisions flagged "
          f"{int(log['collided'].sum())}", flush=True)
    h1 = pl.plan_create(pl.plan_config_init(max_requests=1, **kw))
    for e in (0, 97, 255):
        _, alone = pl.plan_mpc_run(h1, [reqs[e]], cycles, N_EXEC)
        for k in ("ego", "xi", "mu", "collided"):
            assert np.array_equal(alone[k][0], log[k][e]), (e, k)
