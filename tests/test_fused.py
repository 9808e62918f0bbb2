"""GPU tests of the fused iterations (plan_config.fused_iters, include/plan.h):
every upper iteration of a launch group in one launch, each request's
selection and update (Alg. 1) run on the device by the workgroup that
finishes its last samples. The per-request arithmetic is that of the
per-iteration launches, so results must be bitwise the same in every mode;
the bounded device-side waits must give up cleanly and leave the handle
usable."""
import numpy as np
import pytest

from paper_2212_02224_amd import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pl():
    import paper_2212_02224_amd as pl
    pl.load()
    return pl


def same(a, b):
    """Every field of two results bitwise equal (latency aside)."""
    return (a.status == b.status == 0 and a.best_index == b.best_index and a.flags == b.flags
            and a.iterations == b.iterations and np.array_equal(a.p_best, b.p_best)
            and np.array_equal(a.xi_best, b.xi_best) and np.array_equal(a.mu, b.mu)
            and np.array_equal(a.sigma, b.sigma) and a.residual == b.residual and a.cost_upper == b.cost_upper
            and np.array_equal(a.traj, b.traj))


def reqs_for(pl, case):
    out = []
    if case == "single":  # one plan of N = 1000, T = 100, M = 10
        s = workload.scene(2, 0, 10)
        return [pl.Request(N=1000, T=100, ego=s.ego, obstacles=s.obstacles, seed=s.seed)]
    if case == "mix":  # uneven N, T and M in one batch
        for i, (N, T, M) in enumerate([(64, 50, 4), (300, 100, 10), (17, 100, 20), (512, 50, 10), (1, 100, 4),
                                       (250, 100, 20), (700, 100, 4)]):
            s = workload.scene(4, 30 + i, M)
            out.append(pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, request_id=i))
        return out
    if case == "road":  # requests with and without a road profile: two launch groups
        for i in range(4):
            s = workload.scene(2, 60 + i, 10)
            kw = {}
            if i % 2 == 0:
                rp, rx0, rdx = workload.curved_road(2, 60 + i)
                kw = dict(road=rp, road_x0=rx0, road_dx=rdx)
            out.append(pl.Request(N=400 + 100 * i, T=100, ego=s.ego, obstacles=s.obstacles, seed=s.seed, **kw))
        return out
    if case == "ipl2":  # a launch of two instants per lane (T = 200, three 4096-sample requests)
        for i, N in enumerate([4096, 4096, 4096, 64]):
            s = workload.scene(4, 400 + i, 10)
            out.append(pl.Request(N=N, T=200, ego=s.ego, obstacles=s.obstacles, seed=s.seed, request_id=i))
        return out
    raise ValueError(case)


def cfg_for(pl, case, fused, **over):
    kw = dict(T_set=[50, 100], M_set=[4, 10, 20], proj_iters=20, upper_iters=5, max_N=1024, max_requests=8,
              fused_iters=fused)
    if case == "ipl2":
        kw.update(T_set=[200], M_set=[10], proj_iters=10, upper_iters=3, max_N=4096, max_requests=4)
    kw.update(over)
    return pl.plan_config_init(**kw)


@pytest.mark.parametrize("case", ["single", "mix", "road", "ipl2"])
def test_fused_equals_per_iteration(pl, case):
    reqs = reqs_for(pl, case)
    got = {}
    for fused in (0, 1):
        h = pl.plan_create(cfg_for(pl, case, fused))
        got[fused] = pl.plan_solve_batch(h, reqs)
        # a second launch of the same handle: the control words were reset
        again = pl.plan_solve_batch(h, reqs)
        for a, b in zip(got[fused], again):
            assert same(a, b)
    for i, (a, b) in enumerate(zip(got[1], got[0])):
        assert same(a, b), (case, i)


def test_fused_trace_and_sessions_equal_per_iteration(pl):
    """The per-iteration trace (samples, residuals, costs, elite sets, mu,
    Sigma) and session warm starts are those of the per-iteration launches."""
    s = [workload.scene(2, 80 + i, 10) for i in range(3)]
    first = [pl.Request(N=500, T=100, ego=x.ego, obstacles=x.obstacles, seed=x.seed, session_id=7 + i)
             for i, x in enumerate(s)]
    second = [pl.Request(N=500, T=100, ego=x.ego, obstacles=x.obstacles, seed=x.seed + 1, session_id=7 + i)
              for i, x in enumerate(s)]
    res, tr = {}, {}
    for fused in (0, 1):
        cfg = pl.plan_config_init(T_set=[100], M_set=[10], max_N=1024, max_requests=4, trace=1, fused_iters=fused)
        h = pl.plan_create(cfg)
        a = pl.plan_solve_batch(h, first)
        n, q = pl.elite_sizes(cfg, 500)
        tr[fused] = [pl.plan_get_trace(h, i, 500, n, q) for i in range(len(first))]
        b = pl.plan_solve_batch(h, second)
        res[fused] = a + b
    for x, y in zip(res[0], res[1]):
        assert same(x, y)
        assert y.flags & pl.PLAN_F_WARM or y.iterations == 5
    for t0, t2 in zip(tr[0], tr[1]):
        assert t0.keys() == t2.keys()
        for k in t0:
            assert np.array_equal(t0[k], t2[k]), k


def test_fused_decoder_sampler_equals_per_iteration(pl):
    """Iteration 0 from the decoder sampler's samples (decoded before the
    fused launch), then the Gaussian updates."""
    dec = workload.decoder_weights(0)
    res = {}
    for fused in (0, 1):
        h = pl.plan_create(pl.plan_config_init(T_set=[100], M_set=[10], max_N=1024, max_requests=4,
                                               sampler=pl.PLAN_SAMPLER_DECODER, fused_iters=fused))
        pl.plan_set_decoder(h, dec)
        reqs = []
        for i in range(3):
            s = workload.scene(2, 90 + i, 10)
            reqs.append(pl.Request(N=300 + 200 * i, T=100, ego=s.ego, obstacles=s.obstacles, seed=s.seed,
                                   observation=workload.observation(s)))
        res[fused] = pl.plan_solve_batch(h, reqs)
    for a, b in zip(res[0], res[1]):
        assert same(a, b)


def test_fused_served_equals_alone(pl):
    """Served mode with fused iterations: each plan_progress call enqueues the
    whole solve of what it admits; staggered arrivals each return their
    result alone (per-iteration launches), bit for bit, and all retire."""
    reqs = reqs_for(pl, "mix")
    h0 = pl.plan_create(cfg_for(pl, "mix", 0))
    ref = [pl.plan_solve_batch(h0, [r])[0] for r in reqs]
    h = pl.plan_create(cfg_for(pl, "mix", 1, max_requests=4, sample_budget=1500))
    tickets, got = [], {}
    for i, r in enumerate(reqs):
        tickets.append(pl.plan_submit(h, r))
        if i % 2 == 1:
            pl.plan_progress(h)
    for _ in range(100):
        act, q = pl.plan_progress(h)
        for t, r in pl.plan_poll_done(h, 8):
            got[t] = r
        if len(got) == len(tickets):
            break
    assert sorted(got) == sorted(tickets)
    for i, t in enumerate(tickets):
        assert same(got[t], ref[i]), i
    act, q = pl.plan_progress(h)
    assert act == 0 and q == 0
    assert pl.plan_solve_batch(h, [reqs[0]])[0].status == 0


def test_fused_wait_gives_up_and_handle_stays_usable(pl):
    """With a wait bound of 1 us the workgroups of iteration 1 cannot wait for
    the update of iteration 0 (it takes microseconds): they give up, the
    launch ends, the request fails with PLAN_E_TIMEOUT, and the control words
    are reset (a second call behaves the same; a request of one iteration,
    which never waits, still solves, and equals its per-iteration result)."""
    s = workload.scene(2, 5, 10)
    req = pl.Request(N=4096, T=100, ego=s.ego, obstacles=s.obstacles, seed=s.seed)
    cfg = pl.plan_config_init(T_set=[100], M_set=[10], max_N=4096, max_requests=2, upper_iters=3,
                              fused_iters=1, fused_wait_us=1)
    h = pl.plan_create(cfg)
    for _ in range(2):
        r = pl.plan_solve_batch(h, [req], check=False)[0]
        assert r.status == pl.PLAN_E_TIMEOUT
    with pytest.raises(pl.PlanError) as e:
        pl.plan_solve_batch(h, [req])
    assert e.value.status == pl.PLAN_E_TIMEOUT
    assert "fused_wait_us" in pl.plan_last_error(h)
    one = dict(T_set=[100], M_set=[10], max_N=4096, max_requests=2, upper_iters=1)
    h1 = pl.plan_create(pl.plan_config_init(fused_iters=1, fused_wait_us=1, **one))
    h0 = pl.plan_create(pl.plan_config_init(fused_iters=0, **one))
    assert same(pl.plan_solve_batch(h1, [req])[0], pl.plan_solve_batch(h0, [req])[0])
