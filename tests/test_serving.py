"""GPU tests of the served mode (continuous batching, include/plan.h):
requests submitted at different times join the resident set at the next
upper iteration, share the kernel launches with whatever is resident, are
admitted by slot and sample-row budget, and return exactly the result they
have when solved alone."""
import numpy as np
import pytest

from paper_2212_02224_amd import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pl():
    import paper_2212_02224_amd as pl
    pl.load()
    return pl


@pytest.fixture(params=[0, 1], ids=["ticked", "fused"])
def mode(request):
    """plan_config.fused_iters: per-iteration host ticks, or each admission's
    whole solve enqueued at once (fused launches)."""
    return request.param


MIX = [(64, 50, 4), (300, 100, 10), (17, 100, 20), (512, 50, 10), (1, 100, 4), (250, 100, 20),
       (128, 50, 20), (700, 100, 4)]


def reqs_of(pl, cfgid=4):
    out = []
    for i, (N, T, M) in enumerate(MIX):
        s = workload.scene(cfgid, 100 + i, M)
        out.append(pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, request_id=i))
    return out


def cfg_of(pl, mode=1, **over):
    kw = dict(T_set=[50, 100], M_set=[4, 10, 20], proj_iters=8, upper_iters=3, max_N=1024, max_requests=8,
              fused_iters=mode)
    kw.update(over)
    return pl.plan_config_init(**kw)


def alone_results(pl, reqs):
    h = pl.plan_create(cfg_of(pl, 0))
    return [pl.plan_solve_batch(h, [r])[0] for r in reqs]


def drain(pl, h, tickets, max_ticks=200):
    """Drive plan_progress and poll every ticket until all are done; the
    counts are those of one more plan_progress call (results can also be
    retired by plan_poll)."""
    got = {}
    for _ in range(max_ticks):
        pl.plan_progress(h)
        for t in tickets:
            if t not in got:
                r = pl.plan_poll(h, t)
                if r is not None:
                    got[t] = r
        if len(got) == len(tickets):
            act, q = pl.plan_progress(h)
            return got, act, q
    raise AssertionError("requests did not finish")


def same(a, b):
    return (a.status == b.status == 0 and a.best_index == b.best_index and np.array_equal(a.xi_best, b.xi_best)
            and np.array_equal(a.mu, b.mu) and np.array_equal(a.sigma, b.sigma))


def test_served_all_at_once_equals_alone(pl, mode):
    reqs = reqs_of(pl)
    ref = alone_results(pl, reqs)
    h = pl.plan_create(cfg_of(pl, mode))
    tickets = [pl.plan_submit(h, r) for r in reqs]
    got, _, _ = drain(pl, h, tickets)
    for i, t in enumerate(tickets):
        assert same(got[t], ref[i]), i
        assert got[t].latency_s > 0


def test_poll_done_returns_each_ticket_once_and_equals_alone(pl, mode):
    """plan_poll_done hands back every finished request in ticket order,
    each exactly once, with the result (and trajectory) it has alone; a
    capacity smaller than the finished count leaves the rest for the next
    call; plan_poll then knows none of them."""
    reqs = reqs_of(pl)
    ref = alone_results(pl, reqs)
    h = pl.plan_create(cfg_of(pl, mode))
    assert pl.plan_poll_done(h, 4) == []
    tickets = []
    for i, r in enumerate(reqs):
        tickets.append(pl.plan_submit(h, r))
        if i % 3 == 2:
            pl.plan_progress(h)
    got, order = {}, []
    for _ in range(200):
        pl.plan_progress(h)
        batch = pl.plan_poll_done(h, 3)
        assert len(batch) <= 3
        ts = [t for t, _ in batch]
        assert ts == sorted(ts)
        for t, r in batch:
            assert t not in got
            got[t] = r
            order.append(t)
        if len(got) == len(tickets):
            break
    assert sorted(got) == sorted(tickets)
    for i, t in enumerate(tickets):
        assert same(got[t], ref[i]), i
        assert got[t].traj is not None and got[t].traj.shape == (reqs[i].T, 2)
        assert np.array_equal(got[t].traj, ref[i].traj)
    with pytest.raises(pl.PlanError):
        pl.plan_poll(h, tickets[0])
    assert pl.plan_poll_done(h, 8) == []


def test_served_staggered_arrivals_equal_alone(pl, mode):
    reqs = reqs_of(pl)
    ref = alone_results(pl, reqs)
    h = pl.plan_create(cfg_of(pl, mode))
    tickets = []
    for i, r in enumerate(reqs):
        tickets.append(pl.plan_submit(h, r))
        if i % 3 == 2:
            pl.plan_progress(h)  # earlier requests are mid-flight when the next ones arrive
    got, act, q = drain(pl, h, tickets)
    assert act == 0 and q == 0
    for i, t in enumerate(tickets):
        assert same(got[t], ref[i]), i


@pytest.mark.parametrize("ahead", [1, 3])
def test_served_run_ahead_equals_alone(pl, mode, ahead):
    """With iterations enqueued ahead of the GPU (served_run_ahead), arrivals
    during the run still give each request its result alone, bit for bit,
    and every request retires."""
    reqs = reqs_of(pl)
    ref = alone_results(pl, reqs)
    h = pl.plan_create(cfg_of(pl, mode, served_run_ahead=ahead))
    tickets = []
    for i, r in enumerate(reqs):
        tickets.append(pl.plan_submit(h, r))
        if i % 2 == 1:
            pl.plan_progress(h)
    got, act, q = drain(pl, h, tickets)
    assert act == 0 and q == 0
    for i, t in enumerate(tickets):
        assert same(got[t], ref[i]), i
    # the handle is idle again: batch calls work
    assert pl.plan_solve_batch(h, [reqs[0]])[0].status == 0


def test_served_admission_respects_sample_budget(pl, mode):
    reqs = reqs_of(pl)
    ref = alone_results(pl, reqs)
    budget = 800
    h = pl.plan_create(cfg_of(pl, mode, sample_budget=budget, max_requests=3))
    tickets = [pl.plan_submit(h, r) for r in reqs]
    done, ticks = {}, 0
    while len(done) < len(tickets):
        act, q = pl.plan_progress(h)
        ticks += 1
        assert act <= 3
        for t in tickets:
            if t not in done:
                r = pl.plan_poll(h, t)
                if r is not None:
                    done[t] = r
        assert ticks < 400
    for i, t in enumerate(tickets):
        assert same(done[t], ref[i]), i
    # a request larger than the budget is refused at submit
    big = pl.Request(N=1000, T=50, ego=reqs[0].ego, obstacles=reqs[0].obstacles, seed=1)
    with pytest.raises(pl.PlanError) as e:
        pl.plan_submit(h, big)
    assert e.value.status == pl.PLAN_E_NOMEM


def test_served_rejects_bad_requests_and_mixing(pl, mode):
    reqs = reqs_of(pl)
    h = pl.plan_create(cfg_of(pl, mode))
    bad = pl.Request(N=10, T=70, ego=reqs[0].ego, obstacles=reqs[0].obstacles, seed=1)
    with pytest.raises(pl.PlanError) as e:
        pl.plan_submit(h, bad)
    assert e.value.status == pl.PLAN_E_INVALID
    t = pl.plan_submit(h, reqs[0])
    assert pl.plan_poll(h, t) is None
    with pytest.raises(pl.PlanError) as e:
        pl.plan_solve_batch(h, [reqs[1]])
    assert e.value.status == pl.PLAN_E_BUSY
    drain(pl, h, [t])
    assert pl.plan_solve_batch(h, [reqs[1]])[0].status == 0


@pytest.mark.parametrize("T", [100, 200])
def test_instants_per_lane_do_not_change_results(pl, T):
    """A small launch runs one horizon instant per lane, a large one two; the
    sums are formed per 64-instant block in a fixed order, so every request's
    result is bitwise the same either way (here: a 64-sample request alone =
    one per lane, inside a batch of 3 x 4096 samples = two per lane)."""
    M = 10
    cfg = pl.plan_config_init(T_set=[T], M_set=[M], proj_iters=10, upper_iters=2, max_N=4096, max_requests=4)
    h = pl.plan_create(cfg)
    reqs = []
    for i, N in enumerate([4096, 4096, 4096, 64]):
        s = workload.scene(4, 400 + i, M)
        reqs.append(pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, request_id=i))
    big = pl.plan_solve_batch(h, reqs)
    alone = pl.plan_solve_batch(h, [reqs[3]])[0]
    assert same(alone, big[3])
