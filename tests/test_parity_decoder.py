"""GPU parity of the decoder sampler (the learned initial sampler of Sec.
III-D at inference: the App. A decoder MLP applied to [o, z_j], z_j ~ N(0, I)
from the samplers' Philox block) against the FP64 oracle, with random
weights of the App. A sizes: the samples of ragged, maximum-size and
multi-chunk batches, goal positions, Alg. 1 one iteration at a time from
the decoder's samples, and batch / served invariance and the error paths.

Tolerance of the samples: blocks 2-5 run as FP16 high/low products with
FP32 accumulation (about 22 significant bits per product) and every
activation is split the same way; block 1 and the output layer are FP32.
That is FP32 accuracy: rounding every activation of these 1024-wide layers
to FP32 already moves p by about 1e-6 of its size (a plain FP32 forward
pass of the same network and inputs, BatchNorm folded or not, is off by up
to 1.7e-5 at |p| about 20; a CPU emulation of the split arithmetic by
1.6e-5). The bar is twice that level with margin: 1e-5 + 2e-6 (1 + P_a),
P_a the largest |p_a| of the batch for input a."""
import numpy as np
import pytest

from paper_2212_02224_amd import workload
from test_parity_plan import run_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pl():
    import paper_2212_02224_amd as pl
    pl.load()
    return pl


def p_tol(p):
    """Bar of each sample input: the rounding of an output scales with the
    size of that output's terms, i.e. with the output's magnitude over the
    batch, not with one sample's value (a speed set-point drawn near 0 is
    still a sum of terms of size 15)."""
    return 1e-5 + 2e-6 * (1.0 + np.abs(p).max(axis=0, keepdims=True))


def decoder_handle(pl, dec, N_max, n_req, behaviour=0, precision=0, T_set=(50, 100), M_set=(4, 10, 20),
                   upper_iters=1, trace=1):
    cfg = pl.plan_config_init(T_set=list(T_set), M_set=list(M_set), proj_iters=10, upper_iters=upper_iters,
                              max_N=N_max, max_requests=n_req, trace=trace, precision=precision,
                              behaviour=behaviour, sampler=pl.PLAN_SAMPLER_DECODER)
    h = pl.plan_create(cfg)
    pl.plan_set_decoder(h, dec)
    return h


def decoder_samples(orc, pl, h, reqs, dec, behaviour=0):
    """GPU samples of iteration 0 (trace) and the oracle's, per request."""
    res = pl.plan_solve_batch(h, reqs)
    out = []
    par = orc.default_params(behaviour=behaviour)
    for i, r in enumerate(reqs):
        assert res[i].status == 0, pl.plan_last_error(h)
        n, q = pl.elite_sizes(h.cfg, r.N)
        g = pl.plan_get_trace(h, i, r.N, n, q)["p"][0]
        o = orc.decoder_sample(par, dec, r.observation, r.seed, r.N)
        out.append((g, o))
    return out


@pytest.mark.parametrize("N,T,M", [(1000, 100, 10), (37, 50, 4), (4096, 100, 20), (1, 50, 4)])
def test_decoder_samples_match_oracle(orc, pl, N, T, M):
    dec = workload.decoder_weights(0)
    h = decoder_handle(pl, dec, max(N, 16), 1)
    s = workload.scene(2, 11, M)
    req = pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, observation=workload.observation(s))
    print(f"[decoder parity] N={N} T={T} M={M}", flush=True)
    (g, o), = decoder_samples(orc, pl, h, [req], dec)
    err = np.abs(g - o)
    print(f"   max |dp| {err.max():.2e} (per input {np.round(err.max(axis=0), 7)}); |p| up to "
          f"{np.abs(o).max():.1f}", flush=True)
    assert np.all(err <= p_tol(o))
    if N > 1:
        assert np.std(o[:, 4]) > 0.3  # the latent spreads the samples


def test_decoder_chunks_and_segments(orc, pl):
    """Five requests of 4096 samples (20480 rows: two chunks of decoder
    rows, one request split across them) and a small one, with different
    observations and seeds: every sample matches the oracle."""
    dec = workload.decoder_weights(5)
    h = decoder_handle(pl, dec, 4096, 6)
    reqs = []
    for i, N in enumerate([4096, 4096, 4096, 4096, 4096, 123]):
        s = workload.scene(4, 20 + i, 10)
        reqs.append(pl.Request(N=N, T=100, ego=s.ego, obstacles=s.obstacles, seed=s.seed,
                               observation=workload.observation(s)))
    print("[decoder parity] 6 requests, 20603 rows", flush=True)
    worst = 0.0
    for g, o in decoder_samples(orc, pl, h, reqs, dec):
        err = np.abs(g - o)
        worst = max(worst, err.max())
        assert np.all(err <= p_tol(o))
    print(f"   max |dp| {worst:.2e}", flush=True)


def test_decoder_goal_positions(orc, pl):
    dec = workload.decoder_weights(2, behaviour=1)
    h = decoder_handle(pl, dec, 512, 1, behaviour=1)
    s = workload.scene(2, 12, 10)
    req = pl.Request(N=512, T=100, ego=s.ego, obstacles=s.obstacles, seed=s.seed,
                     observation=workload.observation(s))
    (g, o), = decoder_samples(orc, pl, h, [req], dec, behaviour=1)
    assert np.all(g[:, 2:] == 0)
    err = np.abs(g - o)
    print(f"[decoder goals] max |dp| {err.max():.2e}; x_f - x0 in [{o[:, 0].min():.1f}, {o[:, 0].max():.1f}]",
          flush=True)
    assert np.all(err <= p_tol(o))


@pytest.mark.parametrize("cfgid,scene_idx", [(1, 0), (2, 0)])
def test_decoder_plan_parity_per_iteration(orc, pl, cfgid, scene_idx):
    run_config(orc, pl, cfgid, scene_idx, decoder_seed=0, p0_tol=p_tol)


def test_decoder_plan_parity_fp16_split(orc, pl):
    run_config(orc, pl, 1, 1, precision=1, tol_scale=10.0, pos_tol=1e-3, decoder_seed=1, p0_tol=p_tol)


def test_decoder_goal_plan_parity(orc, pl):
    run_config(orc, pl, 1, 2, behaviour=1, decoder_seed=2, p0_tol=p_tol)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_decoder_batch_and_served_equal_alone(pl, precision):
    """Decoder rows of several requests share the decoder launches (in a
    batch, and in the served mode next to requests mid-flight); each
    request's plan is the one it gets alone, bit for bit."""
    dec = workload.decoder_weights(3)
    mix = [(64, 50, 4), (300, 100, 10), (17, 100, 20), (512, 50, 10), (250, 100, 20)]
    reqs = []
    for i, (N, T, M) in enumerate(mix):
        s = workload.scene(4, 40 + i, M)
        reqs.append(pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, request_id=i,
                               observation=workload.observation(s)))

    def handle():
        return decoder_handle(pl, dec, 1024, 8, precision=precision, upper_iters=3, trace=0)
    h1 = handle()
    alone = [pl.plan_solve_batch(h1, [r])[0] for r in reqs]
    batch = pl.plan_solve_batch(handle(), reqs)
    h3 = handle()
    tickets = []
    for i, r in enumerate(reqs):
        tickets.append(pl.plan_submit(h3, r))
        if i % 2 == 1:
            pl.plan_progress(h3)
    got = {}
    for _ in range(100):
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


def test_decoder_error_paths(pl):
    dec = workload.decoder_weights(0)
    s = workload.scene(2, 13, 4)
    base = dict(N=64, T=50, ego=s.ego, obstacles=s.obstacles, seed=s.seed)
    cfg = pl.plan_config_init(T_set=[50], M_set=[4], max_N=64, max_requests=1, sampler=pl.PLAN_SAMPLER_DECODER)
    h = pl.plan_create(cfg)
    obs = workload.observation(s)
    # weights not loaded yet
    assert pl.plan_solve_batch(h, [pl.Request(**base, observation=obs)])[0].status == pl.PLAN_E_INVALID
    bad = workload.decoder_weights(0)
    bad.var[2] = -np.ones_like(bad.var[2])
    with pytest.raises(pl.PlanError):
        pl.plan_set_decoder(h, bad)
    bad = workload.decoder_weights(0)
    bad.W[3] = bad.W[3].copy()
    bad.W[3][5, 7] = np.nan
    with pytest.raises(pl.PlanError):
        pl.plan_set_decoder(h, bad)
    pl.plan_set_decoder(h, dec)
    # an observation is required and must be finite
    assert pl.plan_solve_batch(h, [pl.Request(**base)])[0].status == pl.PLAN_E_INVALID
    nan_obs = obs.copy()
    nan_obs[10] = np.inf
    assert pl.plan_solve_batch(h, [pl.Request(**base, observation=nan_obs)])[0].status == pl.PLAN_E_INVALID
    assert pl.plan_solve_batch(h, [pl.Request(**base, observation=obs)])[0].status == 0
    # the closed loop has no per-cycle observation
    with pytest.raises(pl.PlanError) as e:
        pl.plan_mpc_run(h, [pl.Request(**base, observation=obs)], 2, 5)
    assert e.value.status == pl.PLAN_E_UNSUPPORTED
    # weights only for a handle with the decoder sampler
    h2 = pl.plan_create(pl.plan_config_init(T_set=[50], M_set=[4], max_N=64, max_requests=1))
    with pytest.raises(pl.PlanError):
        pl.plan_set_decoder(h2, dec)


def test_decoder_activation_overflow_fails_the_request(pl):
    """Weights that drive a hidden activation beyond the FP16 range make the
    request fail (status PLAN_E_INVALID), not return a plan."""
    dec = workload.decoder_weights(0)
    dec.b[1] = dec.b[1] + 1e6  # block 2 pre-activations about 1e6 > 65504
    h = decoder_handle(pl, dec, 64, 1, trace=0)
    s = workload.scene(2, 14, 4)
    r = pl.plan_solve_batch(h, [pl.Request(N=64, T=50, ego=s.ego, obstacles=s.obstacles, seed=s.seed,
                                           observation=workload.observation(s))])[0]
    assert r.status == pl.PLAN_E_INVALID
