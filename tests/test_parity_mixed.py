"""GPU parity of the matrix-core lower level against the FP64 oracle, in
both of its forms:
  PLAN_PREC_FP16_SPLIT  FP16 products with FP32 accumulation, every operand
                        split into high and low FP16 halves (reduced
                        precision);
  PLAN_PREC_FP32_MFMA   FP32 products with FP32 accumulation (FP32).

Bar per sample j (parity_common): every trajectory within tol + C m_j of the
oracle at every instant (max over t_k of the Euclidean position error), tol
= 1e-3 m for the FP16 split and 1e-4 m (the FP32 bar) for FP32 on the matrix
cores; residual r within 1e-2 + 1e-3 r + C m_r,j and upper cost c_u within
1e-3 c_u + C m_c,j, with m the oracle's own spread under FP32-sized
perturbations of xi_bar and C = 2 sqrt(K). The measured errors are printed
per case.
"""
import numpy as np
import pytest

from paper_2212_02224_amd import workload
from parity_common import Spread, check_positions

pytestmark = pytest.mark.gpu

POS_TOL = 1e-3
# matrix-core precisions and their position bars
PRECS = [pytest.param(1, 1e-3, id="fp16_split"), pytest.param(2, 1e-4, id="fp32_mfma")]


def pos_err(orc, T, t_f, xa, xb):
    W, _, _ = orc.basis(T, t_f)
    dx = (xa[:, :11] - xb[:, :11]) @ W.T
    dy = (xa[:, 11:] - xb[:, 11:]) @ W.T
    return np.sqrt(dx ** 2 + dy ** 2).max(axis=1)


@pytest.fixture(scope="module")
def pl():
    import paper_2212_02224_amd as pl
    pl.load()
    return pl


def make_handle(pl, T_set, M_set, K, max_N=4096, precision=1):
    cfg = pl.plan_config_init(T_set=T_set, M_set=M_set, proj_iters=K, max_N=max_N, max_requests=1,
                              precision=precision)
    return pl.plan_create(cfg)


def run_case(orc, pl, handle, par, req, p, tag, pos_tol=POS_TOL):
    print(f"[mixed parity] {tag}: N={p.shape[0]} T={req.T} M={req.M} K={par.K} bar {pos_tol:g} m", flush=True)
    sc = orc.Scene(np.asarray(req.ego, float), np.asarray(req.obstacles, float).reshape(-1, 4),
                   req.kappa_road)
    xb_o = orc.step1(par, sc, p)
    xs_o = orc.project(par, sc, xb_o)
    r_o, c_o = orc.residual_cost(par, sc, xs_o)
    xb_g, xs_g, r_g, c_g = pl.plan_lower_solve(handle, req, p)
    e_bar = pos_err(orc, par.T, par.t_f, xb_g, xb_o)
    e_star = pos_err(orc, par.T, par.t_f, xs_g, xs_o)
    sp = Spread(orc, par, sc, xb_o, xs_o)
    dr = np.abs(r_g - r_o)
    dc = np.abs(c_g - c_o)
    print(f"   xi_bar err max {e_bar.max():.2e}  xi* err p50 {np.median(e_star):.2e}  |dr| max {dr.max():.2e} "
          f"|dc|/c max {np.max(dc / np.maximum(np.abs(c_o), 1e-12)):.2e}", flush=True)
    check_positions("xi*", e_star, sp, pos_tol)
    assert e_bar.max() <= 1e-4, e_bar.max()  # Step 1 is FP32 in every mode
    assert np.all(dr <= sp.r_bar(1e-2 + 1e-3 * np.abs(r_o))), dr.max()
    assert np.all(dc <= sp.cu_bar(1e-3 * np.abs(c_o) + 1e-4)), dc.max()
    W, Wd, _ = orc.basis(par.T, par.t_f)
    ego = np.asarray(req.ego, float)
    assert np.allclose(xs_g[:, :11] @ W[0], ego[0], atol=1e-9)
    assert np.allclose(xs_g[:, :11] @ Wd[0], ego[2], atol=1e-9)
    assert np.allclose(xs_g[:, 11:] @ Wd[-1], 0.0, atol=1e-9)
    return e_star, xs_g


@pytest.mark.parametrize("precision,tol", PRECS)
@pytest.mark.parametrize("cfgid", [1, 2])
def test_mixed_lower_parity_configs(orc, pl, cfgid, precision, tol):
    c = workload.CONFIGS[cfgid]
    orc.set_threads(8)
    par = orc.default_params(T=c["T"], M=c["M"], K=c["K"])
    h = make_handle(pl, [c["T"]], [c["M"]], c["K"], precision=precision)
    for idx in range(2):
        s = workload.scene(cfgid, idx, c["M"])
        req = pl.Request(N=c["N"], T=c["T"], ego=s.ego, obstacles=s.obstacles, seed=s.seed)
        p = orc.sample(par, s.seed, 0, c["N"], True)
        run_case(orc, pl, h, par, req, p, f"config {cfgid} scene {idx}", tol)


@pytest.mark.parametrize("precision,tol", PRECS)
def test_mixed_lower_parity_headline_shape(orc, pl, precision, tol):
    """The headline batch's shape (T = 100, M = 20, K = 20), 512 oracle samples
    of each of two of its scenes."""
    c = workload.CONFIGS[5]
    orc.set_threads(8)
    par = orc.default_params(T=c["T"], M=c["M"], K=c["K"])
    h = make_handle(pl, [c["T"]], [c["M"]], c["K"], max_N=512, precision=precision)
    for idx in range(2):
        s = workload.scene(5, idx, c["M"])
        req = pl.Request(N=512, T=c["T"], ego=s.ego, obstacles=s.obstacles, seed=s.seed)
        p = orc.sample(par, s.seed, 0, 512, True)
        run_case(orc, pl, h, par, req, p, f"headline scene {idx}", tol)


@pytest.mark.parametrize("precision,tol", PRECS)
@pytest.mark.parametrize("N,T,M", [(1, 50, 4), (7, 64, 3), (17, 65, 2), (33, 128, 5), (16, 16, 1),
                                   (15, 37, 0), (40, 100, 20), (31, 113, 7)])
def test_mixed_lower_parity_ragged_shapes(orc, pl, N, T, M, precision, tol):
    K = 12
    par = orc.default_params(T=T, M=M, K=K)
    h = make_handle(pl, [T], [M], K, max_N=64, precision=precision)
    s = workload.scene(7, N * 1000 + T * 10 + M, M)
    req = pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed)
    p = orc.sample(par, s.seed, 0, N, True)
    run_case(orc, pl, h, par, req, p, "ragged", tol)


@pytest.mark.parametrize("precision,tol", PRECS)
def test_mixed_lower_general_ego_and_curved_road(orc, pl, precision, tol):
    T, M, K, N = 100, 10, 20, 96
    par = orc.default_params(T=T, M=M, K=K)
    h = make_handle(pl, [T], [M], K, max_N=128, precision=precision)
    s = workload.scene(9, 1, M)
    ego = np.array([12.5, 1.2, 17.0, 0.4, 1.5, -0.6])
    obs = s.obstacles.copy()
    obs[:, 0] += 12.5
    rng = np.random.default_rng(3)
    mu = np.r_[rng.uniform(-3, 3, 4), rng.uniform(12, 24, 4)]
    Sg = np.diag(np.r_[np.full(4, 2.0), np.full(4, 9.0)])
    p = orc.sample(par, 77, 1, N, False, mu, orc.cholesky(Sg))
    for kappa in (0.0, 0.02):
        req = pl.Request(N=N, T=T, ego=ego, obstacles=obs, seed=1, kappa_road=kappa)
        run_case(orc, pl, h, par, req, p, f"kappa {kappa}", tol)


@pytest.mark.parametrize("precision,tol", PRECS)
def test_mixed_agrees_with_fp32_path(orc, pl, precision, tol):
    """Same samples through both kernels: trajectories within the mode's bar
    of each other (and the same draws: Step 1 is shared)."""
    c = workload.CONFIGS[2]
    par = orc.default_params(T=c["T"], M=c["M"], K=c["K"])
    s = workload.scene(2, 3, c["M"])
    req = pl.Request(N=c["N"], T=c["T"], ego=s.ego, obstacles=s.obstacles, seed=s.seed)
    p = orc.sample(par, s.seed, 0, c["N"], True)
    out = {}
    for prec in (0, precision):
        h = make_handle(pl, [c["T"]], [c["M"]], c["K"], precision=prec)
        out[prec] = pl.plan_lower_solve(h, req, p)
    e = pos_err(orc, par.T, par.t_f, out[0][1], out[precision][1])
    print(f"[precision {precision} vs fp32] xi* difference max {e.max():.2e} p99 {np.percentile(e, 99):.2e}",
          flush=True)
    assert np.array_equal(out[0][0], out[precision][0])
    assert e.max() <= tol


@pytest.mark.parametrize("precision,tol", PRECS)
def test_mixed_inactive_constraints_fixed_point(pl, precision, tol):
    T, M, K = 60, 3, 15
    h = make_handle(pl, [T], [M], K, max_N=8, precision=precision)
    obs = np.array([[400.0 + 50 * i, 3.5, 15.0, 0.0] for i in range(M)])
    req = pl.Request(N=2, T=T, ego=[0, 0, 15.0, 0, 0, 0], obstacles=obs, seed=1)
    p = np.array([[0.5, 1.0, 1.0, 0.5, 15, 16, 17, 17.5], [0, 0, 0, 0, 15, 15, 15, 15]])
    xb, xs, r, c = pl.plan_lower_solve(h, req, p)
    assert np.abs(xs - xb).max() < 1e-5
    assert np.all(r == 0.0)


@pytest.mark.parametrize("precision,tol", PRECS)
@pytest.mark.parametrize("cfgid,scene_idx", [(1, 0), (2, 0)])
def test_mixed_plan_parity_per_iteration(orc, pl, cfgid, scene_idx, precision, tol):
    from test_parity_plan import run_config
    run_config(orc, pl, cfgid, scene_idx, precision=precision, tol_scale=10.0 if precision == 1 else 1.0,
               pos_tol=tol)


@pytest.mark.parametrize("precision", [1, 2])
def test_mixed_result_alone_equals_result_in_a_mix(pl, precision):
    """Requests of two horizon lengths (two launch groups) batched together:
    each result is bitwise the one it has alone."""
    cfg = pl.plan_config_init(T_set=[50, 100], M_set=[4, 10, 20], proj_iters=10, upper_iters=3,
                              max_N=512, max_requests=6, precision=precision)
    h = pl.plan_create(cfg)
    reqs = []
    for i, (N, T, M) in enumerate([(64, 50, 4), (300, 100, 10), (17, 100, 20), (512, 50, 10), (1, 100, 4)]):
        s = workload.scene(4, i, M)
        reqs.append(pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, request_id=i))
    mixed = pl.plan_solve_batch(h, reqs)
    for i, r in enumerate(reqs):
        alone = pl.plan_solve_batch(h, [r])[0]
        assert mixed[i].status == 0 and alone.status == 0
        assert np.array_equal(alone.xi_best, mixed[i].xi_best), i
        assert np.array_equal(alone.mu, mixed[i].mu) and np.array_equal(alone.sigma, mixed[i].sigma)


@pytest.mark.parametrize("precision", [1, 2])
def test_mixed_served_equals_alone(pl, precision):
    cfg = dict(T_set=[50, 100], M_set=[4, 10, 20], proj_iters=8, upper_iters=3, max_N=1024, max_requests=4,
               precision=precision)
    mix = [(64, 50, 4), (300, 100, 10), (17, 100, 20), (512, 50, 10), (1, 100, 4), (250, 100, 20)]
    reqs = []
    for i, (N, T, M) in enumerate(mix):
        s = workload.scene(4, 200 + i, M)
        reqs.append(pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, request_id=i))
    h1 = pl.plan_create(pl.plan_config_init(**cfg))
    ref = [pl.plan_solve_batch(h1, [r])[0] for r in reqs]
    h = pl.plan_create(pl.plan_config_init(**cfg))
    tickets = []
    got = {}
    for i, r in enumerate(reqs):
        tickets.append(pl.plan_submit(h, r))
        pl.plan_progress(h)
    for _ in range(100):
        pl.plan_progress(h)
        for t in tickets:
            if t not in got:
                res = pl.plan_poll(h, t)
                if res is not None:
                    got[t] = res
        if len(got) == len(tickets):
            break
    assert len(got) == len(tickets)
    for i, t in enumerate(tickets):
        a, b = got[t], ref[i]
        assert a.status == b.status == 0 and a.best_index == b.best_index, i
        assert np.array_equal(a.xi_best, b.xi_best) and np.array_equal(a.mu, b.mu), i


@pytest.mark.parametrize("precision", [1, 2])
def test_mixed_tiles_per_wave_does_not_change_results(pl, precision):
    """The matrix-core launch shape follows the load: four instant tiles per
    wave for a large launch, two for a middle one, and one tile pair per wave
    over 8-sample workgroups while those fit the chip at once. The sums are
    formed per tile pair in one fixed chain, so every request's result is
    bitwise the same in each (on 256 CUs: the 12k-sample batch runs four,
    request 0 alone, 4096 samples, two, and request 3 alone, 64 samples, one
    pair per wave)."""
    cfg = pl.plan_config_init(T_set=[100], M_set=[10], proj_iters=10, upper_iters=2, max_N=4096, max_requests=4,
                              precision=precision)
    h = pl.plan_create(cfg)
    reqs = []
    for i, N in enumerate([4096, 4096, 4096, 64]):
        s = workload.scene(4, 300 + i, 10)
        reqs.append(pl.Request(N=N, T=100, ego=s.ego, obstacles=s.obstacles, seed=s.seed, request_id=i))
    big = pl.plan_solve_batch(h, reqs)
    for i in (0, 3):
        alone = pl.plan_solve_batch(h, [reqs[i]])[0]
        assert big[i].status == 0 and alone.status == 0
        assert alone.best_index == big[i].best_index, i
        assert np.array_equal(alone.xi_best, big[i].xi_best), i
        assert np.array_equal(alone.mu, big[i].mu) and np.array_equal(alone.sigma, big[i].sigma), i
