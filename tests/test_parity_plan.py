"""GPU parity of Alg. 1 against the FP64 oracle, one upper iteration at a time.

Alg. 1 is a stochastic iteration whose selection steps are discontinuous, so
an FP32 run cannot follow an FP64 run through several iterations: the
weights exp(-(c - c_min)/gamma) amplify the ~1e-7 relative rounding of the
costs into ~1e-3 changes of mu, and the next samples move with them. Each
iteration is therefore checked teacher-forced from the oracle: the GPU gets
the oracle's distribution before iteration l (and the same sample-stream
index), and must reproduce
  * the samples p (FP32 Box-Muller vs FP64: |dp| <= 2e-5 + 1e-6 |p|),
  * r and c_u of every sample, each within the lower-level bar plus C times
    the oracle's own spread at that sample (parity_common; at most a tenth
    of the samples flagged, a quarter on the fixed grid),
  * the ConstraintEliteSet and EliteSet, up to swaps of members whose oracle
    keys are within the two members' key tolerances of each other (near
    ties; counted and reported),
  * mu and Sigma after the update, within the bound that the cost tolerance
    implies through the weights (derived below), and the returned best
    sample (position bar plus C times its spread), at every iteration: the
    expected update is the oracle's over the EliteSet the GPU took, which is
    the oracle's own set or, after near-tie swaps, another resolution of the
    ties checked member by member against the oracle's keys.
Inputs flow only from the oracle to the GPU, never back.
"""
import numpy as np
import pytest

from paper_2212_02224_amd import workload
from parity_common import Spread

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pl():
    import paper_2212_02224_amd as pl
    pl.load()
    return pl


def r_tol(r, scale=1.0):
    return scale * (1e-3 + 1e-4 * np.abs(r))


def c_tol(c, scale=1.0):
    return scale * (1e-4 * np.abs(c) + 1e-6)


def set_check(name, gpu_idx, orc_idx, orc_key, tol):
    """Sets equal up to swaps of near-tied members: every member of the
    symmetric difference has an oracle key within its own tolerance plus the
    largest tolerance among the swapped members and the boundary member, of
    the set's boundary key (tol: per-sample key tolerance). Returns the swap
    count."""
    g, o = set(map(int, gpu_idx)), set(map(int, orc_idx))
    if g == o:
        return 0
    ol = list(o)
    jb = ol[int(np.argmax(orc_key[ol]))]
    boundary = orc_key[jb]
    diff = g.symmetric_difference(o)
    t_pair = max(tol[jb], max(tol[j] for j in diff))
    for j in diff:
        assert abs(orc_key[j] - boundary) <= 2 * (tol[j] + t_pair), \
            f"{name}: sample {j} key {orc_key[j]} (tol {tol[j]:.2e}) not near the boundary {boundary}"
    return len(diff) // 2


def run_config(orc, pl, cfgid, scene_idx, precision=0, tol_scale=1.0, pos_tol=1e-4, behaviour=0, sampler=0,
               L=None, road=False, decoder_seed=None, p0_tol=None, method=None, max_flagged=None):
    c = workload.CONFIGS[cfgid]
    N, T, M, K = c["N"], c["T"], c["M"], c["K"]
    L = c["L"] if L is None else L
    orc.set_threads(8)
    method = method or {}  # method parameters set alike on both sides
    par = orc.default_params(T=T, M=M, K=K, L=L, behaviour=behaviour, sampler=sampler, **method)
    s = workload.scene(cfgid, scene_idx, M)
    rk = {}
    if road:
        rp, rx0, rdx = workload.curved_road(cfgid, scene_idx)
        rk = dict(road=rp, road_x0=rx0, road_dx=rdx)
    sc = orc.Scene(s.ego, s.obstacles, **rk)
    dec, ok_kw, p0 = None, {}, None
    if decoder_seed is not None:
        # the decoder sampler: the oracle plans from its own FP64 decoder samples
        sampler = pl.PLAN_SAMPLER_DECODER
        dec = workload.decoder_weights(decoder_seed, behaviour)
        ok_kw = dict(observation=workload.observation(s, **rk))
        p0 = orc.decoder_sample(par, dec, ok_kw["observation"], s.seed, N)
    ref = orc.plan(par, sc, s.seed, N, trace=True, p0=p0)
    tr = ref.trace
    n, q = orc.elite_sizes(par, N)
    cfg = pl.plan_config_init(T_set=[T], M_set=[M], proj_iters=K, upper_iters=1, max_N=N,
                              max_requests=1, trace=1, precision=precision, behaviour=behaviour,
                              sampler=sampler, **method)
    h = pl.plan_create(cfg)
    if dec is not None:
        pl.plan_set_decoder(h, dec)
    swaps_total, compared = 0, 0
    if max_flagged is None:
        # the fixed grid's lane-centred samples ride along neighbours' centre
        # lines, where the obstacle step's direction flips (about 15-18% of
        # its 1000 samples flagged, measured on the oracle alone)
        max_flagged = 0.25 if sampler == 1 else 0.1
    rt = lambda r: r_tol(r, tol_scale)  # noqa: E731
    ct = lambda c: c_tol(c, tol_scale)  # noqa: E731
    for l in range(L):
        print(f"[plan parity] config {cfgid} scene {scene_idx} precision {precision} behaviour {behaviour} "
              f"sampler {sampler} road {road} iteration {l}", flush=True)
        kw = {}
        if l > 0:
            kw = dict(mu0=tr["mu"][l - 1], sigma0=tr["Sigma"][l - 1])
        req = pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, first_iter=l, **rk, **ok_kw,
                         **kw)
        res = pl.plan_solve_batch(h, [req])[0]
        assert res.status == 0, pl.plan_last_error(h)
        g = pl.plan_get_trace(h, 0, N, n, q)
        # samples
        dp = np.abs(g["p"][0] - tr["p"][l])
        if l == 0 and p0_tol is not None:
            assert np.all(dp <= p0_tol(tr["p"][l])), dp.max()
        else:
            assert np.all(dp <= 2e-5 + 1e-6 * np.abs(tr["p"][l])), dp.max()
        # residuals and costs, each within its bar plus C times the oracle's spread
        sp = Spread(orc, par, sc, tr["xi_bar"][l], tr["xi_star"][l], p=tr["p"][l])
        fl = sp.flagged(pos_tol)
        dr = np.abs(g["r"][0] - tr["r"][l])
        dc = np.abs(g["cu"][0] - tr["cu"][l])
        tol_r = sp.r_bar(rt(tr["r"][l]))
        tol_c = sp.cu_bar(ct(tr["cu"][l]))
        print(f"   |dp| {dp.max():.2e} |dr| {dr.max():.2e} |dc|/c {np.max(dc / tr['cu'][l]):.2e}; flagged "
              f"{int(fl.sum())} of {N} (|dr| there {dr[fl].max() if fl.any() else 0:.2e}, |dc| "
              f"{dc[fl].max() if fl.any() else 0:.2e})", flush=True)
        assert np.all(dr <= tol_r), dr.max()
        assert np.all(dc <= tol_c), dc.max()
        assert fl.sum() <= max(1, int(max_flagged * N)), fl.mean()
        # elite sets
        sw = set_check("ConstraintEliteSet", g["ces"][0], tr["ces"][l], tr["r"][l], tol_r)
        c_full = tr["cu"][l] + tr["r"][l]
        tol_full = tol_r + tol_c
        if sw == 0:
            sw += set_check("EliteSet", g["es"][0], tr["es"][l], c_full, tol_full)
        else:
            # the EliteSets are drawn from different ConstraintEliteSets: a
            # member common to both that fewer than q members of either
            # ConstraintEliteSet could undercut (within the two tolerances)
            # must be in both EliteSets
            common = np.intersect1d(g["ces"][0], tr["ces"][l])
            gc = np.union1d(g["ces"][0], tr["ces"][l])
            sure = [int(j) for j in common
                    if np.sum((c_full[gc] - tol_full[gc] <= c_full[j] + tol_full[j]) & (gc != j)) < q]
            assert set(sure) <= set(map(int, g["es"][0])) and set(sure) <= set(map(int, tr["es"][l]))
            # and the GPU's EliteSet is, by the oracle's costs, the q lowest of
            # the GPU's ConstraintEliteSet up to near ties
            gces = np.asarray(g["ces"][0], np.int64)
            alt = gces[np.lexsort((gces, c_full[gces]))][:q]
            set_check("EliteSet of the GPU's ConstraintEliteSet", g["es"][0], alt, c_full, tol_full)
            print(f"   ConstraintEliteSet differs by {sw} near-tied swap(s): EliteSets compared on "
                  f"{len(sure)} common members that cannot be undercut", flush=True)
        swaps_total += sw
        # mu, Sigma after the update, over the EliteSet the GPU took. With no
        # swap that is the oracle's own set. With near-tie swaps it is another
        # resolution of the ties, each member of which was checked above
        # against the oracle's keys; the oracle's update over that set (its
        # own samples, costs and prior) is then the expected value, since the
        # update is a function of the set alone (eqs. s_formula, mean_update,
        # cov_update).
        es = np.asarray(g["es"][0], np.int64)
        es = es[np.lexsort((es, c_full[es]))]
        if l > 0:
            prior = (tr["mu"][l - 1], tr["Sigma"][l - 1])
        elif p0 is not None:
            prior = orc.sample_moments(p0)
        else:
            prior = orc.initial_moments(par)
        mu_ref, S_ref = orc.update(par, prior[0], prior[1], tr["p"][l], es, c_full[es])
        if sw == 0:
            # the prior is the one the oracle's plan used: its update over its
            # own set is the trace's, to rounding
            assert np.allclose(mu_ref, tr["mu"][l], rtol=1e-12, atol=1e-12)
            assert np.allclose(S_ref, tr["Sigma"][l], rtol=1e-10, atol=1e-12)
        # a cost error dc changes each weight by a factor exp(+-2 dc / gamma);
        # the weighted mean moves by at most eta (e^{2 dc/gamma} - 1)
        # max_j |p_j - m|, the covariance by the same factor times
        # max_j |p_j - m|^2 (plus FP32 sample rounding)
        dcm = np.max(dc[es] + dr[es])
        w = np.expm1(2 * dcm / par.gamma)
        spread = np.abs(tr["p"][l][es] - mu_ref).max()
        tol_mu = par.eta * w * spread + 5e-5 * tol_scale * (1 + np.abs(mu_ref))
        tol_S = par.eta * (w * spread ** 2 + 2 * spread * tol_mu.max()) + 1e-4 * tol_scale * (1 + np.abs(S_ref))
        assert np.all(np.abs(g["mu"][0] - mu_ref) <= tol_mu), np.abs(g["mu"][0] - mu_ref).max()
        assert np.all(np.abs(g["sigma"][0] - S_ref) <= tol_S), np.abs(g["sigma"][0] - S_ref).max()
        # returned sample: the lowest (c, j) of that EliteSet, up to a near tie
        # at the top; its trajectory against the oracle's projection of it
        jb = res.best_index
        assert jb in set(map(int, es)), jb
        assert jb == es[0] or abs(c_full[jb] - c_full[es[0]]) <= 2 * (tol_full[jb] + tol_full[es[0]]), \
            (jb, int(es[0]))
        W, _, _ = orc.basis(T, par.t_f)
        e = np.sqrt((((res.xi_best[:11] - tr["xi_star"][l][jb][:11]) @ W.T) ** 2 +
                     ((res.xi_best[11:] - tr["xi_star"][l][jb][11:]) @ W.T) ** 2)).max()
        assert e <= sp.pos_bar(pos_tol)[jb], (e, sp.pos_bar(pos_tol)[jb])
        if sw:
            print(f"   {sw} near-tie swap(s): update compared over the EliteSet the GPU took", flush=True)
        compared += 1
    assert compared >= 1, "no iteration compared mu, Sigma and the returned sample"
    print(f"   near-tie swaps over {L} iterations: {swaps_total}", flush=True)
    return swaps_total


@pytest.mark.parametrize("cfgid,scene_idx", [(1, 0), (1, 1), (2, 0)])
def test_plan_parity_per_iteration(orc, pl, cfgid, scene_idx):
    run_config(orc, pl, cfgid, scene_idx)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_plan_parity_mostly_infeasible(orc, pl, precision):
    """a_max = 1 m/s^2 leaves 10-20 of the 1000 samples feasible (r = 0), so
    the ConstraintEliteSet of 150 is not a run of equal smallest keys: the
    selection kernel takes its radix passes over the residual keys and the
    position-ordered scan of the boundary bin."""
    kw = dict(tol_scale=10.0, pos_tol=1e-3) if precision == 1 else {}
    run_config(orc, pl, 2, 0, precision=precision, L=3, method=dict(a_max=1.0), **kw)


def test_plan_parity_large_elite_sets(orc, pl):
    """One request of the 1024-request workload's size, N = 4096, T = 100,
    M = 20, two iterations: ConstraintEliteSet of 614 and EliteSet of 205
    members, more than one per thread of the selection workgroup, so the
    EliteSet takes the radix select, its rows the batched loads, and the
    update sums about 51 elites per wave."""
    run_config(orc, pl, 5, 0, L=2)


def test_full_plan_consistency_and_determinism(orc, pl):
    """Full L-iteration plan on the GPU: the first iteration equals the
    teacher-forced one bit for bit, the trace is self-consistent, and two runs
    are identical."""
    c = workload.CONFIGS[1]
    N, T, M, L, K = c["N"], c["T"], c["M"], c["L"], c["K"]
    n, q = orc.elite_sizes(orc.default_params(), N)
    cfg = pl.plan_config_init(T_set=[T], M_set=[M], proj_iters=K, upper_iters=L, max_N=N,
                              max_requests=1, trace=1)
    h = pl.plan_create(cfg)
    s = workload.scene(1, 3, M)
    req = pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed)
    a = pl.plan_solve_batch(h, [req])[0]
    ga = pl.plan_get_trace(h, 0, N, n, q)
    b = pl.plan_solve_batch(h, [req])[0]
    gb = pl.plan_get_trace(h, 0, N, n, q)
    assert a.status == 0 and a.iterations == L
    for k in ga:
        assert np.array_equal(ga[k], gb[k]), k
    assert np.array_equal(a.xi_best, b.xi_best)
    for l in range(L):
        assert set(ga["es"][l]) <= set(ga["ces"][l])
        assert np.all(np.linalg.eigvalsh(ga["sigma"][l]) > -1e-12)
        assert np.array_equal(ga["sigma"][l], ga["sigma"][l].T)  # exactly symmetric as formed
        # ConstraintEliteSet holds the n lowest residuals of the GPU's own r
        kth = np.sort(ga["r"][l])[n - 1]
        assert np.all(ga["r"][l][ga["ces"][l]] <= kth)
    es = ga["es"][L - 1]
    c_es = (ga["cu"][L - 1][es] + ga["r"][L - 1][es]).astype(np.float32)
    assert a.best_index == es[np.lexsort((es, c_es))[0]]
    assert np.isclose(a.cost_upper, ga["cu"][L - 1][a.best_index])
    cfg1 = pl.plan_config_init(T_set=[T], M_set=[M], proj_iters=K, upper_iters=1, max_N=N,
                               max_requests=1, trace=1)
    h1 = pl.plan_create(cfg1)
    pl.plan_solve_batch(h1, [req])
    g1 = pl.plan_get_trace(h1, 0, N, n, q)
    for k in ("p", "r", "cu", "ces", "es", "mu", "sigma"):
        assert np.array_equal(g1[k][0], ga[k][0]), k


def test_result_alone_equals_result_in_a_mix(pl):
    """Each request's result is the same alone and batched with others of
    other sizes (bitwise: requests share no arithmetic)."""
    cfg = pl.plan_config_init(T_set=[50, 100], M_set=[4, 10, 20], proj_iters=10, upper_iters=3,
                              max_N=512, max_requests=6)
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
        assert alone.best_index == mixed[i].best_index


def test_bad_request_fails_alone(pl):
    cfg = pl.plan_config_init(T_set=[50], M_set=[4], proj_iters=5, upper_iters=2, max_N=64, max_requests=3)
    h = pl.plan_create(cfg)
    s = workload.scene(4, 9, 4)
    good = pl.Request(N=32, T=50, ego=s.ego, obstacles=s.obstacles, seed=1)
    bad_T = pl.Request(N=32, T=60, ego=s.ego, obstacles=s.obstacles, seed=1)
    bad_nan = pl.Request(N=32, T=50, ego=[np.nan, 0, 10, 0, 0, 0], obstacles=s.obstacles, seed=1)
    out = pl.plan_solve_batch(h, [bad_T, good, bad_nan])
    assert out[0].status == pl.PLAN_E_INVALID and out[2].status == pl.PLAN_E_INVALID
    assert out[1].status == 0
    alone = pl.plan_solve_batch(h, [good])[0]
    assert np.array_equal(alone.xi_best, out[1].xi_best)
    # sizes outside [1, max_N] fail alone too; an empty batch is a no-op
    out = pl.plan_solve_batch(h, [pl.Request(N=0, T=50, ego=s.ego, obstacles=s.obstacles, seed=1), good,
                                  pl.Request(N=65, T=50, ego=s.ego, obstacles=s.obstacles, seed=1)])
    assert out[0].status == pl.PLAN_E_INVALID and out[2].status == pl.PLAN_E_INVALID
    assert out[1].status == 0 and np.array_equal(out[1].xi_best, alone.xi_best)
    assert pl.plan_solve_batch(h, []) == []
    # one sample: it is its own elite sets and the returned trajectory
    one = pl.plan_solve_batch(h, [pl.Request(N=1, T=50, ego=s.ego, obstacles=s.obstacles, seed=3)])[0]
    assert one.status == 0 and one.best_index == 0 and np.all(np.isfinite(one.xi_best))


def test_session_warm_start(pl):
    """A second request of a session starts from the distribution the first
    one left on the device."""
    cfg = pl.plan_config_init(T_set=[50], M_set=[4], proj_iters=5, upper_iters=2, max_N=64, max_requests=2)
    h = pl.plan_create(cfg)
    s = workload.scene(4, 11, 4)
    r1 = pl.Request(N=64, T=50, ego=s.ego, obstacles=s.obstacles, seed=5, session_id=77)
    a = pl.plan_solve_batch(h, [r1])[0]
    assert a.status == 0 and not (a.flags & pl.PLAN_F_WARM)
    r2 = pl.Request(N=64, T=50, ego=s.ego, obstacles=s.obstacles, seed=6, session_id=77)
    b = pl.plan_solve_batch(h, [r2])[0]
    assert b.flags & pl.PLAN_F_WARM
    # same as an explicit warm start with the first result's distribution
    r3 = pl.Request(N=64, T=50, ego=s.ego, obstacles=s.obstacles, seed=6, mu0=a.mu, sigma0=a.sigma)
    c = pl.plan_solve_batch(h, [r3])[0]
    assert np.array_equal(b.xi_best, c.xi_best) and np.array_equal(b.mu, c.mu)
