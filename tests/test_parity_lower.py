"""GPU parity of the lower level (Alg. 1 Steps 1-2 + residual/cost) against
the FP64 oracle, teacher-forced: both sides get the oracle's samples p.

Bar (FP32 path), per sample j (parity_common): every trajectory within
1e-4 m + C m_j of the oracle at every instant of the horizon (max over t_k
of the Euclidean position error), residual r within 1e-3 + 1e-4 r + C m_r,j
and upper cost c_u within 1e-4 c_u + C m_c,j, where m is the oracle's own
spread under FP32-sized perturbations of xi_bar and C = 2 sqrt(K). Step 1
(xi_bar) is held to 1e-4 m flat. The positions compared are both evaluated
in FP64 from the returned coefficients. At most a tenth of a case may be
flagged (C m_j > 1e-4 m).
"""
import numpy as np
import pytest

from paper_2212_02224_amd import workload
from parity_common import Spread, check_positions

pytestmark = pytest.mark.gpu

POS_TOL = 1e-4


def pos_err(orc, T, t_f, xa, xb):
    W, _, _ = orc.basis(T, t_f)
    dx = (xa[:, :11] - xb[:, :11]) @ W.T
    dy = (xa[:, 11:] - xb[:, 11:]) @ W.T
    return np.sqrt(dx ** 2 + dy ** 2).max(axis=1)


def run_case(orc, pl, handle, par, req, p, tag):
    print(f"[lower parity] {tag}: N={p.shape[0]} T={req.T} M={req.M} K={par.K}", flush=True)
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
    print(f"   xi_bar err max {e_bar.max():.2e}  |dr| max {dr.max():.2e}", flush=True)
    check_positions("xi*", e_star, sp, POS_TOL)
    assert e_bar.max() <= POS_TOL, e_bar.max()
    assert np.all(dr <= sp.r_bar(1e-3 + 1e-4 * np.abs(r_o))), dr.max()
    assert np.all(dc <= sp.cu_bar(1e-4 * np.abs(c_o) + 1e-6)), dc.max()
    # boundary conditions hold exactly in the returned coefficients
    W, Wd, Wdd = orc.basis(par.T, par.t_f)
    ego = np.asarray(req.ego, float)
    assert np.allclose(xs_g[:, :11] @ W[0], ego[0], atol=1e-9)
    assert np.allclose(xs_g[:, :11] @ Wd[0], ego[2], atol=1e-9)
    assert np.allclose(xs_g[:, 11:] @ Wd[-1], 0.0, atol=1e-9)
    return e_star


@pytest.fixture(scope="module")
def pl():
    import paper_2212_02224_amd as pl
    pl.load()
    return pl


def make_handle(pl, T_set, M_set, K, max_N=4096):
    cfg = pl.plan_config_init(T_set=T_set, M_set=M_set, proj_iters=K, max_N=max_N, max_requests=1)
    return pl.plan_create(cfg)


@pytest.mark.parametrize("cfgid", [1, 2])
def test_lower_parity_configs(orc, pl, cfgid):
    c = workload.CONFIGS[cfgid]
    orc.set_threads(8)
    par = orc.default_params(T=c["T"], M=c["M"], K=c["K"])
    h = make_handle(pl, [c["T"]], [c["M"]], c["K"])
    for idx in range(2):
        s = workload.scene(cfgid, idx, c["M"])
        req = pl.Request(N=c["N"], T=c["T"], ego=s.ego, obstacles=s.obstacles, seed=s.seed)
        p = orc.sample(par, s.seed, 0, c["N"], True)
        e = run_case(orc, pl, h, par, req, p, f"config {cfgid} scene {idx}")
        # the scene must exercise the projection, or the test proves little
        assert np.isfinite(e).all()


@pytest.mark.parametrize("N,T,M", [(1, 50, 4), (7, 64, 3), (9, 65, 2), (33, 128, 5), (5, 200, 6),
                                   (17, 100, 0), (40, 100, 20), (3, 16, 1)])
def test_lower_parity_ragged_shapes(orc, pl, N, T, M):
    K = 12
    par = orc.default_params(T=T, M=M, K=K)
    h = make_handle(pl, [T], [M], K, max_N=64)
    s = workload.scene(7, N * 1000 + T * 10 + M, M)
    req = pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed)
    p = orc.sample(par, s.seed, 0, N, True)
    run_case(orc, pl, h, par, req, p, "ragged")


@pytest.mark.parametrize("T,M", [(100, 10), (200, 6)])
def test_lower_parity_two_instants_per_lane(orc, pl, T, M):
    """2048 samples fill a launch enough for two horizon instants per lane."""
    N, K = 2048, 12
    par = orc.default_params(T=T, M=M, K=K)
    h = make_handle(pl, [T], [M], K, max_N=N)
    s = workload.scene(7, 9000 + T, M)
    req = pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed)
    p = orc.sample(par, s.seed, 0, N, True)
    run_case(orc, pl, h, par, req, p, "two instants per lane")


def test_lower_parity_general_ego_and_curved_road(orc, pl):
    """Nonzero x0, lateral velocity and accelerations, curved road (the
    centripetal clip of step clip_d_v), Gaussian samples."""
    T, M, K, N = 100, 10, 20, 96
    par = orc.default_params(T=T, M=M, K=K)
    h = make_handle(pl, [T], [M], K, max_N=128)
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
        run_case(orc, pl, h, par, req, p, f"kappa {kappa}")


def test_lower_inactive_constraints_fixed_point(orc, pl):
    """Far neighbours and gentle set-points: no constraint is active, so the
    projection returns xi_bar."""
    T, M, K = 60, 3, 15
    h = make_handle(pl, [T], [M], K, max_N=8)
    obs = np.array([[400.0 + 50 * i, 3.5, 15.0, 0.0] for i in range(M)])
    req = pl.Request(N=2, T=T, ego=[0, 0, 15.0, 0, 0, 0], obstacles=obs, seed=1)
    p = np.array([[0.5, 1.0, 1.0, 0.5, 15, 16, 17, 17.5], [0, 0, 0, 0, 15, 15, 15, 15]])
    xb, xs, r, c = pl.plan_lower_solve(h, req, p)
    assert np.abs(xs - xb).max() < 1e-5
    assert np.all(r == 0.0)
