"""Pins of every step of the oracle's Alg. 2, from its per-step record.

The matrices of the projection problem are built here from the basis alone
(itself pinned by exact polynomial reproduction in test_oracle_basis_step1):
F = blkdiag([W (once per neighbour); Wd; Wdd]) per axis (eq. for F), the lane
rows G = [W; -W] on c_y (eq. lane_reform) and the boundary rows A_eq (eqs.
boundary_cond_initial, final_boundary). The record's targets h, slack s,
lane bound e and multipliers lambda are then checked against properties the
paper's equations fix, with nothing taken from the oracle's own matrices:

  * the first xi-update (lambda^0 = 0, targets from the target pass at
    xi_bar) equals an independent equality-constrained least-squares solve
    of eq. split_xy by a null-space method (SVD of A_eq, then lstsq);
  * every xi-update k = 1..K satisfies the stationarity condition of eq.
    aug_lag in xi with lambda^(k-1), h^(k-1), e^(k-1), s^(k-1), up to a
    multiple of the boundary rows, and the boundary rows themselves;
  * the recorded targets are the target pass (steps split_alpha_o ..
    update_slack) at the recorded iterate;
  * at a fixed point of the iteration the multiplier step of eq.
    update_lagrange leaves the penalty gradient F^T(F xi - h) + G^T(G xi - e
    + s) zero, so the xi-step's stationarity gives lambda* = xi* - xi_bar up
    to a multiple of the boundary rows, whatever the step length.

The multiplier step's length (the printed rho/2, reading Z15) is the one part
of Alg. 2 no property here fixes: any positive length has the same fixed
points, so its finite-K values stay "parity unpinned". The scene is chosen
so that neighbours, the lane rows and the speed and acceleration clips are
all active, and rho != 1 so that a misplaced rho shows.
"""
import numpy as np
import pytest


def problem_matrices(orc, par, ego):
    W, Wd, Wdd = orc.basis(par.T, par.t_f)
    T, M = par.T, par.M
    blk = np.vstack([W] * M + [Wd, Wdd])
    zb = np.zeros_like(blk)
    F = np.vstack([np.hstack([blk, zb]), np.hstack([zb, blk])])
    Z = np.zeros((T, 11))
    G = np.vstack([np.hstack([Z, W]), np.hstack([Z, -W])])
    A = np.zeros((7, 22))
    A[0, :11], A[1, :11], A[2, :11] = W[0], Wd[0], Wdd[0]
    A[3, 11:], A[4, 11:], A[5, 11:], A[6, 11:] = W[0], Wd[0], Wdd[0], Wd[-1]
    b = np.array([ego[0], ego[2], ego[4], ego[1], ego[3], ego[5], 0.0])
    return W, Wd, Wdd, F, G, A, b


def active_scene(orc, rho, K, T=50):
    """Lane bound at y = 3 with a set-point at 3.5, speed set-points above
    v_max with a jump that exceeds a_max, and neighbours on the path."""
    par = orc.default_params(T=T, M=3, K=K, rho=rho, y_ub=3.0)
    ego = np.array([0.0, 0.0, 14.0, 0.0, 0.0, 0.0])
    obs = np.array([[20.0, 0.0, 8.0, 0.0], [35.0, 3.5, 9.0, 0.0], [30.0, -3.5, 10.0, 0.0]])
    sc = orc.Scene(ego, obs)
    p = np.array([3.5, 3.5, 3.5, 3.5, 10.0, 34.0, 36.0, 36.0])
    xb = orc.step1(par, sc, p)[0]
    return par, ego, sc, xb


def range_projector(A):
    """Orthogonal projector onto the range of A^T (the boundary rows)."""
    return A.T @ np.linalg.pinv(A.T)


@pytest.mark.parametrize("rho", [2.5, 0.3])
def test_scene_has_every_constraint_active(orc, rho):
    par, ego, sc, xb = active_scene(orc, rho, K=2)
    d = orc.project_dump(par, sc, xb)
    _, _, _, F, G, _, _ = problem_matrices(orc, par, ego)
    T, M = par.T, par.M
    Fx = F @ xb
    h0 = d["h"][0]
    assert np.abs(h0[:M * T] - Fx[:M * T]).max() > 0.1                      # neighbours, x rows
    assert np.abs(h0[M * T:(M + 1) * T] - Fx[M * T:(M + 1) * T]).max() > 1.0  # speed clip
    assert np.abs(h0[(M + 1) * T:(M + 2) * T] - Fx[(M + 1) * T:(M + 2) * T]).max() > 1.0  # acceleration
    assert (G @ xb - d["e"][0]).max() > 0.1                                   # lane rows


@pytest.mark.parametrize("rho", [2.5, 0.3])
def test_first_xi_update_is_the_constrained_least_squares_solution(orc, rho):
    """xi^1 = argmin 1/2|xi - xi_bar|^2 + rho/2 |F xi - h^0|^2 + rho/2
    |G xi - e + s^0|^2 s.t. A_eq xi = b (eq. split_xy with lambda^0 = 0),
    with h^0, s^0 from the target pass at xi_bar (d_a of the previous pass:
    |a(xi_bar)| clipped to [0, a_max]) and e the constant lane bounds."""
    par, ego, sc, xb = active_scene(orc, rho, K=1)
    W, Wd, Wdd, F, G, A, b = problem_matrices(orc, par, ego)
    T = par.T
    da0 = np.minimum(np.hypot(Wdd @ xb[:11], Wdd @ xb[11:]), par.a_max)
    h0, s0, _ = orc.targets(par, sc, xb, da0)
    e0 = np.r_[np.full(T, par.y_ub), np.full(T, -par.y_lb)]
    # null space of A_eq and a particular solution, then least squares
    _, _, Vt = np.linalg.svd(A)
    Z = Vt[A.shape[0]:].T
    xp = np.linalg.pinv(A) @ b
    D = np.vstack([np.eye(22), np.sqrt(rho) * F, np.sqrt(rho) * G])
    t = np.concatenate([xb, np.sqrt(rho) * h0, np.sqrt(rho) * (e0 - s0)])
    y = np.linalg.lstsq(D @ Z, t - D @ xp, rcond=None)[0]
    x1 = xp + Z @ y
    d = orc.project_dump(par, sc, xb)
    assert np.abs(d["h"][0] - h0).max() == 0.0 and np.abs(d["s"][0] - s0).max() == 0.0
    assert np.abs(d["e"][0] - e0).max() == 0.0
    scale = max(1.0, np.abs(x1).max())
    assert np.abs(d["xi"][1] - x1).max() <= 1e-10 * scale


@pytest.mark.parametrize("rho", [2.5, 0.3])
def test_every_xi_update_meets_its_kkt_system(orc, rho):
    """Stationarity of eq. aug_lag in xi at every iterate k = 1..K:
    (xi^k - xi_bar - lambda^(k-1)) + rho F^T (F xi^k - h^(k-1))
    + rho G^T (G xi^k - e^(k-1) + s^(k-1)) lies in the range of A_eq^T, to
    1e-10 of the right-hand side's size; and A_eq xi^k = b."""
    par, ego, sc, xb = active_scene(orc, rho, K=20)
    _, _, _, F, G, A, b = problem_matrices(orc, par, ego)
    P = range_projector(A)
    d = orc.project_dump(par, sc, xb)
    worst = 0.0
    for k in range(1, par.K + 1):
        lam, h, s, e = d["lam"][k - 1], d["h"][k - 1], d["s"][k - 1], d["e"][k - 1]
        x = d["xi"][k]
        r = (x - xb - lam) + rho * F.T @ (F @ x - h) + rho * G.T @ (G @ x - e + s)
        rhs = xb + lam + rho * F.T @ h + rho * G.T @ (e - s)
        worst = max(worst, np.linalg.norm(r - P @ r) / np.linalg.norm(rhs))
        assert np.abs(A @ x - b).max() <= 1e-10 * max(1.0, np.abs(x).max())
    assert worst <= 1e-10, worst


def test_record_is_the_target_pass_of_each_iterate(orc):
    """The recorded h^k, s^k, d_a^k equal the target pass at xi^k with
    d_a^(k-1) (steps split_alpha_o .. update_slack), and s^k is the lane
    slack max(0, e^k - G xi^k) of step update_slack."""
    par, ego, sc, xb = active_scene(orc, 2.5, K=6)
    _, _, _, _, G, _, _ = problem_matrices(orc, par, ego)
    d = orc.project_dump(par, sc, xb)
    for k in range(1, par.K + 1):
        h, s, da = orc.targets(par, sc, d["xi"][k], d["da"][k - 1])
        assert np.array_equal(h, d["h"][k]) and np.array_equal(s, d["s"][k])
        assert np.array_equal(da, d["da"][k])
        assert np.allclose(d["s"][k], np.maximum(0.0, d["e"][k] - G @ d["xi"][k]), rtol=0, atol=1e-12)


def test_fixed_point_multiplier_equals_the_projection_step(orc):
    """Run Alg. 2 to its fixed point (rho = 0.3, K = 3000; the iterates stop
    moving). There the multiplier step leaves the penalty gradient zero and
    the xi-step's stationarity gives lambda* = xi* - xi_bar, both up to a
    multiple of the boundary rows. A sign error of lambda in eq. split_xy or
    a multiplier step that does not follow the penalty gradient breaks it;
    the step length does not."""
    par, ego, sc, xb = active_scene(orc, 0.3, K=3000)
    _, _, _, F, G, A, b = problem_matrices(orc, par, ego)
    P = range_projector(A)
    d = orc.project_dump(par, sc, xb)
    K = par.K
    x, lam = d["xi"][K], d["lam"][K]
    assert np.abs(x - d["xi"][K - 1]).max() < 1e-12            # converged
    g = F.T @ (F @ x - d["h"][K]) + G.T @ (G @ x - d["e"][K] + d["s"][K])
    assert np.linalg.norm(g - P @ g) <= 1e-9 * np.linalg.norm(F.T @ d["h"][K])
    q = lam - (x - xb)
    assert np.linalg.norm(q - P @ q) <= 1e-9 * np.linalg.norm(lam)
    assert np.linalg.norm(lam) > 1.0                           # the multipliers are not trivially zero
