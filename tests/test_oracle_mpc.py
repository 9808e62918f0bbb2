"""Pins of the oracle's receding-horizon step (MPC-Bi-Level, Sec. V-A): the
state reached after n_exec instants, the neighbours' constant-velocity
motion, the collision test over the executed instants, and the closed loop's
invariance under a shift along the road."""
import numpy as np
import pytest


def quad_xi(x0, v, a, y0, vy, ay, t_f):
    """Bernstein coefficients (degree 10) of x0 + v t + a t^2 / 2 per axis:
    tau = sum (i/n) B_i and tau^2 = sum i(i-1)/(n(n-1)) B_i."""
    i = np.arange(11.0)
    lin, sq = i / 10.0, i * (i - 1) / 90.0
    return np.r_[x0 + v * t_f * lin + 0.5 * a * t_f ** 2 * sq,
                 y0 + vy * t_f * lin + 0.5 * ay * t_f ** 2 * sq]


@pytest.mark.parametrize("T,n_exec,cycle", [(100, 5, 0), (50, 1, 3), (64, 63, 1), (37, 7, 12)])
def test_advance_state_of_quadratic_motion(orc, T, n_exec, cycle):
    """Closed form: x(t) = x0 + v t + a t^2 / 2 gives the state
    (x0 + v t + a t^2 / 2, ..., v + a t, ..., a, ...) at t = n_exec t_f / (T - 1)."""
    par = orc.default_params(T=T, M=0)
    x0, v, a, y0, vy, ay = 12.5, 17.0, -0.8, 1.2, 0.4, 0.15
    xi = quad_xi(x0, v, a, y0, vy, ay, par.t_f)
    ego, obs, hit = orc.advance(par, xi, np.zeros((0, 4)), cycle, n_exec)
    t = n_exec * par.t_f / (T - 1)
    want = [x0 + v * t + 0.5 * a * t * t, y0 + vy * t + 0.5 * ay * t * t, v + a * t, vy + ay * t, a, ay]
    assert np.allclose(ego, want, rtol=0, atol=1e-11), ego - np.array(want)
    assert obs.shape == (0, 4) and not hit


def test_advance_moves_neighbours_at_constant_velocity(orc):
    T, n_exec = 100, 5
    par = orc.default_params(T=T, M=3)
    obs0 = np.array([[50.0, 0.0, 10.0, 0.0], [-40.0, 3.5, 20.0, 0.0], [80.0, -3.5, 15.0, 0.3]])
    xi = quad_xi(0, 15, 0, -7.0, 0, 0, par.t_f)  # far from all of them laterally
    for cycle in (0, 1, 7):
        _, obs, hit = orc.advance(par, xi, obs0, cycle, n_exec)
        s = (cycle + 1) * n_exec * par.t_f / (T - 1)
        want = obs0.copy()
        want[:, 0] += obs0[:, 2] * s
        want[:, 1] += obs0[:, 3] * s
        assert np.allclose(obs, want, rtol=0, atol=1e-12)
        assert np.array_equal(obs[:, 2:], obs0[:, 2:])
        assert not hit


def test_advance_collision_cases(orc):
    """Hand-built cases: a neighbour on the ego's path at an executed
    instant collides; one just outside the ellipse, or reaching the ego's
    position one instant after the executed part, does not; the cycle index
    sets the scene time."""
    T, n_exec = 100, 5
    par = orc.default_params(T=T, M=1)
    dt = par.t_f / (T - 1)
    v = 15.0
    xi = quad_xi(0.0, v, 0.0, 0.0, 0.0, 0.0, par.t_f)  # x = v t, y = 0
    # standing at the ego's position of instant 3 (same x, same lane)
    _, _, hit = orc.advance(par, xi, np.array([[3 * dt * v, 0.0, 0.0, 0.0]]), 0, n_exec)
    assert hit
    # 1% outside the ellipse laterally at every instant
    _, _, hit = orc.advance(par, xi, np.array([[0.0, 1.01 * par.ell_b, v, 0.0]]), 0, n_exec)
    assert not hit
    # same, 1% inside
    _, _, hit = orc.advance(par, xi, np.array([[0.0, 0.99 * par.ell_b, v, 0.0]]), 0, n_exec)
    assert hit
    # a neighbour moving at v + w that is at the ego's x exactly at instant
    # n_exec + 1 + (a margin of a full ellipse): ahead of it before then
    w = 100.0
    k_meet = n_exec + 1
    gap = par.ell_a * 1.001
    x_meet = k_meet * dt * v
    o = np.array([[x_meet - (v + w) * k_meet * dt - gap, 0.0, v + w, 0.0]])
    _, _, hit = orc.advance(par, xi, o, 0, n_exec)
    assert not hit
    o2 = o.copy()
    o2[0, 0] += 2 * gap  # now it meets the ego a little earlier, inside the executed part
    _, _, hit = orc.advance(par, xi, o2, 0, n_exec)
    assert hit
    # cycle index: a neighbour at rest at x = X meets the ego's instant-0
    # position only in the cycle whose scene time puts it there: with the
    # neighbour moving at -u, x_o(s) = X - u s is at 0 when s = X / u
    u = 10.0
    c_hit = 4
    X = u * c_hit * n_exec * dt
    o3 = np.array([[X, 0.0, -u, 0.0]])
    xi0 = quad_xi(0.0, 0.0, 0.0, 0.0, 0.0, 0.0, par.t_f)  # ego at rest at the origin
    hits = [orc.advance(par, xi0, o3, c, n_exec)[2] for c in range(8)]
    # inside the ellipse (a = 4.5 m) while |X - u s| < 4.5: s within 0.45 s of
    # c_hit * 0.2525 s, i.e. the executed parts of cycles 2 .. 5 touch it
    s_lo, s_hi = (X - par.ell_a) / u, (X + par.ell_a) / u
    want = []
    for c in range(8):
        times = [(c * n_exec + k) * dt for k in range(n_exec + 1)]
        want.append(any(s_lo < t < s_hi for t in times))
    assert hits == want and hits[c_hit]


def test_advance_rejects_bad_instant_counts(orc):
    par = orc.default_params(T=50, M=0)
    xi = quad_xi(0, 10, 0, 0, 0, 0, par.t_f)
    with pytest.raises(ValueError):
        orc.advance(par, xi, np.zeros((0, 4)), 0, 50)
    with pytest.raises(ValueError):
        orc.advance(par, xi, np.zeros((0, 4)), 0, 0)


def test_closed_loop_shift_invariance(orc):
    """Shifting the ego and every neighbour by D along the road shifts every
    cycle's state and trajectory by D and changes nothing else (the method
    depends only on relative positions along x)."""
    par = orc.default_params(T=50, M=4, K=10, L=3)
    ego = np.array([0.0, 0.0, 14.0, 0.0, 0.0, 0.0])
    obs = np.array([[25.0, 0.0, 9.0, 0.0], [-15.0, 3.5, 18.0, 0.0], [40.0, -3.5, 11.0, 0.0],
                    [8.0, 3.5, 13.0, 0.0]])
    D = 64.0
    sh_ego = ego.copy()
    sh_ego[0] += D
    sh_obs = obs.copy()
    sh_obs[:, 0] += D
    for warm in (False, True):
        a = orc.closed_loop(par, orc.Scene(ego, obs), 11, 64, 3, 5, warm=warm)
        b = orc.closed_loop(par, orc.Scene(sh_ego, sh_obs), 11, 64, 3, 5, warm=warm)
        check_shifted(orc, par, obs, a, b, D)


def check_shifted(orc, par, obs, a, b, D):
    assert np.allclose(b["ego"][:, 0] - D, a["ego"][:, 0], atol=1e-7)
    assert np.allclose(b["ego"][:, 1:], a["ego"][:, 1:], atol=1e-7)
    assert np.allclose(b["xi"][:, :11] - D, a["xi"][:, :11], atol=1e-7)
    assert np.allclose(b["xi"][:, 11:], a["xi"][:, 11:], atol=1e-7)
    assert np.allclose(b["mu"], a["mu"], atol=1e-7)
    assert np.array_equal(a["collided"], b["collided"])
    # the loop moves forward and each cycle starts where the last one ended
    assert np.all(np.diff(a["ego"][:, 0]) > 0)
    for c in range(3):
        e_next, _, _ = orc.advance(par, a["xi"][c], obs, c, 5)
        assert np.array_equal(e_next, a["ego"][c + 1])
