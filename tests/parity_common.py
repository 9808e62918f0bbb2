"""Conditioning of the projection, shared by the GPU parity tests.

Alg. 2 is not a continuous function of its input everywhere: the (alpha, d)
step takes the direction atan2(dy/b, dx/a) from a neighbour's centre to the
trajectory, which turns through pi as the trajectory passes the centre, and
the velocity step the direction atan2(ydot, xdot), which is undefined at
rest. Near those points an FP32 run cannot follow the FP64 oracle, however it
is implemented. The oracle itself shows it: its own answer moves far more
than its input when the input is perturbed by a rounding-sized amount.

ill_conditioned() flags the samples whose FP64 projection moves by more than
`limit` (2e-5 m, i.e. 20 times) when xi_bar is perturbed by `noise` (1e-6 m,
about the FP32 rounding of the coefficients, seeded), or whose projection
iterates pass below the speed floor v_eps. The parity tests count those
samples, print their largest error, and hold every other sample to the full
bar; a flagged sample that changes an elite set is treated like a near tie.
"""
import numpy as np


def ill_conditioned(orc, par, sc, xi_bar, xi_star, p=None, noise=1e-6, limit=2e-5, seed=1):
    rng = np.random.default_rng(seed)
    xb2 = xi_bar + noise * rng.standard_normal(xi_bar.shape)
    xs2, it = orc.project(par, sc, xb2, return_iterates=True, p=p)
    W, Wd, _ = orc.basis(par.T, par.t_f)
    dx = (xs2[:, :11] - xi_star[:, :11]) @ W.T
    dy = (xs2[:, 11:] - xi_star[:, 11:]) @ W.T
    move = np.sqrt(dx ** 2 + dy ** 2).max(axis=1)
    vx = np.einsum('jkc,tc->jkt', it[:, :, :11], Wd)
    vy = np.einsum('jkc,tc->jkt', it[:, :, 11:], Wd)
    slow = np.hypot(vx, vy).min(axis=(1, 2)) < par.v_eps
    return (move > limit) | slow
