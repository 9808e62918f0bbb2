"""Seeded synthetic planning scenes (inputs only; none of the method's
arithmetic lives here).

The paper evaluates on highway-env scenes with IDM/MOBIL traffic (Sec. V);
that simulator is not available, so these scenes stand in for them with the
same structure: a straight multi-lane road, an ego vehicle in a lane, and
neighbours moving along straight lines at constant speed in their lanes
(Fig. learned_sampler), of which the planner sees the M nearest.

    road        straight, lane centres {-3.5, 0, 3.5} m, bounds y in [-7, 7]
    ego         x0 = 0, y0 = a lane centre, vx0 ~ U[10, 20] m/s, other terms 0
    neighbours  lane centre, x ~ U[-20, 120] m, vx ~ U[8, 25] m/s, vy = 0;
                rejected if closer than 1.5 (ellipse-normalised) to the ego or
                than 1.0 to another neighbour at t = 0
    seeds       scene seed = 1000 * config + request index; the request's
                sample-stream key is scene seed XOR 0x9E3779B9

curved_road() gives a road profile for the same scenes (curvature and lane
limits along x, in the road-aligned frame the neighbours' lanes follow):
knots every 20 m from x = -40 to 280 m; the curvature ramps linearly from 0
to +-U[0.01, 0.02] 1/m (radius 50..100 m) over 60 m from a start in
U[0, 60] m, holds for 60 m and ramps back; with probability 1/2 the left
lane closes (y_ub from 7 to 5.25 m over 40 m from a start in U[40, 120] m).
At the scenes' speeds the centripetal row v^2 |kappa| <= c_max (c_max 4)
is active inside the bend.

observation() and decoder_weights() are the inputs of the decoder sampler
(the CVAE decoder of App. A, whose trained weights are not published):
    observation  55 values, scaled to O(1): ego heading, vx0 / 20, vy0 / 20;
                 the 10 nearest neighbours (Euclidean at t = 0) as
                 (dx / 50, dy / 7, vx / 20, vy / 20), missing ones at
                 dx / 50 = 4, the rest 0; lane limits (y_lb - y0) / 7,
                 (y_ub - y0) / 7 at the first 6 profile knots from x0 on (the
                 constant limits without a profile)
    weights      random: Linear weights N(0, 2 / fan_in) (the latent
                 columns of the first layer x 4, so that z spreads the
                 samples), biases U(-0.05, 0.05); BatchNorm gamma U(0.9, 1.1),
                 beta, running mean U(-0.05, 0.05), running variance
                 U(0.9, 1.1), eps 1e-5; the output layer scaled so that p
                 spreads like behavioural inputs (lateral set-points about
                 +-2 m around 0, velocity set-points about 15 +- 4 m/s; goals
                 75 +- 20 m ahead, y_f about +-2 m)
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

LANES = (-3.5, 0.0, 3.5)
ELL_A, ELL_B = 4.5, 2.0


@dataclass
class Scene:
    ego: np.ndarray        # (6,)  x0, y0, vx0, vy0, ax0, ay0
    obstacles: np.ndarray  # (M, 4) x, y, vx, vy at t = 0
    seed: int              # key of the request's sample stream


def scene(config: int, index: int, M: int) -> Scene:
    s = 1000 * int(config) + int(index)
    rng = np.random.default_rng(s)
    ego = np.array([0.0, rng.choice(LANES), rng.uniform(10.0, 20.0), 0.0, 0.0, 0.0])
    obs = []
    tries = 0
    while len(obs) < M:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place neighbours")
        o = np.array([rng.uniform(-20.0, 120.0), rng.choice(LANES), rng.uniform(8.0, 25.0), 0.0])
        d_ego = np.hypot((o[0] - ego[0]) / ELL_A, (o[1] - ego[1]) / ELL_B)
        if d_ego < 1.5:
            continue
        if any(np.hypot((o[0] - q[0]) / ELL_A, (o[1] - q[1]) / ELL_B) < 1.0 for q in obs):
            continue
        obs.append(o)
    obs = np.array(obs, dtype=np.float64).reshape(M, 4)
    return Scene(ego, obs, s ^ 0x9E3779B9)


def served_mix(n_req: int, seed: int = 4) -> list[tuple[int, int, int]]:
    """(N, M, T) of the served workload's requests: N in {256, 512, 1000,
    2048}, M in {4, 10, 20}, T in {50, 100}, drawn per request in that
    order from one seeded generator. Request i uses scene(4, i, M)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_req):
        N = int(rng.choice([256, 512, 1000, 2048]))
        M = int(rng.choice([4, 10, 20]))
        T = int(rng.choice([50, 100]))
        out.append((N, M, T))
    return out


def curved_road(config: int, index: int):
    """(road (n x 3: kappa, y_lb, y_ub), road_x0, road_dx) for scene
    (config, index); an independent stream of the scene's seed."""
    rng = np.random.default_rng([1000 * int(config) + int(index), 7])
    x0, dx, n = -40.0, 20.0, 17
    x = x0 + dx * np.arange(n)
    k_c = rng.choice((-1.0, 1.0)) * rng.uniform(0.01, 0.02)
    a = rng.uniform(0.0, 60.0)
    kappa = k_c * np.clip(np.minimum((x - a) / 60.0, (a + 180.0 - x) / 60.0), 0.0, 1.0)
    y_ub = np.full(n, 7.0)
    if rng.uniform() < 0.5:
        b = rng.uniform(40.0, 120.0)
        y_ub = 7.0 - 1.75 * np.clip((x - b) / 40.0, 0.0, 1.0)
    road = np.stack([kappa, np.full(n, -7.0), y_ub], axis=1)
    return road, x0, dx


OBS_DIM, LATENT_DIM = 55, 2
DECODER_SIZES = (OBS_DIM + LATENT_DIM, 1024, 1024, 1024, 1024, 256, 8)


@dataclass
class Decoder:
    W: list          # 6 weight matrices, out x in
    b: list          # 6 biases
    gamma: list      # BatchNorm of blocks 1-5
    beta: list
    mean: list
    var: list
    eps: float = 1e-5


def observation(s: Scene, road=None, road_x0: float = 0.0, road_dx: float = 1.0,
                y_lb: float = -7.0, y_ub: float = 7.0) -> np.ndarray:
    """The 55-value observation of scene s (layout in the module docstring)."""
    ego = np.asarray(s.ego, np.float64)
    o = np.zeros(OBS_DIM)
    o[0] = np.arctan2(ego[3], ego[2])
    o[1], o[2] = ego[2] / 20.0, ego[3] / 20.0
    obs = np.asarray(s.obstacles, np.float64).reshape(-1, 4)
    order = np.argsort(np.hypot(obs[:, 0] - ego[0], obs[:, 1] - ego[1]), kind="stable")[:10]
    for i in range(10):
        k = 3 + 4 * i
        if i < len(order):
            q = obs[order[i]]
            o[k:k + 4] = [(q[0] - ego[0]) / 50.0, (q[1] - ego[1]) / 7.0, q[2] / 20.0, q[3] / 20.0]
        else:
            o[k] = 4.0
    lim = np.tile([y_lb, y_ub], (6, 1))
    if road is not None and np.size(road):
        r = np.asarray(road, np.float64).reshape(-1, 3)
        first = int(np.clip(np.ceil((ego[0] - road_x0) / road_dx), 0, len(r) - 1))
        idx = np.minimum(first + np.arange(6), len(r) - 1)
        lim = r[idx, 1:3]
    o[43:] = ((lim - ego[1]) / 7.0).ravel()
    return o


def decoder_weights(seed: int = 0, behaviour: int = 0) -> Decoder:
    """Random decoder weights of the App. A sizes (recipe in the module
    docstring); behaviour 1 shapes the output for goal positions."""
    rng = np.random.default_rng([int(seed), 11])
    W, b, g, be, m, v = [], [], [], [], [], []
    for i in range(6):
        fi, fo = DECODER_SIZES[i], DECODER_SIZES[i + 1]
        Wi = rng.standard_normal((fo, fi)) * np.sqrt(2.0 / fi)
        bi = rng.uniform(-0.05, 0.05, fo)
        if i == 0:
            Wi[:, OBS_DIM:] *= 4.0
        if i == 5:
            if behaviour:
                scale, centre = np.r_[20.0, 2.0, np.zeros(6)], np.r_[75.0, np.zeros(7)]
            else:
                scale, centre = np.r_[np.full(4, 2.0), np.full(4, 4.0)], np.r_[np.zeros(4), np.full(4, 15.0)]
            Wi *= (scale / np.sqrt(2.0 * 0.9))[:, None]
            bi = bi + centre
        W.append(Wi)
        b.append(bi)
        if i < 5:
            g.append(rng.uniform(0.9, 1.1, fo))
            be.append(rng.uniform(-0.05, 0.05, fo))
            m.append(rng.uniform(-0.05, 0.05, fo))
            v.append(rng.uniform(0.9, 1.1, fo))
    return Decoder(W, b, g, be, m, v)


# Workload configurations (sizes of the planning problem).
CONFIGS = {
    1: dict(name="small-N64-T50-M4", N=64, T=50, M=4, L=3, K=10),
    2: dict(name="plan-N1000-T100-M10", N=1000, T=100, M=10, L=5, K=20),
    4: dict(name="served-poisson-256", N=(256, 512, 1000, 2048), T=(50, 100), M=(4, 10, 20), L=5, K=20),
    5: dict(name="served-1024x-N4096-T100-M20", N=4096, T=100, M=20, L=5, K=20),
}
