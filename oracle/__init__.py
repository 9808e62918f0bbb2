"""FP64 CPU oracle of the bi-level planner hot path (arXiv 2212.02224).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. It shares no
code with the HIP path (``paper_2212_02224_amd``) and never imports it.

The arithmetic lives in ``oracle.c`` (plain C, FP64, literal), except the
decoder MLP of the learned sampler (``decoder_forward``: numpy FP64, layer by
layer as App. A lists them). This module is the ctypes marshalling around the
C code and its build step (``gcc``).

Parity status: pinned by the CPU tests in ``tests/test_oracle_*.py``. Of the
projection (Alg. 2), every xi-update, every target pass and the fixed point
of the multiplier step are pinned; the multiplier step's length (the printed
rho/2 of eq. update_lagrange) is not, so the iterate values at finite K are
"parity unpinned" in that one factor.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "_oracle.so")
_lib = None

NC, NX, NP = 11, 22, 8


def build(force: bool = True) -> str:
    """Compile oracle.c into oracle/_oracle.so with gcc (OpenMP, FP64)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-ffp-contract=off",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Params(C.Structure):
    _fields_ = [
        ("T", C.c_int), ("M", C.c_int), ("K", C.c_int), ("L", C.c_int),
        ("t_f", C.c_double),
        ("k_p", C.c_double), ("k_v", C.c_double),
        ("w_s", C.c_double), ("w_l", C.c_double), ("w_v", C.c_double),
        ("rho", C.c_double),
        ("ell_a", C.c_double), ("ell_b", C.c_double),
        ("v_min", C.c_double), ("v_max", C.c_double), ("a_max", C.c_double),
        ("kappa_max", C.c_double), ("c_max", C.c_double),
        ("y_lb", C.c_double), ("y_ub", C.c_double),
        ("v_eps", C.c_double),
        ("eta", C.c_double), ("gamma", C.c_double),
        ("cov_jitter", C.c_double),
        ("frac_ces", C.c_double), ("frac_es", C.c_double),
        ("lane_c", C.c_double * 3), ("lane_sigma", C.c_double),
        ("vd_lo", C.c_double), ("vd_hi", C.c_double),
        ("behaviour", C.c_int), ("sampler", C.c_int),
    ]


class _Scene(C.Structure):
    _fields_ = [("ego", C.c_double * 6), ("kappa_road", C.c_double),
                ("obs", C.POINTER(C.c_double)),
                ("n_road", C.c_int), ("road_x0", C.c_double), ("road_dx", C.c_double),
                ("road", C.POINTER(C.c_double))]


class _PlanOut(C.Structure):
    _fields_ = [("best_index", C.c_int), ("p_best", C.c_double * NP),
                ("xi_best", C.c_double * NX), ("cost_upper", C.c_double),
                ("residual", C.c_double), ("mu", C.c_double * NP),
                ("Sigma", C.c_double * (NP * NP))]


_PD = C.POINTER(C.c_double)
_PI = C.POINTER(C.c_int)


class _Trace(C.Structure):
    _fields_ = [("p", _PD), ("xi_bar", _PD), ("xi_star", _PD), ("r", _PD),
                ("cu", _PD), ("ces", _PI), ("es", _PI), ("c_es", _PD),
                ("mu", _PD), ("Sigma", _PD)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = C.CDLL(_LIB_PATH)
    P = C.POINTER(Params)
    S = C.POINTER(_Scene)
    lib.orc_default_params.argtypes = [P]
    lib.orc_elite_sizes.argtypes = [P, C.c_int, _PI, _PI]
    lib.orc_basis.argtypes = [C.c_int, C.c_double, _PD, _PD, _PD]
    lib.orc_lower_cost.argtypes = [P, _PD, _PD]
    lib.orc_lower_cost.restype = C.c_double
    lib.orc_step1.argtypes = [P, S, _PD, C.c_int, _PD]
    lib.orc_project.argtypes = [P, S, _PD, _PD, C.c_int, _PD, _PD]
    lib.orc_project_dump.argtypes = [P, S, _PD, _PD, _PD, _PD, _PD, _PD, _PD, _PD]
    lib.orc_targets.argtypes = [P, S, _PD, _PD, _PD, _PD, _PD]
    lib.orc_residual_cost.argtypes = [P, S, _PD, C.c_int, _PD, _PD]
    lib.orc_select.argtypes = [_PD, _PD, C.c_int, C.c_int, C.c_int, _PI, _PI, _PD]
    lib.orc_update.argtypes = [P, _PD, _PD, _PD, _PI, _PD, C.c_int, _PD, _PD]
    lib.orc_cholesky.argtypes = [_PD, C.c_int, C.c_double, _PD]
    lib.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                      C.POINTER(C.c_uint32)]
    lib.orc_initial_moments.argtypes = [P, _PD, _PD]
    lib.orc_sample.argtypes = [P, C.c_uint64, C.c_int, C.c_int, C.c_int, _PD, _PD, _PD]
    lib.orc_plan.argtypes = [P, S, C.c_uint64, C.c_int, _PD, _PD,
                             C.POINTER(_PlanOut), C.POINTER(_Trace)]
    lib.orc_advance.argtypes = [P, _PD, _PD, C.c_int, C.c_int, C.c_int, _PD, _PD, _PI]
    lib.orc_plan_p0.argtypes = [P, S, C.c_uint64, C.c_int, _PD, C.POINTER(_PlanOut), C.POINTER(_Trace)]
    lib.orc_decoder_latent.argtypes = [C.c_uint64, C.c_int, _PD]
    lib.orc_sample_moments.argtypes = [_PD, C.c_int, _PD, _PD]
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_get_threads.restype = C.c_int
    _lib = lib
    return lib


def _pd(a: np.ndarray):
    return a.ctypes.data_as(_PD)


def _pi(a: np.ndarray):
    return a.ctypes.data_as(_PI)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_load().orc_get_threads())


def default_params(**over) -> Params:
    """Parameters with the default reading of every open point, overridden
    by keyword (e.g. ``default_params(T=50, M=4, K=10, L=3)``)."""
    par = Params()
    _load().orc_default_params(C.byref(par))
    for k, v in over.items():
        if k == "lane_c":
            par.lane_c = (C.c_double * 3)(*v)
        else:
            setattr(par, k, v)
    return par


@dataclass
class Scene:
    """Ego state b_0 = (x0, y0, vx0, vy0, ax0, ay0), neighbours (M x 4:
    x, y, vx, vy at t = 0, constant velocity) and the road: a constant
    curvature, or a profile ``road`` (n x 3: kappa, y_lb, y_ub at knots
    road_x0 + i road_dx, linear between them, constant beyond)."""
    ego: np.ndarray
    obs: np.ndarray
    kappa_road: float = 0.0
    road: np.ndarray | None = None
    road_x0: float = 0.0
    road_dx: float = 1.0
    _keep: list = field(default_factory=list, repr=False)

    def c(self) -> _Scene:
        obs = _f64(self.obs).reshape(-1, 4) if np.size(self.obs) else np.zeros((1, 4))
        obs = np.ascontiguousarray(obs)
        self._keep = [obs]
        s = _Scene()
        s.ego = (C.c_double * 6)(*[float(v) for v in np.asarray(self.ego).ravel()])
        s.kappa_road = float(self.kappa_road)
        s.obs = _pd(obs)
        if self.road is not None and np.size(self.road):
            road = np.ascontiguousarray(_f64(self.road).reshape(-1, 3))
            self._keep.append(road)
            s.n_road = road.shape[0]
            s.road = _pd(road)
        else:
            s.n_road = 0
            s.road = None
        s.road_x0 = float(self.road_x0)
        s.road_dx = float(self.road_dx)
        return s


def elite_sizes(par: Params, N: int):
    n, q = C.c_int(), C.c_int()
    _load().orc_elite_sizes(C.byref(par), int(N), C.byref(n), C.byref(q))
    return n.value, q.value


def basis(T: int, t_f: float):
    W = np.zeros((T, NC)); Wd = np.zeros((T, NC)); Wdd = np.zeros((T, NC))
    _load().orc_basis(int(T), float(t_f), _pd(W), _pd(Wd), _pd(Wdd))
    return W, Wd, Wdd


def lower_cost(par: Params, p, xi) -> float:
    p = _f64(p); xi = _f64(xi)
    return float(_load().orc_lower_cost(C.byref(par), _pd(p), _pd(xi)))


def step1(par: Params, scene: Scene, p) -> np.ndarray:
    p = _f64(p).reshape(-1, NP)
    out = np.zeros((p.shape[0], NX))
    sc = scene.c()
    rc = _load().orc_step1(C.byref(par), C.byref(sc), _pd(p), p.shape[0], _pd(out))
    if rc != 0:
        raise RuntimeError("oracle step1 failed: singular KKT")
    return out


def project(par: Params, scene: Scene, xi_bar, return_iterates: bool = False, p=None):
    """Alg. 2 for every row of xi_bar. p (N x 8, the samples) is needed with
    goal positions (behaviour 1): their final boundary rows come from it."""
    xb = _f64(xi_bar).reshape(-1, NX)
    N = xb.shape[0]
    out = np.zeros((N, NX))
    it = np.zeros((N, par.K + 1, NX)) if return_iterates else None
    pp = _f64(p).reshape(N, NP) if p is not None else None
    sc = scene.c()
    rc = _load().orc_project(C.byref(par), C.byref(sc), _pd(xb), _pd(pp) if pp is not None else None, N,
                             _pd(out), _pd(it) if it is not None else None)
    if rc != 0:
        raise ValueError("oracle project: goal positions need the samples p")
    return (out, it) if return_iterates else out


def project_dump(par: Params, scene: Scene, xi_bar, p=None) -> dict:
    """Alg. 2 for one sample with every intermediate, k = 0..K: ``xi``
    (K+1 x 22; xi^0 = xi_bar, then each xi-update of eq. split_xy), the
    target pass at xi^k: ``h`` (K+1 x 2(M+2)T, rows of F), ``s`` and ``e``
    (K+1 x 2T, lane slack and bound), ``da`` (K+1 x T), and ``lam`` (K+1 x
    22: lambda^0 = 0, lambda^k after the step update_lagrange of iteration
    k). The xi-update of iteration k uses row k - 1 of lam, h, s and e."""
    xb = _f64(xi_bar).reshape(NX)
    K, T, M = par.K, par.T, par.M
    out = dict(xi=np.zeros((K + 1, NX)), h=np.zeros((K + 1, 2 * (M + 2) * T)), s=np.zeros((K + 1, 2 * T)),
               e=np.zeros((K + 1, 2 * T)), da=np.zeros((K + 1, T)), lam=np.zeros((K + 1, NX)))
    pp = _f64(p).reshape(NP) if p is not None else None
    sc = scene.c()
    rc = _load().orc_project_dump(C.byref(par), C.byref(sc), _pd(xb), _pd(pp) if pp is not None else None,
                                  *[_pd(out[k]) for k in ("xi", "h", "s", "e", "da", "lam")])
    if rc != 0:
        raise ValueError("oracle project_dump: goal positions need the sample p")
    return out


def targets(par: Params, scene: Scene, xi, da_prev):
    xi = _f64(xi); da_prev = _f64(da_prev)
    T, M = par.T, par.M
    h = np.zeros(2 * (M + 2) * T); s = np.zeros(2 * T); da = np.zeros(T)
    sc = scene.c()
    _load().orc_targets(C.byref(par), C.byref(sc), _pd(xi), _pd(da_prev),
                        _pd(h), _pd(s), _pd(da))
    return h, s, da


def residual_cost(par: Params, scene: Scene, xi):
    xi = _f64(xi).reshape(-1, NX)
    N = xi.shape[0]
    r = np.zeros(N); cu = np.zeros(N)
    sc = scene.c()
    _load().orc_residual_cost(C.byref(par), C.byref(sc), _pd(xi), N, _pd(r), _pd(cu))
    return r, cu


def select(r, cu, n: int, q: int):
    r = _f64(r); cu = _f64(cu)
    ces = np.zeros(n, np.int32); es = np.zeros(q, np.int32); c_es = np.zeros(q)
    _load().orc_select(_pd(r), _pd(cu), r.size, int(n), int(q), _pi(ces), _pi(es), _pd(c_es))
    return ces, es, c_es


def update(par: Params, mu, Sigma, p, es, c_es):
    mu = _f64(mu); Sigma = _f64(Sigma); p = _f64(p).reshape(-1, NP)
    es = np.ascontiguousarray(np.asarray(es, np.int32)); c_es = _f64(c_es)
    mo = np.zeros(NP); So = np.zeros((NP, NP))
    _load().orc_update(C.byref(par), _pd(mu), _pd(Sigma), _pd(p), _pi(es), _pd(c_es),
                       es.size, _pd(mo), _pd(So))
    return mo, So


def cholesky(A, jitter: float = 0.0):
    A = _f64(A)
    n = A.shape[0]
    L = np.zeros((n, n))
    rc = _load().orc_cholesky(_pd(A), n, float(jitter), _pd(L))
    if rc != 0:
        raise np.linalg.LinAlgError("oracle cholesky: not positive definite")
    return L


def philox4x32_10(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(v) & 0xffffffff for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    o = (C.c_uint32 * 4)()
    _load().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def initial_moments(par: Params):
    mu = np.zeros(NP); S = np.zeros((NP, NP))
    _load().orc_initial_moments(C.byref(par), _pd(mu), _pd(S))
    return mu, S


def sample(par: Params, seed: int, l: int, N: int, structured: bool,
           mu=None, Lchol=None) -> np.ndarray:
    mu = _f64(mu if mu is not None else np.zeros(NP))
    Lc = _f64(Lchol if Lchol is not None else np.eye(NP))
    p = np.zeros((N, NP))
    _load().orc_sample(C.byref(par), C.c_uint64(int(seed)), int(l), int(N),
                       1 if structured else 0, _pd(mu), _pd(Lc), _pd(p))
    return p


@dataclass
class PlanResult:
    best_index: int
    p_best: np.ndarray
    xi_best: np.ndarray
    cost_upper: float
    residual: float
    mu: np.ndarray
    Sigma: np.ndarray
    trace: dict | None = None


def plan(par: Params, scene: Scene, seed: int, N: int, mu0=None, Sigma0=None,
         trace: bool = False, p0=None) -> PlanResult:
    """Alg. 1 with the lower level of Alg. 2, FP64. p0 (N x 8): samples of
    the first iteration (the decoder sampler's, ``decoder_sample``); the
    prior of the first update is then their sample moments."""
    n, q = elite_sizes(par, N)
    L = par.L
    out = _PlanOut()
    tr = None
    arrays = None
    if trace:
        arrays = dict(p=np.zeros((L, N, NP)), xi_bar=np.zeros((L, N, NX)),
                      xi_star=np.zeros((L, N, NX)), r=np.zeros((L, N)),
                      cu=np.zeros((L, N)), ces=np.zeros((L, n), np.int32),
                      es=np.zeros((L, q), np.int32), c_es=np.zeros((L, q)),
                      mu=np.zeros((L, NP)), Sigma=np.zeros((L, NP, NP)))
        tr = _Trace()
        for k, v in arrays.items():
            setattr(tr, k, _pi(v) if v.dtype == np.int32 else _pd(v))
    sc = scene.c()
    m0 = _f64(mu0) if mu0 is not None else None
    S0 = _f64(Sigma0) if Sigma0 is not None else None
    if p0 is not None:
        q0 = np.ascontiguousarray(_f64(p0).reshape(N, NP))
        rc = _load().orc_plan_p0(C.byref(par), C.byref(sc), C.c_uint64(int(seed)), int(N), _pd(q0),
                                 C.byref(out), C.byref(tr) if tr is not None else None)
    else:
        rc = _load().orc_plan(C.byref(par), C.byref(sc), C.c_uint64(int(seed)), int(N),
                              _pd(m0) if m0 is not None else None,
                              _pd(S0) if S0 is not None else None,
                              C.byref(out), C.byref(tr) if tr is not None else None)
    if rc != 0:
        raise RuntimeError(f"oracle plan failed rc={rc}")
    return PlanResult(out.best_index, np.array(out.p_best), np.array(out.xi_best),
                      out.cost_upper, out.residual, np.array(out.mu),
                      np.array(out.Sigma).reshape(NP, NP), arrays)


def decoder_latent(seed: int, N: int) -> np.ndarray:
    """Latent draws z (N x 2, z ~ N(0, I) of App. A) of the decoder sampler:
    Box-Muller of words 0, 1 of Philox block (j, 0, 0, 0) under the key seed."""
    z = np.zeros((N, 2))
    _load().orc_decoder_latent(C.c_uint64(int(seed)), int(N), _pd(z))
    return z


def sample_moments(p):
    """Sample mean and covariance (normalised by N) of p (N x 8)."""
    p = np.ascontiguousarray(_f64(p).reshape(-1, NP))
    mu, S = np.zeros(NP), np.zeros((NP, NP))
    _load().orc_sample_moments(_pd(p), p.shape[0], _pd(mu), _pd(S))
    return mu, S


def decoder_forward(dec, obs, z, behaviour: int = 0) -> np.ndarray:
    """Decoder MLP of the CVAE (App. A, decoder table): the input [o, z]
    (55 + 2) goes through five blocks of Linear, BatchNorm (inference form:
    running mean and variance, eps, then gamma and beta) and ReLU with 1024,
    1024, 1024, 1024 and 256 outputs, then a Linear layer to the 8
    behavioural inputs p. FP64. ``dec`` holds W (6 weight matrices, out x
    in), b (6 biases), gamma, beta, mean, var (5 each) and eps. With goal
    positions (behaviour 1) only p[0], p[1] are inputs; the others are 0."""
    z = _f64(z).reshape(-1, 2)
    x = np.concatenate([np.broadcast_to(_f64(obs).reshape(1, -1), (z.shape[0], 55)), z], axis=1)
    for i in range(5):
        h = x @ _f64(dec.W[i]).T + _f64(dec.b[i])
        h = (h - _f64(dec.mean[i])) / np.sqrt(_f64(dec.var[i]) + dec.eps) * _f64(dec.gamma[i]) + _f64(dec.beta[i])
        x = np.maximum(h, 0.0)
    p = x @ _f64(dec.W[5]).T + _f64(dec.b[5])
    if behaviour:
        p[:, 2:] = 0.0
    return p


def decoder_sample(par: Params, dec, obs, seed: int, N: int) -> np.ndarray:
    """N samples of p from the decoder sampler (App. A inference: z drawn
    from N(0, I), passed through the decoder MLP with the observation o)."""
    return decoder_forward(dec, obs, decoder_latent(seed, N), par.behaviour)


def advance(par: Params, xi, obs0, cycle: int, n_exec: int):
    """One step of the receding-horizon loop (MPC-Bi-Level, Sec. V-A): the
    state (x, y, vx, vy, ax, ay) of trajectory xi at t_{n_exec}, the
    neighbours (M x 4, first-cycle states obs0) at the start of cycle + 1,
    and whether an executed instant t_0..t_{n_exec} of cycle ``cycle`` meets
    a neighbour's ellipse."""
    xi = _f64(xi).reshape(NX)
    obs0 = np.ascontiguousarray(_f64(obs0).reshape(-1, 4))
    M = obs0.shape[0]
    ego = np.zeros(6)
    obs = np.zeros((max(M, 1), 4))
    hit = C.c_int()
    rc = _load().orc_advance(C.byref(par), _pd(xi), _pd(obs0 if M else np.zeros((1, 4))), M, int(cycle),
                             int(n_exec), _pd(ego), _pd(obs), C.byref(hit))
    if rc != 0:
        raise ValueError("oracle advance: n_exec out of [1, T - 1] or negative cycle")
    return ego, obs[:M], bool(hit.value)


def closed_loop(par: Params, scene: Scene, seed: int, N: int, cycles: int, n_exec: int,
                warm: bool = False, mu0=None, Sigma0=None) -> dict:
    """Receding-horizon loop of one episode (MPC-Bi-Level, Sec. V-A): Alg. 1
    per cycle (seed + c at cycle c), then ``advance``. Cycles after the first
    start from the initial sampler, or with ``warm`` from the previous
    cycle's final mu, Sigma (Sec. IV). Returns per-cycle logs shaped like the
    library's plan_mpc_run logs."""
    obs0 = np.asarray(scene.obs, float).reshape(-1, 4)
    ego = np.asarray(scene.ego, float).copy()
    obs = obs0.copy()
    out = dict(ego=np.zeros((cycles + 1, 6)), xi=np.zeros((cycles, NX)), mu=np.zeros((cycles, NP)),
               sigma=np.zeros((cycles, NP, NP)), cost=np.zeros((cycles, 2)), collided=np.zeros(cycles, np.int32))
    out["ego"][0] = ego
    m, S = mu0, Sigma0
    for c in range(cycles):
        res = plan(par, Scene(ego, obs, scene.kappa_road, scene.road, scene.road_x0, scene.road_dx),
                   (int(seed) + c) % 2 ** 64, N, m, S)
        out["xi"][c], out["mu"][c], out["sigma"][c] = res.xi_best, res.mu, res.Sigma
        out["cost"][c] = (res.cost_upper, res.residual)
        ego, obs, hit = advance(par, res.xi_best, obs0, c, n_exec)
        out["ego"][c + 1] = ego
        out["collided"][c] = int(hit)
        m, S = (res.mu, res.Sigma) if warm else (None, None)
    return out
