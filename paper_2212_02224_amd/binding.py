"""ctypes binding of ``include/plan.h`` (``libplan.so``).

Argument marshalling only: every step of the planner runs in the HIP kernels
of the library. The binding raises when the library is missing or was built
for something else; there is no other execution path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libplan.so")

PLAN_OK, PLAN_E_INVALID, PLAN_E_NOMEM, PLAN_E_DEVICE, PLAN_E_BUSY, PLAN_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
PLAN_E_TIMEOUT = -6
PLAN_PREC_FP32, PLAN_PREC_FP16_SPLIT, PLAN_PREC_FP32_MFMA = 0, 1, 2
PLAN_F_INFEASIBLE, PLAN_F_WARM = 1, 2
PLAN_MPC_SAMPLER, PLAN_MPC_WARM = 0, 1
PLAN_BEHAV_SETPOINTS, PLAN_BEHAV_GOALS = 0, 1
PLAN_SAMPLER_RANDOM, PLAN_SAMPLER_GRID, PLAN_SAMPLER_DECODER = 0, 1, 2
PLAN_OBS_DIM = 55  # observation of the decoder sampler
PLAN_MAX_ROAD = 64  # knots of a request's road profile
NC, NX, NP = 11, 22, 8
MAX_N, MAX_M, MAX_T, MAX_ROAD = 4096, 32, 256, 64


class PlanError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"plan status {status}: {msg}")
        self.status = status


class plan_config(C.Structure):
    _fields_ = [
        ("T_set", C.c_int32 * 4), ("n_T", C.c_int32),
        ("M_set", C.c_int32 * 8), ("n_M", C.c_int32),
        ("t_f", C.c_double),
        ("max_N", C.c_int32), ("max_requests", C.c_int32),
        ("proj_iters", C.c_int32), ("upper_iters", C.c_int32),
        ("frac_ces", C.c_double), ("frac_es", C.c_double),
        ("eta", C.c_double), ("gamma", C.c_double), ("rho", C.c_double),
        ("k_p", C.c_double), ("k_v", C.c_double), ("w_s", C.c_double), ("w_l", C.c_double),
        ("w_v", C.c_double),
        ("cov_jitter", C.c_double),
        ("v_min", C.c_double), ("v_max", C.c_double), ("a_max", C.c_double),
        ("kappa_max", C.c_double), ("c_max", C.c_double), ("y_lb", C.c_double), ("y_ub", C.c_double),
        ("ell_a", C.c_double), ("ell_b", C.c_double), ("v_eps", C.c_double),
        ("lane_c", C.c_double * 3),
        ("lane_sigma", C.c_double), ("vd_lo", C.c_double), ("vd_hi", C.c_double),
        ("precision", C.c_int32), ("trace", C.c_int32),
        ("behaviour", C.c_int32), ("sampler", C.c_int32), ("served_run_ahead", C.c_int32),
        ("fused_iters", C.c_int32), ("fused_wait_us", C.c_int32),
        ("sample_budget", C.c_int64),
        ("device_workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
        ("stream", C.c_void_p),
    ]


_PD = C.POINTER(C.c_double)
_PI = C.POINTER(C.c_int32)


class plan_request(C.Structure):
    _fields_ = [
        ("request_id", C.c_uint64), ("session_id", C.c_uint64), ("seed", C.c_uint64),
        ("N", C.c_int32), ("M", C.c_int32), ("T", C.c_int32),
        ("ego", C.c_double * 6),
        ("obstacles", _PD),
        ("kappa_road", C.c_double),
        ("mu0", _PD), ("sigma0", _PD),
        ("first_iter", C.c_int32),
        ("n_road", C.c_int32), ("road_x0", C.c_double), ("road_dx", C.c_double),
        ("road", _PD),
        ("observation", _PD),
    ]


class plan_decoder(C.Structure):
    _fields_ = [
        ("W", _PD * 6), ("b", _PD * 6),
        ("bn_gamma", _PD * 5), ("bn_beta", _PD * 5), ("bn_mean", _PD * 5), ("bn_var", _PD * 5),
        ("bn_eps", C.c_double),
    ]


class plan_result(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("flags", C.c_uint32),
        ("best_index", C.c_int32), ("iterations", C.c_int32),
        ("p_best", C.c_double * NP), ("xi_best", C.c_double * NX),
        ("cost_upper", C.c_double), ("residual", C.c_double),
        ("mu", C.c_double * NP), ("sigma", C.c_double * (NP * NP)),
        ("latency_s", C.c_double),
        ("traj_xy", _PD),
    ]


class plan_mpc_log(C.Structure):
    _fields_ = [("ego", _PD), ("xi", _PD), ("mu", _PD), ("sigma", _PD), ("cost", _PD),
                ("collided", _PI), ("status", _PI)]


_lib = None


def load():
    """Load libplan.so (built by ``paper_2212_02224_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2212_02224_amd.build`")
    lib = C.CDLL(LIB_PATH)
    H = C.c_void_p
    Cfg = C.POINTER(plan_config)
    Req = C.POINTER(plan_request)
    Res = C.POINTER(plan_result)
    lib.plan_config_init.argtypes = [Cfg]
    lib.plan_config_init.restype = None
    lib.plan_workspace_bytes.argtypes = [Cfg]
    lib.plan_workspace_bytes.restype = C.c_size_t
    lib.plan_create.argtypes = [Cfg, C.POINTER(H)]
    lib.plan_destroy.argtypes = [H]
    lib.plan_destroy.restype = None
    lib.plan_last_error.argtypes = [H]
    lib.plan_last_error.restype = C.c_char_p
    lib.plan_solve_batch.argtypes = [H, Req, C.c_int32, Res]
    lib.plan_stage.argtypes = [H, Req, C.c_int32]
    lib.plan_launch.argtypes = [H]
    lib.plan_collect.argtypes = [H, Res]
    lib.plan_lower_solve.argtypes = [H, Req, _PD, C.c_int32, _PD, _PD, _PD, _PD]
    lib.plan_lower_solve_static.argtypes = [H, Req, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_void_p]
    lib.plan_get_trace.argtypes = [H, C.c_int32, _PD, _PD, _PD, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), _PD, _PD]
    lib.plan_submit.argtypes = [H, Req, C.POINTER(C.c_uint64)]
    lib.plan_progress.argtypes = [H, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.plan_poll.argtypes = [H, C.c_uint64, Res]
    lib.plan_poll_done.argtypes = [H, C.POINTER(C.c_uint64), Res, C.c_int32, C.POINTER(C.c_int32)]
    lib.plan_mpc_run.argtypes = [H, Req, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(plan_mpc_log), Res]
    lib.plan_profile.argtypes = [H, C.c_int32]
    lib.plan_profile_read.argtypes = [H, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.plan_set_decoder.argtypes = [H, C.POINTER(plan_decoder)]
    lib.plan_elite_sizes.argtypes = [Cfg, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    for name in ("plan_create", "plan_solve_batch", "plan_stage", "plan_launch", "plan_collect",
                 "plan_lower_solve", "plan_lower_solve_static", "plan_get_trace", "plan_submit",
                 "plan_progress", "plan_poll", "plan_poll_done", "plan_mpc_run", "plan_profile",
                 "plan_profile_read", "plan_set_decoder", "plan_elite_sizes"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def exported_symbols() -> list[str]:
    return ["plan_config_init", "plan_workspace_bytes", "plan_create", "plan_destroy",
            "plan_last_error", "plan_solve_batch", "plan_stage", "plan_launch", "plan_collect",
            "plan_lower_solve", "plan_lower_solve_static", "plan_get_trace", "plan_submit",
            "plan_progress", "plan_poll", "plan_poll_done", "plan_mpc_run", "plan_profile",
            "plan_profile_read", "plan_set_decoder", "plan_elite_sizes"]


def _check(status: int, handle=None) -> int:
    if status != PLAN_OK:
        msg = load().plan_last_error(handle)
        raise PlanError(status, msg.decode() if msg else "")
    return status


def _pd(a: np.ndarray):
    return a.ctypes.data_as(_PD)


# --------------------------------------------------------------- requests

@dataclass
class Request:
    """One planning request (see ``plan_request`` in include/plan.h)."""
    N: int
    T: int
    ego: Sequence[float]
    obstacles: np.ndarray  # M x 4: x, y, vx, vy at t = 0
    seed: int = 0
    request_id: int = 0
    session_id: int = 0
    kappa_road: float = 0.0
    mu0: np.ndarray | None = None
    sigma0: np.ndarray | None = None
    first_iter: int = 0
    road: np.ndarray | None = None  # n x 3: kappa, y_lb, y_ub at road_x0 + i road_dx
    road_x0: float = 0.0
    road_dx: float = 1.0
    observation: np.ndarray | None = None  # PLAN_OBS_DIM values (decoder sampler)

    @property
    def M(self) -> int:
        return int(np.asarray(self.obstacles).reshape(-1, 4).shape[0])


class _Marshalled:
    """plan_request array plus the numpy buffers its pointers refer to."""

    def __init__(self, reqs: Sequence[Request]):
        self.keep = []
        self.arr = (plan_request * max(1, len(reqs)))()
        for i, r in enumerate(reqs):
            c = self.arr[i]
            c.request_id, c.session_id, c.seed = int(r.request_id), int(r.session_id), int(r.seed) & (2**64 - 1)
            c.N, c.T = int(r.N), int(r.T)
            obs = np.ascontiguousarray(np.asarray(r.obstacles, np.float64).reshape(-1, 4))
            c.M = obs.shape[0]
            c.ego = (C.c_double * 6)(*[float(v) for v in r.ego])
            self.keep.append(obs)
            c.obstacles = _pd(obs) if obs.size else None
            c.kappa_road = float(r.kappa_road)
            c.first_iter = int(r.first_iter)
            c.road_x0, c.road_dx = float(r.road_x0), float(r.road_dx)
            if r.road is not None and np.size(r.road):
                road = np.ascontiguousarray(np.asarray(r.road, np.float64).reshape(-1, 3))
                self.keep.append(road)
                c.n_road, c.road = road.shape[0], _pd(road)
            else:
                c.n_road, c.road = 0, None
            if r.mu0 is not None:
                mu = np.ascontiguousarray(np.asarray(r.mu0, np.float64).reshape(8))
                sg = np.ascontiguousarray(np.asarray(r.sigma0, np.float64).reshape(64))
                self.keep += [mu, sg]
                c.mu0, c.sigma0 = _pd(mu), _pd(sg)
            else:
                c.mu0 = c.sigma0 = None
            if r.observation is not None:
                o = np.ascontiguousarray(np.asarray(r.observation, np.float64).reshape(PLAN_OBS_DIM))
                self.keep.append(o)
                c.observation = _pd(o)
            else:
                c.observation = None


@dataclass
class Result:
    status: int
    flags: int
    best_index: int
    iterations: int
    p_best: np.ndarray
    xi_best: np.ndarray
    cost_upper: float
    residual: float
    mu: np.ndarray
    sigma: np.ndarray
    latency_s: float
    traj: np.ndarray | None = None  # T x 2 positions of the returned trajectory (FP64, from the device)


class _Results:
    """plan_result array whose traj_xy members point at T x 2 numpy
    buffers, one per request."""

    def __init__(self, Ts: Sequence[int]):
        self.arr = (plan_result * max(1, len(Ts)))()
        self.traj = []
        for i, T in enumerate(Ts):
            a = np.full((max(int(T), 1), 2), np.nan)
            self.traj.append(a)
            self.arr[i].traj_xy = _pd(a)

    def result(self, i: int) -> Result:
        r = self.arr[i]
        return Result(r.status, r.flags, r.best_index, r.iterations, np.array(r.p_best), np.array(r.xi_best),
                      r.cost_upper, r.residual, np.array(r.mu), np.array(r.sigma).reshape(8, 8), r.latency_s,
                      self.traj[i] if r.status == 0 else None)


# ----------------------------------------------------------- entry points

def plan_config_init(**over) -> plan_config:
    cfg = plan_config()
    load().plan_config_init(C.byref(cfg))
    for k, v in over.items():
        if k in ("T_set", "M_set"):
            arr = getattr(cfg, k)
            for i, x in enumerate(v):
                arr[i] = int(x)
            setattr(cfg, "n_T" if k == "T_set" else "n_M", len(v))
        elif k == "lane_c":
            cfg.lane_c = (C.c_double * 3)(*v)
        else:
            setattr(cfg, k, v)
    return cfg


def plan_workspace_bytes(cfg: plan_config) -> int:
    return int(load().plan_workspace_bytes(C.byref(cfg)))


class Handle:
    """Owner of a plan_handle (and of the workspace tensor, if any)."""

    def __init__(self, ptr, cfg, workspace=None):
        self.ptr = ptr
        self.cfg = cfg
        self.workspace = workspace

    def __del__(self):
        try:
            plan_destroy(self)
        except Exception:
            pass


def plan_create(cfg: plan_config, workspace=None, stream=None) -> Handle:
    """Create a handle. ``workspace``: optional device tensor (e.g. a torch
    uint8 CUDA tensor) used as the library's device memory; ``stream``:
    optional hipStream_t handle (int) to enqueue on."""
    if workspace is not None:
        cfg.device_workspace = C.c_void_p(int(workspace.data_ptr()))
        cfg.workspace_bytes = int(workspace.numel() * workspace.element_size())
    if stream is not None:
        cfg.stream = C.c_void_p(int(stream))
    h = C.c_void_p()
    _check(load().plan_create(C.byref(cfg), C.byref(h)), None)
    return Handle(h, cfg, workspace)


def plan_destroy(h: Handle) -> None:
    if h.ptr:
        load().plan_destroy(h.ptr)
        h.ptr = None


def plan_last_error(h: Handle | None = None) -> str:
    m = load().plan_last_error(h.ptr if h else None)
    return m.decode() if m else ""


def plan_solve_batch(h: Handle, reqs: Sequence[Request], check: bool = True) -> list[Result]:
    m = _Marshalled(reqs)
    out = _Results([r.T for r in reqs])
    st = load().plan_solve_batch(h.ptr, m.arr, len(reqs), out.arr)
    if check and st not in (PLAN_OK, PLAN_E_INVALID, PLAN_E_NOMEM):
        _check(st, h.ptr)
    return [out.result(i) for i in range(len(reqs))]


def plan_stage(h: Handle, reqs: Sequence[Request]) -> None:
    m = _Marshalled(reqs)
    h._staged_T = [r.T for r in reqs]
    _check(load().plan_stage(h.ptr, m.arr, len(reqs)), h.ptr)


def plan_launch(h: Handle) -> None:
    _check(load().plan_launch(h.ptr), h.ptr)


def plan_collect(h: Handle) -> list[Result]:
    Ts = getattr(h, "_staged_T", [])
    out = _Results(Ts)
    st = load().plan_collect(h.ptr, out.arr)
    if st not in (PLAN_OK, PLAN_E_INVALID, PLAN_E_NOMEM):
        _check(st, h.ptr)
    return [out.result(i) for i in range(len(Ts))]


def plan_lower_solve(h: Handle, req: Request, p: np.ndarray):
    """Steps 1-2 of Alg. 1 and the residual/cost for given samples p (N x 8).
    Returns (xi_bar, xi_star, resid, cost_upper)."""
    p = np.ascontiguousarray(np.asarray(p, np.float64).reshape(-1, 8))
    N = p.shape[0]
    xb, xs = np.zeros((N, NX)), np.zeros((N, NX))
    r, c = np.zeros(N), np.zeros(N)
    m = _Marshalled([req])
    _check(load().plan_lower_solve(h.ptr, m.arr, _pd(p), N, _pd(xb), _pd(xs), _pd(r), _pd(c)), h.ptr)
    return xb, xs, r, c


def plan_lower_solve_static(h: Handle, req: Request, p_ptr: int, N: int, xi_bar_ptr: int, xi_star_ptr: int,
                            resid_ptr: int, cost_ptr: int) -> None:
    """plan_lower_solve on device arrays (addresses as integers, e.g. a torch
    tensor's data_ptr(); xi pointers may both be 0), with the library's
    working memory in its static device array: allocates nothing."""
    m = _Marshalled([req])
    vp = lambda a: C.c_void_p(a) if a else None
    _check(load().plan_lower_solve_static(h.ptr, m.arr, vp(p_ptr), N, vp(xi_bar_ptr), vp(xi_star_ptr),
                                          vp(resid_ptr), vp(cost_ptr)), h.ptr)


def plan_get_trace(h: Handle, i: int, N: int, n: int, q: int) -> dict:
    L = h.cfg.upper_iters
    out = dict(p=np.zeros((L, N, 8)), r=np.zeros((L, N)), cu=np.zeros((L, N)),
               ces=np.zeros((L, n), np.int32), es=np.zeros((L, q), np.int32),
               mu=np.zeros((L, 8)), sigma=np.zeros((L, 8, 8)))
    ip = C.POINTER(C.c_int32)
    _check(load().plan_get_trace(h.ptr, i, _pd(out["p"]), _pd(out["r"]), _pd(out["cu"]),
                                 out["ces"].ctypes.data_as(ip), out["es"].ctypes.data_as(ip),
                                 _pd(out["mu"]), _pd(out["sigma"])), h.ptr)
    return out


def plan_submit(h: Handle, req: Request) -> int:
    """Queue a request for the served mode; returns its ticket."""
    m = _Marshalled([req])
    t = C.c_uint64()
    _check(load().plan_submit(h.ptr, m.arr, C.byref(t)), h.ptr)
    if not hasattr(h, "_ticket_T"):
        h._ticket_T = {}
    h._ticket_T[int(t.value)] = int(req.T)
    return int(t.value)


def plan_progress(h: Handle) -> tuple[int, int]:
    """Admit, run one upper iteration of everything resident, retire.
    Returns (resident, queued) counts."""
    a, q = C.c_int32(), C.c_int32()
    _check(load().plan_progress(h.ptr, C.byref(a), C.byref(q)), h.ptr)
    return int(a.value), int(q.value)


def plan_poll(h: Handle, ticket: int) -> Result | None:
    """The result of a finished ticket, or None while it is queued/resident."""
    T = getattr(h, "_ticket_T", {}).get(int(ticket), 1)
    out = _Results([T])
    st = load().plan_poll(h.ptr, C.c_uint64(int(ticket)), out.arr)
    if st == PLAN_E_BUSY:
        return None
    _check(st, h.ptr)
    h._ticket_T.pop(int(ticket), None)
    return out.result(0)


def plan_poll_done(h: Handle, max_n: int = 64) -> list[tuple[int, Result]]:
    """Every finished served request (up to max_n), in ticket order, as
    (ticket, Result) pairs; an empty list while none has finished."""
    Tmax = max(int(h.cfg.T_set[i]) for i in range(h.cfg.n_T))
    # one result buffer per handle, grown on demand: a served loop calls this
    # every tick, and building max_n trajectory buffers each time would cost
    # more host time than the tick itself
    buf = getattr(h, "_poll_buf", None)
    if buf is None or buf[0] < max(1, max_n):
        cap = max(1, max_n)
        buf = (cap, _Results([Tmax] * cap), (C.c_uint64 * cap)())
        h._poll_buf = buf
    _, out, tickets = buf
    n = C.c_int32()
    _check(load().plan_poll_done(h.ptr, tickets, out.arr, max_n, C.byref(n)), h.ptr)
    got = []
    for i in range(n.value):
        t = int(tickets[i])
        T = getattr(h, "_ticket_T", {}).pop(t, Tmax)
        r = out.result(i)
        if r.traj is not None:
            r.traj = r.traj[:T].copy()  # the buffer is reused by the next call
        got.append((t, r))
    return got


MPC_LOGS = ("ego", "xi", "mu", "sigma", "cost", "collided", "status")


def plan_mpc_run(h: Handle, reqs: Sequence[Request], cycles: int, n_exec: int = 5,
                 init: int = PLAN_MPC_SAMPLER, log=MPC_LOGS) -> tuple[list[Result], dict]:
    """Receding-horizon closed loop of len(reqs) episodes (see plan_mpc_run in
    include/plan.h). ``init``: PLAN_MPC_SAMPLER or PLAN_MPC_WARM. ``log``:
    names of the per-cycle logs to record (a subset of MPC_LOGS). Returns
    (results of the last cycle, {name: array})."""
    n = len(reqs)
    m = _Marshalled(reqs)
    out = _Results([r.T for r in reqs])
    shapes = dict(ego=(n, cycles + 1, 6), xi=(n, cycles, NX), mu=(n, cycles, NP), sigma=(n, cycles, NP, NP),
                  cost=(n, cycles, 2), collided=(n, cycles), status=(n, cycles))
    logs = {}
    lg = plan_mpc_log()
    for name in log:
        if name not in shapes:
            raise ValueError(f"unknown log {name!r}")
        a = np.zeros(shapes[name], np.int32 if name in ("collided", "status") else np.float64)
        logs[name] = a
        setattr(lg, name, a.ctypes.data_as(_PI if a.dtype == np.int32 else _PD))
    _check(load().plan_mpc_run(h.ptr, m.arr, n, int(cycles), int(n_exec), int(init), C.byref(lg), out.arr), h.ptr)
    return [out.result(i) for i in range(n)], logs


def plan_profile(h: Handle, enable: bool = True) -> None:
    _check(load().plan_profile(h.ptr, 1 if enable else 0), h.ptr)


def plan_profile_read(h: Handle):
    """Returns ({'lower','select','decoder'}: total ms, same: launch count)."""
    ms = (C.c_double * 3)()
    cnt = (C.c_int64 * 3)()
    _check(load().plan_profile_read(h.ptr, ms, cnt), h.ptr)
    names = ("lower", "select", "decoder")
    return {k: ms[i] for i, k in enumerate(names)}, {k: cnt[i] for i, k in enumerate(names)}


def plan_set_decoder(h: Handle, dec) -> None:
    """Load the decoder sampler's weights. ``dec`` has W, b (6 each, W out x
    in), gamma, beta, mean, var (5 each) and eps, as workload.Decoder."""
    c = plan_decoder()
    keep = []

    def arr(v):
        a = np.ascontiguousarray(np.asarray(v, np.float64))
        keep.append(a)
        return _pd(a)
    for i in range(6):
        c.W[i], c.b[i] = arr(dec.W[i]), arr(dec.b[i])
    for i in range(5):
        c.bn_gamma[i], c.bn_beta[i] = arr(dec.gamma[i]), arr(dec.beta[i])
        c.bn_mean[i], c.bn_var[i] = arr(dec.mean[i]), arr(dec.var[i])
    c.bn_eps = float(dec.eps)
    _check(load().plan_set_decoder(h.ptr, C.byref(c)), h.ptr)


def elite_sizes(cfg: plan_config, N: int) -> tuple[int, int]:
    """(n, q) of the ConstraintEliteSet / EliteSet for N samples, as the
    library sizes them."""
    n, q = C.c_int32(), C.c_int32()
    st = load().plan_elite_sizes(C.byref(cfg), int(N), C.byref(n), C.byref(q))
    if st != PLAN_OK:
        raise PlanError(st, f"elite sizes: N = {N} outside [1, max_N]")
    return int(n.value), int(q.value)
