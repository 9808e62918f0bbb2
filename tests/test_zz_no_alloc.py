"""plan_lower_solve_static (working memory in a static device array, no
allocation) against plan_lower_solve (the handle's own device memory) on the
same inputs: the same kernels on the same samples, so every output must be
bitwise equal. Three calls in a row on one handle, each smaller than the one
before (the last with a road profile, the kernel variant with the profile
lookup), in both precisions; the static array keeps the previous call's
contents, so a stale descriptor or row would show.
"""
import numpy as np
import pytest

from paper_2212_02224_amd import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pl():
    import paper_2212_02224_amd as pl
    pl.load()
    return pl


class Hip:
    """Device buffers for the test through the HIP runtime libplan.so is
    linked against (already loaded with it, so both share one runtime)."""

    def __init__(self):
        import ctypes as C
        self.C = C
        self.lib = C.CDLL("libamdhip64.so.7")
        self.lib.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        self.lib.hipFree.argtypes = [C.c_void_p]
        self.lib.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        self.bufs = []

    def alloc_from(self, a: np.ndarray) -> int:
        a = np.ascontiguousarray(a)
        ptr = self.C.c_void_p()
        assert self.lib.hipMalloc(self.C.byref(ptr), max(1, a.nbytes)) == 0
        self.bufs.append(ptr.value)
        assert self.lib.hipMemcpy(ptr.value, a.ctypes.data, a.nbytes, 1) == 0  # host to device
        return ptr.value

    def read(self, ptr: int, shape, dtype) -> np.ndarray:
        out = np.empty(shape, dtype)
        assert self.lib.hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2) == 0  # device to host
        return out

    def free(self):
        for b in self.bufs:
            self.lib.hipFree(b)
        self.bufs = []


@pytest.fixture(scope="module")
def hip(pl):
    h = Hip()
    yield h
    h.free()


def samples(N, seed):
    """Seeded behavioural inputs (lateral offsets, velocities), FP32-exact so
    both entry points see the same values."""
    rng = np.random.default_rng(seed)
    p = np.concatenate([rng.uniform(-5.0, 5.0, (N, 4)), rng.uniform(5.0, 25.0, (N, 4))], axis=1)
    return p.astype(np.float32)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_static_equals_allocating(pl, hip, precision):
    cfg = pl.plan_config_init(T_set=[50, 100], M_set=[4, 10], proj_iters=20, upper_iters=5, max_N=1000,
                              max_requests=1, precision=precision)
    h = pl.plan_create(cfg)
    cases = [(1000, 100, 10, 0, False), (300, 50, 4, 1, False), (77, 100, 10, 2, True)]
    for N, T, M, idx, road in cases:
        s = workload.scene(2, idx, M)
        kw = {}
        if road:
            rp, rx0, rdx = workload.curved_road(6, idx)
            kw = dict(road=rp, road_x0=rx0, road_dx=rdx)
        req = pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, **kw)
        p32 = samples(N, 100 + idx)
        print(f"[no-alloc] precision {precision} N={N} T={T} M={M} road={road}", flush=True)
        xb_a, xs_a, r_a, c_a = pl.plan_lower_solve(h, req, p32.astype(np.float64))
        nan22 = np.full((N, 22), np.nan)
        nan1 = np.full(N, np.nan, np.float32)
        p_d = hip.alloc_from(p32)
        xb_d, xs_d = hip.alloc_from(nan22), hip.alloc_from(nan22)
        r_d, c_d = hip.alloc_from(nan1), hip.alloc_from(nan1)
        pl.plan_lower_solve_static(h, req, p_d, N, xb_d, xs_d, r_d, c_d)
        assert np.array_equal(hip.read(xb_d, (N, 22), np.float64), xb_a)
        assert np.array_equal(hip.read(xs_d, (N, 22), np.float64), xs_a)
        r_s = hip.read(r_d, N, np.float32)
        c_s = hip.read(c_d, N, np.float32)
        assert np.array_equal(r_s.astype(np.float64), r_a)
        assert np.array_equal(c_s.astype(np.float64), c_a)
        # without the coefficient outputs
        r2, c2 = hip.alloc_from(nan1), hip.alloc_from(nan1)
        pl.plan_lower_solve_static(h, req, p_d, N, 0, 0, r2, c2)
        assert np.array_equal(hip.read(r2, N, np.float32), r_s)
        assert np.array_equal(hip.read(c2, N, np.float32), c_s)
    pl.plan_destroy(h)


def test_static_rejects_bad_calls(pl, hip):
    cfg = pl.plan_config_init(T_set=[50], M_set=[4], proj_iters=5, upper_iters=1, max_N=64, max_requests=1)
    h = pl.plan_create(cfg)
    s = workload.scene(1, 0, 4)
    ptr = hip.alloc_from(np.zeros(128 * 22))
    for N, xb, xs, st in ((65, ptr, ptr, pl.PLAN_E_INVALID),   # beyond max_N
                          (0, ptr, ptr, pl.PLAN_E_INVALID),    # empty
                          (8, ptr, 0, pl.PLAN_E_INVALID)):     # one coefficient output only
        req = pl.Request(N=max(N, 1), T=50, ego=s.ego, obstacles=s.obstacles, seed=s.seed)
        with pytest.raises(pl.PlanError) as ei:
            pl.plan_lower_solve_static(h, req, ptr, N, xb, xs, ptr, ptr)
        assert ei.value.status == st
    pl.plan_destroy(h)
