"""CPU checks of the HIP library's host side: the shared library loads, it
exports every function include/plan.h declares, the binding's structs match
the header's layout, and configuration validation rejects bad input before
any device call. No kernel runs here."""
import ctypes as C
import os
import re

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pl():
    import paper_2212_02224_amd as pl
    try:
        pl.load()
    except ImportError:
        pytest.skip("libplan.so not built (run __graft_entry__.build())")
    return pl


def header_functions():
    src = open(os.path.join(ROOT, "include", "plan.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(plan_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(pl):
    lib = pl.load()
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(pl.exported_symbols()) <= set(names)


def test_struct_layout_matches_header(pl):
    # sizes the C compiler gives the header's structs (built into a probe)
    import subprocess
    import tempfile
    probe = r'''
#include <stdio.h>
#include <stddef.h>
#include "plan.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(plan_config), sizeof(plan_request),
         sizeof(plan_result), offsetof(plan_config, stream), offsetof(plan_request, first_iter),
         offsetof(plan_result, latency_s), sizeof(plan_mpc_log), offsetof(plan_mpc_log, status),
         offsetof(plan_request, road), offsetof(plan_request, observation), sizeof(plan_decoder),
         offsetof(plan_decoder, bn_eps), offsetof(plan_result, traj_xy));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        open(c, "w").write(probe)
        exe = os.path.join(d, "probe")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    got = [int(x) for x in out]
    b = pl.binding
    want = [C.sizeof(b.plan_config), C.sizeof(b.plan_request), C.sizeof(b.plan_result),
            b.plan_config.stream.offset, b.plan_request.first_iter.offset, b.plan_result.latency_s.offset,
            C.sizeof(b.plan_mpc_log), b.plan_mpc_log.status.offset, b.plan_request.road.offset,
            b.plan_request.observation.offset, C.sizeof(b.plan_decoder), b.plan_decoder.bn_eps.offset,
            b.plan_result.traj_xy.offset]
    assert got == want


def test_config_defaults_and_workspace(pl):
    cfg = pl.plan_config_init()
    assert cfg.proj_iters == 20 and cfg.upper_iters == 5 and abs(cfg.gamma - 0.9) < 1e-15
    assert list(cfg.T_set[:cfg.n_T]) == [50, 100] and list(cfg.M_set[:cfg.n_M]) == [4, 10, 20]
    small = pl.plan_workspace_bytes(cfg)
    big = pl.plan_workspace_bytes(pl.plan_config_init(max_requests=64, max_N=4096))
    assert 0 < small < big


@pytest.mark.parametrize("over", [dict(max_N=0), dict(max_N=5000), dict(T_set=[8]), dict(M_set=[40]),
                                  dict(upper_iters=0), dict(gamma=0.0), dict(y_lb=3.0, y_ub=-3.0),
                                  dict(frac_ces=0.01, frac_es=0.05), dict(precision=7), dict(precision=3),
                                  dict(precision=1, T_set=[50, 200]), dict(precision=2, T_set=[50, 200]),
                                  dict(behaviour=2), dict(sampler=3),
                                  dict(behaviour=1, w_s=0.0), dict(served_run_ahead=4),
                                  dict(served_run_ahead=-1), dict(fused_iters=2), dict(fused_iters=-1),
                                  dict(fused_iters=1, fused_wait_us=0)])
def test_invalid_config_rejected_before_device(pl, over):
    cfg = pl.plan_config_init(**over)
    assert pl.plan_workspace_bytes(cfg) == 0
    with pytest.raises(pl.PlanError) as e:
        pl.plan_create(cfg)
    assert e.value.status == pl.PLAN_E_INVALID


def test_fp16_split_config_accepted(pl):
    """The matrix-core mode adds its FP16 tables to the workspace."""
    base = pl.plan_workspace_bytes(pl.plan_config_init())
    mixed = pl.plan_workspace_bytes(pl.plan_config_init(precision=pl.PLAN_PREC_FP16_SPLIT))
    # per T: 4 ceil(T/4) instants x 224 bytes; per (T, M): 1 KiB (A^-1 halves)
    tables = sum(4 * ((T + 3) // 4) * 224 for T in (50, 100)) + 2 * 3 * 1024
    assert mixed - base >= tables
    assert pl.plan_workspace_bytes(pl.plan_config_init(precision=1, T_set=[128])) > 0


def test_elite_sizes_match_oracle(pl, orc):
    """The library's sizes (plan_elite_sizes, no device needed) against the
    oracle's, and its argument checks."""
    cfg = pl.plan_config_init(max_N=4096)
    par = orc.default_params()
    for N in (1, 5, 64, 256, 512, 1000, 2048, 4096, 333):
        assert pl.elite_sizes(cfg, N) == orc.elite_sizes(par, N)
    for N in (0, 4097):
        with pytest.raises(pl.PlanError):
            pl.elite_sizes(cfg, N)


def test_workload_scenes_are_seeded(pl):
    from paper_2212_02224_amd import workload
    a, b = workload.scene(2, 5, 10), workload.scene(2, 5, 10)
    assert (a.ego == b.ego).all() and (a.obstacles == b.obstacles).all() and a.seed == b.seed
    assert a.obstacles.shape == (10, 4)


def test_curved_road_profile_is_seeded_and_valid(pl):
    from paper_2212_02224_amd import workload
    a, b = workload.curved_road(6, 3), workload.curved_road(6, 3)
    assert np.array_equal(a[0], b[0]) and a[1:] == b[1:]
    road, x0, dx = a
    assert road.shape == (17, 3) and dx > 0
    assert np.all(road[:, 1] < road[:, 2]) and np.abs(road[:, 0]).max() <= 0.02
    bends = [np.abs(workload.curved_road(6, i)[0][:, 0]).max() for i in range(20)]
    assert min(bends) >= 0.01  # every profile has a bend of radius 50..100 m


def test_decoder_inputs_are_seeded_and_shaped(pl):
    from paper_2212_02224_amd import workload
    s = workload.scene(2, 4, 10)
    o = workload.observation(s)
    assert o.shape == (55,) and np.array_equal(o, workload.observation(s))
    # nearest neighbour first; a scene with fewer than 10 neighbours pads
    d = np.hypot(o[3:43:4] * 50.0, o[4:43:4] * 7.0)
    assert np.all(np.diff(d) >= -1e-12)
    few = workload.observation(workload.scene(1, 0, 4))
    assert np.all(few[3 + 16:43:4] == 4.0)
    a, b = workload.decoder_weights(2), workload.decoder_weights(2)
    assert all(np.array_equal(x, y) for x, y in zip(a.W, b.W))
    assert [w.shape for w in a.W] == [(1024, 57), (1024, 1024), (1024, 1024), (1024, 1024), (256, 1024), (8, 256)]
