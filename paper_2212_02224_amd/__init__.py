"""MI355X batched bi-level trajectory planner (arXiv 2212.02224 hot path).

The planner runs as HIP kernels in ``libplan.so`` behind the C ABI of
``include/plan.h``; ``binding`` is its ctypes binding (same names), and
``workload`` builds seeded synthetic scenes.
"""
from .binding import (PLAN_BEHAV_GOALS, PLAN_BEHAV_SETPOINTS, PLAN_SAMPLER_GRID,  # noqa: F401
                      PLAN_SAMPLER_DECODER, PLAN_OBS_DIM, PLAN_SAMPLER_RANDOM, PLAN_E_BUSY, PLAN_E_DEVICE, PLAN_E_INVALID, PLAN_E_NOMEM,
                      PLAN_E_TIMEOUT, PLAN_E_UNSUPPORTED, PLAN_F_INFEASIBLE, PLAN_F_WARM, PLAN_MPC_SAMPLER,
                      PLAN_MAX_ROAD, PLAN_MPC_WARM, PLAN_OK,
                      PLAN_PREC_FP16_SPLIT, PLAN_PREC_FP32, PLAN_PREC_FP32_MFMA, Handle,
                      PlanError, Request, Result, elite_sizes, exported_symbols, load,
                      plan_collect, plan_config_init, plan_create, plan_destroy,
                      MPC_LOGS, plan_get_trace, plan_last_error, plan_launch, plan_lower_solve,
                      plan_lower_solve_static,
                      plan_mpc_run,
                      plan_poll, plan_poll_done, plan_progress, plan_submit,
                      plan_profile, plan_profile_read, plan_set_decoder, plan_solve_batch, plan_stage,
                      plan_workspace_bytes)
