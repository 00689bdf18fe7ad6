// Heterogeneous batches: plans, the task list of the persistent kernel,
// hipGraph capture, and the schedule autotuner.
#pragma once
#include "hk_plan.hpp"

namespace hk {

Status plan_create(hk_plan_t *plan, hk_dtype_t dt, const hk_problem_t *probs, int64_t count, unsigned flags);
Status plan_ws_size(hk_plan_t plan, size_t *bytes);
Status plan_execute(hk_plan_t plan, void *ws, size_t ws_bytes, hipStream_t st);
Status plan_status(hk_plan_t plan);
Status plan_destroy(hk_plan_t plan);
Status plan_set_wait_bound(hk_plan_t plan, uint32_t spins);
Status plan_pass_bytes(hk_plan_t plan, int64_t *bytes);
Status plan_tune_times(hk_plan_t plan, double *ms_default, double *ms_tuned, uint32_t *pow2_buckets);
// One-shot execution keeps the descriptor tables in the caller's workspace
// (no plan-owned device memory).
Status plan_set_oneshot(hk_plan_t plan);
// Waits for the stream, then frees a one-shot plan.
Status plan_release_after(hk_plan_t plan, hipStream_t st);

// Times the candidate schedules of one shape and stores the winner in the
// schedule cache.  kind 0: forward 1D equal vectors (m, n); 1: adjoint 1D;
// 2: forward BHHB equal vectors (inner/blocks); batch = instances per call.
Status autotune_tvp(hk_dtype_t dt, int m, int64_t n, bool verbose);
Status autotune_shape(hk_dtype_t dt, int kind, int m, int64_t n, const int64_t *inner, const int64_t *blocks,
                      int64_t batch, bool verbose);

}  // namespace hk
