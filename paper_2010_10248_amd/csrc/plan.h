// Work plans: the forward run and the gradient as ordered lists of
// propagation passes (one wave-front launch of T steps of one job) and side
// actions (copies, trace reduction, residual, imaging). tb_forward and
// tb_gradient execute a plan in order on one stream; the serving runtime
// interleaves the plans of several jobs, batching the passes of a round into
// one launch. Both issue the same per-job computations, so a job's results
// are the same alone and in a mix.
#pragma once

#include <functional>
#include <vector>

#include "acoustic_params.h"
#include "tb_internal.h"

namespace tbw {

struct SchedChoice {
    int T, tile_y, chunk, wgs_per_cu;
};

// Resolve a caller schedule (NULL: the tuned choice for the model if one is
// cached, else the default).
tb_status resolve_schedule(const tb_model *m, const tb_schedule *s, SchedChoice *out);

// Per-segment lists of the schedule, within the kernel's LDS capacities.
tb_status lists_for(const tb_model *m, tb_sparse *s, int adjoint, const SchedChoice &sc, int T,
                    TileLists **out);

// One wave-front launch of T updates of one job: from (u = u^{n0},
// v = u^{n0} - u^{n0-1}) to out_u = u^{n0+T}, out_v = v^{n0+T} and, if
// out_mid is set and T > 1, out_mid = u^{n0+T-1}.
struct Pass {
    int adjoint = 0, T = 1;
    const float *u = nullptr, *v = nullptr;
    float *out_u = nullptr, *out_v = nullptr, *out_mid = nullptr;
    int n0 = 0;
    const float *dcmp = nullptr;
    int ninj = 0;
    float *rec = nullptr;
    int nrecp = 0;
};

struct Item {
    bool is_pass = false;
    Pass pass;
    std::function<tb_status(hipStream_t)> act;
};
using Plan = std::vector<Item>;

// Kernel parameters of a pass (lists resolved for the job's schedule); *gl
// is set when a segment's lists exceed the LDS capacities (the pass then
// needs the global-list kernel and cannot join a batched launch).
tb_status pass_params(const tb_model *m, tb_sparse *s, const SchedChoice &sc, const Pass &p,
                      AcParams *out, const TileGeom **geom, bool *gl);

size_t forward_ws_bytes(const tb_model *m, const tb_sparse *s, const SchedChoice &sc);
size_t gradient_ws_bytes(const tb_model *m, const tb_sparse *s, const SchedChoice &sc, int every);

tb_status plan_forward(const tb_model *m, tb_sparse *s, const SchedChoice &sc, void *ws,
                       float *rec_out, float *field_out, float *field_prev_out, Plan *plan);
// The first nsteps updates of a TTI or elastic forward (no outputs), for
// timing schedules.
tb_status plan_forward_steps(const tb_model *m, tb_sparse *s, const SchedChoice &sc, void *ws,
                             int nsteps, Plan *plan);
// loss_dst: host memory that receives J by an asynchronous copy (NULL: none).
tb_status plan_gradient(const tb_model *m, tb_sparse *s, const SchedChoice &sc, int every,
                        void *ws, const float *d_obs, float *grad_m, double *loss_dst,
                        Plan *plan);
tb_status run_plan(const tb_model *m, tb_sparse *s, const SchedChoice &sc, const Plan &plan,
                   hipStream_t st);
// True when the per-segment lists of every pass of the plan are already
// cached in the sparse handle (running the plan then allocates nothing).
bool plan_lists_cached(const tb_model *m, tb_sparse *s, const SchedChoice &sc, const Plan &plan);

// Tuned schedules (tb_autotune), keyed by physics, space order and shape.
bool tuned_schedule(const tb_model *m, SchedChoice *out);

}  // namespace tbw
