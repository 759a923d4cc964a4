// Schedule autotuner. The paper tunes tile and block sizes by an exhaustive
// sweep per kernel and platform (Section IV-C, Table 1) and does not report
// the depth of a time tile; here every valid schedule of the library is timed
// on the device for a model — acoustic: (time_tile, tile_y, chunk_x and the
// resident workgroups per compute unit); TTI and elastic: (time_tile, slab
// width) — and the fastest is cached per (physics, space order, grid shape).
// A NULL schedule then resolves to the cached choice. All candidates give
// bit-identical results, so tuning changes speed only.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "plan.h"

namespace tbw {
namespace {

using TuneKey = std::tuple<int, int, int, int, int>;  // physics, so, nx, ny, nz
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<SchedChoice, double>> g_tuned;

TuneKey key_of(const tb_model *m) { return {m->physics, m->so, m->n[0], m->n[1], m->n[2]}; }

}  // namespace

bool tuned_schedule(const tb_model *m, SchedChoice *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key_of(m));
    if (it == g_tuned.end()) return false;
    *out = it->second.first;
    return true;
}

}  // namespace tbw

using namespace tbw;

namespace {

struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

struct Ev {
    hipEvent_t e = nullptr;
    ~Ev()
    {
        if (e) (void)hipEventDestroy(e);
    }
};

void store(const tb_model *m, const SchedChoice &c, double ms, tb_schedule *best,
           double *ms_per_step)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[key_of(m)] = {c, ms};
    }
    if (best) {
        best->mode = c.T == 1 ? TB_SCHED_SB : TB_SCHED_TB;
        best->time_tile = c.T;
        best->tile_y = c.tile_y;
        best->chunk_x = c.chunk;
    }
    if (ms_per_step) *ms_per_step = ms;
}

// TTI and elastic: depth 1..3 and slab widths of 16, 32 and 64 planes.
tb_status tune_slabs(const tb_model *m, tb_sparse *s, int steps, hipStream_t st,
                     tb_schedule *best, double *ms_per_step)
{
    std::vector<SchedChoice> cands;
    for (int T = 1; T <= 3; T++)
        for (int w : {16, 32, 64}) {
            if (T == 1 && w != 16) continue;
            tb_schedule c{T == 1 ? TB_SCHED_SB : TB_SCHED_TB, T, 0, T == 1 ? 0 : w};
            SchedChoice sc;
            if (resolve_schedule(m, &c, &sc) == TB_OK) cands.push_back(sc);
        }
    size_t need = 0;
    for (const SchedChoice &c : cands) need = std::max(need, forward_ws_bytes(m, s, c));
    DevBuf buf;
    TB_HIP(hipMalloc(&buf.p, need));
    Ev e0, e1;
    TB_HIP(hipEventCreate(&e0.e));
    TB_HIP(hipEventCreate(&e1.e));
    SchedChoice bestc{};
    double best_ms = INFINITY;
    for (const SchedChoice &c : cands) {
        Plan plan;
        tb_status rc = plan_forward_steps(m, s, c, buf.p, steps, &plan);
        if (rc) return rc;
        float ms = 0.0f;
        for (int rep = 0; rep < 2; rep++) {
            TB_HIP(hipEventRecord(e0.e, st));
            if ((rc = run_plan(m, s, c, plan, st))) return rc;
            TB_HIP(hipEventRecord(e1.e, st));
            TB_HIP(hipEventSynchronize(e1.e));
            TB_HIP(hipEventElapsedTime(&ms, e0.e, e1.e));
        }
        if (ms / steps < best_ms) {
            best_ms = ms / steps;
            bestc = c;
        }
    }
    if (!std::isfinite(best_ms)) {
        set_error("tb_autotune: no schedule ran");
        return TB_EUNSUPPORTED;
    }
    store(m, bestc, best_ms, best, ms_per_step);
    return TB_OK;
}

}  // namespace

extern "C" {

tb_status tb_autotune(const tb_model *m, const tb_sparse *s_, int32_t steps, void *stream,
                      tb_schedule *best, double *ms_per_step)
{
    tb_sparse *s = const_cast<tb_sparse *>(s_);
    if (!m || !s || s->m != m || steps < 1) {
        set_error("tb_autotune: invalid argument");
        return TB_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    steps = std::min<int32_t>(steps, std::max(m->nt, 1));
    if (m->physics != TB_ACOUSTIC) return tune_slabs(m, s, steps, st, best, ms_per_step);
    const size_t fb = (m->field_elems() * sizeof(float) + 255) & ~(size_t)255;
    const size_t recb = ((size_t)m->nt + 1) * std::max(s->nrid, 1) * sizeof(float);
    DevBuf buf;
    TB_HIP(hipMalloc(&buf.p, 4 * fb + recb));
    char *base = (char *)buf.p;
    float *F[4] = {(float *)base, (float *)(base + fb), (float *)(base + 2 * fb),
                   (float *)(base + 3 * fb)};
    float *rec = (float *)(base + 4 * fb);
    Ev e0, e1;
    TB_HIP(hipEventCreate(&e0.e));
    TB_HIP(hipEventCreate(&e1.e));

    const int Tmax = m->r >= 4 ? 3 : 4;
    const int tiles[3] = {32, 16, 0};
    const int chunks[5] = {0, 32, 64, 128, kMaxChunk};
    // Resident workgroups per compute unit of the even (tile, x) partition
    // (chunk 0); the chunked and whole-x schedules keep one per unit.
    const int wgs_axis[3] = {1, 2, 3};
    SchedChoice bestc{};
    double best_ms = INFINITY;
    for (int T = 1; T <= Tmax; T++)
        for (int ty : tiles)
            for (int ch : chunks)
                for (int wpc : wgs_axis) {
                    if (ch != 0 && wpc != 2) continue;
                    tb_schedule cand{T == 1 ? TB_SCHED_SB : TB_SCHED_TB, T, ty, ch};
                    SchedChoice sc;
                    if (resolve_schedule(m, &cand, &sc) != TB_OK) continue;
                    sc.wgs_per_cu = wpc;
                    // One warm-up run (builds the lists), then the timed run.
                    double ms = 0.0;
                    bool ok = true;
                    for (int rep = 0; rep < 2 && ok; rep++) {
                        Plan plan;
                        int ua = 0, va = 0;
                        const size_t fe = m->field_elems();
                        tb_status rc = launch_fill(F[0], fe, 0.0f, st);
                        if (!rc) rc = launch_fill(F[2], fe, 0.0f, st);
                        if (rc) return rc;
                        // Passes of `steps` updates from zero state (u in F[0..1],
                        // v in F[2..3]).
                        int n = 0;
                        while (n < steps) {
                            const int Tp = std::min(sc.T, steps - n);
                            Item it;
                            it.is_pass = true;
                            it.pass.T = Tp;
                            it.pass.u = F[ua];
                            it.pass.v = F[2 + va];
                            it.pass.out_u = F[1 - ua];
                            it.pass.out_v = F[3 - va];
                            it.pass.n0 = n;
                            it.pass.dcmp = s->d_dcmp;
                            it.pass.ninj = s->npts;
                            it.pass.rec = rec;
                            it.pass.nrecp = s->nrid;
                            plan.push_back(it);
                            ua = 1 - ua;
                            va = 1 - va;
                            n += Tp;
                        }
                        TB_HIP(hipEventRecord(e0.e, st));
                        rc = run_plan(m, s, sc, plan, st);
                        if (rc == TB_EUNSUPPORTED) {  // lists beyond capacity: skip
                            ok = false;
                            break;
                        }
                        if (rc) return rc;
                        TB_HIP(hipEventRecord(e1.e, st));
                        TB_HIP(hipEventSynchronize(e1.e));
                        float t = 0.0f;
                        TB_HIP(hipEventElapsedTime(&t, e0.e, e1.e));
                        ms = t;
                    }
                    if (!ok) continue;
                    const double per = ms / steps;
                    if (per < best_ms) {
                        best_ms = per;
                        bestc = sc;
                    }
                }
    if (!std::isfinite(best_ms)) {
        set_error("tb_autotune: no schedule ran");
        return TB_EUNSUPPORTED;
    }
    store(m, bestc, best_ms, best, ms_per_step);
    return TB_OK;
}

tb_status tb_autotune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
    return TB_OK;
}

}  // extern "C"
