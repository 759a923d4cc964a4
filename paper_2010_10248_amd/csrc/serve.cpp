// Serving runtime: continuous batching of shots (forward runs or checkpointed
// gradients) on one device.
//
// * Admission: requests queue in arrival order; the head is admitted when a
//   slot is free and its workspace fits in the server's device arena
//   (first-fit with coalescing), so shots of different grid sizes share HBM
//   by footprint. Models, sparse operators and wavefields stay resident.
// * Execution: every job is a plan (propagation passes and side actions, the
//   same plan tb_forward / tb_gradient run alone). A step runs the pending
//   side actions of every job, then an epoch of up to kMaxRounds rounds: in
//   each round every active job advances by one pass, and the passes that
//   share a kernel shape go into one batched launch. Parameters live in a
//   device table refreshed by one copy per epoch, so an epoch of the same
//   structure is captured once as a hipGraph and replayed.
// * Everything runs in order on the server's stream, so a job's arena region
//   can be handed to the next job as soon as its last item is enqueued, and a
//   job's arithmetic is exactly that of a run alone.
#include <algorithm>
#include <deque>
#include <map>
#include <memory>
#include <vector>

#include "plan.h"

using namespace tbw;

namespace {

constexpr int kMaxRounds = 8;  // passes per job per epoch

struct Job {
    int64_t id = 0;
    tb_request rq{};
    SchedChoice sc{};
    Plan plan;
    size_t pos = 0;
    size_t ws_off = 0, ws_bytes = 0;
    double *loss = nullptr;  // pinned host
    hipEvent_t done = nullptr;
    ~Job()
    {
        if (loss) (void)hipHostFree(loss);
        if (done) (void)hipEventDestroy(done);
    }
};

// First-fit arena with coalescing of free neighbours.
struct Arena {
    size_t bytes = 0;
    std::map<size_t, size_t> free_;  // offset -> size
    void init(size_t b)
    {
        bytes = b;
        free_.clear();
        free_[0] = b;
    }
    bool alloc(size_t need, size_t *off)
    {
        need = (need + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                *off = it->first;
                const size_t rest = it->second - need;
                const size_t at = it->first + need;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t size)
    {
        size = (size + 255) & ~(size_t)255;
        auto it = free_.emplace(off, size).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// One batched launch of an epoch (offsets into the parameter tables).
struct LaunchRec {
    int r, T, LZ, BYE, njobs, total_wg;
    int poff, woff;
    int round = 0;
};

}  // namespace

struct tb_server {
    int device = 0;
    hipStream_t st = nullptr;
    int max_active = 1;
    int flags = 0;
    void *arena_mem = nullptr;
    Arena arena;
    int64_t next_id = 1;
    std::deque<std::unique_ptr<Job>> queue;
    std::vector<std::unique_ptr<Job>> active, retiring;
    struct Done {
        int64_t id;
        double loss;
    };
    std::vector<Done> done;
    // Parameter tables (pinned staging and device copies).
    int cap = 0;
    AcParams *h_par = nullptr, *d_par = nullptr;
    int *h_wg = nullptr, *d_wg = nullptr;
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
    std::map<std::vector<int>, hipGraphExec_t> graphs;
    int64_t stats[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    ~tb_server()
    {
        if (st) (void)hipStreamSynchronize(st);
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
        if (staged) (void)hipEventDestroy(staged);
        if (h_par) (void)hipHostFree(h_par);
        if (h_wg) (void)hipHostFree(h_wg);
        if (d_par) (void)hipFree(d_par);
        if (d_wg) (void)hipFree(d_wg);
        if (arena_mem) (void)hipFree(arena_mem);
        queue.clear();
        active.clear();
        retiring.clear();
        if (st) (void)hipStreamDestroy(st);
    }
};

namespace {

// Statistics slots (tb_server_stats).
enum { kEpochs, kRounds, kLaunches, kPassesBatched, kGraphCaptures, kGraphReplays, kActions,
       kCompleted };

tb_status admit(tb_server *sv)
{
    while (!sv->queue.empty() && (int)sv->active.size() < sv->max_active) {
        Job &j = *sv->queue.front();
        size_t off = 0;
        if (!sv->arena.alloc(j.ws_bytes, &off)) break;  // in order: wait for memory
        j.ws_off = off;
        void *ws = (char *)sv->arena_mem + off;
        tb_sparse *s = const_cast<tb_sparse *>(j.rq.sparse);
        tb_status rc = j.rq.op == TB_OP_FORWARD
                           ? plan_forward(j.rq.model, s, j.sc, ws, j.rq.rec_out, nullptr, nullptr,
                                          &j.plan)
                           : plan_gradient(j.rq.model, s, j.sc, j.rq.checkpoint_every, ws,
                                           j.rq.d_obs, j.rq.grad_out, j.loss, &j.plan);
        if (rc) {
            sv->arena.release(off, j.ws_bytes);
            return rc;
        }
        sv->active.push_back(std::move(sv->queue.front()));
        sv->queue.pop_front();
    }
    return TB_OK;
}

// Run side actions at the head of every job's plan; retire finished jobs.
tb_status run_actions(tb_server *sv)
{
    for (size_t i = 0; i < sv->active.size();) {
        Job &j = *sv->active[i];
        while (j.pos < j.plan.size() && !j.plan[j.pos].is_pass) {
            tb_status rc = j.plan[j.pos].act(sv->st);
            if (rc) return rc;
            j.pos++;
            sv->stats[kActions]++;
        }
        if (j.pos == j.plan.size()) {
            TB_HIP(hipEventRecord(j.done, sv->st));
            sv->arena.release(j.ws_off, j.ws_bytes);
            sv->retiring.push_back(std::move(sv->active[i]));
            sv->active.erase(sv->active.begin() + i);
        } else {
            i++;
        }
    }
    return TB_OK;
}

tb_status collect(tb_server *sv)
{
    for (size_t i = 0; i < sv->retiring.size();) {
        hipError_t e = hipEventQuery(sv->retiring[i]->done);
        if (e == hipSuccess) {
            Job &j = *sv->retiring[i];
            sv->done.push_back({j.id, j.rq.op == TB_OP_GRADIENT ? *j.loss : 0.0});
            sv->stats[kCompleted]++;
            sv->retiring.erase(sv->retiring.begin() + i);
        } else if (e == hipErrorNotReady) {
            i++;
        } else {
            TB_HIP(e);
        }
    }
    return TB_OK;
}

tb_status ensure_tables(tb_server *sv, int need)
{
    if (need <= sv->cap) return TB_OK;
    // Grow (rare): wait for the device to finish with the old tables.
    TB_HIP(hipStreamSynchronize(sv->st));
    for (auto &g : sv->graphs) (void)hipGraphExecDestroy(g.second);
    sv->graphs.clear();
    if (sv->h_par) (void)hipHostFree(sv->h_par);
    if (sv->h_wg) (void)hipHostFree(sv->h_wg);
    if (sv->d_par) (void)hipFree(sv->d_par);
    if (sv->d_wg) (void)hipFree(sv->d_wg);
    sv->h_par = nullptr;
    sv->h_wg = nullptr;
    sv->d_par = nullptr;
    sv->d_wg = nullptr;
    int cap = std::max(need, 64);
    TB_HIP(hipHostMalloc((void **)&sv->h_par, cap * sizeof(AcParams), hipHostMallocDefault));
    TB_HIP(hipHostMalloc((void **)&sv->h_wg, cap * sizeof(int), hipHostMallocDefault));
    TB_HIP(hipMalloc((void **)&sv->d_par, cap * sizeof(AcParams)));
    TB_HIP(hipMalloc((void **)&sv->d_wg, cap * sizeof(int)));
    sv->cap = cap;
    sv->staged_pending = false;
    return TB_OK;
}

tb_status issue(tb_server *sv, const std::vector<LaunchRec> &L,
                 const std::vector<std::vector<std::pair<Job *, Pass>>> &singles, bool timing)
{
    size_t k = 0;
    for (size_t round = 0; round < singles.size(); round++) {
        for (; k < L.size() && L[k].round == (int)round; k++) {
            const LaunchRec &l = L[k];
            tb_status rc = launch_acoustic_batch(l.r, sv->d_par + l.poff, sv->d_wg + l.woff,
                                                 l.njobs, l.total_wg, l.T, l.LZ, l.BYE, sv->st,
                                                 timing);
            if (rc) return rc;
        }
        for (const auto &jp : singles[round]) {
            Plan one;
            Item it;
            it.is_pass = true;
            it.pass = jp.second;
            one.push_back(it);
            tb_sparse *s = const_cast<tb_sparse *>(jp.first->rq.sparse);
            tb_status rc = run_plan(jp.first->rq.model, s, jp.first->sc, one, sv->st);
            if (rc) return rc;
        }
    }
    return TB_OK;
}

tb_status epoch(tb_server *sv)
{
    if (sv->active.empty()) return TB_OK;
    int P = kMaxRounds;
    for (auto &jp : sv->active) {
        Job &j = *jp;
        int k = 0;
        while (k < P && j.pos + k < j.plan.size() && j.plan[j.pos + k].is_pass) k++;
        P = std::min(P, k);
    }
    if (P == 0) return TB_OK;
    // The host may rewrite the staging tables once the previous epoch's copy
    // has executed (it runs behind the work already on the stream).
    if (sv->staged_pending) {
        TB_HIP(hipEventSynchronize(sv->staged));
        sv->staged_pending = false;
    }
    tb_status rc = ensure_tables(sv, P * (int)sv->active.size());
    if (rc) return rc;
    struct Entry {
        int r, T, LZ, BYE;
        AcParams p;
    };
    std::vector<LaunchRec> L;
    std::vector<int> key;
    // Passes whose lists exceed the LDS capacities run as launches of their
    // own (the global-list kernel), after the batched launches of the round.
    std::vector<std::vector<std::pair<Job *, Pass>>> singles(P);
    int np = 0;
    for (int round = 0; round < P; round++) {
        std::vector<Entry> ents;
        for (auto &jp : sv->active) {
            Job &j = *jp;
            const Pass &ps = j.plan[j.pos + round].pass;
            Entry e;
            const TileGeom *g = nullptr;
            bool gl = false;
            tb_sparse *s = const_cast<tb_sparse *>(j.rq.sparse);
            if ((rc = pass_params(j.rq.model, s, j.sc, ps, &e.p, &g, &gl))) return rc;
            if (gl) {
                singles[round].push_back({&j, ps});
                continue;
            }
            e.r = j.rq.model->r;
            e.T = g->T;
            e.LZ = g->LZ;
            e.BYE = g->BYE;
            ents.push_back(e);
        }
        std::stable_sort(ents.begin(), ents.end(), [](const Entry &a, const Entry &b) {
            return std::make_tuple(a.r, a.T, a.LZ, a.BYE) < std::make_tuple(b.r, b.T, b.LZ, b.BYE);
        });
        for (size_t a = 0; a < ents.size();) {
            size_t b = a;
            LaunchRec l{ents[a].r, ents[a].T, ents[a].LZ, ents[a].BYE, 0, 0, np, np};
            int wg = 0;
            while (b < ents.size() && ents[b].r == l.r && ents[b].T == l.T &&
                   ents[b].LZ == l.LZ && ents[b].BYE == l.BYE) {
                sv->h_par[np] = ents[b].p;
                sv->h_wg[np] = wg;
                wg += (ents[b].p.nwg + 7) & ~7;
                np++;
                b++;
            }
            l.njobs = (int)(b - a);
            l.total_wg = wg;
            l.round = round;
            L.push_back(l);
            for (int v : {l.r, l.T, l.LZ, l.BYE, l.njobs, l.total_wg, l.poff}) key.push_back(v);
            sv->stats[kPassesBatched] += l.njobs;
            a = b;
        }
    }
    bool any_single = false;
    for (auto &v : singles) any_single |= !v.empty();
    TB_HIP(hipMemcpyAsync(sv->d_par, sv->h_par, np * sizeof(AcParams), hipMemcpyHostToDevice,
                          sv->st));
    TB_HIP(hipMemcpyAsync(sv->d_wg, sv->h_wg, np * sizeof(int), hipMemcpyHostToDevice, sv->st));
    TB_HIP(hipEventRecord(sv->staged, sv->st));
    sv->staged_pending = true;
    if ((sv->flags & TB_SERVE_GRAPHS) && !any_single) {
        auto it = sv->graphs.find(key);
        if (it == sv->graphs.end()) {
            hipGraph_t graph = nullptr;
            TB_HIP(hipStreamBeginCapture(sv->st, hipStreamCaptureModeThreadLocal));
            rc = issue(sv, L, singles, false);
            hipError_t e = hipStreamEndCapture(sv->st, &graph);
            if (rc) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            TB_HIP(e);
            hipGraphExec_t exec = nullptr;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            TB_HIP(e);
            it = sv->graphs.emplace(key, exec).first;
            sv->stats[kGraphCaptures]++;
        }
        TB_HIP(hipGraphLaunch(it->second, sv->st));
        sv->stats[kGraphReplays]++;
    } else {
        if ((rc = issue(sv, L, singles, true))) return rc;
    }
    for (auto &jp : sv->active) jp->pos += P;
    sv->stats[kLaunches] += (int64_t)L.size();
    for (auto &v : singles) sv->stats[kLaunches] += (int64_t)v.size();
    sv->stats[kEpochs]++;
    sv->stats[kRounds] += P;
    return TB_OK;
}

}  // namespace

extern "C" {

tb_status tb_server_create(size_t arena_bytes, int32_t max_active, int32_t flags,
                           tb_server **out)
{
    if (!out || max_active < 1 || arena_bytes == 0) {
        set_error("tb_server_create: invalid argument");
        return TB_EINVAL;
    }
    *out = nullptr;
    auto sv = std::make_unique<tb_server>();
    TB_HIP(hipGetDevice(&sv->device));
    TB_HIP(hipStreamCreateWithFlags(&sv->st, hipStreamNonBlocking));
    TB_HIP(hipEventCreateWithFlags(&sv->staged, hipEventDisableTiming));
    hipError_t e = hipMalloc(&sv->arena_mem, arena_bytes);
    if (e != hipSuccess) {
        set_error("arena of %zu bytes: %s", arena_bytes, hipGetErrorString(e));
        return TB_ENOMEM;
    }
    sv->arena.init(arena_bytes);
    sv->max_active = max_active;
    sv->flags = flags;
    *out = sv.release();
    return TB_OK;
}

tb_status tb_server_submit(tb_server *sv, const tb_request *rq, int64_t *id)
{
    if (!sv || !rq || !rq->model || !rq->sparse || rq->sparse->m != rq->model ||
        (rq->op != TB_OP_FORWARD && rq->op != TB_OP_GRADIENT) ||
        (rq->op == TB_OP_GRADIENT && (!rq->grad_out || rq->checkpoint_every < 0 ||
                                      (rq->sparse->nrec > 0 && rq->model->nt > 0 && !rq->d_obs)))) {
        set_error("tb_server_submit: invalid argument");
        return TB_EINVAL;
    }
    auto j = std::make_unique<Job>();
    j->rq = *rq;
    j->rq.sched = nullptr;
    tb_status rc = resolve_schedule(rq->model, rq->sched, &j->sc);
    if (rc) return rc;
    tb_sparse *s = const_cast<tb_sparse *>(rq->sparse);
    j->ws_bytes = rq->op == TB_OP_FORWARD
                      ? forward_ws_bytes(rq->model, s, j->sc)
                      : gradient_ws_bytes(rq->model, s, j->sc, rq->checkpoint_every);
    if (j->ws_bytes > sv->arena.bytes) {
        set_error("request needs %zu bytes of workspace; the arena holds %zu", j->ws_bytes,
                  sv->arena.bytes);
        return TB_EWORKSPACE;
    }
    TB_HIP(hipHostMalloc((void **)&j->loss, sizeof(double), hipHostMallocDefault));
    *j->loss = 0.0;
    TB_HIP(hipEventCreateWithFlags(&j->done, hipEventDisableTiming));
    j->id = sv->next_id++;
    if (id) *id = j->id;
    sv->queue.push_back(std::move(j));
    return TB_OK;
}

tb_status tb_server_step(tb_server *sv, int32_t *n_active, int32_t *n_queued)
{
    if (!sv) {
        set_error("tb_server_step: NULL server");
        return TB_EINVAL;
    }
    tb_status rc;
    if ((rc = collect(sv))) return rc;
    if ((rc = admit(sv))) return rc;
    if ((rc = run_actions(sv))) return rc;
    if ((rc = admit(sv))) return rc;  // slots freed by jobs that just finished
    if ((rc = run_actions(sv))) return rc;
    if ((rc = epoch(sv))) return rc;
    if ((rc = collect(sv))) return rc;
    if (n_active) *n_active = (int32_t)(sv->active.size() + sv->retiring.size());
    if (n_queued) *n_queued = (int32_t)sv->queue.size();
    return TB_OK;
}

tb_status tb_server_poll(tb_server *sv, int32_t cap, int64_t *ids, double *losses,
                         int32_t *n_done)
{
    if (!sv || cap < 0 || (cap > 0 && !ids) || !n_done) {
        set_error("tb_server_poll: invalid argument");
        return TB_EINVAL;
    }
    tb_status rc = collect(sv);
    if (rc) return rc;
    const int n = std::min<int>(cap, (int)sv->done.size());
    for (int i = 0; i < n; i++) {
        ids[i] = sv->done[i].id;
        if (losses) losses[i] = sv->done[i].loss;
    }
    sv->done.erase(sv->done.begin(), sv->done.begin() + n);
    *n_done = n;
    return TB_OK;
}

tb_status tb_server_stats(const tb_server *sv, int64_t *stats, int32_t n)
{
    if (!sv || !stats || n < 0) {
        set_error("tb_server_stats: invalid argument");
        return TB_EINVAL;
    }
    for (int i = 0; i < n && i < 8; i++) stats[i] = sv->stats[i];
    return TB_OK;
}

void tb_server_destroy(tb_server *sv) { delete sv; }

}  // extern "C"
