// C ABI of the temporal-blocking library: model and sparse handles, the
// time loop of the forward and adjoint propagators (host side), status codes.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "plan.h"
#include "elastic_params.h"
#include "tti_params.h"

namespace tbw {
const char *last_error();
tb_status inspect_into(tb_sparse *s, int nsrc, const double *src_xyz, const double *wav, int nrec,
                       const double *rec_xyz);
}  // namespace tbw

using namespace tbw;

tb_model::~tb_model()
{
    if (d_c) (void)hipFree(d_c);
    if (d_damp) (void)hipFree(d_damp);
    if (d_zero) (void)hipFree(d_zero);
    if (d_tti) (void)hipFree(d_tti);
    if (d_el) (void)hipFree(d_el);
}

tb_sparse::~tb_sparse()
{
    tiles.clear();
    for (void *p : {(void *)d_dcmp, (void *)d_rc_ptr, (void *)d_rc_id, (void *)d_rc_w,
                    (void *)d_sc_ptr, (void *)d_sc_id, (void *)d_sc_w, (void *)d_rr_ptr,
                    (void *)d_rr_rec, (void *)d_rr_w, (void *)d_rid_scale, (void *)d_src_off,
                    (void *)d_src_alpha, (void *)d_rid_off, (void *)d_rc2_ptr, (void *)d_rc2_id,
                    (void *)d_rc2_w, (void *)d_rid2_off, (void *)d_rr2_ptr, (void *)d_rr2_rec,
                    (void *)d_rr2_w})
        if (p) (void)hipFree(p);
}

namespace {

// Finite-difference weights on unit spacing, exact rationals (Fornberg 1988)
// for space orders 4, 8 and 12; the kernels take them rounded to FP32.
// Centred second derivative, offsets 0..r.
const double *d2_weights(int so)
{
    static const double w4[3] = {-5.0 / 2.0, 4.0 / 3.0, -1.0 / 12.0};
    static const double w8[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
    static const double w12[7] = {-5369.0 / 1800.0, 12.0 / 7.0, -15.0 / 56.0, 10.0 / 189.0,
                                  -1.0 / 112.0,     2.0 / 1925.0, -1.0 / 16632.0};
    return so == 4 ? w4 : (so == 8 ? w8 : (so == 12 ? w12 : nullptr));
}
// Centred first derivative, offsets 1..r (offset -j has the opposite sign).
const double *d1_weights(int so)
{
    static const double w4[2] = {2.0 / 3.0, -1.0 / 12.0};
    static const double w8[4] = {4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};
    static const double w12[6] = {6.0 / 7.0, -15.0 / 56.0, 5.0 / 63.0,
                                  -1.0 / 56.0, 1.0 / 385.0, -1.0 / 5544.0};
    return so == 4 ? w4 : (so == 8 ? w8 : (so == 12 ? w12 : nullptr));
}
// Staggered first derivative, offsets 1/2 .. r-1/2.
const double *stag_weights(int so)
{
    static const double w4[2] = {9.0 / 8.0, -1.0 / 24.0};
    static const double w8[4] = {1225.0 / 1024.0, -245.0 / 3072.0, 49.0 / 5120.0, -5.0 / 7168.0};
    static const double w12[6] = {160083.0 / 131072.0, -12705.0 / 131072.0, 22869.0 / 1310720.0,
                                  -5445.0 / 1835008.0, 847.0 / 2359296.0,   -63.0 / 2883584.0};
    return so == 4 ? w4 : (so == 8 ? w8 : (so == 12 ? w12 : nullptr));
}

// Damping profile along one axis: d0 (k/nbl)^2 with k the depth into the
// absorbing layer, d0 = 3 vmax ln(1/R) / (2 nbl h), R = 1e-3.
void damping_axis(int n, int nbl, double h, double vmax, float *out)
{
    for (int i = 0; i < n; i++) {
        double v = 0.0;
        if (nbl > 0) {
            int k = std::max(std::max(nbl - i, i - (n - 1 - nbl)), 0);
            double d0 = 3.0 * vmax * std::log(1.0 / 1e-3) / (2.0 * nbl * h);
            double q = (double)k / nbl;
            v = d0 * q * q;
        }
        out[i] = (float)v;
    }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

template <class T>
tb_status upload(T **dst, const std::vector<T> &src)
{
    size_t n = std::max<size_t>(src.size(), 1);
    TB_HIP(hipMalloc(dst, n * sizeof(T)));
    if (!src.empty()) TB_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return TB_OK;
}

}  // namespace

namespace tbw {

size_t field_bytes(const tb_model *m) { return align256(m->field_elems() * sizeof(float)); }

tb_status resolve_schedule(const tb_model *m, const tb_schedule *s, SchedChoice *out)
{
    // Default: three steps per pass at space order 4, two at space order 8,
    // one (spatial blocking) at space order 12, where the radius-6 halos of a
    // two-step tile cost more than the pass saves (measured at 512^3: 178
    // against 249 GPts/s), on 32-row tiles. When the tiles fill at least half
    // the CUs but not all, each tile
    // streams whole x (neighbouring tiles in step, sharing their halo reads in
    // L2) and the spare workgroups take the tails; otherwise long x axes use
    // 64-plane chunks dispatched chunk-major, short ones the even partition of
    // the tile-x space. A schedule tuned for the model's shape (tb_autotune)
    // replaces the default.
    const int T0 = m->r == 2 && acoustic_shape_ok(2, 3, 16, 32) ? 3 : (m->r >= 6 ? 1 : 2);
    SchedChoice c{T0, 32, m->n[0] >= 256 ? 64 : 0, 2};
    if (m->n[0] <= kMaxChunk) {
        const int nt = make_geom(m->r, T0, 32, kMaxChunk, m->ncu, m->n[0], m->n[1], m->n[2]).ntiles();
        if (2 * nt >= m->ncu && nt < m->ncu) c.chunk = kMaxChunk;
    }
    if (s) {
        if (s->mode == TB_SCHED_SB) c.T = 1;
        else if (s->mode == TB_SCHED_TB) c.T = s->time_tile;
        else {
            set_error("schedule mode %d unknown", s->mode);
            return TB_EINVAL;
        }
        c.tile_y = s->tile_y;
        c.chunk = s->chunk_x;
    } else {
        SchedChoice t;
        if (m->physics != TB_ACOUSTIC) c = SchedChoice{1, 0, 0, 1};
        if (tuned_schedule(m, &t)) c = t;
    }
    if (c.T < 1 || c.T > 4) {
        set_error("time_tile %d not in 1..4", c.T);
        return TB_EUNSUPPORTED;
    }
    if (m->physics != TB_ACOUSTIC) {
        // TTI and elastic: passes of T steps over x-slabs of chunk_x owned
        // planes (0: the default width); tile_y does not apply.
        if (c.chunk < 0) {
            set_error("chunk_x %d negative", c.chunk);
            return TB_EINVAL;
        }
        *out = c;
        return TB_OK;
    }
    if (m->r >= 4 && c.T > 3) {
        set_error("time_tile %d exceeds 3 at space order %d", c.T, m->so);
        return TB_EUNSUPPORTED;
    }
    if (c.tile_y != 0 && c.tile_y != 16 && c.tile_y != 32) {
        set_error("tile_y %d not in {0 (default), 16, 32}", c.tile_y);
        return TB_EUNSUPPORTED;
    }
    if (c.tile_y != 0 && c.tile_y - 2 * m->r * (c.T - 1) <= 0) {
        set_error("tile_y %d too small for time_tile %d at radius %d", c.tile_y, c.T, m->r);
        return TB_EUNSUPPORTED;
    }
    if (c.chunk < 0) {
        set_error("chunk_x %d negative", c.chunk);
        return TB_EINVAL;
    }
    if (m->physics == TB_ACOUSTIC) {
        // Every depth up to T is launched (the remainder of nt), so each one
        // needs a kernel of the selected shape.
        for (int t = 1; t <= c.T; t++) {
            int lz = 0, bye = 0;
            tile_shape(m->r, t, c.tile_y, &lz, &bye);
            if (!acoustic_shape_ok(m->r, t, lz, bye)) {
                set_error("no wave-front kernel for radius %d, time_tile %d, tile %dx%d (LDS)",
                          m->r, t, bye, 4 * lz);
                return TB_EUNSUPPORTED;
            }
        }
    }
    *out = c;
    return TB_OK;
}

namespace {

// Cached per-segment lists for (direction, T, tile_y, chunk, workgroups).
tb_status get_lists(const tb_model *m, tb_sparse *s, int adjoint, int T, int tile_y, int chunk,
                    int wgs, TileLists **out)
{
    std::lock_guard<std::mutex> lk(s->mu);
    auto key = std::make_tuple(adjoint, T, tile_y, chunk, wgs);
    auto it = s->tiles.find(key);
    if (it != s->tiles.end()) {
        *out = it->second.get();
        return TB_OK;
    }
    auto tl = std::make_unique<TileLists>();
    tl->g = make_geom(m->r, T, tile_y, chunk, wgs, m->n[0], m->n[1], m->n[2]);
    if (tl->g.nwg == 0) {
        set_error("empty tile geometry");
        return TB_EINVAL;
    }
    tb_status st = adjoint ? build_tile_lists(m, s->rid_nodes, s->src_nodes, tl.get())
                           : build_tile_lists(m, s->src_nodes, s->rid_nodes, tl.get());
    if (st) return st;
    *out = tl.get();
    s->tiles[key] = std::move(tl);
    return TB_OK;
}

}  // namespace

// Lists of the schedule (segments whose lists exceed the LDS capacities are
// walked in global memory by the kernel).
tb_status lists_for(const tb_model *m, tb_sparse *s, int adjoint, const SchedChoice &sc, int T,
                    TileLists **out)
{
    // Chunked schedules keep one workgroup per compute unit resident (their
    // LDS footprint allows no more) and hand each a list of segments.
    const int wgs = m->ncu * (sc.chunk > 0 ? 1 : sc.wgs_per_cu);
    return get_lists(m, s, adjoint, T, sc.tile_y, sc.chunk, wgs, out);
}

bool plan_lists_cached(const tb_model *m, tb_sparse *s, const SchedChoice &sc, const Plan &plan)
{
    const int wgs = m->ncu * (sc.chunk > 0 ? 1 : sc.wgs_per_cu);
    std::lock_guard<std::mutex> lk(s->mu);
    for (const Item &it : plan) {
        if (!it.is_pass) continue;
        auto key = std::make_tuple(it.pass.adjoint, it.pass.T, sc.tile_y, sc.chunk, wgs);
        if (s->tiles.find(key) == s->tiles.end()) return false;
    }
    return true;
}

namespace {

AcLaunch to_launch(const Pass &p)
{
    AcLaunch a{};
    a.u = p.u;
    a.v = p.v;
    a.out_u = p.out_u;
    a.out_v = p.out_v;
    a.out_mid = p.out_mid;
    a.n0 = p.n0;
    a.dcmp = p.dcmp;
    a.npts = p.ninj;
    a.rec_dcmp = p.rec;
    a.nrid = p.nrecp;
    return a;
}

Item pass_item(const Pass &p)
{
    Item it;
    it.is_pass = true;
    it.pass = p;
    return it;
}

Item act_item(std::function<tb_status(hipStream_t)> f)
{
    Item it;
    it.act = std::move(f);
    return it;
}

// Append the passes of a time loop of `steps` updates from level n0 with the
// state in U[*ua] = u^{n0} and V[*va] = v^{n0}: each pass reads one u and one
// v buffer and writes the other two. mid (may be NULL) receives u^{n0+steps-1}
// from the last pass when that pass advances two or more steps. after(n, ua,
// va) is called after each pass ending at level n.
void plan_time_loop(Plan *plan, int adjoint, int Tmax, float *U[2], float *V[2], float *mid,
                    int n0, int steps, const float *dcmp, int ninj, float *rec, int nrecp,
                    int *ua, int *va, const std::function<void(int, int, int)> &after)
{
    int n = n0;
    while (n < n0 + steps) {
        const int T = std::min(Tmax, n0 + steps - n);
        Pass p;
        p.adjoint = adjoint;
        p.T = T;
        p.u = U[*ua];
        p.v = V[*va];
        p.out_u = U[1 - *ua];
        p.out_v = V[1 - *va];
        p.out_mid = (T > 1 && n + T == n0 + steps) ? mid : nullptr;
        p.n0 = n;
        p.dcmp = dcmp;
        p.ninj = ninj;
        p.rec = rec;
        p.nrecp = nrecp;
        plan->push_back(pass_item(p));
        *ua = 1 - *ua;
        *va = 1 - *va;
        n += T;
        if (after) after(n, *ua, *va);
    }
}

Item fill_item(float *p, size_t n)
{
    return act_item([=](hipStream_t st) { return launch_fill(p, n, 0.0f, st); });
}

Item copy_item(void *dst, const void *src, size_t bytes)
{
    return act_item([=](hipStream_t st) -> tb_status {
        TB_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
        return TB_OK;
    });
}

// Workspace of the gradient (offsets in bytes from the base).
struct GradLayout {
    int K = 0;       // checkpoint interval (a multiple of the forward depth)
    int ncp = 0;     // stored checkpoints (u^{jK}, v^{jK} for j >= 1)
    int nslot = 0;   // segment slots (u levels jK .. jK+K-1)
    size_t F = 0, A = 0, RV = 0, slots = 0, cps = 0, g = 0, gs = 0, rec = 0, traces = 0, res = 0,
           adj_dcmp = 0, adj_rec = 0, loss = 0, total = 0;
};

int ceil_sqrt(int n)
{
    int k = (int)std::ceil(std::sqrt((double)n));
    while (k > 1 && (k - 1) * (k - 1) >= n) k--;
    return std::max(k, 1);
}

GradLayout grad_layout(const tb_model *m, const tb_sparse *s, const SchedChoice &sc, int every)
{
    GradLayout L;
    const int nt = m->nt;
    int K = every > 0 ? every : ceil_sqrt(std::max(nt, 1));
    K = (K + sc.T - 1) / sc.T * sc.T;
    L.K = K;
    // Checkpoints at levels jK for j >= 1 with jK <= nt - 2 (level 0 is zero).
    L.ncp = nt >= 2 ? (nt - 2) / K : 0;
    L.nslot = K;
    const size_t fb = field_bytes(m);
    const size_t nt1 = (size_t)nt + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    L.F = take(4 * fb);   // forward u, u', v, v'
    L.A = take(5 * fb);   // adjoint u, u', v, v', intermediate level
    L.RV = take(2 * fb);  // v of the recomputed segment
    L.slots = take(L.nslot * fb);
    L.cps = take(2 * (size_t)L.ncp * fb);
    L.g = take(m->field_elems() * sizeof(double));
    L.gs = take((size_t)std::max(s->npts, 1) * sizeof(double));
    L.rec = take(nt1 * std::max(s->nrid, 1) * sizeof(float));
    L.traces = take((size_t)nt * std::max(s->nrec, 1) * sizeof(float));
    L.res = take((size_t)nt * std::max(s->nrec, 1) * sizeof(float));
    L.adj_dcmp = take((size_t)nt * std::max(s->nrid, 1) * sizeof(float));
    L.adj_rec = take(nt1 * std::max(s->npts, 1) * sizeof(float));
    L.loss = take(sizeof(double));
    L.total = o;
    return L;
}

// Centred second-derivative weights per axis scaled by h^-2 (FP64).
void image_weights(const tb_model *m, double w[3][7])
{
    const double *d2 = d2_weights(m->so);
    for (int a = 0; a < 3; a++)
        for (int j = 0; j < 7; j++) w[a][j] = j <= m->r ? d2[j] / (m->h[a] * m->h[a]) : 0.0;
}

}  // namespace

tb_status pass_params(const tb_model *m, tb_sparse *s, const SchedChoice &sc, const Pass &p,
                      AcParams *out, const TileGeom **geom, bool *gl)
{
    TileLists *tl = nullptr;
    tb_status rc = lists_for(m, s, p.adjoint, sc, p.T, &tl);
    if (rc) return rc;
    *out = make_params(m, *tl, to_launch(p));
    if (geom) *geom = &tl->g;
    if (gl)
        *gl = tl->max_src > kSrcCap || !acoustic_lists_in_lds(m->r, tl->g.T, tl->g.LZ, tl->g.BYE);
    return TB_OK;
}

tb_status run_plan(const tb_model *m, tb_sparse *s, const SchedChoice &sc, const Plan &plan,
                   hipStream_t st)
{
    for (const Item &it : plan) {
        tb_status rc;
        if (it.is_pass) {
            TileLists *tl = nullptr;
            if ((rc = lists_for(m, s, it.pass.adjoint, sc, it.pass.T, &tl))) return rc;
            rc = launch_acoustic(m, *tl, to_launch(it.pass), st);
        } else {
            rc = it.act(st);
        }
        if (rc) return rc;
    }
    return TB_OK;
}

namespace {

// Overlapped x-slab passes of the TTI and elastic propagators (layout and
// widths; see plan_slab_passes).
constexpr int kSlabDefault = 32;

int slab_fields(const tb_model *m) { return m->physics == TB_TTI ? 4 : 9; }

// Skew per step: two chained first-derivative stages of radius r (the rotated
// gradient and its divergence; the velocity and the stress pass).
int slab_skew(const tb_model *m) { return 2 * m->r; }

int slab_width(const tb_model *m, const SchedChoice &sc)
{
    if (sc.T == 1) return m->n[0];
    return sc.chunk > 0 ? std::min(sc.chunk, m->n[0]) : std::min(kSlabDefault, m->n[0]);
}

// Planes a step writes beyond its range on each side: the elastic velocity
// pass runs r planes wider than the stress pass that reads it.
int slab_margin(const tb_model *m) { return m->physics == TB_ELASTIC ? m->r : 0; }

// Planes of one scratch level: the widest written range of a slab.
size_t slab_ext(const tb_model *m, const SchedChoice &sc)
{
    if (sc.T == 1) return 0;
    return (size_t)std::min(m->n[0], slab_width(m, sc) + 2 * (sc.T - 1) * slab_skew(m) +
                                         2 * slab_margin(m));
}

}  // namespace

size_t forward_ws_bytes(const tb_model *m, const tb_sparse *s, const SchedChoice &sc)
{
    const size_t rec =
        align256(((size_t)m->nt + 1) * std::max(s->nrid + s->nrid2, 1) * sizeof(float));
    if (m->physics == TB_ACOUSTIC) return 5 * field_bytes(m) + rec;
    // States A and B, the rotated gradients (TTI), p^{nt-1} (TTI), then two
    // scratch levels of the slabs.
    const size_t nf = slab_fields(m);
    const size_t plane = (size_t)m->n[1] * m->nzp * sizeof(float);
    const size_t extra = m->physics == TB_TTI ? 3 : 0;
    return (2 * nf + extra) * field_bytes(m) + 2 * align256(nf * slab_ext(m, sc) * plane) + rec;
}

namespace {

// Model part of the TTI kernel parameters (forward and adjoint).
TtiParams tti_params(const tb_model *m)
{
    const size_t fe = m->field_elems();
    TtiParams P{};
    P.ncu = m->ncu;
    P.ax = m->d_tti;
    P.ay = m->d_tti + fe;
    P.az = m->d_tti + 2 * fe;
    P.e1 = m->d_tti + 3 * fe;
    P.sd = m->d_tti + 4 * fe;
    P.c = m->d_c;
    P.dx = m->d_damp;
    P.dy = m->d_damp + m->n[0];
    P.dz = m->d_damp + m->n[0] + m->n[1];
    P.hdt = (float)(m->dt / 2.0);
    // Centred weights on unit spacing (Fornberg rationals).
    const double *d1 = d1_weights(m->so);
    const double *d2 = d2_weights(m->so);
    for (int j = 0; j < 6; j++) P.w1[j] = j < m->r ? (float)d1[j] : 0.0f;
    for (int j = 0; j < 7; j++) P.w2[j] = j <= m->r ? (float)d2[j] : 0.0f;
    for (int a = 0; a < 3; a++) {
        P.ih[a] = (float)(1.0 / m->h[a]);
        P.ih2[a] = (float)(1.0 / (m->h[a] * m->h[a]));
    }
    P.nx = m->n[0];
    P.ny = m->n[1];
    P.nz = m->n[2];
    P.nzp = m->nzp;
    return P;
}

// Model part of the elastic kernel parameters, with the nine fields at F.
ElParams el_params(const tb_model *m, float *const *F)
{
    const size_t fe = m->field_elems();
    ElParams P{};
    P.ncu = m->ncu;
    for (int k = 0; k < 3; k++) P.v[k] = F[k];
    for (int k = 0; k < 6; k++) P.t[k] = F[3 + k];
    for (int k = 0; k < 3; k++) P.bq[k] = m->d_el + k * fe;
    P.lam = m->d_el + 3 * fe;
    P.mu = m->d_el + 4 * fe;
    for (int k = 0; k < 3; k++) P.ms[k] = m->d_el + (5 + k) * fe;
    P.dx = m->d_damp;
    P.dy = m->d_damp + m->n[0];
    P.dz = m->d_damp + m->n[0] + m->n[1];
    P.hdt = (float)(m->dt / 2.0);
    const double *sw = stag_weights(m->so);
    for (int j = 0; j < 6; j++) P.w[j] = j < m->r ? (float)sw[j] : 0.0f;
    for (int a = 0; a < 3; a++) P.ih[a] = (float)(1.0 / m->h[a]);
    P.nx = m->n[0];
    P.ny = m->n[1];
    P.nz = m->n[2];
    P.nzp = m->nzp;
    return P;
}

// Forward of the TTI and elastic propagators as passes over x-slabs.
//
// A pass of T' steps advances the state from A (level n0) to B (level
// n0 + T'), slab after slab. The slab owning planes [x0, x1) computes step s
// over U_s = [x0 - (T'-1-s) h, x1 + (T'-1-s) h) clipped to the grid, with h
// the skew per step (slab_skew): it reads level n0 + s from A (s = 0) or
// from the slab's scratch level, and writes level n0 + s + 1 to the other
// scratch level, or to B at s = T' - 1. U_s widened by h is U_{s-1}, exactly
// what step s reads. Injection of step s reaches every point of U_s — the
// redundant copies in the slab's halo included, which is what makes the
// reordering legal (Section II-B, Fig. 4b) — and receivers record the owned
// planes [x0, x1) only, each level from the copy of its own slab. A is only
// read and B only written during a pass, so slabs do not interact, and each
// point is computed by the expression of the one-step schedule: every slab
// width and depth gives the same bits. The scratch levels are addressed with
// the global plane offsets (their base pointer is moved back by the first
// plane they hold). T = 1 is spatial blocking: one slab of all of x.
//
// The state is (p, r, w_p, w_r) for TTI (w = u^n - u^{n-1}) and (vx, vy, vz,
// txx, tyy, tzz, txy, txz, tyz) for elastic; receiver rows are indexed by
// level. field_prev (TTI: p^{nt-1}) is gathered from the owned planes of the
// level before the last.
tb_status plan_slab_passes(const tb_model *m, tb_sparse *s, const SchedChoice &sc, void *ws,
                           float *rec_out, float *field_out, float *field_prev_out, Plan *plan,
                           int nsteps)
{
    const bool tti = m->physics == TB_TTI;
    const int NF = slab_fields(m);
    const size_t fb = field_bytes(m), fe = m->field_elems();
    const long long plane = (long long)m->n[1] * m->nzp;
    const int nx = m->n[0], ny = m->n[1], nz = m->n[2], nzp = m->nzp, r = m->r;
    char *base = (char *)ws;
    auto field = [&](int k) { return (float *)(base + (size_t)k * fb); };
    float *A[9], *B[9];
    for (int f = 0; f < NF; f++) {
        A[f] = field(f);
        B[f] = field(NF + f);
    }
    float *qp = tti ? field(2 * NF) : nullptr, *qr = tti ? field(2 * NF + 1) : nullptr;
    float *mid = tti ? field(2 * NF + 2) : nullptr;
    const int nfull = 2 * NF + (tti ? 3 : 0);
    const size_t ext = slab_ext(m, sc);
    const size_t sbytes = align256((size_t)NF * ext * plane * sizeof(float));
    float *scr[2] = {(float *)(base + nfull * fb), (float *)(base + nfull * fb + sbytes)};
    float *rec = (float *)(base + nfull * fb + 2 * sbytes);
    const int nrid = s->nrid, nrid2 = s->nrid2, npts = s->npts;
    const int nt = nsteps >= 0 ? std::min(nsteps, m->nt) : m->nt;
    const int stride = nrid + nrid2;  // elastic rows: P (nrid), then vz (nrid2)
    for (int f = 0; f < NF; f++) plan->push_back(fill_item(A[f], fe));
    if (tti) plan->push_back(fill_item(B[0], fe));  // p^{-1} when nt = 0
    if (stride > 0) plan->push_back(fill_item(rec, (size_t)stride));
    const TtiParams PT = tti ? tti_params(m) : TtiParams{};
    float *F0[9] = {};
    const ElParams PE = tti ? ElParams{} : el_params(m, F0);
    const float *dcmp = s->d_dcmp;
    const long long *soff = s->d_src_off, *roff = s->d_rid_off, *roff2 = s->d_rid2_off;
    const int h = slab_skew(m), wm = slab_margin(m);
    const int W = slab_width(m, sc);
    // x of every source and receiver point (sorted): a slab step whose range
    // holds none skips the injection or the gather launch.
    const long long nyz = (long long)m->n[1] * m->n[2];
    auto xs_of = [&](const std::vector<int64_t> &nodes) {
        std::vector<int> xs;
        for (int64_t r : nodes) xs.push_back((int)(r / nyz));
        std::sort(xs.begin(), xs.end());
        return xs;
    };
    const std::vector<int> sx = xs_of(s->src_nodes), rx = xs_of(s->rid_nodes),
                           rx2 = xs_of(s->rid2_nodes);
    auto any_in = [](const std::vector<int> &xs, int lo, int hi) {
        auto it = std::lower_bound(xs.begin(), xs.end(), lo);
        return it != xs.end() && *it < hi;
    };

    // One step of one slab: level n from `in` to `out` over [lo, hi), owned
    // planes [x0, x1).
    auto step = [&](float *const *in, float *const *out, int n, int lo, int hi, int x0,
                    int x1) -> Item {
        const float *inc = dcmp + (size_t)n * npts;
        float *row = rec + (size_t)(n + 1) * (tti ? nrid : stride);
        // Launch counts of the sparse kernels (0: no point in the range).
        const int ninj = any_in(sx, lo, hi) ? npts : 0;
        const bool rec_here = any_in(rx, x0, x1) || any_in(rx2, x0, x1);
        const int rlo = rec_here ? x0 : 0, rhi = rec_here ? x1 : 0;
        if (tti) {
            TtiParams Q = PT;
            Q.p = in[0];
            Q.r = in[1];
            Q.vp = in[2];
            Q.vr = in[3];
            Q.pn = out[0];
            Q.rn = out[1];
            Q.vpo = out[2];
            Q.vro = out[3];
            Q.qp = qp;
            Q.qr = qr;
            Q.xlo = lo;
            Q.xhi = hi;
            return act_item([=](hipStream_t st) {
                return launch_tti_step(Q, r, inc, soff, ninj, row, roff, nrid, rlo, rhi, st);
            });
        }
        ElParams E = PE;
        for (int c = 0; c < 3; c++) {
            E.v[c] = in[c];
            E.vo[c] = out[c];
        }
        for (int c = 0; c < 6; c++) {
            E.t[c] = in[3 + c];
            E.to[c] = out[3 + c];
        }
        E.xlo = lo;
        E.xhi = hi;
        return act_item([=](hipStream_t st) {
            return launch_elastic_step(E, r, inc, soff, ninj, row, roff, nrid, row + nrid, roff2,
                                       nrid2, rlo, rhi, st);
        });
    };

    float **cur = A, **nxt = B;
    int n0 = 0;
    float *prev_level = A[0];  // p^{nt-1} when the last pass is one step
    while (n0 < nt) {
        const int Tp = std::min(sc.T, nt - n0);
        const bool last = n0 + Tp == nt;
        const int width = Tp == 1 ? nx : W;
        for (int x0 = 0; x0 < nx; x0 += width) {
            const int x1 = std::min(nx, x0 + width);
            const int e_lo = std::max(0, x0 - (Tp - 1) * h - wm);
            float *lv[2][9];
            for (int k = 0; k < 2; k++)
                for (int f = 0; f < NF; f++)
                    lv[k][f] = scr[k] + (ptrdiff_t)f * (ptrdiff_t)ext * plane -
                               (ptrdiff_t)e_lo * plane;
            for (int st_ = 0; st_ < Tp; st_++) {
                const int lo = std::max(0, x0 - (Tp - 1 - st_) * h);
                const int hi = std::min(nx, x1 + (Tp - 1 - st_) * h);
                // Host check before anything is launched: a scratch level
                // must hold every plane the step writes into it ([lo, hi)
                // widened by the margin) and every plane the next step reads
                // from it (its range widened by the skew, which is this one).
                if (st_ < Tp - 1 && (std::max(0, lo - wm) < e_lo ||
                                     std::min(nx, hi + wm) > e_lo + (int)ext)) {
                    set_error("internal: slab step [%d, %d) beyond its scratch [%d, %d)", lo, hi,
                              e_lo, e_lo + (int)ext);
                    return TB_EINVAL;
                }
                float *const *in = st_ == 0 ? cur : lv[(st_ - 1) & 1];
                float *const *out = st_ == Tp - 1 ? nxt : lv[st_ & 1];
                plan->push_back(step(in, out, n0 + st_, lo, hi, x0, x1));
                if (tti && last && field_prev_out && Tp >= 2 && st_ == Tp - 2) {
                    // p^{nt-1} of the owned planes.
                    plan->push_back(copy_item(mid + (size_t)x0 * plane, out[0] + (size_t)x0 * plane,
                                              (size_t)(x1 - x0) * plane * sizeof(float)));
                }
            }
        }
        if (last) prev_level = Tp >= 2 ? mid : cur[0];
        std::swap(cur, nxt);
        n0 += Tp;
    }
    if (rec_out && s->nrec > 0 && nt > 0) {
        const int nrec = s->nrec;
        if (tti) {
            const int *ptr = s->d_rc_ptr, *id = s->d_rc_id;
            const float *w = s->d_rc_w;
            plan->push_back(act_item([=](hipStream_t st) {
                return launch_trace_reduce(rec, nrid, nt, ptr, id, w, nrec, rec_out, 0, st);
            }));
        } else {
            // Rows are [P (nrid) | vz (nrid2)]: reduce each part with its mirror.
            const int *p1 = s->d_rc_ptr, *i1 = s->d_rc_id, *p2 = s->d_rc2_ptr,
                      *i2 = s->d_rc2_id;
            const float *w1 = s->d_rc_w, *w2 = s->d_rc2_w;
            plan->push_back(act_item([=](hipStream_t st) -> tb_status {
                tb_status rc =
                    launch_trace_reduce(rec + nrid, stride, nt, p2, i2, w2, nrec, rec_out, 0, st);
                if (rc) return rc;
                return launch_trace_reduce(rec, stride, nt, p1, i1, w1, nrec,
                                           rec_out + (size_t)nt * nrec, 0, st);
            }));
        }
    }
    // Field outputs. TTI: p^{nt}, p^{nt-1}; elastic: vz^{nt-1/2}, tzz^{nt}.
    float *fc = tti ? cur[0] : cur[2];
    float *fp = tti ? (nt == 0 ? B[0] : prev_level) : cur[5];
    if (field_out)
        plan->push_back(act_item([=](hipStream_t st) {
            return launch_unpad(fc, field_out, nx, ny, nz, nzp, st);
        }));
    if (field_prev_out)
        plan->push_back(act_item([=](hipStream_t st) {
            return launch_unpad(fp, field_prev_out, nx, ny, nz, nzp, st);
        }));
    return TB_OK;
}

}  // namespace

// TTI gradient workspace: forward state (p, r two levels each, w_p, w_r,
// q_p, q_r), adjoint state (lambda_p, lambda_r two levels each, psi_p,
// psi_r, z_p, z_r; q shared), K level slots of (p, r), a checkpoint of
// (p, r, w_p, w_r) at the start of every segment, then the FP64 image and
// the per-step rows.
struct TtiGradLayout {
    int K = 1, nseg = 0;
    size_t F = 0, A = 0, slots = 0, cps = 0, g = 0, gs = 0, rec = 0, traces = 0, res = 0,
           adj = 0, srec = 0, loss = 0, total = 0;
};

TtiGradLayout tti_grad_layout(const tb_model *m, const tb_sparse *s, int every)
{
    TtiGradLayout L;
    const int nt = m->nt;
    L.K = every > 0 ? every : ceil_sqrt(std::max(nt, 1));
    L.nseg = (nt + L.K - 1) / L.K;
    const size_t fb = field_bytes(m), nt1 = (size_t)nt + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    L.F = take(8 * fb);
    L.A = take(8 * fb);
    L.slots = take(2 * (size_t)L.K * fb);
    L.cps = take(4 * (size_t)L.nseg * fb);
    L.g = take(m->field_elems() * sizeof(double));
    L.gs = take((size_t)std::max(s->npts, 1) * sizeof(double));
    L.rec = take(nt1 * std::max(s->nrid, 1) * sizeof(float));
    L.traces = take((size_t)nt * std::max(s->nrec, 1) * sizeof(float));
    L.res = take((size_t)nt * std::max(s->nrec, 1) * sizeof(float));
    L.adj = take((size_t)nt * std::max(s->nrid, 1) * sizeof(float));
    L.srec = take(nt1 * std::max(s->npts, 1) * sizeof(float));
    L.loss = take(sizeof(double));
    L.total = o;
    return L;
}

// Elastic gradient workspace: the forward state (9 fields), the multipliers
// and scratch (15), K level slots of (v^{t+1/2}, t^t) (9 each), a checkpoint
// of the 9 fields at the start of every segment, nine FP64 accumulators, the
// per-step rows, traces, residual and loss.
struct ElGradLayout {
    int K = 1, nseg = 0;
    size_t F = 0, A = 0, slots = 0, cps = 0, acc = 0, rec = 0, traces = 0, res = 0, adj = 0,
           loss = 0, total = 0;
};

ElGradLayout el_grad_layout(const tb_model *m, const tb_sparse *s, int every)
{
    ElGradLayout L;
    const int nt = m->nt;
    L.K = every > 0 ? every : ceil_sqrt(std::max(nt, 1));
    L.nseg = (nt + L.K - 1) / L.K;
    const size_t fb = field_bytes(m), nt1 = (size_t)nt + 1;
    const size_t nr = (size_t)std::max(s->nrid + s->nrid2, 1);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    L.F = take(9 * fb);
    L.A = take(15 * fb);
    L.slots = take(9 * (size_t)L.K * fb);
    L.cps = take(9 * (size_t)L.nseg * fb);
    L.acc = take(9 * m->field_elems() * sizeof(double));
    L.rec = take(nt1 * nr * sizeof(float));
    L.traces = take(2 * (size_t)nt * std::max(s->nrec, 1) * sizeof(float));
    L.res = take(2 * (size_t)nt * std::max(s->nrec, 1) * sizeof(float));
    L.adj = take((size_t)nt * nr * sizeof(float));
    L.loss = take(sizeof(double));
    L.total = o;
    return L;
}

size_t gradient_ws_bytes(const tb_model *m, const tb_sparse *s, const SchedChoice &sc, int every)
{
    if (m->physics == TB_TTI) return tti_grad_layout(m, s, every).total;
    if (m->physics == TB_ELASTIC) return el_grad_layout(m, s, every).total;
    return grad_layout(m, s, sc, every).total;
}

tb_status plan_forward_steps(const tb_model *m, tb_sparse *s, const SchedChoice &sc, void *ws,
                             int nsteps, Plan *plan)
{
    if (m->physics == TB_ACOUSTIC) {
        set_error("plan_forward_steps covers the slab passes of TTI and elastic");
        return TB_EUNSUPPORTED;
    }
    return plan_slab_passes(m, s, sc, ws, nullptr, nullptr, nullptr, plan, nsteps);
}

tb_status plan_forward(const tb_model *m, tb_sparse *s, const SchedChoice &sc, void *ws,
                       float *rec_out, float *field_out, float *field_prev_out, Plan *plan)
{
    if (m->physics != TB_ACOUSTIC)
        return plan_slab_passes(m, s, sc, ws, rec_out, field_out, field_prev_out, plan, -1);
    const size_t fb = field_bytes(m), fe = m->field_elems();
    char *base = (char *)ws;
    float *U[2] = {(float *)base, (float *)(base + fb)};
    float *V[2] = {(float *)(base + 2 * fb), (float *)(base + 3 * fb)};
    float *mid = (float *)(base + 4 * fb);
    float *rec = (float *)(base + 5 * fb);
    // u^0 = u^{-1} = 0: both u buffers (the second is u^{-1} when nt = 0)
    // and v^0.
    plan->push_back(fill_item(U[0], fe));
    plan->push_back(fill_item(U[1], fe));
    plan->push_back(fill_item(V[0], fe));
    if (s->nrid > 0) plan->push_back(fill_item(rec, (size_t)s->nrid));
    int ua = 0, va = 0;
    plan_time_loop(plan, 0, sc.T, U, V, mid, 0, m->nt, s->d_dcmp, s->npts, rec, s->nrid, &ua,
                   &va, nullptr);
    // u^{nt-1}: the intermediate level of a last pass of two or more steps,
    // else the input of the last (single-step) pass.
    const int tl = m->nt == 0 ? 1 : (m->nt % sc.T == 0 ? sc.T : m->nt % sc.T);
    if (rec_out && s->nrec > 0 && m->nt > 0) {
        const int nrid = s->nrid, nt = m->nt, nrec = s->nrec;
        const int *pp = s->d_rc_ptr, *id = s->d_rc_id;
        const float *w = s->d_rc_w;
        plan->push_back(act_item([=](hipStream_t st) {
            return launch_trace_reduce(rec, nrid, nt, pp, id, w, nrec, rec_out, 0, st);
        }));
    }
    const int nx = m->n[0], ny = m->n[1], nz = m->n[2], nzp = m->nzp;
    float *fc = U[ua], *fp = tl > 1 ? mid : U[1 - ua];
    if (field_out)
        plan->push_back(act_item([=](hipStream_t st) {
            return launch_unpad(fc, field_out, nx, ny, nz, nzp, st);
        }));
    if (field_prev_out)
        plan->push_back(act_item([=](hipStream_t st) {
            return launch_unpad(fp, field_prev_out, nx, ny, nz, nzp, st);
        }));
    return TB_OK;
}

tb_status plan_gradient(const tb_model *m, tb_sparse *s, const SchedChoice &sc, int every,
                        void *ws, const float *d_obs, float *grad_m, double *loss_dst, Plan *plan)
{
    if (m->physics != TB_ACOUSTIC) {
        set_error("this gradient plan is built for the acoustic propagator only");
        return TB_EUNSUPPORTED;
    }
    const GradLayout L = grad_layout(m, s, sc, every);
    const int nt = m->nt, K = L.K;
    const size_t fb = field_bytes(m), fe = m->field_elems();
    char *base = (char *)ws;
    auto fld = [=](size_t off, int i) { return (float *)(base + off + (size_t)i * fb); };
    float *FU[2] = {fld(L.F, 0), fld(L.F, 1)}, *FV[2] = {fld(L.F, 2), fld(L.F, 3)};
    float *AU[2] = {fld(L.A, 0), fld(L.A, 1)}, *AV[2] = {fld(L.A, 2), fld(L.A, 3)};
    float *AM = fld(L.A, 4);
    float *RV[2] = {fld(L.RV, 0), fld(L.RV, 1)};
    double *g = (double *)(base + L.g);
    double *gs = (double *)(base + L.gs);
    float *rec = (float *)(base + L.rec), *traces = (float *)(base + L.traces);
    float *res = (float *)(base + L.res), *adj_dcmp = (float *)(base + L.adj_dcmp);
    float *adj_rec = (float *)(base + L.adj_rec);
    double *loss = (double *)(base + L.loss);
    const int nrec = s->nrec, nrid = s->nrid, npts = s->npts;

    // 1. Forward run from zero state, keeping (u^{jK}, v^{jK}) for j >= 1.
    plan->push_back(fill_item(FU[0], fe));
    plan->push_back(fill_item(FV[0], fe));
    if (nrid > 0) plan->push_back(fill_item(rec, (size_t)nrid));
    int ua = 0, va = 0, j = 1;
    plan_time_loop(plan, 0, sc.T, FU, FV, nullptr, 0, nt, s->d_dcmp, npts, rec, nrid, &ua, &va,
                   [&](int n, int cu, int cv) {
                       if (j <= L.ncp && n == j * K) {
                           plan->push_back(copy_item(fld(L.cps, 2 * (j - 1)), FU[cu], fb));
                           plan->push_back(copy_item(fld(L.cps, 2 * (j - 1) + 1), FV[cv], fb));
                           j++;
                       }
                   });
    // 2. Traces, residual and misfit; the adjoint source.
    {
        const int *pp = s->d_rc_ptr, *id = s->d_rc_id, *rp = s->d_rr_ptr, *rr = s->d_rr_rec;
        const float *w = s->d_rc_w, *rw = s->d_rr_w, *rs = s->d_rid_scale;
        plan->push_back(act_item([=](hipStream_t st) -> tb_status {
            tb_status rc;
            if (nrec > 0 && nt > 0 &&
                (rc = launch_trace_reduce(rec, nrid, nt, pp, id, w, nrec, traces, 0, st)))
                return rc;
            if ((rc = launch_residual_loss(traces, d_obs, (long long)nt * nrec, res, loss, st)))
                return rc;
            if (nrid > 0 && nt > 0 &&
                (rc = launch_adj_inject(res, nt, nrec, nrid, rp, rr, rw, rs, adj_dcmp, st)))
                return rc;
            return TB_OK;
        }));
    }
    // 3. Segments in reverse: recompute levels k0 .. e into the slots, then
    //    run the adjoint through levels e+1 .. k0+1 and image each one.
    plan->push_back(act_item([=](hipStream_t st) -> tb_status {
        tb_status rc = launch_zero64(g, fe, st);
        if (rc) return rc;
        return launch_zero64(gs, (size_t)npts, st);
    }));
    plan->push_back(fill_item(AU[0], fe));
    plan->push_back(fill_item(AV[0], fe));
    if (npts > 0) plan->push_back(fill_item(adj_rec, (size_t)npts));
    ImageArgs ia{};
    ia.c = m->d_c;
    ia.g = g;
    ia.nx = m->n[0];
    ia.ny = m->n[1];
    ia.nz = m->n[2];
    ia.nzp = m->nzp;
    ia.r = m->r;
    image_weights(m, ia.w);
    const float *dcmp = s->d_dcmp;
    const long long *soff = s->d_src_off;
    const double *salpha = s->d_src_alpha;
    const int Td = std::min(sc.T, 2);  // every level of these passes is stored
    int au = 0, av = 0;
    for (int seg = L.ncp; seg >= 0 && nt >= 2; seg--) {
        const int k0 = seg * K;
        const int e = std::min(k0 + K - 1, nt - 2);
        // slot i holds u^{k0 + i}; RV holds v of the recomputed levels.
        if (seg == 0) {
            plan->push_back(fill_item(fld(L.slots, 0), fe));
            plan->push_back(fill_item(RV[0], fe));
        } else {
            plan->push_back(copy_item(fld(L.slots, 0), fld(L.cps, 2 * (seg - 1)), fb));
            plan->push_back(copy_item(RV[0], fld(L.cps, 2 * (seg - 1) + 1), fb));
        }
        int rv = 0;
        for (int nn = k0; nn < e;) {
            const int T = std::min(Td, e - nn);
            const int b = nn - k0;
            Pass p;
            p.T = T;
            p.u = fld(L.slots, b);
            p.v = RV[rv];
            p.out_u = fld(L.slots, b + T);
            p.out_v = RV[1 - rv];
            p.out_mid = T > 1 ? fld(L.slots, b + 1) : nullptr;
            p.n0 = nn;
            p.dcmp = dcmp;
            p.ninj = npts;
            p.rec = rec;
            p.nrecp = nrid;
            plan->push_back(pass_item(p));
            rv = 1 - rv;
            nn += T;
        }
        // Adjoint step na produces nu^{nt-1-na}.
        int na = nt - 2 - e;
        for (int left = e - k0 + 1; left > 0;) {
            const int T = std::min(Td, left);
            Pass p;
            p.adjoint = 1;
            p.T = T;
            p.u = AU[au];
            p.v = AV[av];
            p.out_u = AU[1 - au];
            p.out_v = AV[1 - av];
            p.out_mid = T > 1 ? AM : nullptr;
            p.n0 = na;
            p.dcmp = adj_dcmp;
            p.ninj = nrid;
            p.rec = adj_rec;
            p.nrecp = npts;
            plan->push_back(pass_item(p));
            // Image the levels of this pass in one sweep, newest-in-k first
            // (the intermediate level is overwritten by the next pass); the
            // source-point terms go to their own accumulator in the same
            // level order, so the sums do not depend on the pass depth.
            ImageArgs a2 = ia;
            a2.nlev = T;
            const float *srow[2] = {nullptr, nullptr};
            for (int t = 0; t < T; t++) {
                const int k = nt - 1 - na - t;
                a2.nu[t] = (t == T - 1) ? p.out_u : p.out_mid;
                a2.u[t] = fld(L.slots, k - 1 - k0);
                srow[t] = dcmp + (size_t)(k - 1) * npts;
            }
            plan->push_back(act_item([=](hipStream_t st) -> tb_status {
                tb_status rc = launch_image(a2, st);
                for (int t = 0; t < a2.nlev && !rc; t++)
                    rc = launch_image_sparse(a2.nu[t], srow[t], npts, soff, salpha, gs, st);
                return rc;
            }));
            au = 1 - au;
            av = 1 - av;
            na += T;
            left -= T;
        }
    }
    const int nx = m->n[0], ny = m->n[1], nz = m->n[2], nzp = m->nzp;
    const double scale = -1.0 / (m->dt * m->dt);
    plan->push_back(act_item([=](hipStream_t st) -> tb_status {
        tb_status rc = launch_image_merge(gs, npts, soff, g, st);
        if (rc) return rc;
        return launch_finish_grad(g, grad_m, nx, ny, nz, nzp, scale, st);
    }));
    if (loss_dst)
        plan->push_back(act_item([=](hipStream_t st) -> tb_status {
            TB_HIP(hipMemcpyAsync(loss_dst, loss, sizeof(double), hipMemcpyDeviceToHost, st));
            return TB_OK;
        }));
    return TB_OK;
}

// Adjoint time loop (tb_adjoint): nt updates from zero state in F[0..3].
// Adjoint of the TTI map q -> d (spatially blocked), backwards in time from
// lambda = psi = 0: the decomposed residual of each step enters the p
// component; the source-point samples c (lambda_p + lambda_r)^{k+1} / alpha,
// reduced with the weights W alpha, give qhat^k.
tb_status tti_adjoint(const tb_model *m, tb_sparse *s, void *ws, const float *rec_in,
                      float *src_out, hipStream_t strm)
{
    const size_t fb = field_bytes(m), fe = m->field_elems();
    const size_t nt1 = (size_t)m->nt + 1;
    const int nt = m->nt, npts = s->npts, nrid = s->nrid;
    char *base = (char *)ws;
    float *F[10];
    for (int k = 0; k < 10; k++) F[k] = (float *)(base + k * fb);
    float *srec = (float *)(base + 10 * fb);
    float *adj = (float *)(base + 10 * fb + align256(nt1 * std::max(npts, 1) * sizeof(float)));
    tb_status st;
    for (int k = 0; k < 10; k++)
        if ((st = launch_fill(F[k], fe, 0.0f, strm))) return st;
    if (nrid > 0 && nt > 0)
        if ((st = launch_adj_inject(rec_in, nt, s->nrec, nrid, s->d_rr_ptr, s->d_rr_rec,
                                    s->d_rr_w, nullptr, adj, strm)))
            return st;
    TtiParams P = tti_params(m);
    P.vp = F[4];
    P.vr = F[5];
    P.zp = F[6];
    P.zr = F[7];
    P.p = F[6];
    P.r = F[7];
    P.qp = F[8];
    P.qr = F[9];
    int lc = 0, ln = 1;  // lambda_p^{k+1} in F[lc], lambda_r^{k+1} in F[lc + 2]
    for (int tau = 0; tau < nt; tau++) {
        TtiParams Q = P;
        Q.lp = F[lc];
        Q.lr = F[lc + 2];
        Q.pn = F[ln];
        Q.rn = F[ln + 2];
        if ((st = launch_tti_adjoint_step(Q, m->r, adj + (size_t)tau * std::max(nrid, 1),
                                          s->d_rid_off, nrid, srec + (size_t)tau * npts,
                                          s->d_src_off, s->d_src_alpha, npts, strm)))
            return st;
        std::swap(lc, ln);
    }
    if (src_out && s->nsrc > 0 && nt > 0)
        if ((st = launch_trace_reduce(srec, npts, nt, s->d_sc_ptr, s->d_sc_id, s->d_sc_w, s->nsrc,
                                      src_out, 1, strm)))
            return st;
    return TB_OK;
}


// Gradient of J = 1/2 |traces - d_obs|^2 (traces [2][nt][nrec]: vz, then P)
// of the elastic propagator with respect to lambda, mu and b = 1/rho at the
// nodes, by checkpointing with recomputation: the forward run stores the nine
// fields at the start of every segment of K steps; the backward run
// recomputes a segment's levels (v^{t+1/2}, t^t) into the slots, then for
// each step images them against the multipliers and takes the adjoint step
// (elastic_adjoint's recursion). grad_out is [3][nx][ny][nz].
tb_status elastic_gradient(const tb_model *m, tb_sparse *s, int every, void *ws,
                           const float *d_obs, float *grad_out, double *loss_out, hipStream_t strm)
{
    const ElGradLayout L = el_grad_layout(m, s, every);
    const size_t fb = field_bytes(m), fe = m->field_elems();
    const int nt = m->nt, npts = s->npts, nrid = s->nrid, nrid2 = s->nrid2, nrec = s->nrec;
    const int K = L.K, stride = nrid + nrid2;
    char *base = (char *)ws;
    auto fld = [&](size_t off, size_t k) { return (float *)(base + off + k * fb); };
    float *rec = (float *)(base + L.rec), *traces = (float *)(base + L.traces);
    float *res = (float *)(base + L.res);
    float *adjP = (float *)(base + L.adj), *adjV = adjP + (size_t)nt * nrid;
    double *loss = (double *)(base + L.loss);
    tb_status st;
    float *Ff[9], *Af[9];
    for (int k = 0; k < 9; k++) {
        Ff[k] = fld(L.F, k);
        Af[k] = fld(L.A, k);
        if ((st = launch_fill(Ff[k], fe, 0.0f, strm)) || (st = launch_fill(Af[k], fe, 0.0f, strm)))
            return st;
    }
    ElGradAcc G{};
    double *acc = (double *)(base + L.acc);
    if ((st = launch_zero64(acc, 9 * fe, strm))) return st;
    G.lam = acc;
    G.mu = acc + fe;
    for (int c = 0; c < 3; c++) {
        G.sh[c] = acc + (2 + c) * fe;
        G.bv[c] = acc + (5 + c) * fe;
    }
    if (stride > 0 && (st = launch_fill(rec, (size_t)stride, 0.0f, strm))) return st;
    const ElParams PF = el_params(m, Ff), PA = el_params(m, Af);
    const long long *soff = s->d_src_off, *roff = s->d_rid_off, *roff2 = s->d_rid2_off;
    for (int t = 0; t < nt; t++) {
        if (t % K == 0)
            for (int f = 0; f < 9; f++)
                TB_HIP(hipMemcpyAsync(fld(L.cps, 9 * (size_t)(t / K) + f), Ff[f], fb,
                                      hipMemcpyDeviceToDevice, strm));
        float *row = rec + (size_t)(t + 1) * stride;
        if ((st = launch_elastic_step(PF, m->r, s->d_dcmp + (size_t)t * npts, soff, npts, row, roff,
                                      nrid, row + nrid, roff2, nrid2, 0, m->n[0], strm)))
            return st;
    }
    if (nt > 0 && nrec > 0) {
        if ((st = launch_trace_reduce(rec + nrid, stride, nt, s->d_rc2_ptr, s->d_rc2_id,
                                      s->d_rc2_w, nrec, traces, 0, strm)) ||
            (st = launch_trace_reduce(rec, stride, nt, s->d_rc_ptr, s->d_rc_id, s->d_rc_w, nrec,
                                      traces + (size_t)nt * nrec, 0, strm)))
            return st;
    }
    if ((st = launch_residual_loss(traces, d_obs, 2LL * nt * nrec, res, loss, strm))) return st;
    if (loss_out)
        TB_HIP(hipMemcpyAsync(loss_out, loss, sizeof(double), hipMemcpyDeviceToHost, strm));
    if (nt > 0 && nrec > 0) {
        if (nrid > 0 && (st = launch_adj_inject(res + (size_t)nt * nrec, nt, nrec, nrid,
                                                s->d_rr_ptr, s->d_rr_rec, s->d_rr_w, nullptr, adjP,
                                                strm)))
            return st;
        if (nrid2 > 0 && (st = launch_adj_inject(res, nt, nrec, nrid2, s->d_rr2_ptr, s->d_rr2_rec,
                                                 s->d_rr2_w, nullptr, adjV, strm)))
            return st;
    }
    ElScratch S{};
    for (int k = 0; k < 6; k++) S.f[k] = fld(L.A, 9 + k);
    for (int j = L.nseg - 1; j >= 0; j--) {
        const int k0 = j * K, k1 = std::min(nt, k0 + K);
        for (int f = 0; f < 9; f++)
            TB_HIP(hipMemcpyAsync(Ff[f], fld(L.cps, 9 * (size_t)j + f), fb,
                                  hipMemcpyDeviceToDevice, strm));
        for (int t = k0; t < k1; t++) {
            float *sl = fld(L.slots, 9 * (size_t)(t - k0));
            for (int f = 0; f < 6; f++)
                TB_HIP(hipMemcpyAsync(sl + (3 + f) * (fb / sizeof(float)), Ff[3 + f], fb,
                                      hipMemcpyDeviceToDevice, strm));
            if ((st = launch_elastic_step(PF, m->r, s->d_dcmp + (size_t)t * npts, soff, npts,
                                          nullptr, roff, 0, nullptr, roff2, 0, 0, 0, strm)))
                return st;
            for (int f = 0; f < 3; f++)
                TB_HIP(hipMemcpyAsync(sl + f * (fb / sizeof(float)), Ff[f], fb,
                                      hipMemcpyDeviceToDevice, strm));
        }
        for (int t = k1 - 1; t >= k0; t--) {
            const int tau = nt - 1 - t;
            float *sl = fld(L.slots, 9 * (size_t)(t - k0));
            ElScratch fv{}, ft{};
            for (int f = 0; f < 3; f++) fv.f[f] = sl + f * (fb / sizeof(float));
            for (int f = 0; f < 6; f++) ft.f[f] = sl + (3 + f) * (fb / sizeof(float));
            if ((st = launch_elastic_gradient_step(PA, S, fv, ft, G, m->r,
                                                   adjP + (size_t)tau * nrid, roff, nrid,
                                                   adjV + (size_t)tau * nrid2, roff2, nrid2,
                                                   m->dt, strm)))
                return st;
        }
    }
    return launch_elastic_grad_finish(PA, G, grad_out, strm);
}

// Adjoint of the elastic map q -> (vz, P) (spatially blocked), backwards from
// zero multipliers; rec_in is [2][nt][nrec] (vz block, then P). The samples
// dt tr(th) / alpha at the source points, reduced with the weights W alpha,
// give qhat.
tb_status elastic_adjoint(const tb_model *m, tb_sparse *s, void *ws, const float *rec_in,
                          float *src_out, hipStream_t strm)
{
    const size_t fb = field_bytes(m), fe = m->field_elems();
    const size_t nt1 = (size_t)m->nt + 1;
    const int nt = m->nt, npts = s->npts, nrid = s->nrid, nrid2 = s->nrid2, nrec = s->nrec;
    char *base = (char *)ws;
    float *F[15];
    for (int k = 0; k < 15; k++) F[k] = (float *)(base + k * fb);
    float *srec = (float *)(base + 15 * fb);
    float *adjP = (float *)(base + 15 * fb + align256(nt1 * std::max(npts, 1) * sizeof(float)));
    float *adjV = adjP + (size_t)nt * nrid;
    tb_status st;
    for (int k = 0; k < 9; k++)
        if ((st = launch_fill(F[k], fe, 0.0f, strm))) return st;
    if (nt > 0 && nrec > 0) {
        if (nrid > 0 && (st = launch_adj_inject(rec_in + (size_t)nt * nrec, nt, nrec, nrid,
                                                s->d_rr_ptr, s->d_rr_rec, s->d_rr_w, nullptr, adjP,
                                                strm)))
            return st;
        if (nrid2 > 0 && (st = launch_adj_inject(rec_in, nt, nrec, nrid2, s->d_rr2_ptr,
                                                 s->d_rr2_rec, s->d_rr2_w, nullptr, adjV, strm)))
            return st;
    }
    const ElParams P = el_params(m, F);
    ElScratch S{};
    for (int k = 0; k < 6; k++) S.f[k] = F[9 + k];
    for (int tau = 0; tau < nt; tau++) {
        if ((st = launch_elastic_adjoint_step(P, S, m->r, adjP + (size_t)tau * nrid, s->d_rid_off,
                                              nrid, adjV + (size_t)tau * nrid2, s->d_rid2_off,
                                              nrid2, srec + (size_t)tau * npts, s->d_src_off,
                                              s->d_src_alpha, m->dt, npts, strm)))
            return st;
    }
    if (src_out && s->nsrc > 0 && nt > 0)
        if ((st = launch_trace_reduce(srec, npts, nt, s->d_sc_ptr, s->d_sc_id, s->d_sc_w, s->nsrc,
                                      src_out, 1, strm)))
            return st;
    return TB_OK;
}

// Gradient of J = 1/2 sum_k |P_r p^k - d_obs^k|^2 of the TTI propagator with
// respect to m = 1/vp^2, by checkpointing with recomputation:
//   grad = -(1/dt^2) sum_{k=0}^{nt-2} sum_f y_f^{k+1} (c (A w^k)_f + alpha s^k),
//   y^{k+1} = (c/alpha) lambda^{k+1},
// with lambda the multiplier of tti_adjoint driven by the residual. The
// forward run stores (p, r, w_p, w_r) at the start of every segment of K
// levels; the backward run recomputes a segment's levels into the slots,
// then images each level against the multiplier and takes the adjoint step.
tb_status tti_gradient(const tb_model *m, tb_sparse *s, int every, void *ws, const float *d_obs,
                       float *grad_m, double *loss_out, hipStream_t strm)
{
    const TtiGradLayout L = tti_grad_layout(m, s, every);
    const size_t fb = field_bytes(m), fe = m->field_elems();
    const int nt = m->nt, npts = s->npts, nrid = s->nrid, nrec = s->nrec, K = L.K;
    char *base = (char *)ws;
    auto fld = [&](size_t off, int k) { return (float *)(base + off + (size_t)k * fb); };
    float *rec = (float *)(base + L.rec), *traces = (float *)(base + L.traces);
    float *res = (float *)(base + L.res), *adj = (float *)(base + L.adj);
    float *srec = (float *)(base + L.srec);
    double *g = (double *)(base + L.g), *gs = (double *)(base + L.gs);
    double *loss = (double *)(base + L.loss);
    tb_status st;
    for (int k = 0; k < 8; k++) {
        if ((st = launch_fill(fld(L.F, k), fe, 0.0f, strm))) return st;
        if ((st = launch_fill(fld(L.A, k), fe, 0.0f, strm))) return st;
    }
    if (nrid > 0 && (st = launch_fill(rec, (size_t)nrid, 0.0f, strm))) return st;
    if ((st = launch_zero64(g, fe, strm)) || (st = launch_zero64(gs, std::max(npts, 1), strm)))
        return st;
    const TtiParams P0 = tti_params(m);
    // Forward: p in F0/F1, r in F2/F3, w_p F4, w_r F5, q F6/F7.
    TtiParams P = P0;
    P.vp = fld(L.F, 4);
    P.vr = fld(L.F, 5);
    P.qp = fld(L.F, 6);
    P.qr = fld(L.F, 7);
    const long long *soff = s->d_src_off, *roff = s->d_rid_off;
    int pc = 0, pp = 1;
    for (int n = 0; n < nt; n++) {
        if (n % K == 0) {
            const int j = n / K;
            const float *src4[4] = {fld(L.F, pc), fld(L.F, pc + 2), P.vp, P.vr};
            for (int f = 0; f < 4; f++)
                TB_HIP(hipMemcpyAsync(fld(L.cps, 4 * j + f), src4[f], fb, hipMemcpyDeviceToDevice,
                                      strm));
        }
        TtiParams Q = P;
        Q.p = fld(L.F, pc);
        Q.pn = fld(L.F, pp);
        Q.r = fld(L.F, pc + 2);
        Q.rn = fld(L.F, pp + 2);
        if ((st = launch_tti_step(Q, m->r, s->d_dcmp + (size_t)n * npts, soff, npts,
                                  rec + (size_t)(n + 1) * nrid, roff, nrid, 0, m->n[0], strm)))
            return st;
        std::swap(pc, pp);
    }
    if (nt > 0 && nrec > 0) {
        if ((st = launch_trace_reduce(rec, nrid, nt, s->d_rc_ptr, s->d_rc_id, s->d_rc_w, nrec,
                                      traces, 0, strm)))
            return st;
    }
    if ((st = launch_residual_loss(traces, d_obs, (long long)nt * nrec, res, loss, strm)))
        return st;
    if (loss_out)
        TB_HIP(hipMemcpyAsync(loss_out, loss, sizeof(double), hipMemcpyDeviceToHost, strm));
    if (nrid > 0 && nt > 0)
        if ((st = launch_adj_inject(res, nt, nrec, nrid, s->d_rr_ptr, s->d_rr_rec, s->d_rr_w,
                                    nullptr, adj, strm)))
            return st;
    // Backward. Adjoint: lambda_p A0/A1, lambda_r A2/A3, psi A4/A5, z A6/A7.
    TtiParams PA = P0;
    PA.vp = fld(L.A, 4);
    PA.vr = fld(L.A, 5);
    PA.zp = fld(L.A, 6);
    PA.zr = fld(L.A, 7);
    PA.p = PA.zp;
    PA.r = PA.zr;
    PA.qp = P.qp;
    PA.qr = P.qr;
    int lc = 0, ln = 1;
    for (int j = L.nseg - 1; j >= 0; j--) {
        const int k0 = j * K, k1 = std::min(nt, k0 + K);
        // Recompute levels k0 .. k1-1 into the slots (p in slot 2i, r in 2i+1).
        TB_HIP(hipMemcpyAsync(fld(L.slots, 0), fld(L.cps, 4 * j), fb, hipMemcpyDeviceToDevice,
                              strm));
        TB_HIP(hipMemcpyAsync(fld(L.slots, 1), fld(L.cps, 4 * j + 1), fb,
                              hipMemcpyDeviceToDevice, strm));
        TB_HIP(hipMemcpyAsync(P.vp, fld(L.cps, 4 * j + 2), fb, hipMemcpyDeviceToDevice, strm));
        TB_HIP(hipMemcpyAsync(P.vr, fld(L.cps, 4 * j + 3), fb, hipMemcpyDeviceToDevice, strm));
        for (int k = k0; k + 1 < k1; k++) {
            const int i = k - k0;
            TtiParams Q = P;
            Q.p = fld(L.slots, 2 * i);
            Q.r = fld(L.slots, 2 * i + 1);
            Q.pn = fld(L.slots, 2 * i + 2);
            Q.rn = fld(L.slots, 2 * i + 3);
            if ((st = launch_tti_step(Q, m->r, s->d_dcmp + (size_t)k * npts, soff, npts, nullptr,
                                      roff, 0, 0, 0, strm)))
                return st;
        }
        for (int k = k1 - 1; k >= k0; k--) {
            const int tau = nt - 1 - k, i = k - k0;
            TtiParams Q = PA;
            Q.lp = fld(L.A, lc);
            Q.lr = fld(L.A, lc + 2);
            Q.pn = fld(L.A, ln);
            Q.rn = fld(L.A, ln + 2);
            if (k <= nt - 2) {
                TtiParams I = P0;
                I.p = fld(L.slots, 2 * i);
                I.r = fld(L.slots, 2 * i + 1);
                I.qp = P.qp;
                I.qr = P.qr;
                I.lp = Q.lp;
                I.lr = Q.lr;
                if ((st = launch_tti_image(I, m->r, g, strm))) return st;
            }
            float *srow = srec + (size_t)tau * npts;
            if ((st = launch_tti_adjoint_step(Q, m->r, adj + (size_t)tau * nrid, roff, nrid, srow,
                                              soff, s->d_src_alpha, npts, strm)))
                return st;
            if (k <= nt - 2 && npts > 0)
                if ((st = launch_tti_image_sparse(srow, s->d_src_alpha,
                                                  s->d_dcmp + (size_t)k * npts, npts, gs, strm)))
                    return st;
            std::swap(lc, ln);
        }
    }
    if ((st = launch_image_merge(gs, npts, soff, g, strm))) return st;
    return launch_finish_grad(g, grad_m, m->n[0], m->n[1], m->n[2], m->nzp,
                              -1.0 / (m->dt * m->dt), strm);
}

tb_status time_loop(const tb_model *m, tb_sparse *s, const SchedChoice &sc, int adjoint,
                    float *F[4], const float *dcmp, int ninj, float *rec_dcmp, int nrecp,
                    hipStream_t st)
{
    Plan plan;
    const size_t fe = m->field_elems();
    float *U[2] = {F[0], F[1]}, *V[2] = {F[2], F[3]};
    plan.push_back(fill_item(U[0], fe));
    plan.push_back(fill_item(V[0], fe));
    if (nrecp > 0) plan.push_back(fill_item(rec_dcmp, (size_t)nrecp));
    int ua = 0, va = 0;
    plan_time_loop(&plan, adjoint, sc.T, U, V, nullptr, 0, m->nt, dcmp, ninj, rec_dcmp, nrecp,
                   &ua, &va, nullptr);
    return run_plan(m, s, sc, plan, st);
}

}  // namespace tbw

namespace {

}  // namespace

extern "C" {

const char *tb_last_error(void) { return tbw::last_error(); }

const char *tb_version(void) { return "tbwave 0.1 (gfx950)"; }

tb_status tb_kernel_timing(int32_t enable) { return tbw::kernel_timing(enable); }

tb_status tb_kernel_timing_read(int32_t *launches, double *total_ms)
{
    int n = 0;
    tb_status st = tbw::kernel_timing_read(&n, total_ms);
    if (launches) *launches = n;
    return st;
}

tb_status tb_create_model(const tb_model_desc *d, tb_model **out)
{
    if (!out) {
        set_error("tb_create_model: out is NULL");
        return TB_EINVAL;
    }
    *out = nullptr;
    if (!d) {
        set_error("tb_create_model: desc is NULL");
        return TB_EINVAL;
    }
    if (d->physics != TB_ACOUSTIC && d->physics != TB_TTI && d->physics != TB_ELASTIC) {
        set_error("physics %d is not built", d->physics);
        return TB_EUNSUPPORTED;
    }
    if (d->physics == TB_ELASTIC && (!d->vs || !d->rho)) {
        set_error("the elastic model needs vs and rho");
        return TB_EINVAL;
    }
    if (d->physics == TB_TTI && (!d->epsilon || !d->delta || !d->theta || !d->phi)) {
        set_error("TTI needs epsilon, delta, theta and phi");
        return TB_EINVAL;
    }
    if (d->space_order != 4 && d->space_order != 8 && d->space_order != 12) {
        set_error("space order %d not supported (4, 8 or 12)", d->space_order);
        return TB_EUNSUPPORTED;
    }
    for (int a = 0; a < 3; a++) {
        if (d->shape[a] < 1 || !(d->spacing[a] > 0.0) || !std::isfinite(d->origin[a])) {
            set_error("shape/spacing/origin of axis %d invalid", a);
            return TB_EINVAL;
        }
    }
    if (!(d->dt > 0.0) || d->nt < 0 || d->nbl < 0) {
        set_error("dt, nt or nbl invalid");
        return TB_EINVAL;
    }
    if ((d->vp == nullptr) == (d->slowness2 == nullptr)) {
        set_error("give exactly one of vp and slowness2");
        return TB_EINVAL;
    }
    if (d->slowness2 && d->physics != TB_ACOUSTIC) {
        set_error("slowness2 is accepted for the acoustic physics only");
        return TB_EUNSUPPORTED;
    }
    const int nx = d->shape[0], ny = d->shape[1], nz = d->shape[2];
    if ((long long)ny * nz > (1LL << 30) || (long long)nx * ny * nz > (1LL << 36)) {
        set_error("grid too large");
        return TB_EINVAL;
    }
    if (nx > 65535) {
        set_error("nx %d above 65535 (the sparse-list keys hold x in 16 bits)", nx);
        return TB_EUNSUPPORTED;
    }
    if ((long long)ny * ((nz + 3) & ~3) * 4 >= (1LL << 31)) {
        set_error("a padded y-z plane of %lld bytes reaches 2 GiB (planes are addressed with "
                  "32-bit offsets)", (long long)ny * ((nz + 3) & ~3) * 4);
        return TB_EUNSUPPORTED;
    }
    auto m = std::make_unique<tb_model>();
    m->physics = d->physics;
    std::memcpy(m->n, d->shape, sizeof m->n);
    m->nzp = (nz + 3) & ~3;
    std::memcpy(m->h, d->spacing, sizeof m->h);
    std::memcpy(m->o, d->origin, sizeof m->o);
    m->so = d->space_order;
    m->r = d->space_order / 2;
    m->nbl = d->nbl;
    m->dt = d->dt;
    m->nt = d->nt;
    TB_HIP(hipGetDevice(&m->device));
    TB_HIP(hipDeviceGetAttribute(&m->ncu, hipDeviceAttributeMultiprocessorCount, m->device));
    if (m->ncu < 1) m->ncu = 1;

    const size_t N = (size_t)nx * ny * nz;
    // The host copy holds vp, or m = 1/vp^2 when the caller gave slowness2.
    const bool by_m = d->slowness2 != nullptr;
    std::vector<float> vp(N);
    TB_HIP(hipMemcpy(vp.data(), by_m ? d->slowness2 : d->vp, N * sizeof(float),
                     hipMemcpyDeviceToHost));
    double vpmax = 0.0;
    for (size_t i = 0; i < N; i++) {
        if (!(vp[i] > 0.0f) || !std::isfinite(vp[i])) {
            set_error("%s[%zu] = %g is not positive and finite", by_m ? "slowness2" : "vp", i,
                      (double)vp[i]);
            return TB_EINVAL;
        }
        vpmax = std::max(vpmax, by_m ? 1.0 / std::sqrt((double)vp[i]) : (double)vp[i]);
    }
    m->vmax = d->damp_vmax > 0.0 ? d->damp_vmax : vpmax;
    // TTI parameters: the fastest phase velocity is vp sqrt(1 + 2 eps).
    std::vector<float> tti_host;
    double vstab = vpmax;
    if (d->physics == TB_TTI) {
        std::vector<float> ep(N), de(N), th(N), ph(N);
        TB_HIP(hipMemcpy(ep.data(), d->epsilon, N * sizeof(float), hipMemcpyDeviceToHost));
        TB_HIP(hipMemcpy(de.data(), d->delta, N * sizeof(float), hipMemcpyDeviceToHost));
        TB_HIP(hipMemcpy(th.data(), d->theta, N * sizeof(float), hipMemcpyDeviceToHost));
        TB_HIP(hipMemcpy(ph.data(), d->phi, N * sizeof(float), hipMemcpyDeviceToHost));
        const size_t fe = m->field_elems();
        tti_host.assign(5 * fe, 0.0f);
        for (size_t x = 0; x < (size_t)nx; x++)
            for (size_t y = 0; y < (size_t)ny; y++)
                for (size_t z = 0; z < (size_t)nz; z++) {
                    const size_t i = (x * ny + y) * nz + z, q = (x * ny + y) * m->nzp + z;
                    const double e = ep[i], dl = std::min((double)de[i], e);
                    if (!(e >= 0.0) || !(dl > -0.5) || !std::isfinite(th[i]) ||
                        !std::isfinite(ph[i])) {
                        set_error("TTI parameters at node %zu invalid", i);
                        return TB_EINVAL;
                    }
                    const double t = th[i], f = ph[i];
                    tti_host[q] = (float)(std::sin(t) * std::cos(f));
                    tti_host[fe + q] = (float)(std::sin(t) * std::sin(f));
                    tti_host[2 * fe + q] = (float)std::cos(t);
                    tti_host[3 * fe + q] = (float)(1.0 + 2.0 * e);
                    tti_host[4 * fe + q] = (float)std::sqrt(1.0 + 2.0 * dl);
                    vstab = std::max(vstab, (double)vp[i] * std::sqrt(1.0 + 2.0 * e));
                }
    }
    // Elastic parameters at their staggered positions, times dt (FP64, one
    // rounding): b averaged over the 2 nodes of a velocity point, mu over the
    // 4 nodes of a shear point (a node outside the grid takes the nearest
    // inside value).
    std::vector<float> el_host;
    if (d->physics == TB_ELASTIC) {
        std::vector<float> vsh(N), rh(N);
        TB_HIP(hipMemcpy(vsh.data(), d->vs, N * sizeof(float), hipMemcpyDeviceToHost));
        TB_HIP(hipMemcpy(rh.data(), d->rho, N * sizeof(float), hipMemcpyDeviceToHost));
        std::vector<double> b(N), mu(N), lam(N);
        for (size_t i = 0; i < N; i++) {
            const double r = rh[i], sv = vsh[i], p = vp[i];
            if (!(r > 0.0) || !(sv >= 0.0) || !(p * p - 2.0 * sv * sv >= -1e-12 * p * p)) {
                set_error("elastic parameters at node %zu invalid", i);
                return TB_EINVAL;
            }
            b[i] = 1.0 / r;
            mu[i] = r * sv * sv;
            lam[i] = r * (p * p - 2.0 * sv * sv);
        }
        auto cl = [&](const std::vector<double> &f, long x, long y, long z) {
            x = std::min<long>(std::max<long>(x, 0), nx - 1);
            y = std::min<long>(std::max<long>(y, 0), ny - 1);
            z = std::min<long>(std::max<long>(z, 0), nz - 1);
            return f[((size_t)x * ny + y) * nz + z];
        };
        const size_t fe = m->field_elems();
        el_host.assign(8 * fe, 0.0f);
        const double dt = m->dt;
        for (long x = 0; x < nx; x++)
            for (long y = 0; y < ny; y++)
                for (long z = 0; z < nz; z++) {
                    const size_t q = ((size_t)x * ny + y) * m->nzp + z;
                    const size_t i = ((size_t)x * ny + y) * nz + z;
                    el_host[q] = (float)(dt * 0.5 * (cl(b, x, y, z) + cl(b, x + 1, y, z)));
                    el_host[fe + q] = (float)(dt * 0.5 * (cl(b, x, y, z) + cl(b, x, y + 1, z)));
                    el_host[2 * fe + q] = (float)(dt * 0.5 * (cl(b, x, y, z) + cl(b, x, y, z + 1)));
                    el_host[3 * fe + q] = (float)(dt * lam[i]);
                    el_host[4 * fe + q] = (float)(dt * mu[i]);
                    el_host[5 * fe + q] =
                        (float)(dt * 0.25 * (cl(mu, x, y, z) + cl(mu, x + 1, y, z) +
                                             cl(mu, x, y + 1, z) + cl(mu, x + 1, y + 1, z)));
                    el_host[6 * fe + q] =
                        (float)(dt * 0.25 * (cl(mu, x, y, z) + cl(mu, x + 1, y, z) +
                                             cl(mu, x, y, z + 1) + cl(mu, x + 1, y, z + 1)));
                    el_host[7 * fe + q] =
                        (float)(dt * 0.25 * (cl(mu, x, y, z) + cl(mu, x, y + 1, z) +
                                             cl(mu, x, y, z + 1) + cl(mu, x, y + 1, z + 1)));
                }
    }
    // Leapfrog stability: dt^2 v_max^2 * sum_a |symbol max| / h_a^2 <= 4, with
    // the symbol of the centred second derivative, or for the staggered
    // system the square of that of the staggered first derivative.
    const double *w = d2_weights(m->so);
    double sym = w[0];
    for (int j = 1; j <= m->r; j++) sym += 2.0 * w[j] * ((j & 1) ? -1.0 : 1.0);
    sym = std::fabs(sym);
    if (d->physics == TB_ELASTIC) {
        const double *sw = stag_weights(m->so);
        double a = 0.0;
        for (int j = 0; j < m->r; j++) a += 2.0 * std::fabs(sw[j]);
        sym = a * a;
    }
    double rho = 0.0;
    for (int a = 0; a < 3; a++) rho += sym / (m->h[a] * m->h[a]);
    if (m->dt * m->dt * vstab * vstab * rho > 4.0) {
        set_error("dt = %g exceeds the stability bound %g for the fastest velocity %g", m->dt,
                  2.0 / (vstab * std::sqrt(rho)), vstab);
        return TB_EUNSTABLE;
    }
    m->damp.assign((size_t)nx + ny + m->nzp, 0.0f);
    damping_axis(nx, m->nbl, m->h[0], m->vmax, m->damp.data());
    damping_axis(ny, m->nbl, m->h[1], m->vmax, m->damp.data() + nx);
    damping_axis(nz, m->nbl, m->h[2], m->vmax, m->damp.data() + nx + ny);
    // c = dt^2 vp^2 (or dt^2/m) on the device from the caller's array (the
    // same FP64 expression the inspector evaluates at its points from the
    // host copy).
    TB_HIP(hipMalloc(&m->d_c, m->field_elems() * sizeof(float)));
    {
        tb_status rc = launch_c_from_vp(by_m ? d->slowness2 : d->vp, m->d_c, nx, ny, nz, m->nzp,
                                        m->dt, by_m, nullptr);
        if (rc) return rc;
        TB_HIP(hipDeviceSynchronize());
    }
    m->vp_host = std::move(vp);
    m->host_is_m = by_m;
    TB_HIP(hipMalloc(&m->d_zero, 256));
    TB_HIP(hipMemset(m->d_zero, 0, 256));
    if (!el_host.empty()) {
        TB_HIP(hipMalloc(&m->d_el, el_host.size() * sizeof(float)));
        TB_HIP(hipMemcpy(m->d_el, el_host.data(), el_host.size() * sizeof(float),
                         hipMemcpyHostToDevice));
    }
    if (!tti_host.empty()) {
        TB_HIP(hipMalloc(&m->d_tti, tti_host.size() * sizeof(float)));
        TB_HIP(hipMemcpy(m->d_tti, tti_host.data(), tti_host.size() * sizeof(float),
                         hipMemcpyHostToDevice));
    }
    TB_HIP(hipMalloc(&m->d_damp, m->damp.size() * sizeof(float)));
    TB_HIP(hipMemcpy(m->d_damp, m->damp.data(), m->damp.size() * sizeof(float),
                     hipMemcpyHostToDevice));
    *out = m.release();
    return TB_OK;
}

void tb_destroy_model(tb_model *m) { delete m; }

tb_status tb_inspect_sparse(const tb_model *m, int32_t nsrc, const double *src_xyz,
                            const double *src_wavelet, int32_t nrec, const double *rec_xyz,
                            tb_sparse **out)
{
    if (!out) {
        set_error("tb_inspect_sparse: out is NULL");
        return TB_EINVAL;
    }
    *out = nullptr;
    if (!m || nsrc < 0 || nrec < 0 || (nsrc && (!src_xyz || (m->nt && !src_wavelet))) ||
        (nrec && !rec_xyz)) {
        set_error("tb_inspect_sparse: invalid argument");
        return TB_EINVAL;
    }
    auto s = std::make_unique<tb_sparse>();
    s->m = m;
    tb_status st = inspect_into(s.get(), nsrc, src_xyz, src_wavelet, nrec, rec_xyz);
    if (st) return st;
    if ((st = upload(&s->d_dcmp, s->dcmp))) return st;
    // Receiver read-out: per receiver corners (rid, W).
    std::vector<float> rw(s->rc_w.begin(), s->rc_w.end());
    if ((st = upload(&s->d_rc_ptr, s->rc_ptr)) || (st = upload(&s->d_rc_id, s->rc_id)) ||
        (st = upload(&s->d_rc_w, rw)))
        return st;
    // Adjoint read-out at the sources: weights W alpha(node).
    const int nx = m->n[0], ny = m->n[1], nz = m->n[2];
    auto alpha_at = [&](int64_t r) {
        const int z = (int)(r % nz), y = (int)((r / nz) % ny), x = (int)(r / ((int64_t)nz * ny));
        const double d = (double)m->damp[x] + (double)m->damp[nx + y] + (double)m->damp[nx + ny + z];
        return 1.0 + d * m->dt / 2.0;
    };
    (void)nx;
    std::vector<float> sw(s->sc_w.size());
    for (int p = 0; p < nsrc; p++)
        for (int k = s->sc_ptr[p]; k < s->sc_ptr[p + 1]; k++)
            sw[k] = (float)(s->sc_w[k] * alpha_at(s->src_nodes[s->sc_id[k]]));
    if ((st = upload(&s->d_sc_ptr, s->sc_ptr)) || (st = upload(&s->d_sc_id, s->sc_id)) ||
        (st = upload(&s->d_sc_w, sw)))
        return st;
    // Adjoint injection at receiver points: rid -> (receiver, W), scale c/alpha.
    std::vector<int> cnt(s->nrid + 1, 0);
    for (size_t k = 0; k < s->rc_id.size(); k++) cnt[s->rc_id[k] + 1]++;
    for (int i = 0; i < s->nrid; i++) cnt[i + 1] += cnt[i];
    std::vector<int> rr_rec(s->rc_id.size());
    std::vector<float> rr_w(s->rc_id.size());
    std::vector<int> fillp(cnt.begin(), cnt.end() - 1);
    for (int r = 0; r < nrec; r++)
        for (int k = s->rc_ptr[r]; k < s->rc_ptr[r + 1]; k++) {
            const int pos = fillp[s->rc_id[k]]++;
            rr_rec[pos] = r;
            rr_w[pos] = (float)s->rc_w[k];
        }
    std::vector<float> scale(s->nrid);
    for (int i = 0; i < s->nrid; i++)
        scale[i] = (float)(m->inj_coef(s->rid_nodes[i]) / alpha_at(s->rid_nodes[i]));
    if ((st = upload(&s->d_rr_ptr, cnt)) || (st = upload(&s->d_rr_rec, rr_rec)) ||
        (st = upload(&s->d_rr_w, rr_w)) || (st = upload(&s->d_rid_scale, scale)))
        return st;
    // Imaging at the injection points: padded offsets and alpha per SID.
    std::vector<long long> soff(s->npts);
    std::vector<double> salpha(s->npts);
    for (int i = 0; i < s->npts; i++) {
        const int64_t r = s->src_nodes[i];
        const int64_t xy = r / nz;
        soff[i] = (long long)(xy * m->nzp + r % nz);
        salpha[i] = alpha_at(r);
    }
    if ((st = upload(&s->d_src_off, soff)) || (st = upload(&s->d_src_alpha, salpha))) return st;
    std::vector<long long> roff(s->nrid);
    for (int i = 0; i < s->nrid; i++) {
        const int64_t r = s->rid_nodes[i];
        roff[i] = (long long)((r / nz) * m->nzp + r % nz);
    }
    if ((st = upload(&s->d_rid_off, roff))) return st;
    if (m->physics == TB_ELASTIC) {
        std::vector<float> w2(s->rc2_w.begin(), s->rc2_w.end());
        std::vector<long long> roff2(s->nrid2);
        for (int i = 0; i < s->nrid2; i++) {
            const int64_t r = s->rid2_nodes[i];
            roff2[i] = (long long)((r / nz) * m->nzp + r % nz);
        }
        if ((st = upload(&s->d_rc2_ptr, s->rc2_ptr)) || (st = upload(&s->d_rc2_id, s->rc2_id)) ||
            (st = upload(&s->d_rc2_w, w2)) || (st = upload(&s->d_rid2_off, roff2)))
            return st;
        // Transposed vz mirror (adjoint injection at the vz points).
        std::vector<int> c2(s->nrid2 + 1, 0);
        for (size_t k = 0; k < s->rc2_id.size(); k++) c2[s->rc2_id[k] + 1]++;
        for (int i = 0; i < s->nrid2; i++) c2[i + 1] += c2[i];
        std::vector<int> rr2_rec(s->rc2_id.size());
        std::vector<float> rr2_w(s->rc2_id.size());
        std::vector<int> fill2(c2.begin(), c2.end() - 1);
        for (int r = 0; r < nrec; r++)
            for (int k = s->rc2_ptr[r]; k < s->rc2_ptr[r + 1]; k++) {
                const int pos = fill2[s->rc2_id[k]]++;
                rr2_rec[pos] = r;
                rr2_w[pos] = (float)s->rc2_w[k];
            }
        if ((st = upload(&s->d_rr2_ptr, c2)) || (st = upload(&s->d_rr2_rec, rr2_rec)) ||
            (st = upload(&s->d_rr2_w, rr2_w)))
            return st;
    }
    *out = s.release();
    return TB_OK;
}

void tb_destroy_sparse(tb_sparse *s) { delete s; }

tb_status tb_sparse_counts(const tb_sparse *s, int32_t *npts, int32_t *nrid)
{
    if (!s) {
        set_error("tb_sparse_counts: NULL handle");
        return TB_EINVAL;
    }
    if (npts) *npts = s->npts;
    if (nrid) *nrid = s->nrid;
    return TB_OK;
}

tb_status tb_workspace_size(const tb_model *m, const tb_sparse *s, const tb_schedule *sched,
                            int32_t op, size_t *bytes)
{
    if (!m || !s || !bytes) {
        set_error("tb_workspace_size: invalid argument");
        return TB_EINVAL;
    }
    SchedChoice sc;
    tb_status st = resolve_schedule(m, sched, &sc);
    if (st) return st;
    const size_t fb = field_bytes(m);
    const size_t nt1 = (size_t)m->nt + 1;
    switch (op) {
    case TB_OP_FORWARD:
        *bytes = forward_ws_bytes(m, s, sc);
        return TB_OK;
    case TB_OP_ADJOINT:
        // Acoustic: u, v (two levels each); TTI: lambda_p, lambda_r (two
        // levels each), psi_p, psi_r, z_p, z_r, q_p, q_r. Then the samples at
        // the source points and the decomposed residual.
        // Elastic: the nine multipliers and six scratch fields; its residual
        // rows cover both receiver mirrors.
        *bytes = (m->physics == TB_TTI ? 10 : (m->physics == TB_ELASTIC ? 15 : 4)) * fb +
                 align256(nt1 * std::max(s->npts, 1) * sizeof(float)) +
                 align256((size_t)m->nt * std::max(s->nrid + s->nrid2, 1) * sizeof(float));
        return TB_OK;
    case TB_OP_GRADIENT:
        *bytes = gradient_ws_bytes(m, s, sc, 0);
        return TB_OK;
    default:
        set_error("operation %d has no workspace query", op);
        return TB_EUNSUPPORTED;
    }
}

tb_status tb_forward(const tb_model *m, const tb_sparse *s_, const tb_schedule *sched, void *ws,
                     size_t ws_bytes, float *rec_out, float *field_out, float *field_prev_out,
                     void *stream)
{
    tb_sparse *s = const_cast<tb_sparse *>(s_);
    if (!m || !s || s->m != m || !ws) {
        set_error("tb_forward: invalid argument");
        return TB_EINVAL;
    }
    SchedChoice sc;
    tb_status st = resolve_schedule(m, sched, &sc);
    if (st) return st;
    size_t need = 0;
    if ((st = tb_workspace_size(m, s, sched, TB_OP_FORWARD, &need))) return st;
    if (ws_bytes < need) {
        set_error("workspace %zu bytes < %zu needed", ws_bytes, need);
        return TB_EWORKSPACE;
    }
    Plan plan;
    if ((st = plan_forward(m, s, sc, ws, rec_out, field_out, field_prev_out, &plan))) return st;
    return run_plan(m, s, sc, plan, (hipStream_t)stream);
}

tb_status tb_adjoint(const tb_model *m, const tb_sparse *s_, const tb_schedule *sched, void *ws,
                     size_t ws_bytes, const float *rec_in, float *src_out, void *stream)
{
    tb_sparse *s = const_cast<tb_sparse *>(s_);
    if (!m || !s || s->m != m || !ws || (s->nrec > 0 && m->nt > 0 && !rec_in)) {
        set_error("tb_adjoint: invalid argument");
        return TB_EINVAL;
    }
    SchedChoice sc;
    tb_status st = resolve_schedule(m, sched, &sc);
    if (st) return st;
    size_t need = 0;
    if ((st = tb_workspace_size(m, s, sched, TB_OP_ADJOINT, &need))) return st;
    if (ws_bytes < need) {
        set_error("workspace %zu bytes < %zu needed", ws_bytes, need);
        return TB_EWORKSPACE;
    }
    hipStream_t strm = (hipStream_t)stream;
    if (m->physics == TB_TTI) return tti_adjoint(m, s, ws, rec_in, src_out, strm);
    if (m->physics == TB_ELASTIC) return elastic_adjoint(m, s, ws, rec_in, src_out, strm);
    const size_t fb = field_bytes(m);
    const size_t nt1 = (size_t)m->nt + 1;
    char *base = (char *)ws;
    float *F[4] = {(float *)base, (float *)(base + fb), (float *)(base + 2 * fb),
                   (float *)(base + 3 * fb)};
    float *rec_dcmp = (float *)(base + 4 * fb);  // recorded at source points
    float *adj_dcmp = (float *)(base + 4 * fb + align256(nt1 * std::max(s->npts, 1) * sizeof(float)));
    if (s->nrid > 0 && m->nt > 0)
        if ((st = launch_adj_inject(rec_in, m->nt, s->nrec, s->nrid, s->d_rr_ptr, s->d_rr_rec,
                                    s->d_rr_w, s->d_rid_scale, adj_dcmp, strm)))
            return st;
    st = time_loop(m, s, sc, 1, F, adj_dcmp, s->nrid, rec_dcmp, s->npts, strm);
    if (st) return st;
    // qhat^n = P_s (alpha nu^{n+1}); nu^{n+1} is adjoint level nt-1-n.
    if (src_out && s->nsrc > 0 && m->nt > 0)
        if ((st = launch_trace_reduce(rec_dcmp, s->npts, m->nt, s->d_sc_ptr, s->d_sc_id, s->d_sc_w,
                                      s->nsrc, src_out, 1, strm)))
            return st;
    return TB_OK;
}

tb_status tb_gradient_workspace_size(const tb_model *m, const tb_sparse *s,
                                     const tb_schedule *sched, int32_t checkpoint_every,
                                     size_t *bytes)
{
    if (!m || !s || !bytes || checkpoint_every < 0) {
        set_error("tb_gradient_workspace_size: invalid argument");
        return TB_EINVAL;
    }
    SchedChoice sc;
    tb_status st = resolve_schedule(m, sched, &sc);
    if (st) return st;
    *bytes = gradient_ws_bytes(m, s, sc, checkpoint_every);
    return TB_OK;
}

tb_status tb_gradient(const tb_model *m, const tb_sparse *s_, const tb_schedule *sched, void *ws,
                      size_t ws_bytes, const float *d_obs, float *grad_m, double *loss_out,
                      int32_t checkpoint_every, void *stream)
{
    tb_sparse *s = const_cast<tb_sparse *>(s_);
    if (!m || !s || s->m != m || !ws || !grad_m || checkpoint_every < 0 ||
        (s->nrec > 0 && m->nt > 0 && !d_obs)) {
        set_error("tb_gradient: invalid argument");
        return TB_EINVAL;
    }
    SchedChoice sc;
    tb_status st = resolve_schedule(m, sched, &sc);
    if (st) return st;
    const size_t need = gradient_ws_bytes(m, s, sc, checkpoint_every);
    if (ws_bytes < need) {
        set_error("workspace %zu bytes < %zu needed", ws_bytes, need);
        return TB_EWORKSPACE;
    }
    hipStream_t strm = (hipStream_t)stream;
    if (m->physics == TB_TTI || m->physics == TB_ELASTIC) {
        if ((st = m->physics == TB_TTI
                      ? tti_gradient(m, s, checkpoint_every, ws, d_obs, grad_m, loss_out, strm)
                      : elastic_gradient(m, s, checkpoint_every, ws, d_obs, grad_m, loss_out,
                                         strm)))
            return st;
        if (loss_out) TB_HIP(hipStreamSynchronize(strm));
        return TB_OK;
    }
    Plan plan;
    if ((st = plan_gradient(m, s, sc, checkpoint_every, ws, d_obs, grad_m, loss_out, &plan)))
        return st;
    if ((st = run_plan(m, s, sc, plan, strm))) return st;
    if (loss_out) TB_HIP(hipStreamSynchronize(strm));
    return TB_OK;
}

}  // extern "C"
