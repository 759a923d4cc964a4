// Inspector (Section II-A of the paper): turns off-grid sources and receivers
// into grid-aligned data so that injection and interpolation become plain
// per-grid-point operations that any iteration order may apply.
//
//  * support: the grid points with non-zero trilinear weight around each
//    off-grid point (the paper's empty-grid injection: its non-zero points);
//  * unique ascending IDs over those points (the paper's source mask and ID
//    arrays, kept here in sparse form: a sorted list of raster indices);
//  * the decomposed per-point wavelets src_dcmp[t][id] (the paper's
//    decomposition listing), summed in FP64 and rounded once to FP32;
//  * per-tile lists, the GPU form of the paper's per-column count and
//    compressed z-index arrays: for one schedule, every affected point that
//    falls in a workgroup's extended (halo) region, sorted by x, so the fused
//    injection of the time-tiled loop touches only real points.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "tb_internal.h"

namespace tbw {

namespace {
thread_local char g_err[512] = "";
}

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

const char *last_error() { return g_err; }

// Trilinear support of every point: corners (bx, by, bz) in lexicographic
// order with z fastest; zero-weight corners are dropped; a point counts as
// inside when 0 <= (p - o)/h <= n - 1 on every axis.
tb_status build_support(const int n[3], const double h[3], const double o[3], int np,
                        const double *xyz, Support *out)
{
    out->nodes.clear();
    out->ptr.assign(1, 0);
    out->id.clear();
    out->w.clear();
    std::vector<int64_t> raster;
    for (int p = 0; p < np; p++) {
        int64_t base[3];
        double frac[3];
        for (int a = 0; a < 3; a++) {
            double xi = (xyz[3 * p + a] - o[a]) / h[a];
            if (!(xi >= 0.0) || !(xi <= (double)(n[a] - 1))) {
                set_error("point %d coordinate %d = %.9g outside [%g, %g]", p, a, xyz[3 * p + a],
                          o[a], o[a] + (n[a] - 1) * h[a]);
                return TB_ERANGE;
            }
            double f = std::floor(xi);
            base[a] = (int64_t)f;
            frac[a] = xi - f;
        }
        for (int corner = 0; corner < 8; corner++) {
            int b[3] = {(corner >> 2) & 1, (corner >> 1) & 1, corner & 1};
            double W = 1.0;
            for (int a = 0; a < 3; a++) W *= b[a] ? frac[a] : 1.0 - frac[a];
            if (W == 0.0) continue;
            int64_t r = ((base[0] + b[0]) * n[1] + (base[1] + b[1])) * (int64_t)n[2] + base[2] + b[2];
            raster.push_back(r);
            out->w.push_back(W);
        }
        out->ptr.push_back((int)raster.size());
    }
    out->nodes = raster;
    std::sort(out->nodes.begin(), out->nodes.end());
    out->nodes.erase(std::unique(out->nodes.begin(), out->nodes.end()), out->nodes.end());
    out->id.resize(raster.size());
    for (size_t k = 0; k < raster.size(); k++)
        out->id[k] = (int)(std::lower_bound(out->nodes.begin(), out->nodes.end(), raster[k]) -
                           out->nodes.begin());
    return TB_OK;
}

// Decomposition: dcmp[t][id] = sum_s sum_corner W c(node) q_s(t_n), FP64
// accumulation in (s ascending, corner ascending) order, one rounding.
static void decompose(const Support &sp, int nsrc, int nt, const double *wav,
                      const std::vector<double> &cnode, std::vector<float> *dcmp)
{
    const size_t npts = sp.nodes.size();
    std::vector<double> acc(npts);
    dcmp->assign((size_t)nt * npts, 0.0f);
    for (int t = 0; t < nt; t++) {
        std::fill(acc.begin(), acc.end(), 0.0);
        for (int s = 0; s < nsrc; s++) {
            double q = wav[(size_t)t * nsrc + s];
            for (int k = sp.ptr[s]; k < sp.ptr[s + 1]; k++)
                acc[sp.id[k]] += sp.w[k] * cnode[sp.id[k]] * q;
        }
        for (size_t i = 0; i < npts; i++) (*dcmp)[(size_t)t * npts + i] = (float)acc[i];
    }
}

static void node_xyz(int64_t r, const int n[3], int *x, int *y, int *z)
{
    *z = (int)(r % n[2]);
    int64_t q = r / n[2];
    *y = (int)(q % n[1]);
    *x = (int)(q / n[1]);
}

// Tile shape for (R, T): 16 lanes (64 z) per row; 32 rows when that shape
// has a kernel (its LDS fits), else 16, unless the schedule names the rows.
void tile_shape(int R, int T, int tile_y, int *LZ, int *BYE)
{
    *LZ = 16;
    *BYE = tile_y > 0 ? tile_y : (acoustic_shape_ok(R, T, 16, 32) ? 32 : 16);
}

TileGeom make_geom(int R, int T, int tile_y, int chunk, int wgs, int nx, int ny, int nz)
{
    TileGeom g;
    g.R = R;
    g.T = T;
    g.HY = R * (T - 1);
    g.HZ = ((R * (T - 1) + 3) / 4) * 4;
    tile_shape(R, T, tile_y, &g.LZ, &g.BYE);
    g.OY = g.BYE - 2 * g.HY;
    g.OZ = 4 * g.LZ - 2 * g.HZ;
    g.tiles_y = g.OY > 0 ? (ny + g.OY - 1) / g.OY : 0;
    g.tiles_z = g.OZ > 0 ? (nz + g.OZ - 1) / g.OZ : 0;
    const int nt = g.ntiles();
    g.segs.clear();
    g.seg_off.assign(1, 0);
    if (nt == 0) return g;
    if (chunk > 0) {
        g.chunk = std::min(std::min(chunk, nx), kMaxChunk);
        const int nch = (nx + g.chunk - 1) / g.chunk;
        auto seg = [&](int c, int t) {
            const int x0 = c * g.chunk;
            return SegDesc{t, x0, std::min(nx, x0 + g.chunk), 0, 0, 0, 0, 0};
        };
        const int W = wgs / 8;  // workgroups per XCD
        if (nch == 1 && nt < wgs && nx > 1) {
            // Whole x per tile, with fewer tiles than resident workgroups.
            // Tile t streams x in [0, s) on workgroup t, so neighbouring
            // tiles stream the same planes together (their halo re-reads
            // meet in L2); the wgs - nt spare workgroups take the tails
            // [s, nx) of tiles j, j + ns, ... (neighbouring tails again run
            // together). s balances the two: a head costs s + R T planes
            // of the stream, a spare k tails of nx - s + 2 R T each.
            const int ns = wgs - nt;
            const int k = (nt + ns - 1) / ns;
            const int H = R * T;
            const int s = std::max(1, std::min(nx - 1, (k * (nx + 2 * H) - H) / (k + 1)));
            for (int t = 0; t < nt; t++) {
                g.segs.push_back(SegDesc{t, 0, s, 0, 0, 0, 0, 0});
                g.seg_off.push_back((int)g.segs.size());
            }
            // (Spares beyond nt would get no tail: none is launched.)
            for (int j = 0; j < std::min(ns, nt); j++) {
                for (int t = j; t < nt; t += ns) g.segs.push_back(SegDesc{t, s, nx, 0, 0, 0, 0, 0});
                g.seg_off.push_back((int)g.segs.size());
            }
        } else if (W < 1 || (long long)nch * nt <= 8LL * W) {
            // One workgroup per (chunk of x, tile), chunk-major so that the
            // workgroups running together stream the same x range of
            // neighbouring tiles.
            for (int c = 0; c < nch; c++)
                for (int t = 0; t < nt; t++) {
                    g.segs.push_back(seg(c, t));
                    g.seg_off.push_back((int)g.segs.size());
                }
        } else {
            // XCD slabs. Workgroups are handed to the 8 XCDs round-robin and
            // the kernel remaps them so that XCD k holds workgroups
            // [k W, (k+1) W). XCD k owns a contiguous run of tiles (a slab in
            // y) and its W workgroups take that slab's segments chunk by
            // chunk in x order, round-robin, so that the workgroups resident
            // on one XCD stream neighbouring tiles of the same x range, and
            // the x halo of a chunk is the end of the chunk the same XCD has
            // just streamed: both share its L2.
            for (int k = 0; k < 8; k++) {
                const int t0 = (int)((long long)nt * k / 8), t1 = (int)((long long)nt * (k + 1) / 8);
                std::vector<SegDesc> list;
                for (int c = 0; c < nch; c++)
                    for (int t = t0; t < t1; t++) list.push_back(seg(c, t));
                for (int j = 0; j < W; j++) {
                    for (size_t q = j; q < list.size(); q += W) g.segs.push_back(list[q]);
                    g.seg_off.push_back((int)g.segs.size());
                }
            }
        }
    } else {
        // Even partition of the (tile, x) space over `wgs` workgroups: each
        // workgroup streams one contiguous range, split where it crosses a
        // tile boundary (or exceeds the longest chunk).
        g.chunk = 0;
        const long long W = (long long)nt * nx;
        const int nwg = (int)std::max<long long>(1, std::min<long long>(wgs, W));
        for (int b = 0; b < nwg; b++) {
            long long a = W * b / nwg, e = W * (b + 1) / nwg;
            while (a < e) {
                const int t = (int)(a / nx), x0 = (int)(a % nx);
                const int x1 = (int)std::min<long long>({(long long)nx, x0 + (e - a),
                                                          (long long)x0 + kMaxChunk});
                g.segs.push_back(SegDesc{t, x0, x1, 0, 0, 0, 0, 0});
                a += x1 - x0;
            }
            g.seg_off.push_back((int)g.segs.size());
        }
    }
    g.nwg = (int)g.seg_off.size() - 1;
    return g;
}

TileLists::~TileLists()
{
    if (d_src) (void)hipFree(d_src);
    if (d_rec) (void)hipFree(d_rec);
    if (d_segs) (void)hipFree(d_segs);
    if (d_seg_off) (void)hipFree(d_seg_off);
}

// Tile index of (tile_y, tile_z), z fastest; the kernels decode it the same way.
static inline int tile_index(const TileGeom &g, int ty, int tz) { return ty * g.tiles_z + tz; }

// Bin points by tile: inj points into every tile whose extended region
// (rows [0, BYE), columns [0, 4 LZ)) holds them, rec points into the tile
// that owns them. Entries carry x in the key (tile_key for injection,
// rec_key for receivers); segments select by x later.
static void bin_points(const TileGeom &g, const int n[3], const std::vector<int64_t> &nodes,
                       bool owned_only, std::vector<std::vector<int2>> *bins)
{
    const int EZ = 4 * g.LZ;
    for (size_t id = 0; id < nodes.size(); id++) {
        int x, y, z;
        node_xyz(nodes[id], n, &x, &y, &z);
        int ty_lo, ty_hi, tz_lo, tz_hi;
        if (owned_only) {
            ty_lo = ty_hi = y / g.OY;
            tz_lo = tz_hi = z / g.OZ;
        } else {
            // tile t covers rows [t*OY - HY, t*OY - HY + BYE); the exact test
            // is applied below, this only bounds the candidates.
            ty_hi = std::min(g.tiles_y - 1, (y + g.HY) / g.OY);
            ty_lo = std::max(0, ty_hi - (g.BYE / g.OY + 2));
            tz_hi = std::min(g.tiles_z - 1, (z + g.HZ) / g.OZ);
            tz_lo = std::max(0, tz_hi - (EZ / g.OZ + 2));
        }
        for (int ty = ty_lo; ty <= ty_hi; ty++) {
            const int row = y - (ty * g.OY - g.HY);
            if (owned_only ? (row < g.HY || row >= g.HY + g.OY) : (row < 0 || row >= g.BYE))
                continue;
            for (int tz = tz_lo; tz <= tz_hi; tz++) {
                const int col = z - (tz * g.OZ - g.HZ);
                if (owned_only ? (col < g.HZ || col >= g.HZ + g.OZ) : (col < 0 || col >= EZ))
                    continue;
                const int key = owned_only ? rec_key(row, col >> 2, x, col & 3)
                                           : tile_key(row, col >> 2, x, col & 3);
                (*bins)[tile_index(g, ty, tz)].push_back(make_int2(key, (int)id));
            }
        }
    }
    for (auto &b : *bins)
        std::sort(b.begin(), b.end(), [](const int2 &a, const int2 &c) { return a.x < c.x; });
}

template <class T>
static tb_status upload_vec(T **d, const std::vector<T> &v)
{
    const size_t n = std::max<size_t>(v.size(), 1);
    TB_HIP(hipMalloc(d, n * sizeof(T)));
    if (!v.empty()) TB_HIP(hipMemcpy(*d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return TB_OK;
}

// Splits every segment whose injection list (entries with x in [xs - halo,
// xe + halo)) would exceed the LDS capacity into consecutive pieces on the
// same workgroup, each within the capacity where one plane allows it; the
// workgroup streams the pieces one after the other (each with its own x
// warm-up), so the staged-list kernel runs instead of the global-list one.
static void split_dense_segments(TileGeom &g, int nx, const std::vector<std::vector<int2>> &sb,
                                 int halo_x)
{
    std::vector<std::vector<int>> pre(sb.size());  // per tile: prefix counts over x
    auto prefix = [&](int t) -> const std::vector<int> & {
        std::vector<int> &P = pre[t];
        if (P.empty()) {
            P.assign(nx + 1, 0);
            for (const int2 &e : sb[t]) P[((e.x >> 2) & 0xffff) + 1]++;
            for (int x = 0; x < nx; x++) P[x + 1] += P[x];
        }
        return P;
    };
    std::vector<SegDesc> segs;
    std::vector<int> off(1, 0);
    for (size_t w = 0; w + 1 < g.seg_off.size(); w++) {
        for (int k = g.seg_off[w]; k < g.seg_off[w + 1]; k++) {
            const SegDesc &sd = g.segs[k];
            if ((int)sb[sd.tile].size() <= kSrcCap) {
                segs.push_back(sd);
                continue;
            }
            const std::vector<int> &P = prefix(sd.tile);
            auto count = [&](int a, int b) {  // entries of the piece [a, b)
                return P[std::min(nx, b + halo_x)] - P[std::max(0, a - halo_x)];
            };
            for (int a = sd.xs; a < sd.xe;) {
                int b = a + 1;
                while (b < sd.xe && count(a, b + 1) <= kSrcCap) b++;
                segs.push_back(SegDesc{sd.tile, a, b, 0, 0, 0, 0, 0});
                a = b;
            }
        }
        off.push_back((int)segs.size());
    }
    g.segs.swap(segs);
    g.seg_off.swap(off);
}

// Per-segment lists: the tile's entries whose x lies in the segment's range
// (extended by the x halo for injection points), kept in key order.
tb_status build_tile_lists(const tb_model *m, const std::vector<int64_t> &inj,
                           const std::vector<int64_t> &rec, TileLists *out)
{
    TileGeom &g = out->g;
    const int nt = g.ntiles();
    std::vector<std::vector<int2>> sb(nt), rb(nt);
    bin_points(g, m->n, inj, false, &sb);
    bin_points(g, m->n, rec, true, &rb);
    const int halo_x = g.R * (g.T - 1);
    split_dense_segments(g, m->n[0], sb, halo_x);
    std::vector<int2> sflat, rflat;
    out->max_src = out->max_rec = 0;
    for (SegDesc &sd : g.segs) {
        sd.sbeg = (int)sflat.size();
        for (const int2 &e : sb[sd.tile]) {
            const int x = (e.x >> 2) & 0xffff;
            if (x >= sd.xs - halo_x && x < sd.xe + halo_x) sflat.push_back(e);
        }
        sd.sn = (int)sflat.size() - sd.sbeg;
        sd.rbeg = (int)rflat.size();
        for (const int2 &e : rb[sd.tile]) {
            const int x = e.x >> 11;
            if (x >= sd.xs && x < sd.xe) rflat.push_back(e);
        }
        sd.rn = (int)rflat.size() - sd.rbeg;
        out->max_src = std::max(out->max_src, sd.sn);
        out->max_rec = std::max(out->max_rec, sd.rn);
    }
    out->nsrc_entries = (int)sflat.size();
    out->nrec_entries = (int)rflat.size();
    tb_status st;
    if ((st = upload_vec(&out->d_src, sflat)) || (st = upload_vec(&out->d_rec, rflat)) ||
        (st = upload_vec(&out->d_segs, g.segs)) || (st = upload_vec(&out->d_seg_off, g.seg_off)))
        return st;
    return TB_OK;
}

}  // namespace tbw

extern "C" tb_status tb_inspect_host(const int32_t shape[3], const double spacing[3],
                                     const double origin[3], double dt, int32_t nt,
                                     const float *vp_host, int32_t nsrc, const double *src_xyz,
                                     const double *src_wavelet, int32_t *npts, int32_t *nodes,
                                     float *dcmp)
{
    if (!shape || !spacing || !origin || !npts || nt < 0 || nsrc < 0 || (nsrc && !src_xyz) ||
        (nsrc && nt && !src_wavelet) || !vp_host) {
        tbw::set_error("tb_inspect_host: invalid argument");
        return TB_EINVAL;
    }
    int n[3] = {shape[0], shape[1], shape[2]};
    tbw::Support sp;
    tb_status st = tbw::build_support(n, spacing, origin, nsrc, src_xyz, &sp);
    if (st) return st;
    int cap = *npts;
    *npts = (int32_t)sp.nodes.size();
    if ((int)sp.nodes.size() > cap) {
        tbw::set_error("tb_inspect_host: %d points exceed capacity %d", *npts, cap);
        return TB_EWORKSPACE;
    }
    std::vector<double> cn(sp.nodes.size());
    for (size_t i = 0; i < sp.nodes.size(); i++) {
        double v = (double)vp_host[sp.nodes[i]];
        cn[i] = dt * dt * v * v;
    }
    std::vector<float> dc;
    tbw::decompose(sp, nsrc, nt, src_wavelet, cn, &dc);
    for (size_t i = 0; i < sp.nodes.size(); i++) {
        int x, y, z;
        tbw::node_xyz(sp.nodes[i], n, &x, &y, &z);
        nodes[3 * i] = x;
        nodes[3 * i + 1] = y;
        nodes[3 * i + 2] = z;
    }
    const size_t np_ = sp.nodes.size();
    if (dcmp)
        for (int t = 0; t < nt; t++)
            for (size_t i = 0; i < np_; i++) dcmp[(size_t)t * cap + i] = dc[(size_t)t * np_ + i];
    return TB_OK;
}

namespace tbw {
tb_status inspect_into(tb_sparse *s, int nsrc, const double *src_xyz, const double *wav,
                       int nrec, const double *rec_xyz)
{
    const tb_model *m = s->m;
    Support ss, rs;
    tb_status st = build_support(m->n, m->h, m->o, nsrc, src_xyz, &ss);
    if (st) return st;
    st = build_support(m->n, m->h, m->o, nrec, rec_xyz, &rs);
    if (st) return st;
    s->nsrc = nsrc;
    s->nrec = nrec;
    s->nt = m->nt;
    s->npts = (int)ss.nodes.size();
    s->src_nodes = ss.nodes;
    s->sc_ptr = ss.ptr;
    s->sc_id = ss.id;
    s->sc_w = ss.w;
    std::vector<double> cn(ss.nodes.size());
    for (size_t i = 0; i < ss.nodes.size(); i++) cn[i] = m->inj_coef(ss.nodes[i]);
    decompose(ss, nsrc, m->nt, wav, cn, &s->dcmp);
    s->nrid = (int)rs.nodes.size();
    s->rid_nodes = rs.nodes;
    s->rc_ptr = rs.ptr;
    s->rc_id = rs.id;
    s->rc_w = rs.w;
    if (m->physics == TB_ELASTIC) {
        // vz lives half a cell above the nodes in z: its own receiver mirror.
        const double o2[3] = {m->o[0], m->o[1], m->o[2] + 0.5 * m->h[2]};
        Support r2;
        if ((st = build_support(m->n, m->h, o2, nrec, rec_xyz, &r2))) return st;
        s->nrid2 = (int)r2.nodes.size();
        s->rid2_nodes = r2.nodes;
        s->rc2_ptr = r2.ptr;
        s->rc2_id = r2.id;
        s->rc2_w = r2.w;
    }
    return TB_OK;
}
}  // namespace tbw

extern "C" tb_status tb_schedule_segments_host(const int32_t shape[3], int32_t space_order,
                                               const tb_schedule *s, int32_t wgs, int32_t tile[4],
                                               int32_t *nseg, int32_t *seg)
{
    if (!shape || !s || !tile || !nseg || wgs < 1 || shape[0] < 1 || shape[1] < 1 ||
        shape[2] < 1) {
        tbw::set_error("tb_schedule_segments_host: invalid argument");
        return TB_EINVAL;
    }
    if (space_order != 4 && space_order != 8 && space_order != 12) {
        tbw::set_error("tb_schedule_segments_host: space order %d not in {4, 8, 12}", space_order);
        return TB_EUNSUPPORTED;
    }
    const int R = space_order / 2;
    const int T = s->mode == TB_SCHED_SB ? 1 : s->time_tile;
    int lz = 0, bye = 0;
    if (T < 1 || T > 4 || s->chunk_x < 0 ||
        (s->tile_y != 0 && s->tile_y != 16 && s->tile_y != 32)) {
        tbw::set_error("tb_schedule_segments_host: schedule out of range");
        return TB_EINVAL;
    }
    tbw::tile_shape(R, T, s->tile_y, &lz, &bye);
    if (!tbw::acoustic_shape_ok(R, T, lz, bye)) {
        tbw::set_error("tb_schedule_segments_host: no kernel for radius %d, depth %d, %d rows", R,
                       T, bye);
        return TB_EUNSUPPORTED;
    }
    const tbw::TileGeom g = tbw::make_geom(R, T, s->tile_y, s->chunk_x, wgs, shape[0], shape[1],
                                           shape[2]);
    tile[0] = g.BYE;
    tile[1] = 4 * g.LZ;
    tile[2] = g.OY;
    tile[3] = g.OZ;
    const int n = (int)g.segs.size();
    const int cap = *nseg;
    *nseg = n;
    if (n > cap || (n > 0 && !seg)) {
        tbw::set_error("tb_schedule_segments_host: %d segments exceed capacity %d", n, cap);
        return TB_EWORKSPACE;
    }
    for (int w = 0; w < g.nwg; w++)
        for (int k = g.seg_off[w]; k < g.seg_off[w + 1]; k++) {
            const tbw::SegDesc &d = g.segs[k];
            int32_t *o = seg + 5 * k;
            o[0] = w;
            o[1] = d.tile / g.tiles_z;
            o[2] = d.tile % g.tiles_z;
            o[3] = d.xs;
            o[4] = d.xe;
        }
    return TB_OK;
}
