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

TileGeom make_geom(int R, int T, int BYE, int chunk, int nx, int ny, int nz)
{
    TileGeom g;
    g.R = R;
    g.T = T;
    g.BYE = BYE;
    g.HY = R * (T - 1);
    g.HZ = ((R * (T - 1) + 3) / 4) * 4;
    g.OY = BYE - 2 * g.HY;
    g.OZ = kTileZ - 2 * g.HZ;
    g.chunk = (chunk <= 0 || chunk > nx) ? nx : chunk;
    if (g.chunk > kMaxChunk) g.chunk = kMaxChunk;
    g.tiles_y = g.OY > 0 ? (ny + g.OY - 1) / g.OY : 0;
    g.tiles_z = g.OZ > 0 ? (nz + g.OZ - 1) / g.OZ : 0;
    g.nchunks = (nx + g.chunk - 1) / g.chunk;
    return g;
}

TileLists::~TileLists()
{
    if (d_src) (void)hipFree(d_src);
    if (d_src_off) (void)hipFree(d_src_off);
    if (d_rec) (void)hipFree(d_rec);
    if (d_rec_off) (void)hipFree(d_rec_off);
}

// Tile index of (chunk, tile_y, tile_z), z fastest: the kernels decode it the
// same way.
static inline int tile_index(const TileGeom &g, int ch, int ty, int tz)
{
    return (ch * g.tiles_y + ty) * g.tiles_z + tz;
}

static void bin_points(const TileGeom &g, const int n[3], const std::vector<int64_t> &nodes,
                       bool owned_only, std::vector<std::vector<int2>> *bins)
{
    const int halo_x = g.R * (g.T - 1);
    for (size_t id = 0; id < nodes.size(); id++) {
        int x, y, z;
        node_xyz(nodes[id], n, &x, &y, &z);
        // Candidate tiles along each axis.
        int ty_lo, ty_hi, tz_lo, tz_hi, ch_lo, ch_hi;
        if (owned_only) {
            ty_lo = ty_hi = y / g.OY;
            tz_lo = tz_hi = z / g.OZ;
            ch_lo = ch_hi = x / g.chunk;
        } else {
            // tile t covers rows [t*OY - HY, t*OY - HY + BYE); the exact test
            // is applied below, this only bounds the candidates.
            ty_hi = std::min(g.tiles_y - 1, (y + g.HY) / g.OY);
            ty_lo = std::max(0, ty_hi - (g.BYE / g.OY + 2));
            tz_hi = std::min(g.tiles_z - 1, (z + g.HZ) / g.OZ);
            tz_lo = std::max(0, tz_hi - (kTileZ / g.OZ + 2));
            ch_lo = 0;
            ch_hi = g.nchunks - 1;
        }
        for (int ch = ch_lo; ch <= ch_hi; ch++) {
            int xc0 = ch * g.chunk, xc1 = std::min(n[0], xc0 + g.chunk);
            if (owned_only) {
                if (x < xc0 || x >= xc1) continue;
            } else if (x < xc0 - halo_x || x >= xc1 + halo_x) {
                continue;
            }
            for (int ty = ty_lo; ty <= ty_hi; ty++) {
                int y0 = ty * g.OY - g.HY;
                int row = y - y0;
                if (owned_only ? (row < g.HY || row >= g.HY + g.OY) : (row < 0 || row >= g.BYE))
                    continue;
                for (int tz = tz_lo; tz <= tz_hi; tz++) {
                    int z0 = tz * g.OZ - g.HZ;
                    int col = z - z0;
                    if (owned_only ? (col < g.HZ || col >= g.HZ + g.OZ)
                                   : (col < 0 || col >= kTileZ))
                        continue;
                    (*bins)[tile_index(g, ch, ty, tz)].push_back(
                        make_int2(tile_key(row, col >> 2, x, col & 3), (int)id));
                }
            }
        }
    }
    for (auto &b : *bins)
        std::sort(b.begin(), b.end(), [](const int2 &a, const int2 &c) { return a.x < c.x; });
}

static tb_status upload_csr(const std::vector<std::vector<int2>> &bins, int2 **d_list,
                            int **d_off, int *count, int *longest)
{
    std::vector<int> off(bins.size() + 1, 0);
    *longest = 0;
    for (size_t t = 0; t < bins.size(); t++) {
        off[t + 1] = off[t] + (int)bins[t].size();
        *longest = std::max(*longest, (int)bins[t].size());
    }
    std::vector<int2> flat;
    flat.reserve(off.back() + 1);
    for (auto &b : bins) flat.insert(flat.end(), b.begin(), b.end());
    flat.push_back(make_int2(0x7fffffff, 0));  // sentinel
    *count = off.back();
    TB_HIP(hipMalloc(d_list, flat.size() * sizeof(int2)));
    TB_HIP(hipMemcpy(*d_list, flat.data(), flat.size() * sizeof(int2), hipMemcpyHostToDevice));
    TB_HIP(hipMalloc(d_off, off.size() * sizeof(int)));
    TB_HIP(hipMemcpy(*d_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice));
    return TB_OK;
}

tb_status build_tile_lists(const tb_model *m, const std::vector<int64_t> &inj,
                           const std::vector<int64_t> &rec, const TileGeom &g, TileLists *out)
{
    const int nb = g.nblocks();
    std::vector<std::vector<int2>> sb(nb), rb(nb);
    bin_points(g, m->n, inj, false, &sb);
    bin_points(g, m->n, rec, true, &rb);
    tb_status st = upload_csr(sb, &out->d_src, &out->d_src_off, &out->nsrc_entries, &out->max_src);
    if (st) return st;
    return upload_csr(rb, &out->d_rec, &out->d_rec_off, &out->nrec_entries, &out->max_rec);
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
    for (size_t i = 0; i < ss.nodes.size(); i++) cn[i] = m->c64[ss.nodes[i]];
    decompose(ss, nsrc, m->nt, wav, cn, &s->dcmp);
    s->nrid = (int)rs.nodes.size();
    s->rid_nodes = rs.nodes;
    s->rc_ptr = rs.ptr;
    s->rc_id = rs.id;
    s->rc_w = rs.w;
    return TB_OK;
}
}  // namespace tbw
