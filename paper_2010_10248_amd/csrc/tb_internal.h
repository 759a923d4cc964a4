// Internal host-side structures of the temporal-blocking library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/tb.h"

namespace tbw {

// Error reporting: thread-local text behind tb_last_error().
void set_error(const char *fmt, ...);
#define TB_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            ::tbw::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),    \
                             __FILE__, __LINE__);                                      \
            return TB_EHIP;                                                            \
        }                                                                              \
    } while (0)

// Each lane of the acoustic kernels holds 4 consecutive z as one float4; a
// tile row has 16 lanes (one DPP row).
constexpr int kMaxThreads = 512;
// LDS of one workgroup on gfx950.
constexpr int kLdsBytes = 160 * 1024;
// Longest x range one work segment streams (its damping values sit in LDS).
constexpr int kMaxChunk = 1024;
// Injection entries one segment can stage in LDS; a segment with more runs
// the variant that walks its injection list in global memory. (Receiver
// lists stay in global memory: they are read a few entries ahead.)
constexpr int kSrcCap = 1024;

// An injection-list entry: key = ((row*32 + lane) << 18) | (x << 2) | k,
// with k the z component inside the lane's float4; id = point ID. Sorted by
// key, so each lane's entries are contiguous and ordered by x.
__host__ __device__ inline int tile_key(int row, int lane, int x, int k)
{
    return ((row * 32 + lane) << 18) | (x << 2) | k;
}
// A receiver-list entry: key = (x << 11) | (row << 6) | (lane << 2) | k
// (row < 32, lane < 16); sorted by key, so the entries of one plane are
// contiguous and the planes come in x order.
__host__ __device__ inline int rec_key(int row, int lane, int x, int k)
{
    return (x << 11) | (row << 6) | (lane << 2) | k;
}

// One unit of work of a workgroup: tile `tile` over planes [xs, xe), with the
// offsets of its injection and receiver lists.
struct SegDesc {
    int tile, xs, xe, pad;
    int sbeg, sn, rbeg, rn;
};

// Geometry of one schedule (shared by the binning and the launch code).
struct TileGeom {
    int R = 0, T = 1;
    int LZ = 16, BYE = 32;  // lanes per tile row, rows per tile
    int HY = 0, HZ = 0;     // halo rows / halo columns (columns multiple of 4)
    int OY = 0, OZ = 0;     // owned rows / owned columns per tile
    int tiles_y = 0, tiles_z = 0;
    int chunk = 0;          // > 0: one workgroup per (tile, chunk of x)
    int nwg = 0;            // workgroups of the launch
    std::vector<SegDesc> segs;  // work segments (list fields filled by binning)
    std::vector<int> seg_off;   // per workgroup: [seg_off[b], seg_off[b+1])
    int ntiles() const { return tiles_y * tiles_z; }
};
// Tile shape: 16 lanes (64 z) and tile_y rows; tile_y == 0 picks 32 rows
// where that shape fits the kernel's LDS for (R, T), else 16. chunk > 0 gives one workgroup per
// (tile, chunk of x); chunk == 0 partitions the tile-x space evenly over
// `wgs` workgroups.
TileGeom make_geom(int R, int T, int tile_y, int chunk, int wgs, int nx, int ny, int nz);
// Lanes per row and rows of the tile a schedule selects.
void tile_shape(int R, int T, int tile_y, int *LZ, int *BYE);
// Whether the wave-front kernel is built for this radius, depth and shape
// (it must fit the LDS of one workgroup).
bool acoustic_shape_ok(int R, int T, int LZ, int BYE);

// Per-segment injection / recording lists, entries {key, id}, and the
// segment table of one schedule geometry.
struct TileLists {
    TileGeom g;
    int2 *d_src = nullptr;
    int2 *d_rec = nullptr;
    SegDesc *d_segs = nullptr;
    int *d_seg_off = nullptr;
    int nsrc_entries = 0, nrec_entries = 0;
    int max_src = 0, max_rec = 0;  // longest list of one segment
    ~TileLists();
};

}  // namespace tbw

struct tb_model {
    int physics = TB_ACOUSTIC;
    int n[3] = {0, 0, 0};
    int nzp = 0;  // padded row length (multiple of 4)
    double h[3] = {0, 0, 0}, o[3] = {0, 0, 0};
    int so = 8, r = 4, nbl = 0;
    double dt = 0;
    int nt = 0;
    double vmax = 0;  // velocity of the damping profile
    int device = 0;
    int ncu = 1;              // compute units of the device
    float *d_c = nullptr;     // dt^2 vp^2, [nx][ny][nzp]
    float *d_damp = nullptr;  // d_x[nx] | d_y[ny] | d_z[nzp]
    float *d_zero = nullptr;  // 256 zeroed bytes
    // TTI: five padded fields ax, ay, az (symmetry axis), 1 + 2 eps and
    // sqrt(1 + 2 min(delta, eps)), each field_elems() long.
    float *d_tti = nullptr;
    // Elastic: eight padded fields, each multiplied by dt: b at the vx, vy,
    // vz points, lambda and mu at the nodes, mu at the txy, txz, tyz points.
    float *d_el = nullptr;
    std::vector<float> vp_host;  // host copy of vp [nx][ny][nz] (of m = 1/vp^2 if host_is_m)
    bool host_is_m = false;
    std::vector<float> damp;     // host copy of the three tables
    // The inspector's scale of injected values at raster point i: dt^2 vp^2
    // or dt^2/m (FP64 from the FP32 input; the value the device field c
    // rounds) for the second-order systems, dt for the stress injection of
    // the elastic one.
    double inj_coef(int64_t i) const
    {
        if (physics == TB_ELASTIC) return dt;
        const double v = (double)vp_host[i];
        return host_is_m ? dt * dt / v : dt * dt * v * v;
    }
    size_t field_elems() const { return (size_t)n[0] * n[1] * nzp; }
    ~tb_model();
};

struct tb_sparse {
    const tb_model *m = nullptr;
    int nsrc = 0, nrec = 0, nt = 0;
    // Source side (inspector, Section II-A): unique affected points.
    int npts = 0;
    std::vector<int64_t> src_nodes;  // raster index x*ny*nz + y*nz + z, ascending = SID
    std::vector<float> dcmp;         // [nt][npts]
    float *d_dcmp = nullptr;
    // Per source: corners (sid, W) in corner order (adjoint read-out).
    std::vector<int> sc_ptr, sc_id;
    std::vector<double> sc_w;
    // Receiver mirror: unique points and per-receiver corners (rid, W).
    int nrid = 0;
    std::vector<int64_t> rid_nodes;
    std::vector<int> rc_ptr, rc_id;
    std::vector<double> rc_w;
    int *d_rc_ptr = nullptr, *d_rc_id = nullptr;
    float *d_rc_w = nullptr;
    // Adjoint: source read-out weights W * alpha(node), and receiver-point
    // injection scale c/alpha at each rid.
    int *d_sc_ptr = nullptr, *d_sc_id = nullptr;
    float *d_sc_w = nullptr;
    // For each rid: receivers hitting it and their weights (adjoint injection).
    int *d_rr_ptr = nullptr, *d_rr_rec = nullptr;
    float *d_rr_w = nullptr;
    float *d_rid_scale = nullptr;  // (c/alpha)(rid node)
    // Imaging at the injection points: padded offset and alpha of each SID.
    long long *d_src_off = nullptr;
    double *d_src_alpha = nullptr;
    // Padded offsets of the receiver points (gathers outside the wave-front
    // kernel).
    long long *d_rid_off = nullptr;
    // Elastic: the receiver mirror on the vz grid (origin + h/2 in z).
    int nrid2 = 0;
    std::vector<int64_t> rid2_nodes;
    std::vector<int> rc2_ptr, rc2_id;
    std::vector<double> rc2_w;
    int *d_rc2_ptr = nullptr, *d_rc2_id = nullptr;
    float *d_rc2_w = nullptr;
    long long *d_rid2_off = nullptr;
    // Transposed vz mirror for the adjoint: rid2 -> (receiver, W).
    int *d_rr2_ptr = nullptr, *d_rr2_rec = nullptr;
    float *d_rr2_w = nullptr;
    std::mutex mu;
    std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<tbw::TileLists>> tiles;
    ~tb_sparse();
};

namespace tbw {

// Host inspector: support, IDs and FP64 decomposition.
struct Support {
    std::vector<int64_t> nodes;  // unique raster indices, ascending
    std::vector<int> ptr, id;    // per point: corners (index into nodes)
    std::vector<double> w;       // corner weights
};
tb_status build_support(const int n[3], const double h[3], const double o[3], int npts_in,
                        const double *xyz, Support *out);

// Bin points into per-tile lists for a schedule geometry.
// inj: points injected at every computed copy (extended region); rec: points
// recorded from the owned copy only.
tb_status build_tile_lists(const tb_model *m, const std::vector<int64_t> &inj,
                           const std::vector<int64_t> &rec, TileLists *out);

// Kernel launchers (acoustic.hip).
struct AcLaunch {
    const float *u, *v;  // u^n, v^n = u^n - u^{n-1}
    float *out_u, *out_v, *out_mid;  // u^{n+T}, v^{n+T}, u^{n+T-1} (or NULL)
    int n0;  // time index of the first update of this pass
    const float *dcmp;
    int npts;
    float *rec_dcmp;
    int nrid;
};
tb_status launch_acoustic(const tb_model *m, const TileLists &tl, const AcLaunch &a,
                          hipStream_t st);
tb_status launch_fill(float *p, size_t n, float v, hipStream_t st);
// c[x][y][z] = dt^2 vp^2 (FP64, rounded once) over the padded layout [nx][ny][nzp]
// (0 in the padding), from vp [nx][ny][nz].
tb_status launch_c_from_vp(const float *vp, float *c, int nx, int ny, int nz, int nzp, double dt,
                           bool is_m, hipStream_t st);
tb_status kernel_timing(int enable);
tb_status kernel_timing_read(int *n, double *ms);
tb_status launch_trace_reduce(const float *rec_dcmp, int nrid, int nt, const int *ptr,
                              const int *id, const float *w, int nrec, float *out,
                              int reverse, hipStream_t st);
tb_status launch_unpad(const float *src, float *dst, int nx, int ny, int nz, int nzp,
                       hipStream_t st);
// rid_scale NULL: unit scale.
tb_status launch_adj_inject(const float *res, int nt, int nrec, int nrid, const int *rr_ptr,
                            const int *rr_rec, const float *rr_w, const float *rid_scale,
                            float *dcmp_out, hipStream_t st);

// Gradient kernels (imaging.hip).
// Imaging of one or two consecutive levels in one pass over memory:
// g += nu[l] * c * L(u[l]) for l = 0 .. nlev-1, in that order.
struct ImageArgs {
    const float *nu[2], *u[2];
    int nlev;
    const float *c;
    double *g;
    int nx, ny, nz, nzp, r;
    double w[3][7];  // centred second-derivative weights per axis, scaled by h^-2
};
tb_status launch_residual_loss(const float *d, const float *dobs, long long n, float *res,
                               double *loss, hipStream_t st);
tb_status launch_image(const ImageArgs &a, hipStream_t st);
// gs[i] += nu[off[i]] * alpha[i] * s[i] at the injection points (a separate
// accumulator, merged into g once by launch_image_merge).
tb_status launch_image_sparse(const float *nu, const float *s, int npts, const long long *off,
                              const double *alpha, double *gs, hipStream_t st);
tb_status launch_image_merge(const double *gs, int npts, const long long *off, double *g,
                             hipStream_t st);
tb_status launch_finish_grad(const double *g, float *out, int nx, int ny, int nz, int nzp,
                             double scale, hipStream_t st);
tb_status launch_zero64(double *p, size_t n, hipStream_t st);

}  // namespace tbw
