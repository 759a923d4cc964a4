// Host launch code of the acoustic propagator and the small auxiliary kernels
// (fill, trace reduction, unpadding, adjoint source assembly). The wave-front
// kernel itself lives in acoustic_kernel.h.
#include "acoustic_params.h"

namespace tbw {
namespace {

__global__ void fill_kernel(float *p, size_t n, float v)
{
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// d[n][r] = sum_k W_rk rec_dcmp[row(n)][rid_k], corners in their fixed order.
__global__ void trace_reduce_kernel(const float *__restrict__ rec_dcmp, int nrid, int nt,
                                    const int *__restrict__ ptr, const int *__restrict__ id,
                                    const float *__restrict__ w, int nrec, float *out, int reverse)
{
    const long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (g >= (long long)nt * nrec) return;
    const int n = (int)(g / nrec), r = (int)(g % nrec);
    const int rowi = reverse ? nt - 1 - n : n;
    const float *src = rec_dcmp + (long long)rowi * nrid;
    float acc = 0.0f;
    for (int k = ptr[r]; k < ptr[r + 1]; k++) acc = __builtin_fmaf(w[k], src[id[k]], acc);
    out[g] = acc;
}

__global__ void unpad_kernel(const float *__restrict__ src, float *__restrict__ dst, int nx,
                             int ny, int nz, int nzp)
{
    const long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long total = (long long)nx * ny * nz;
    if (g >= total) return;
    const int zz = (int)(g % nz);
    const long long xy = g / nz;
    dst[g] = src[xy * nzp + zz];
}

// Adjoint source term: dcmp_out[tau][rid] = scale[rid] * sum W res[nt-1-tau][rec]
// (scale 1 where rid_scale is NULL).
__global__ void adj_inject_kernel(const float *__restrict__ res, int nt, int nrec, int nrid,
                                  const int *__restrict__ rr_ptr, const int *__restrict__ rr_rec,
                                  const float *__restrict__ rr_w,
                                  const float *__restrict__ rid_scale, float *dcmp_out)
{
    const long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (g >= (long long)nt * nrid) return;
    const int tau = (int)(g / nrid), rid = (int)(g % nrid);
    const float *rv = res + (long long)(nt - 1 - tau) * nrec;
    float acc = 0.0f;
    for (int k = rr_ptr[rid]; k < rr_ptr[rid + 1]; k++)
        acc = __builtin_fmaf(rr_w[k], rv[rr_rec[k]], acc);
    dcmp_out[g] = rid_scale ? rid_scale[rid] * acc : acc;
}

}  // namespace

AcParams make_params(const tb_model *m, const TileLists &tl, const AcLaunch &a)
{
    const TileGeom &g = tl.g;
    AcParams p{};
    p.u = a.u;
    p.v = a.v;
    p.c = m->d_c;
    p.zero = m->d_zero;
    p.out_u = a.out_u;
    p.out_v = a.out_v;
    p.out_mid = a.out_mid;
    p.dx = m->d_damp;
    p.dy = m->d_damp + m->n[0];
    p.dz = m->d_damp + m->n[0] + m->n[1];
    p.hdt = (float)(m->dt / 2.0);
    // Centred second-derivative weights of order so (Fornberg), tabulated
    // as exact rationals and scaled by h^-2 per axis; the kernel applies them
    // to differences from the centre, so the centre weight is not needed.
    static const double w4[3] = {-5.0 / 2.0, 4.0 / 3.0, -1.0 / 12.0};
    static const double w8[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
    static const double w12[7] = {-5369.0 / 1800.0, 12.0 / 7.0, -15.0 / 56.0, 10.0 / 189.0,
                                  -1.0 / 112.0,     2.0 / 1925.0, -1.0 / 16632.0};
    const double *w = m->so == 4 ? w4 : (m->so == 8 ? w8 : w12);
    const double ihx = 1.0 / (m->h[0] * m->h[0]), ihy = 1.0 / (m->h[1] * m->h[1]),
                 ihz = 1.0 / (m->h[2] * m->h[2]);
    for (int j = 0; j < 6; j++) {
        const double wj = j < m->r ? w[j + 1] : 0.0;
        p.wx[j] = (float)(wj * ihx);
        p.wy[j] = (float)(wj * ihy);
        p.wz[j] = (float)(wj * ihz);
    }
    p.iso = 1;
    for (int j = 0; j < 6; j++) p.iso &= p.wx[j] == p.wy[j] && p.wx[j] == p.wz[j];
    p.nx = m->n[0];
    p.ny = m->n[1];
    p.nz = m->n[2];
    p.nzp = m->nzp;
    p.sx = (long long)m->n[1] * m->nzp;
    p.tiles_z = g.tiles_z;
    p.nwg = g.nwg;
    p.segs = tl.d_segs;
    p.seg_off = tl.d_seg_off;
    p.src = tl.d_src;
    p.dcmp = a.dcmp;
    p.npts = a.npts;
    p.n0 = a.n0;
    p.rec = tl.d_rec;
    p.rec_dcmp = a.rec_dcmp;
    p.nrid = a.nrid;
    return p;
}

tb_status launch_acoustic(const tb_model *m, const TileLists &tl, const AcLaunch &a,
                          hipStream_t st)
{
    const TileGeom &g = tl.g;
    const AcParams p = make_params(m, tl, a);
    hipError_t e = hipErrorInvalidValue;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (timing_enabled()) timing_begin(st, &ev0, &ev1);
    const bool gl = tl.max_src > kSrcCap;
    if (m->r == 2) e = launch_acoustic_r2(p, g.T, g.LZ, g.BYE, gl, st);
    else if (m->r == 4) e = launch_acoustic_r4(p, g.T, g.LZ, g.BYE, gl, st);
    else if (m->r == 6) e = launch_acoustic_r6(p, g.T, g.LZ, g.BYE, gl, st);
    if (ev0) timing_end(st, ev0, ev1);
    if (e != hipSuccess) {
        set_error("acoustic kernel launch (R=%d T=%d LZ=%d BYE=%d) failed: %s", m->r, g.T, g.LZ,
                  g.BYE, hipGetErrorString(e));
        return TB_EHIP;
    }
    return TB_OK;
}

bool acoustic_shape_ok(int R, int T, int LZ, int BYE)
{
    return R == 2   ? acoustic_shape_ok_r2(T, LZ, BYE)
           : R == 4 ? acoustic_shape_ok_r4(T, LZ, BYE)
           : R == 6 ? acoustic_shape_ok_r6(T, LZ, BYE)
                    : false;
}

bool acoustic_lists_in_lds(int R, int T, int LZ, int BYE)
{
    return R == 2   ? acoustic_lists_in_lds_r2(T, LZ, BYE)
           : R == 4 ? acoustic_lists_in_lds_r4(T, LZ, BYE)
           : R == 6 ? acoustic_lists_in_lds_r6(T, LZ, BYE)
                    : false;
}

tb_status launch_acoustic_batch(int r, const AcParams *d_jobs, const int *d_wgoff, int njobs,
                                int total_wg, int T, int LZ, int BYE, hipStream_t st,
                                bool allow_timing)
{
    if (njobs == 0 || total_wg == 0) return TB_OK;
    hipError_t e = hipErrorInvalidValue;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (allow_timing && timing_enabled()) timing_begin(st, &ev0, &ev1);
    if (r == 2) e = launch_acoustic_batch_r2(d_jobs, d_wgoff, njobs, total_wg, T, LZ, BYE, st);
    else if (r == 4) e = launch_acoustic_batch_r4(d_jobs, d_wgoff, njobs, total_wg, T, LZ, BYE, st);
    else if (r == 6) e = launch_acoustic_batch_r6(d_jobs, d_wgoff, njobs, total_wg, T, LZ, BYE, st);
    if (ev0) timing_end(st, ev0, ev1);
    if (e != hipSuccess) {
        set_error("batched acoustic kernel launch (R=%d T=%d LZ=%d BYE=%d, %d jobs) failed: %s", r,
                  T, LZ, BYE, njobs, hipGetErrorString(e));
        return TB_EHIP;
    }
    return TB_OK;
}

// ---------------------------------------------------------------------------
// Optional per-launch timing (tb_kernel_timing).
namespace {
std::mutex g_tmu;
bool g_timing = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events;
double g_done_ms = 0.0;
int g_done_n = 0;
}  // namespace

bool timing_enabled()
{
    std::lock_guard<std::mutex> lk(g_tmu);
    return g_timing;
}

void timing_begin(hipStream_t st, hipEvent_t *a, hipEvent_t *b)
{
    if (hipEventCreate(a) != hipSuccess || hipEventCreate(b) != hipSuccess) {
        *a = *b = nullptr;
        return;
    }
    (void)hipEventRecord(*a, st);
}

void timing_end(hipStream_t st, hipEvent_t a, hipEvent_t b)
{
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_tmu);
    g_events.emplace_back(a, b);
}

static void timing_drain(bool keep)
{
    for (auto &e : g_events) {
        if (keep) {
            (void)hipEventSynchronize(e.second);
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) {
                g_done_ms += ms;
                g_done_n++;
            }
        }
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    g_events.clear();
}

tb_status kernel_timing(int enable)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    timing_drain(false);
    g_done_ms = 0.0;
    g_done_n = 0;
    g_timing = enable != 0;
    return TB_OK;
}

tb_status kernel_timing_read(int *n, double *ms)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    timing_drain(true);
    if (n) *n = g_done_n;
    if (ms) *ms = g_done_ms;
    return TB_OK;
}

tb_status launch_fill(float *ptr, size_t n, float v, hipStream_t st)
{
    if (n == 0) return TB_OK;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, ptr, n, v);
    TB_HIP(hipGetLastError());
    return TB_OK;
}

// c = dt^2 vp^2, or c = dt^2 / m from the squared slowness (is_m), in FP64
// and rounded once; the padding columns z >= nz are zero.
__global__ void c_from_vp_kernel(const float *__restrict__ vp, float *__restrict__ c, int ny,
                                 int nz, int nzp, long long n, double dt, int is_m)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int z = (int)(i % nzp);
        const long long xy = i / nzp;
        float out = 0.0f;
        if (z < nz) {
            const double v = (double)vp[xy * nz + z];
            out = is_m ? (float)(dt * dt / v) : (float)(dt * dt * v * v);
        }
        c[i] = out;
    }
}

tb_status launch_c_from_vp(const float *vp, float *c, int nx, int ny, int nz, int nzp, double dt,
                           bool is_m, hipStream_t st)
{
    const long long n = (long long)nx * ny * nzp;
    if (n == 0) return TB_OK;
    long long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(c_from_vp_kernel, dim3((unsigned)blocks), dim3(256), 0, st, vp, c, ny, nz,
                       nzp, n, dt, (int)is_m);
    TB_HIP(hipGetLastError());
    return TB_OK;
}

tb_status launch_trace_reduce(const float *rec_dcmp, int nrid, int nt, const int *ptr,
                              const int *id, const float *w, int nrec, float *out, int reverse,
                              hipStream_t st)
{
    const long long total = (long long)nt * nrec;
    if (total == 0) return TB_OK;
    hipLaunchKernelGGL(trace_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       st, rec_dcmp, nrid, nt, ptr, id, w, nrec, out, reverse);
    TB_HIP(hipGetLastError());
    return TB_OK;
}

tb_status launch_unpad(const float *src, float *dst, int nx, int ny, int nz, int nzp,
                       hipStream_t st)
{
    const long long total = (long long)nx * ny * nz;
    if (nz == nzp) {
        TB_HIP(hipMemcpyAsync(dst, src, total * sizeof(float), hipMemcpyDeviceToDevice, st));
        return TB_OK;
    }
    hipLaunchKernelGGL(unpad_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, src,
                       dst, nx, ny, nz, nzp);
    TB_HIP(hipGetLastError());
    return TB_OK;
}

tb_status launch_adj_inject(const float *res, int nt, int nrec, int nrid, const int *rr_ptr,
                            const int *rr_rec, const float *rr_w, const float *rid_scale,
                            float *dcmp_out, hipStream_t st)
{
    const long long total = (long long)nt * nrid;
    if (total == 0) return TB_OK;
    hipLaunchKernelGGL(adj_inject_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       res, nt, nrec, nrid, rr_ptr, rr_rec, rr_w, rid_scale, dcmp_out);
    TB_HIP(hipGetLastError());
    return TB_OK;
}

}  // namespace tbw
