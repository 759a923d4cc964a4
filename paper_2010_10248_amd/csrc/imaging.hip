// Kernels of the squared-slowness gradient of the acoustic propagator: the
// data residual and its misfit, the imaging condition and the final scaling.
//
// With the forward update written as
//   alpha u^k = c L u^{k-1} + 2 u^{k-1} - beta u^{k-2} + alpha s^{k-1},
// (s^{k-1} the injected increment of step k-1, c = dt^2 / m) and nu the
// adjoint wavefield in the scaling that makes the adjoint recursion the same
// update run backward in time, the gradient of J = 1/2 sum_k |P_r u^k - d^k|^2
// with respect to m is
//   dJ/dm = -(1/dt^2) sum_{k>=1} nu^k (c L u^{k-1} + alpha s^{k-1}),
// which includes the m-dependence of the dt^2/m source scaling. The paper
// motivates the adjoint by full-waveform inversion and reverse-time migration
// (Section I) and leaves its form open; this is the exact discrete adjoint of
// the update of equation (acou).
//
// The Laplacian of the imaging term is evaluated in FP64 from the FP32 field,
// and the gradient accumulates in FP64, so that the sum over nt levels adds
// no FP32 rounding of its own.
#include <cstdint>

#include "tb_internal.h"

namespace tbw {
namespace {

// res = d - d_obs over nt x nrec samples.
__global__ void residual_kernel(const float *__restrict__ d, const float *__restrict__ dobs,
                                long long n, float *__restrict__ res)
{
    const long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (g < n) res[g] = d[g] - dobs[g];
}

// J = 1/2 sum res^2 in FP64 by one workgroup in a fixed order (strided
// per-thread partial sums, then a tree), so the value is reproducible.
constexpr int kLossThreads = 1024;
__global__ void __launch_bounds__(kLossThreads)
    loss_kernel(const float *__restrict__ res, long long n, double *__restrict__ out)
{
    __shared__ double part[kLossThreads];
    double acc = 0.0;
    for (long long i = threadIdx.x; i < n; i += kLossThreads) {
        const double r = res[i];
        acc += 0.5 * r * r;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kLossThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0];
}

// g += nu * c * L(u) for one or two levels; each thread takes 4 consecutive z
// (float4 loads of the fields; the z neighbours come from the two float4 on
// each side, enough for radius 6), z padding skipped.
__global__ void __launch_bounds__(256) image_kernel(const ImageArgs a)
{
    const int nz4 = a.nzp / 4;
    const long long total = (long long)a.nx * a.ny * nz4;
    const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (gid >= total) return;
    const int z4 = (int)(gid % nz4) * 4;
    const long long xy = gid / nz4;
    const int y = (int)(xy % a.ny);
    const int x = (int)(xy / a.ny);
    const long long sx = (long long)a.ny * a.nzp;
    const long long off = xy * a.nzp + z4;
    typedef float f4 __attribute__((ext_vector_type(4)));
    auto ld4 = [&](const float *f, long long o, bool in) {
        return in ? *(const f4 *)(f + o) : f4{0.f, 0.f, 0.f, 0.f};
    };
    const f4 cc = ld4(a.c, off, true);
    double acc[4];
#pragma unroll
    for (int k = 0; k < 4; k++) acc[k] = 0.0;
    bool touched = false;
    for (int l = 0; l < a.nlev; l++) {
        const f4 nu = ld4(a.nu[l], off, true);
        // A zero adjoint level adds +0 to a finite g: skip its stencil.
        if (nu[0] == 0.0f && nu[1] == 0.0f && nu[2] == 0.0f && nu[3] == 0.0f) continue;
        const float *u = a.u[l];
        // z window [z4-8, z4+12): two float4 on each side cover radius 6.
        const f4 uc = ld4(u, off, true);
        float zw[20];
#pragma unroll
        for (int o = -8; o <= 8; o += 4) {
            const f4 t = o == 0 ? uc : ld4(u, off + o, z4 + o >= 0 && z4 + o < a.nzp);
#pragma unroll
            for (int k = 0; k < 4; k++) zw[8 + o + k] = t[k];
        }
        double lx[4], ly[4], lz[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            lx[k] = a.w[0][0] * (double)uc[k];
            ly[k] = a.w[1][0] * (double)uc[k];
            lz[k] = a.w[2][0] * (double)uc[k];
        }
        for (int j = 1; j <= a.r; j++) {
            const f4 xm = ld4(u, off - j * sx, x - j >= 0);
            const f4 xp = ld4(u, off + j * sx, x + j < a.nx);
            const f4 ym = ld4(u, off - (long long)j * a.nzp, y - j >= 0);
            const f4 yp = ld4(u, off + (long long)j * a.nzp, y + j < a.ny);
#pragma unroll
            for (int k = 0; k < 4; k++) {
                lx[k] += a.w[0][j] * ((double)xm[k] + (double)xp[k]);
                ly[k] += a.w[1][j] * ((double)ym[k] + (double)yp[k]);
                lz[k] += a.w[2][j] * ((double)zw[8 + k - j] + (double)zw[8 + k + j]);
            }
        }
        double *g = a.g + off;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (z4 + k >= a.nz || nu[k] == 0.0f) continue;
            if (!touched) {
#pragma unroll
                for (int kk = 0; kk < 4; kk++) acc[kk] = z4 + kk < a.nz ? g[kk] : 0.0;
                touched = true;
            }
            acc[k] += (double)nu[k] * ((double)cc[k] * (lx[k] + ly[k] + lz[k]));
        }
    }
    if (touched) {
        double *g = a.g + off;
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (z4 + k < a.nz) g[k] = acc[k];
    }
}

// gs += nu * alpha * s at the injection points (s = the decomposed increment
// of one step, one value per point).
__global__ void image_sparse_kernel(const float *__restrict__ nu, const float *__restrict__ s,
                                    int npts, const long long *__restrict__ off,
                                    const double *__restrict__ alpha, double *__restrict__ gs)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    gs[i] += (double)nu[off[i]] * (alpha[i] * (double)s[i]);
}

__global__ void image_merge_kernel(const double *__restrict__ gs, int npts,
                                   const long long *__restrict__ off, double *__restrict__ g)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npts) g[off[i]] += gs[i];
}

// grad_m = scale * g, unpadded.
__global__ void finish_kernel(const double *__restrict__ g, float *__restrict__ out, int nx,
                              int ny, int nz, int nzp, double scale)
{
    const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (gid >= (long long)nx * ny * nz) return;
    const int z = (int)(gid % nz);
    const long long xy = gid / nz;
    out[gid] = (float)(g[xy * nzp + z] * scale);
}

__global__ void fill64_kernel(double *p, size_t n)
{
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.0;
}

unsigned blocks_for(long long n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

tb_status launch_residual_loss(const float *d, const float *dobs, long long n, float *res,
                               double *loss, hipStream_t st)
{
    if (n > 0) {
        hipLaunchKernelGGL(residual_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, d, dobs,
                           n, res);
        TB_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(kLossThreads), 0, st, res, n, loss);
    TB_HIP(hipGetLastError());
    return TB_OK;
}

tb_status launch_image(const ImageArgs &a, hipStream_t st)
{
    const long long total = (long long)a.nx * a.ny * (a.nzp / 4);
    if (total == 0 || a.nlev == 0) return TB_OK;
    hipLaunchKernelGGL(image_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, st, a);
    TB_HIP(hipGetLastError());
    return TB_OK;
}

tb_status launch_image_sparse(const float *nu, const float *s, int npts, const long long *off,
                              const double *alpha, double *gs, hipStream_t st)
{
    if (npts == 0) return TB_OK;
    hipLaunchKernelGGL(image_sparse_kernel, dim3(blocks_for(npts, 256)), dim3(256), 0, st, nu, s,
                       npts, off, alpha, gs);
    TB_HIP(hipGetLastError());
    return TB_OK;
}

tb_status launch_image_merge(const double *gs, int npts, const long long *off, double *g,
                             hipStream_t st)
{
    if (npts == 0) return TB_OK;
    hipLaunchKernelGGL(image_merge_kernel, dim3(blocks_for(npts, 256)), dim3(256), 0, st, gs,
                       npts, off, g);
    TB_HIP(hipGetLastError());
    return TB_OK;
}

tb_status launch_finish_grad(const double *g, float *out, int nx, int ny, int nz, int nzp,
                             double scale, hipStream_t st)
{
    const long long total = (long long)nx * ny * nz;
    if (total == 0) return TB_OK;
    hipLaunchKernelGGL(finish_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, st, g, out, nx,
                       ny, nz, nzp, scale);
    TB_HIP(hipGetLastError());
    return TB_OK;
}

tb_status launch_zero64(double *p, size_t n, hipStream_t st)
{
    if (n == 0) return TB_OK;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill64_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
    TB_HIP(hipGetLastError());
    return TB_OK;
}

}  // namespace tbw
