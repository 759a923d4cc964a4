// Isotropic elastic velocity-stress propagator (Section III-C) on the
// staggered grid: txx, tyy, tzz at the nodes, vx / vy / vz half a cell above
// the node along x / y / z, txy / txz / tyz half a cell above along both of
// their axes; every array is [nx][ny][nzp] (padded z) and every field is zero
// outside the grid. One time step:
//   el_vel   v^{n+1/2} = (beta v^{n-1/2} + dt b (div t^n)) / alpha
//   el_str   t^{n+1}   = (beta t^n + dt (lambda tr(grad v) I
//                                       + mu (grad v + grad v^T))) / alpha
//   el_src   t_ii^{n+1} += dt W q(t_n) at the inspector's points
//   el_rec   gather of P = (txx + tyy + tzz) / 3 (nodes) and of vz (vz grid)
// Both updates are in place (each element reads its own old value only).
#include "elastic_params.h"

namespace tbw {
namespace {

// Staggered first derivative along axis AX at element (x, y, z). FWD: the
// field sits at integer positions along AX and the target half a cell above
// (samples [i+m+1] - [i-m]); otherwise the field sits half a cell above its
// index and the target at the integer position ([i+m] - [i-m-1]).
template <int R, int AX, bool FWD>
__device__ __forceinline__ float dstg(const float *__restrict__ f, const ElParams &P, int x, int y,
                                      int z, long long gid)
{
    const int c = AX == 0 ? x : (AX == 1 ? y : z);
    const int n = AX == 0 ? P.nx : (AX == 1 ? P.ny : P.nz);
    const long long st = AX == 0 ? (long long)P.ny * P.nzp : (AX == 1 ? (long long)P.nzp : 1);
    float s = 0.0f;
#pragma unroll
    for (int m = 0; m < R; m++) {
        const int a = FWD ? m + 1 : m, b = FWD ? -m : -m - 1;
        const float up = (c + a < n) ? f[gid + a * st] : 0.0f;
        const float dn = (c + b >= 0) ? f[gid + b * st] : 0.0f;
        s = __builtin_fmaf(P.w[m], up - dn, s);
    }
    return s * P.ih[AX];
}

__device__ __forceinline__ void locate(const ElParams &P, long long gid, int &x, int &y, int &z)
{
    z = (int)(gid % P.nzp);
    const long long xy = gid / P.nzp;
    y = (int)(xy % P.ny);
    x = (int)(xy / P.ny);
}

template <int R>
__global__ void __launch_bounds__(256) el_vel(const ElParams P)
{
    const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (gid >= (long long)P.nx * P.ny * P.nzp) return;
    int x, y, z;
    locate(P, gid, x, y, z);
    if (z >= P.nz) return;
    const float fx = dstg<R, 0, true>(P.t[0], P, x, y, z, gid) +
                     dstg<R, 1, false>(P.t[3], P, x, y, z, gid) +
                     dstg<R, 2, false>(P.t[4], P, x, y, z, gid);
    const float fy = dstg<R, 0, false>(P.t[3], P, x, y, z, gid) +
                     dstg<R, 1, true>(P.t[1], P, x, y, z, gid) +
                     dstg<R, 2, false>(P.t[5], P, x, y, z, gid);
    const float fz = dstg<R, 0, false>(P.t[4], P, x, y, z, gid) +
                     dstg<R, 1, false>(P.t[5], P, x, y, z, gid) +
                     dstg<R, 2, true>(P.t[2], P, x, y, z, gid);
    const float d = P.dx[x] + P.dy[y] + P.dz[z];
    const float dd = d * P.hdt;
    const float beta = 1.0f - dd;
    float vx = __builtin_fmaf(beta, P.v[0][gid], P.bq[0][gid] * fx);
    float vy = __builtin_fmaf(beta, P.v[1][gid], P.bq[1][gid] * fy);
    float vz = __builtin_fmaf(beta, P.v[2][gid], P.bq[2][gid] * fz);
    if (d != 0.0f) {
        const float al = 1.0f + dd;
        vx /= al;
        vy /= al;
        vz /= al;
    }
    P.v[0][gid] = vx;
    P.v[1][gid] = vy;
    P.v[2][gid] = vz;
}

template <int R>
__global__ void __launch_bounds__(256) el_str(const ElParams P)
{
    const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (gid >= (long long)P.nx * P.ny * P.nzp) return;
    int x, y, z;
    locate(P, gid, x, y, z);
    if (z >= P.nz) return;
    const float exx = dstg<R, 0, false>(P.v[0], P, x, y, z, gid);
    const float eyy = dstg<R, 1, false>(P.v[1], P, x, y, z, gid);
    const float ezz = dstg<R, 2, false>(P.v[2], P, x, y, z, gid);
    const float gxy = dstg<R, 1, true>(P.v[0], P, x, y, z, gid) + dstg<R, 0, true>(P.v[1], P, x, y, z, gid);
    const float gxz = dstg<R, 2, true>(P.v[0], P, x, y, z, gid) + dstg<R, 0, true>(P.v[2], P, x, y, z, gid);
    const float gyz = dstg<R, 2, true>(P.v[1], P, x, y, z, gid) + dstg<R, 1, true>(P.v[2], P, x, y, z, gid);
    const float tr = exx + eyy + ezz;
    const float lam = P.lam[gid], mu2 = 2.0f * P.mu[gid];
    const float d = P.dx[x] + P.dy[y] + P.dz[z];
    const float dd = d * P.hdt;
    const float beta = 1.0f - dd;
    float t[6];
    t[0] = __builtin_fmaf(beta, P.t[0][gid], __builtin_fmaf(lam, tr, mu2 * exx));
    t[1] = __builtin_fmaf(beta, P.t[1][gid], __builtin_fmaf(lam, tr, mu2 * eyy));
    t[2] = __builtin_fmaf(beta, P.t[2][gid], __builtin_fmaf(lam, tr, mu2 * ezz));
    t[3] = __builtin_fmaf(beta, P.t[3][gid], P.ms[0][gid] * gxy);
    t[4] = __builtin_fmaf(beta, P.t[4][gid], P.ms[1][gid] * gxz);
    t[5] = __builtin_fmaf(beta, P.t[5][gid], P.ms[2][gid] * gyz);
    if (d != 0.0f) {
        const float al = 1.0f + dd;
#pragma unroll
        for (int k = 0; k < 6; k++) t[k] /= al;
    }
#pragma unroll
    for (int k = 0; k < 6; k++) P.t[k][gid] = t[k];
}

__global__ void el_src(float *__restrict__ txx, float *__restrict__ tyy, float *__restrict__ tzz,
                       const float *__restrict__ inc, const long long *__restrict__ soff, int npts)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    const long long o = soff[i];
    txx[o] += inc[i];
    tyy[o] += inc[i];
    tzz[o] += inc[i];
}

__global__ void el_rec(const float *__restrict__ txx, const float *__restrict__ tyy,
                       const float *__restrict__ tzz, const float *__restrict__ vz,
                       float *__restrict__ row_p, const long long *__restrict__ roff, int nrid,
                       float *__restrict__ row_v, const long long *__restrict__ roff2, int nrid2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nrid) {
        const long long o = roff[i];
        row_p[i] = (txx[o] + tyy[o] + tzz[o]) / 3.0f;
    } else if (i < nrid + nrid2) {
        const int j = i - nrid;
        row_v[j] = vz[roff2[j]];
    }
}

unsigned nblocks(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

tb_status launch_elastic_step(const ElParams &P, int r, const float *inc, const long long *soff,
                              int npts, float *row_p, const long long *roff, int nrid,
                              float *row_v, const long long *roff2, int nrid2, hipStream_t st)
{
    const long long total = (long long)P.nx * P.ny * P.nzp;
    if (total == 0) return TB_OK;
    if (r == 2) {
        hipLaunchKernelGGL(el_vel<2>, dim3(nblocks(total)), dim3(256), 0, st, P);
        hipLaunchKernelGGL(el_str<2>, dim3(nblocks(total)), dim3(256), 0, st, P);
    } else if (r == 4) {
        hipLaunchKernelGGL(el_vel<4>, dim3(nblocks(total)), dim3(256), 0, st, P);
        hipLaunchKernelGGL(el_str<4>, dim3(nblocks(total)), dim3(256), 0, st, P);
    } else {
        set_error("elastic radius %d not built", r);
        return TB_EUNSUPPORTED;
    }
    TB_HIP(hipGetLastError());
    if (npts > 0) {
        hipLaunchKernelGGL(el_src, dim3(nblocks(npts)), dim3(256), 0, st, P.t[0], P.t[1], P.t[2],
                           inc, soff, npts);
        TB_HIP(hipGetLastError());
    }
    if (nrid + nrid2 > 0) {
        hipLaunchKernelGGL(el_rec, dim3(nblocks(nrid + nrid2)), dim3(256), 0, st, P.t[0], P.t[1],
                           P.t[2], P.v[2], row_p, roff, nrid, row_v, roff2, nrid2);
        TB_HIP(hipGetLastError());
    }
    return TB_OK;
}

}  // namespace tbw
