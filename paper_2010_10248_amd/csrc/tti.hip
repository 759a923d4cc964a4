// Pseudo-acoustic TTI propagator (Section III-B): one time step is three
// kernels over the padded grid [nx][ny][nzp], z fastest:
//   tti_rot      q_p = a . grad p,  q_r = a . grad r   (a = symmetry axis,
//                centred first derivatives of the space order, zero outside);
//   tti_update   Hz u = sum_b d_b (a_b q_u), H0 p = L p - Hz p, and in the
//                velocity form of the leapfrog (w = u^n - u^{n-1}):
//                w_p' = (c [(1+2e) H0 p + s Hz r] + beta w_p) / alpha,
//                w_r' = (c [s H0 p + Hz r]        + beta w_r) / alpha,
//                p' = p + w_p', r' = r + w_r', s = sqrt(1 + 2 min(delta, eps));
//                L is applied to differences from the centre, so a constant
//                has an exactly zero Laplacian in FP32 (as in the acoustic
//                kernel, this keeps FP32 runs of many steps on the FP64
//                definition); w updates in place, p' and r' go to new buffers;
//   tti_sparse   injection of the inspector's per-point increments into p'
//                and r', and the receiver gather of p'.
// Every field is zero outside the grid (bounds-checked neighbour reads), so
// Hz = -D^T D exactly, as in the definition of the operator.
#include "tti_params.h"

namespace tbw {
namespace {

__device__ __forceinline__ float nb(const float *__restrict__ f, const TtiParams &P, int x, int y,
                                    int z, long long off)
{
    return (x >= 0 && x < P.nx && y >= 0 && y < P.ny && z >= 0 && z < P.nz) ? f[off] : 0.0f;
}

template <int R>
__global__ void __launch_bounds__(256) tti_rot(const TtiParams P)
{
    const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long total = (long long)P.nx * P.ny * P.nzp;
    if (gid >= total) return;
    const int z = (int)(gid % P.nzp);
    if (z >= P.nz) return;
    const long long xy = gid / P.nzp;
    const int y = (int)(xy % P.ny), x = (int)(xy / P.ny);
    const long long sx = (long long)P.ny * P.nzp, sy = P.nzp;
    float gp[3] = {0.f, 0.f, 0.f}, gr[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int m = 1; m <= R; m++) {
        const float w = P.w1[m - 1];
        gp[0] = __builtin_fmaf(w, nb(P.p, P, x + m, y, z, gid + m * sx) -
                                      nb(P.p, P, x - m, y, z, gid - m * sx), gp[0]);
        gp[1] = __builtin_fmaf(w, nb(P.p, P, x, y + m, z, gid + m * sy) -
                                      nb(P.p, P, x, y - m, z, gid - m * sy), gp[1]);
        gp[2] = __builtin_fmaf(w, nb(P.p, P, x, y, z + m, gid + m) -
                                      nb(P.p, P, x, y, z - m, gid - m), gp[2]);
        gr[0] = __builtin_fmaf(w, nb(P.r, P, x + m, y, z, gid + m * sx) -
                                      nb(P.r, P, x - m, y, z, gid - m * sx), gr[0]);
        gr[1] = __builtin_fmaf(w, nb(P.r, P, x, y + m, z, gid + m * sy) -
                                      nb(P.r, P, x, y - m, z, gid - m * sy), gr[1]);
        gr[2] = __builtin_fmaf(w, nb(P.r, P, x, y, z + m, gid + m) -
                                      nb(P.r, P, x, y, z - m, gid - m), gr[2]);
    }
    const float ax = P.ax[gid], ay = P.ay[gid], az = P.az[gid];
    P.qp[gid] = ax * (gp[0] * P.ih[0]) + ay * (gp[1] * P.ih[1]) + az * (gp[2] * P.ih[2]);
    P.qr[gid] = ax * (gr[0] * P.ih[0]) + ay * (gr[1] * P.ih[1]) + az * (gr[2] * P.ih[2]);
}

template <int R>
__global__ void __launch_bounds__(256) tti_update(const TtiParams P)
{
    const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long total = (long long)P.nx * P.ny * P.nzp;
    if (gid >= total) return;
    const int z = (int)(gid % P.nzp);
    if (z >= P.nz) return;
    const long long xy = gid / P.nzp;
    const int y = (int)(xy % P.ny), x = (int)(xy / P.ny);
    const long long sx = (long long)P.ny * P.nzp, sy = P.nzp;
    const float pc = P.p[gid], rc = P.r[gid];
    // L p: centred second derivatives on differences from the centre.
    const float p2 = 2.0f * pc;
    float lx = 0.0f, ly = 0.0f, lz = 0.0f;
    // Hz u = sum_b d_b (a_b q_u).
    float hp[3] = {0.f, 0.f, 0.f}, hr[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int m = 1; m <= R; m++) {
        lx = __builtin_fmaf(P.w2[m], (nb(P.p, P, x + m, y, z, gid + m * sx) +
                                      nb(P.p, P, x - m, y, z, gid - m * sx)) - p2, lx);
        ly = __builtin_fmaf(P.w2[m], (nb(P.p, P, x, y + m, z, gid + m * sy) +
                                      nb(P.p, P, x, y - m, z, gid - m * sy)) - p2, ly);
        lz = __builtin_fmaf(P.w2[m], (nb(P.p, P, x, y, z + m, gid + m) +
                                      nb(P.p, P, x, y, z - m, gid - m)) - p2, lz);
        const float w = P.w1[m - 1];
        const long long o[3] = {m * sx, m * sy, (long long)m};
        const int dx[3] = {m, 0, 0}, dy[3] = {0, m, 0}, dz[3] = {0, 0, m};
        const float *a3[3] = {P.ax, P.ay, P.az};
#pragma unroll
        for (int b = 0; b < 3; b++) {
            const bool inp = x + dx[b] < P.nx && y + dy[b] < P.ny && z + dz[b] < P.nz;
            const bool inm = x - dx[b] >= 0 && y - dy[b] >= 0 && z - dz[b] >= 0;
            const float ap = inp ? a3[b][gid + o[b]] : 0.0f;
            const float am = inm ? a3[b][gid - o[b]] : 0.0f;
            const float qpp = inp ? P.qp[gid + o[b]] : 0.0f, qpm = inm ? P.qp[gid - o[b]] : 0.0f;
            const float qrp = inp ? P.qr[gid + o[b]] : 0.0f, qrm = inm ? P.qr[gid - o[b]] : 0.0f;
            hp[b] = __builtin_fmaf(w, ap * qpp - am * qpm, hp[b]);
            hr[b] = __builtin_fmaf(w, ap * qrp - am * qrm, hr[b]);
        }
    }
    const float lap = lx * P.ih2[0] + ly * P.ih2[1] + lz * P.ih2[2];
    const float hzp = hp[0] * P.ih[0] + hp[1] * P.ih[1] + hp[2] * P.ih[2];
    const float hzr = hr[0] * P.ih[0] + hr[1] * P.ih[1] + hr[2] * P.ih[2];
    const float h0p = lap - hzp;
    const float e1 = P.e1[gid], sd = P.sd[gid], cc = P.c[gid];
    const float rhs_p = __builtin_fmaf(e1, h0p, sd * hzr);
    const float rhs_r = __builtin_fmaf(sd, h0p, hzr);
    const float d = P.dx[x] + P.dy[y] + P.dz[z];
    const float dd = d * P.hdt;
    const float beta = 1.0f - dd;
    float wp = __builtin_fmaf(cc, rhs_p, beta * P.vp[gid]);
    float wr = __builtin_fmaf(cc, rhs_r, beta * P.vr[gid]);
    if (d != 0.0f) {
        wp = wp / (1.0f + dd);
        wr = wr / (1.0f + dd);
    }
    P.vp[gid] = wp;
    P.vr[gid] = wr;
    P.pn[gid] = pc + wp;
    P.rn[gid] = rc + wr;
}

// The injected increment enters the new level and its velocity alike.
__global__ void tti_sparse(float *__restrict__ p, float *__restrict__ r, float *__restrict__ vp,
                           float *__restrict__ vr, const float *__restrict__ inc,
                           const long long *__restrict__ soff, int npts)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npts) {
        const long long o = soff[i];
        p[o] += inc[i];
        r[o] += inc[i];
        vp[o] += inc[i];
        vr[o] += inc[i];
    }
}

__global__ void tti_record(const float *__restrict__ p, float *__restrict__ rec_row,
                           const long long *__restrict__ roff, int nrid)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nrid) rec_row[i] = p[roff[i]];
}

unsigned nblocks(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

tb_status launch_tti_step(const TtiParams &P, int r, const float *inc, const long long *soff,
                          int npts, float *rec_row, const long long *roff, int nrid,
                          hipStream_t st)
{
    const long long total = (long long)P.nx * P.ny * P.nzp;
    if (total == 0) return TB_OK;
    if (r == 2) {
        hipLaunchKernelGGL(tti_rot<2>, dim3(nblocks(total)), dim3(256), 0, st, P);
        hipLaunchKernelGGL(tti_update<2>, dim3(nblocks(total)), dim3(256), 0, st, P);
    } else if (r == 4) {
        hipLaunchKernelGGL(tti_rot<4>, dim3(nblocks(total)), dim3(256), 0, st, P);
        hipLaunchKernelGGL(tti_update<4>, dim3(nblocks(total)), dim3(256), 0, st, P);
    } else {
        set_error("TTI radius %d not built", r);
        return TB_EUNSUPPORTED;
    }
    TB_HIP(hipGetLastError());
    if (npts > 0) {
        hipLaunchKernelGGL(tti_sparse, dim3(nblocks(npts)), dim3(256), 0, st, P.pn, P.rn, P.vp,
                           P.vr, inc, soff, npts);
        TB_HIP(hipGetLastError());
    }
    if (nrid > 0) {
        hipLaunchKernelGGL(tti_record, dim3(nblocks(nrid)), dim3(256), 0, st, P.pn, rec_row, roff,
                           nrid);
        TB_HIP(hipGetLastError());
    }
    return TB_OK;
}

}  // namespace tbw
