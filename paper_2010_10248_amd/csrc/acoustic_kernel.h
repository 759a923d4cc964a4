// Isotropic acoustic propagator kernels for gfx950 (CDNA4).
//
// One kernel template covers both schedules of the paper:
//   T == 1  spatial blocking (Fig. 4a): one time step per pass over memory;
//   T >= 2  wave-front temporal blocking (Section II-B, Fig. 7/8a and the
//           final loop-nest listing): T steps per pass.
//
// A workgroup owns a y-z tile and streams along x. Stage s of the pipeline
// holds the (2R+1)-plane window of time level n+s in registers (the x
// neighbours), publishes its centre plane to LDS (the y neighbours) and
// exchanges z neighbours inside 16-lane DPP rows (each lane holds 4
// consecutive z as one float4, so a single row shift brings all R <= 4 z
// neighbours). Stage s lags stage s-1 by R planes: the wave-front angle the
// stencil radius imposes (Section II-B). The y-z tile carries an overlapped
// halo of R(T-1) so the T stages need no exchange between workgroups.
//
// Injection follows the inspector's decomposition (Section II-A): the
// per-tile list names every affected grid point in the workgroup's extended
// region, and each stage adds src_dcmp[n][id] to every computed copy of such
// a point right after its stencil update — redundant halo copies included,
// which is what makes the reordering legal (the violation of Fig. 4b is a
// halo copy that misses, or precedes, its injection). Receivers record from
// the owned copy only.
//
// Every schedule evaluates the same per-point expression with the same
// operation order, so all schedules give bit-identical fields.
#pragma once

#include <type_traits>

#include "acoustic_params.h"

namespace tbw {
namespace wf {

struct F4 {
    float v[4];
};

__device__ __forceinline__ F4 tof4(float4 a) { return F4{{a.x, a.y, a.z, a.w}}; }
__device__ __forceinline__ float4 tofloat4(const F4 &a)
{
    return make_float4(a.v[0], a.v[1], a.v[2], a.v[3]);
}

__device__ __forceinline__ float4 ld4(const float *__restrict__ base, long long off, bool ok)
{
    return ok ? *reinterpret_cast<const float4 *>(base + off) : make_float4(0.f, 0.f, 0.f, 0.f);
}

// Lane l of a 16-lane DPP row receives lane l-1 (shr) or l+1 (shl); the lane
// at the row edge keeps `old`.
__device__ __forceinline__ float dpp_from_left(float old, float src)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src),
                                                      0x111, 0xF, 0xF, false));
}
__device__ __forceinline__ float dpp_from_right(float old, float src)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src),
                                                      0x101, 0xF, 0xF, false));
}

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// The per-point update shared by every schedule (fixed operation order):
//   lap = w0 u + sum_{j=1..R} [wx_j (x-j + x+j) + wy_j (y-j + y+j) + wz_j (z-j + z+j)]
//   r   = c lap + (2u - beta u^{n-1});  r /= alpha where the damping is non-zero.
template <int R>
__device__ __forceinline__ float point_update(const AcParams &p, float ctr, const float *xm,
                                              const float *xp, const float *ym, const float *yp,
                                              const float *zm, const float *zp, float prev,
                                              float cc, float d)
{
    float lap = p.w0 * ctr;
#pragma unroll
    for (int j = 0; j < R; j++) {
        lap = __builtin_fmaf(p.wx[j], xm[j] + xp[j], lap);
        lap = __builtin_fmaf(p.wy[j], ym[j] + yp[j], lap);
        lap = __builtin_fmaf(p.wz[j], zm[j] + zp[j], lap);
    }
    const float dd = d * p.hdt;
    const float beta = 1.0f - dd;
    float r = __builtin_fmaf(cc, lap, __builtin_fmaf(-beta, prev, 2.0f * ctr));
    if (d != 0.0f) r = r / (1.0f + dd);
    return r;
}

template <int R, int T, int BYE>
__global__ void __launch_bounds__(kLanesZ *BYE) acoustic_wavefront(const AcParams p)
{
    constexpr int Q = 2 * R + 1;  // x window
    constexpr int HY = R * (T - 1);
    constexpr int HZ = ((R * (T - 1) + 3) / 4) * 4;
    constexpr int OY = BYE - 2 * HY;
    constexpr int OZ = kTileZ - 2 * HZ;
    constexpr int LR = BYE + 2 * R;  // LDS rows per stage (with the y ring)
    static_assert(OY > 0 && OZ > 0, "tile too small for this depth");
    static_assert(R >= 1 && R <= 4, "radius must be 1..4");

    __shared__ float4 sh[2][T][LR][kLanesZ];

    const int tid = threadIdx.x;
    const int zl = tid & (kLanesZ - 1);
    const int row = tid >> 4;

    // XCD-aware tile order: hardware hands consecutive workgroups to the 8
    // XCDs round-robin; give each XCD a contiguous run of neighbouring tiles
    // so halo re-reads hit the same L2.
    const int b = blockIdx.x, nb = p.nblocks;
    const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7;
    const int L = xcd * q8 + min(xcd, r8) + (b >> 3);
    const int tz = L % p.tiles_z;
    const int rest = L / p.tiles_z;
    const int tyi = rest % p.tiles_y;
    const int ch = rest / p.tiles_y;

    const int y0 = tyi * OY - HY, z0 = tz * OZ - HZ;
    const int xc0 = ch * p.chunk;
    const int xc1 = min(p.nx, xc0 + p.chunk);
    const int y = y0 + row, z = z0 + 4 * zl;
    const bool yin = (unsigned)y < (unsigned)p.ny;
    const bool ldok = yin && z >= 0 && z < p.nzp;
    const long long rowoff = (long long)y * p.nzp + z;
    bool dm[4];
    float dyz[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        dm[k] = yin && z + k >= 0 && z + k < p.nz;
        dyz[k] = dm[k] ? p.dy[y] + p.dz[z + k] : 0.0f;
    }
    const bool own = row >= HY && row < HY + OY && zl >= HZ / 4 && zl < (HZ + OZ) / 4 && ldok;

    // z ring of stage 0: lane 0 of each row holds z0-4..z0-1, lane 15 holds
    // z0+64..z0+67 (one float4 covers the radius).
    const int zr = zl == 0 ? z - 4 : z + 4;
    const bool rgok = yin && (zl == 0 || zl == kLanesZ - 1) && zr >= 0 && zr < p.nzp;
    const long long rgoff = (long long)y * p.nzp + zr;
    // y ring of stage 0: rows y0-R..y0-1 and y0+BYE..y0+BYE+R-1.
    const bool has_yr = tid < 2 * R * kLanesZ;
    const int rr = row;  // ring row index for threads with has_yr
    const int yr = rr < R ? y0 - R + rr : y0 + BYE + rr - R;
    const int yr_lds = rr < R ? rr : BYE + rr;
    const bool yrok = has_yr && (unsigned)yr < (unsigned)p.ny && z >= 0 && z < p.nzp;
    const long long yroff = (long long)yr * p.nzp + z;

    // Clear the LDS planes so the unused ring rows of stages >= 1 hold zeros.
    for (int k = tid; k < 2 * T * LR * kLanesZ; k += kLanesZ * BYE)
        (&sh[0][0][0][0])[k] = make_float4(0.f, 0.f, 0.f, 0.f);

    // Per-stage x ranges and list cursors.
    int lo[T], hi[T];
#pragma unroll
    for (int s = 0; s < T; s++) {
        lo[s] = max(0, xc0 - R * (T - 1 - s));
        hi[s] = min(p.nx, xc1 + R * (T - 1 - s));
    }
    const int sbeg = p.src_off[L], send = p.src_off[L + 1];
    const int rbeg = p.rec_off[L], rend = p.rec_off[L + 1];
    int scur[T], rcur[T];
#pragma unroll
    for (int s = 0; s < T; s++) {
        scur[s] = sbeg;
        rcur[s] = rbeg;
    }

    F4 q[T][Q];
#pragma unroll
    for (int s = 0; s < T; s++)
#pragma unroll
        for (int k = 0; k < Q; k++) q[s][k] = F4{{0.f, 0.f, 0.f, 0.f}};

    const int i0 = max(0, xc0 - R * T);
    const int ilast = xc1 - 1 + R * T;

    // Prefetch registers for the tick about to run: the new plane of u^n, and
    // at the stage-0 centre plane u^{n-1}, the z ring and the y ring; c at
    // every stage's centre plane (stages >= 1 re-read planes stage 0 read R*s
    // ticks earlier, which the caches still hold).
    auto fetch = [&](int i, float4 &fu, float4 &fum, float4 (&fc)[T], float4 &frg,
                     float4 &fyr) {
        const int c0 = i - R;
        const bool pin = i < p.nx;  // i >= 0 always
        const bool cin = c0 >= 0 && c0 < p.nx;
        fu = ld4(p.u, (long long)i * p.sx + rowoff, ldok && pin);
        fum = ld4(p.um, (long long)c0 * p.sx + rowoff, ldok && cin);
#pragma unroll
        for (int s = 0; s < T; s++) {
            const int cs = c0 - R * s;
            fc[s] = ld4(p.c, (long long)cs * p.sx + rowoff, ldok && cs >= lo[s] && cs < hi[s]);
        }
        frg = ld4(p.u, (long long)c0 * p.sx + rgoff, rgok && cin);
        fyr = ld4(p.u, (long long)c0 * p.sx + yroff, yrok && cin);
    };
    float4 pu, pum, pc[T], prg, pyr;
    fetch(i0, pu, pum, pc, prg, pyr);
    __syncthreads();

    int i = i0;
    int tick = 0;
    while (i <= ilast) {
        static_for<0, Q>([&](auto PC) {
            constexpr int P = decltype(PC)::value;
            if (i > ilast) return;
            const F4 cu = tof4(pu);
            const F4 cum = tof4(pum);
            float4 cc4[T];
#pragma unroll
            for (int s = 0; s < T; s++) cc4[s] = pc[s];
            const float4 crg = prg;
            const float4 cyr = pyr;
            if (i + 1 <= ilast) fetch(i + 1, pu, pum, pc, prg, pyr);

            constexpr int NEW = (P + 2 * R) % Q;
            constexpr int CTR = (P + R) % Q;
            constexpr int OLD = P % Q;
            q[0][NEW] = cu;
            const int buf = tick & 1;
#pragma unroll
            for (int s = 0; s < T; s++) sh[buf][s][row + R][zl] = tofloat4(q[s][CTR]);
            if (has_yr) sh[buf][0][yr_lds][zl] = cyr;
            __syncthreads();

            static_for<0, T>([&](auto SC) {
                constexpr int s = decltype(SC)::value;
                const int cs = i - R * (s + 1);
                F4 v = F4{{0.f, 0.f, 0.f, 0.f}};
                if (cs >= lo[s] && cs < hi[s]) {
                    const F4 ctr = q[s][CTR];
                    const F4 prev = (s == 0) ? cum : q[s > 0 ? s - 1 : 0][OLD];
                    const F4 cf = tof4(cc4[s]);
                    const F4 ring = (s == 0) ? tof4(crg) : F4{{0.f, 0.f, 0.f, 0.f}};
                    float zw[12];
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        zw[k] = dpp_from_left(ring.v[k], ctr.v[k]);
                        zw[4 + k] = ctr.v[k];
                        zw[8 + k] = dpp_from_right(ring.v[k], ctr.v[k]);
                    }
                    F4 ym[R], yp[R];
#pragma unroll
                    for (int j = 1; j <= R; j++) {
                        ym[j - 1] = tof4(sh[buf][s][row + R - j][zl]);
                        yp[j - 1] = tof4(sh[buf][s][row + R + j][zl]);
                    }
                    const float dxs = p.dx[cs];
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        float xm[R], xp[R], a[R], bb[R], zm[R], zp[R];
#pragma unroll
                        for (int j = 1; j <= R; j++) {
                            xm[j - 1] = q[s][(P + R - j) % Q].v[k];
                            xp[j - 1] = q[s][(P + R + j) % Q].v[k];
                            a[j - 1] = ym[j - 1].v[k];
                            bb[j - 1] = yp[j - 1].v[k];
                            zm[j - 1] = zw[4 + k - j];
                            zp[j - 1] = zw[4 + k + j];
                        }
                        v.v[k] = point_update<R>(p, ctr.v[k], xm, xp, a, bb, zm, zp, prev.v[k],
                                                 cf.v[k], dxs + dyz[k]);
                    }
                    // Fused injection at every computed copy (per-tile list).
                    if (sbeg < send) {
                        int kk = scur[s];
                        while (kk < send && p.src[kk].x < cs) kk++;
                        scur[s] = kk;
                        for (; kk < send && p.src[kk].x == cs; kk++) {
                            const int4 e = p.src[kk];
                            if (e.y == row && (e.z >> 2) == zl) {
                                const float add =
                                    p.dcmp[(long long)(p.n0 + s) * p.npts + e.w];
#pragma unroll
                                for (int k = 0; k < 4; k++)
                                    if ((e.z & 3) == k) v.v[k] += add;
                            }
                        }
                    }
#pragma unroll
                    for (int k = 0; k < 4; k++)
                        if (!dm[k]) v.v[k] = 0.0f;
                    // Receiver points: owned copy only.
                    if (rbeg < rend) {
                        int kk = rcur[s];
                        while (kk < rend && p.rec[kk].x < cs) kk++;
                        rcur[s] = kk;
                        for (; kk < rend && p.rec[kk].x == cs; kk++) {
                            const int4 e = p.rec[kk];
                            if (e.y == row && (e.z >> 2) == zl) {
                                float val = v.v[0];
#pragma unroll
                                for (int k = 1; k < 4; k++)
                                    if ((e.z & 3) == k) val = v.v[k];
                                p.rec_dcmp[(long long)(p.n0 + s + 1) * p.nrid + e.w] = val;
                            }
                        }
                    }
                }
                if constexpr (s + 1 < T) {
                    q[s + 1 < T ? s + 1 : 0][NEW] = v;
                } else {
                    if (cs >= xc0 && cs < xc1 && own) {
                        const long long off = (long long)cs * p.sx + rowoff;
                        *reinterpret_cast<float4 *>(p.out0 + off) = tofloat4(v);
                        if constexpr (T > 1)
                            *reinterpret_cast<float4 *>(p.out1 + off) = tofloat4(q[s][CTR]);
                    }
                }
            });
            i++;
            tick++;
        });
    }
}

template <int R, int T, int BYE>
hipError_t launch_rtb(const AcParams &p, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL((acoustic_wavefront<R, T, BYE>), dim3(nblocks), dim3(kLanesZ * BYE), 0,
                       st, p);
    return hipGetLastError();
}

// LDS bytes of one workgroup of acoustic_wavefront<R, T, BYE>.
constexpr int wavefront_lds(int R, int T, int BYE) { return 16 * kLanesZ * 2 * T * (BYE + 2 * R); }

// Instantiated shapes: the halo must leave owned rows, LDS must fit, and a
// 1024-thread workgroup (at most 128 VGPRs per lane) only for the shallow
// pipelines whose register queues fit without spilling.
template <int R, int T, int BYE>
constexpr bool wavefront_fits()
{
    return BYE - 2 * R * (T - 1) > 0 && wavefront_lds(R, T, BYE) <= 160 * 1024 &&
           (BYE <= 32 || (R <= 2 && T <= 2));
}

template <int R, int T>
hipError_t launch_rt(const AcParams &p, int BYE, int nblocks, hipStream_t st)
{
    switch (BYE) {
    case 16:
        if constexpr (wavefront_fits<R, T, 16>()) return launch_rtb<R, T, 16>(p, nblocks, st);
        break;
    case 32:
        if constexpr (wavefront_fits<R, T, 32>()) return launch_rtb<R, T, 32>(p, nblocks, st);
        break;
    case 64:
        if constexpr (wavefront_fits<R, T, 64>()) return launch_rtb<R, T, 64>(p, nblocks, st);
        break;
    }
    return hipErrorInvalidValue;
}

template <int R>
hipError_t launch_r(const AcParams &p, int T, int BYE, int nblocks, hipStream_t st)
{
    switch (T) {
    case 1: return launch_rt<R, 1>(p, BYE, nblocks, st);
    case 2: return launch_rt<R, 2>(p, BYE, nblocks, st);
    case 3: return launch_rt<R, 3>(p, BYE, nblocks, st);
    case 4: return launch_rt<R, 4>(p, BYE, nblocks, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace wf
}  // namespace tbw
