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
// The forward step at radius 2 and 4 runs the x-streaming forms of the two
// passes (el_vel_s, el_str_s; same per-point operations); radius 6 runs the
// tiled ones.
#include <algorithm>

#include "elastic_params.h"
#include "stream_kernel.h"

namespace tbw {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// Each thread takes 4 consecutive z (float4 accesses); neighbours along x and
// y are float4 loads, along z they come from the window [z4-ZB, z4+4+ZB),
// ZB = 4 up to radius 4 and 8 up to radius 6. Reads outside the grid give 0;
// the z padding holds 0 in every field.
struct Site {
    int x, y, z4;
    long long off, sx, sy;
};

// XCD-aware block order. The hardware deals consecutive workgroups to the 8
// XCDs round-robin. With P.band = S > 0 the launch's blocks form runs of 8S
// (S = blocks of one x-plane / 8, rounded up), and XCD k takes the k-th
// contiguous band of S blocks of every run: each XCD streams the same band
// of y rows through the planes, so that neighbour reads along x and most
// along y meet in its own L2 (with plain round-robin order every y neighbour
// of a row sits on another XCD). A permutation of the work; blocks past the
// grid return at once.
template <class Params>
__device__ __forceinline__ long long block_index(const Params &P)
{
    const unsigned b = blockIdx.x;
    if (P.band <= 0) return b;
    const unsigned S = (unsigned)P.band, xcd = b & 7, j = b >> 3;
    return (long long)(j / S) * 8 * S + xcd * S + (j % S);
}

__device__ __forceinline__ bool locate4(const ElParams &P, Site &q)
{
    const int nz4 = P.nzp / 4;
    const int xe = P.xhi > 0 ? P.xhi : P.nx;
    const long long gid = block_index(P) * blockDim.x + threadIdx.x;
    if (gid >= (long long)(xe - P.xlo) * P.ny * nz4) return false;
    q.z4 = (int)(gid % nz4) * 4;
    const long long xy = gid / nz4;
    q.y = (int)(xy % P.ny);
    q.x = P.xlo + (int)(xy / P.ny);
    q.sx = (long long)P.ny * P.nzp;
    q.sy = P.nzp;
    q.off = ((long long)q.x * P.ny + q.y) * P.nzp + q.z4;
    return true;
}

__device__ __forceinline__ f4 ld4(const float *f, long long o, bool in)
{
    return in ? *(const f4 *)(f + o) : f4{0.f, 0.f, 0.f, 0.f};
}

// Staggered first derivative (scaled by 1/h) along AX at the 4 sites. FWD:
// the field sits at integer positions along AX and the target half a cell
// above (samples [i+m+1] - [i-m]); otherwise [i+m] - [i-m-1].
template <int R, int AX, bool FWD>
__device__ __forceinline__ f4 dstg(const float *__restrict__ f, const ElParams &P, const Site &q)
{
    f4 s = f4{0.f, 0.f, 0.f, 0.f};
    if constexpr (AX == 2) {
        static_assert(R >= 1 && R <= 6, "radius must be 1..6");
        constexpr int ZB = R <= 4 ? 4 : 8;
        float w[4 + 2 * ZB];
#pragma unroll
        for (int o = -ZB; o <= ZB; o += 4) {
            const f4 a = ld4(f, q.off + o, q.z4 + o >= 0 && q.z4 + o < P.nzp);
#pragma unroll
            for (int k = 0; k < 4; k++) w[ZB + o + k] = a[k];
        }
#pragma unroll
        for (int k = 0; k < 4; k++)
#pragma unroll
            for (int m = 0; m < R; m++) {
                const int up = FWD ? m + 1 : m, dn = FWD ? -m : -m - 1;
                s[k] = __builtin_fmaf(P.w[m], w[ZB + k + up] - w[ZB + k + dn], s[k]);
            }
    } else {
        const int c = AX == 0 ? q.x : q.y, n = AX == 0 ? P.nx : P.ny;
        const long long st = AX == 0 ? q.sx : q.sy;
        // Two offsets per iteration: unrolled fully, the compiler hoists every
        // neighbour load of the kernel (256 VGPRs, one wave per SIMD); this
        // keeps the stress pass at 4 waves per SIMD and is 23% faster.
#pragma unroll 2
        for (int m = 0; m < R; m++) {
            const int up = FWD ? m + 1 : m, dn = FWD ? -m : -m - 1;
            const f4 fu = ld4(f, q.off + up * st, c + up < n);
            const f4 fd = ld4(f, q.off + dn * st, c + dn >= 0);
#pragma unroll
            for (int k = 0; k < 4; k++) s[k] = __builtin_fmaf(P.w[m], fu[k] - fd[k], s[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; k++) s[k] *= P.ih[AX];
    return s;
}

// Forward passes on 2-D tiles: a workgroup takes 16 y rows x 64 z (16 lanes
// of 4 z) of one x-plane. The three fields each pass differentiates along y
// are staged in LDS with R rows of halo on each side (zero outside the grid),
// so a y neighbour costs an LDS read instead of a vector load; x and z
// neighbours are read as before. The per-point expressions and their order
// are those of the one-point form, so the values are the same bits.
constexpr int kTY = 16, kTZ = 16;  // tile rows, tile lanes (4 z each)

struct TileSite {
    Site q;
    int ty, tz, y0;
    bool valid;
};

// Tile of this workgroup in the banded block order over the planes [xlo,
// xhi); false (for the whole workgroup) past the grid.
__device__ __forceinline__ bool tile_site(const ElParams &P, TileSite &t)
{
    const int nz4 = P.nzp / 4;
    const int nty = (P.ny + kTY - 1) / kTY, ntz = (nz4 + kTZ - 1) / kTZ;
    const long long tpp = (long long)nty * ntz;
    const int xe = P.xhi > 0 ? P.xhi : P.nx;
    const long long L = block_index(P);
    if (L >= (long long)(xe - P.xlo) * tpp) return false;
    const int x = P.xlo + (int)(L / tpp);
    const int tl = (int)(L % tpp);
    t.ty = threadIdx.x / kTZ;
    t.tz = threadIdx.x % kTZ;
    t.y0 = (tl / ntz) * kTY;
    const int y = t.y0 + t.ty, z4 = ((tl % ntz) * kTZ + t.tz) * 4;
    t.valid = y < P.ny && z4 < P.nzp;
    t.q.x = x;
    t.q.y = y;
    t.q.z4 = z4;
    t.q.sx = (long long)P.ny * P.nzp;
    t.q.sy = P.nzp;
    t.q.off = ((long long)x * P.ny + y) * P.nzp + z4;
    return true;
}

// Rows y0-R .. y0+16+R-1 of field f at this tile's x and z columns into
// L[0 .. 16+2R) (row y0 + i - R at L[i]).
template <int R>
__device__ __forceinline__ void stage_rows(f4 (*L)[kTZ], const float *f, const ElParams &P,
                                           const TileSite &t)
{
    const bool zin = t.q.z4 < P.nzp;
    L[t.ty + R][t.tz] = ld4(f, t.q.off, t.valid);
    if ((int)threadIdx.x < 2 * R * kTZ) {
        const int hr = threadIdx.x / kTZ;
        const int row = hr < R ? hr : kTY + hr;
        const int yy = t.y0 + row - R;
        const bool ok = zin && yy >= 0 && yy < P.ny;
        L[row][t.tz] = ld4(f, ((long long)t.q.x * P.ny + yy) * P.nzp + t.q.z4, ok);
    }
}

// The y derivative of dstg<R, 1, FWD> from the staged rows.
template <int R, bool FWD>
__device__ __forceinline__ f4 dy_lds(const f4 (*L)[kTZ], const ElParams &P, const TileSite &t)
{
    f4 s = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int m = 0; m < R; m++) {
        const int up = FWD ? m + 1 : m, dn = FWD ? -m : -m - 1;
        const f4 fu = L[t.ty + R + up][t.tz], fd = L[t.ty + R + dn][t.tz];
#pragma unroll
        for (int k = 0; k < 4; k++) s[k] = __builtin_fmaf(P.w[m], fu[k] - fd[k], s[k]);
    }
#pragma unroll
    for (int k = 0; k < 4; k++) s[k] *= P.ih[1];
    return s;
}

template <int R>
__global__ void __launch_bounds__(256) el_vel(const ElParams P)
{
    __shared__ f4 L[3][kTY + 2 * R][kTZ];
    TileSite t;
    if (!tile_site(P, t)) return;
    stage_rows<R>(L[0], P.t[3], P, t);
    stage_rows<R>(L[1], P.t[1], P, t);
    stage_rows<R>(L[2], P.t[5], P, t);
    __syncthreads();
    if (!t.valid) return;
    const Site &q = t.q;
    const f4 fx = dstg<R, 0, true>(P.t[0], P, q) + dy_lds<R, false>(L[0], P, t) +
                  dstg<R, 2, false>(P.t[4], P, q);
    const f4 fy = dstg<R, 0, false>(P.t[3], P, q) + dy_lds<R, true>(L[1], P, t) +
                  dstg<R, 2, false>(P.t[5], P, q);
    const f4 fz = dstg<R, 0, false>(P.t[4], P, q) + dy_lds<R, false>(L[2], P, t) +
                  dstg<R, 2, true>(P.t[2], P, q);
    const f4 f3[3] = {fx, fy, fz};
    const float dxy = P.dx[q.x] + P.dy[q.y];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        f4 v = ld4(P.v[c], q.off, true);
        const f4 b = ld4(P.bq[c], q.off, true);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int z = q.z4 + k;
            const float d = dxy + (z < P.nz ? P.dz[z] : 0.0f);
            const float dd = d * P.hdt;
            float r = __builtin_fmaf(1.0f - dd, v[k], b[k] * f3[c][k]);
            if (d != 0.0f) r /= 1.0f + dd;
            v[k] = r;
        }
        *(f4 *)((P.vo[c] ? P.vo[c] : P.v[c]) + q.off) = v;
    }
}

template <int R>
__global__ void __launch_bounds__(256) el_str(const ElParams P)
{
    __shared__ f4 L[3][kTY + 2 * R][kTZ];
    TileSite ts;
    if (!tile_site(P, ts)) return;
    stage_rows<R>(L[0], P.v[0], P, ts);
    stage_rows<R>(L[1], P.v[1], P, ts);
    stage_rows<R>(L[2], P.v[2], P, ts);
    __syncthreads();
    if (!ts.valid) return;
    const Site &q = ts.q;
    const f4 exx = dstg<R, 0, false>(P.v[0], P, q);
    const f4 eyy = dy_lds<R, false>(L[1], P, ts);
    const f4 ezz = dstg<R, 2, false>(P.v[2], P, q);
    const f4 gxy = dy_lds<R, true>(L[0], P, ts) + dstg<R, 0, true>(P.v[1], P, q);
    const f4 gxz = dstg<R, 2, true>(P.v[0], P, q) + dstg<R, 0, true>(P.v[2], P, q);
    const f4 gyz = dstg<R, 2, true>(P.v[1], P, q) + dy_lds<R, true>(L[2], P, ts);
    const f4 lam = ld4(P.lam, q.off, true), mu = ld4(P.mu, q.off, true);
    const f4 m0 = ld4(P.ms[0], q.off, true), m1 = ld4(P.ms[1], q.off, true),
             m2 = ld4(P.ms[2], q.off, true);
    f4 t[6];
#pragma unroll
    for (int c = 0; c < 6; c++) t[c] = ld4(P.t[c], q.off, true);
    const float dxy = P.dx[q.x] + P.dy[q.y];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int z = q.z4 + k;
        const float d = dxy + (z < P.nz ? P.dz[z] : 0.0f);
        const float dd = d * P.hdt;
        const float beta = 1.0f - dd;
        const float tr = exx[k] + eyy[k] + ezz[k];
        const float mu2 = 2.0f * mu[k];
        float n[6];
        n[0] = __builtin_fmaf(beta, t[0][k], __builtin_fmaf(lam[k], tr, mu2 * exx[k]));
        n[1] = __builtin_fmaf(beta, t[1][k], __builtin_fmaf(lam[k], tr, mu2 * eyy[k]));
        n[2] = __builtin_fmaf(beta, t[2][k], __builtin_fmaf(lam[k], tr, mu2 * ezz[k]));
        n[3] = __builtin_fmaf(beta, t[3][k], m0[k] * gxy[k]);
        n[4] = __builtin_fmaf(beta, t[4][k], m1[k] * gxz[k]);
        n[5] = __builtin_fmaf(beta, t[5][k], m2[k] * gyz[k]);
        if (d != 0.0f) {
#pragma unroll
            for (int c = 0; c < 6; c++) n[c] /= 1.0f + dd;
        }
#pragma unroll
        for (int c = 0; c < 6; c++) t[c][k] = n[c];
    }
#pragma unroll
    for (int c = 0; c < 6; c++) *(f4 *)((P.to[c] ? P.to[c] : P.t[c]) + q.off) = t[c];
}

// ---------------------------------------------------------------------------
// Streaming forward passes (radius 2 and 4; building blocks in
// stream_kernel.h). Slot k of an x window holds plane j - R + k for the
// centre plane j (a staggered derivative reads slots R - R .. R + R), shifted
// by one slot per tick; the inputs a tick starts with are loaded during the
// previous tick. Per point the operations and their order are those of
// el_vel / el_str above, so the streaming and tiled passes give the same
// bits.
using namespace st;

// Staggered first derivatives (unit weights w, scaled by 1/h) of the PL
// points: along x from a window, along y from staged LDS rows, along z from
// the lane window of zlanes. FWD as in dstg.
template <int R, int PL, bool FWD>
__device__ __forceinline__ vec<PL> sdx(const ElParams &P, const vec<PL> *win)
{
    vec<PL> s = vec<PL>{};
#pragma unroll
    for (int m = 0; m < R; m++) {
        const int up = FWD ? m + 1 : m, dn = FWD ? -m : -m - 1;
#pragma unroll
        for (int k = 0; k < PL; k++) s[k] = __builtin_fmaf(P.w[m], win[R + up][k] - win[R + dn][k], s[k]);
    }
#pragma unroll
    for (int k = 0; k < PL; k++) s[k] *= P.ih[0];
    return s;
}
template <int R, int PL, bool FWD>
__device__ __forceinline__ vec<PL> sdy(const ElParams &P, const vec<PL> (*L)[kSZ], const SSite &s)
{
    vec<PL> a = vec<PL>{};
#pragma unroll
    for (int m = 0; m < R; m++) {
        const int up = FWD ? m + 1 : m, dn = FWD ? -m : -m - 1;
        const vec<PL> fu = L[s.row + R + up][s.zl], fd = L[s.row + R + dn][s.zl];
#pragma unroll
        for (int k = 0; k < PL; k++) a[k] = __builtin_fmaf(P.w[m], fu[k] - fd[k], a[k]);
    }
#pragma unroll
    for (int k = 0; k < PL; k++) a[k] *= P.ih[1];
    return a;
}
template <int R, int PL, bool FWD>
__device__ __forceinline__ vec<PL> sdz(const ElParams &P, const float *w)
{
    vec<PL> a;
#pragma unroll
    for (int k = 0; k < PL; k++) {
        float t = 0.0f;
#pragma unroll
        for (int m = 0; m < R; m++) {
            const int up = FWD ? m + 1 : m, dn = FWD ? -m : -m - 1;
            t = __builtin_fmaf(P.w[m], w[4 + k + up] - w[4 + k + dn], t);
        }
        a[k] = t * P.ih[2];
    }
    return a;
}

template <int R, int PL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
el_vel_s(const ElParams P)
{
    static_assert(R == 2 || R == 4, "streaming passes cover radius 2 and 4");
    using V = vec<PL>;
    constexpr int U = 2 * R + 1, LR = kSY + 2 * R, CTR = R;
    __shared__ V sh[2][3][LR][kSZ];  // txy, tyy, tyz along y
    // The halo values of the x-windowed txy (y halo rows) and txz (outer z
    // values) are loaded with the neighbouring tiles' own loads of the newest
    // plane, while those lines are in L2, and wait R ticks for the centre in
    // thread-private LDS delay lines; tyy, tyz, tzz are read at the centre
    // plane by their owners too, so their halo values load with those.
    __shared__ V yd[R + 1][2 * R * kSZ];
    __shared__ V zd[R + 1][kSY * edge_lanes<R, PL>()];
    SSite s;
    if (!ssite<R, PL>(P, s)) return;
    const int tid = threadIdx.x;
    const float dyv = s.y < P.ny ? P.dy[s.y] : 0.0f;
    float dzv[PL];
#pragma unroll
    for (int k = 0; k < PL; k++) dzv[k] = s.z + k < P.nz ? P.dz[s.z + k] : 0.0f;
    struct In {
        V xx, xy, xz;     // txx, txy, txz at the window plane i
        V yy, yz, zz;     // tyy, tyz, tzz at the centre plane j = i - R
        V hxy, gxz;       // y halo of txy and outer z values of txz at i
        V hyy, hyz;       // y halo at j
        V gyz, gzz;       // outer z values at j
    };
    const int i0 = s.xa - R, ilast = s.xb - 1 + R;
    auto fetch = [&](int i, In &f) {
        const int j = i - R;
        const bool c = j >= s.xa && j < s.xb, w = i <= ilast;
        const PlaneRef xw = plane(P, i, w), xc = plane(P, j, c);
        f.xx = vload<PL>(at(P.t[0], xw), s.off);
        f.xy = vload<PL>(at(P.t[3], xw), s.off);
        f.xz = vload<PL>(at(P.t[4], xw), s.off);
        const PlaneRef xh = plane(P, i, i >= s.xa && i < s.xb);  // a centre later
        const wf::rsrc_t yyj = at(P.t[1], xc), yzj = at(P.t[5], xc), zzj = at(P.t[2], xc);
        f.yy = vload<PL>(yyj, s.off);
        f.yz = vload<PL>(yzj, s.off);
        f.zz = vload<PL>(zzj, s.off);
        f.hxy = vload<PL>(at(P.t[3], xh), s.off_yr);
        f.hyy = vload<PL>(yyj, s.off_yr);
        f.hyz = vload<PL>(yzj, s.off_yr);
        f.gxz = vload<PL>(at(P.t[4], xh), s.off_rg);
        f.gyz = vload<PL>(yzj, s.off_rg);
        f.gzz = vload<PL>(zzj, s.off_rg);
    };
    const V zero = V{};
    V wxx[U], wxy[U], wxz[U];
#pragma unroll
    for (int k = 0; k < U; k++) wxx[k] = wxy[k] = wxz[k] = zero;
    In pf;
    fetch(i0, pf);
    int tick = 0, hs = 0;  // hs: delay slot of plane i, (i - i0) mod (R + 1)
    for (int i = i0; i <= ilast; i++) {
        const In cur = pf;
        if (s.yring) yd[hs][tid] = cur.hxy;
        if (s.edge) zd[hs][s.ze] = cur.gxz;
        const int hc = hs == R ? 0 : hs + 1;  // slot of plane i - R
        hs = hc;
#pragma unroll
        for (int k = 0; k + 1 < U; k++) {
            wxx[k] = wxx[k + 1];
            wxy[k] = wxy[k + 1];
            wxz[k] = wxz[k + 1];
        }
        wxx[U - 1] = cur.xx;
        wxy[U - 1] = cur.xy;
        wxz[U - 1] = cur.xz;
        const int j = i - R;
        const bool out = j >= s.xa;
        const PlaneRef xj = plane(P, j, true);
        const int buf = tick & 1;
        V vo[3], bq[3], dz[3];
        if (out) {
#pragma unroll
            for (int c = 0; c < 3; c++) {
                vo[c] = vload<PL, wf::kStreaming>(at(P.v[c], xj), s.off);
                bq[c] = vload<PL, wf::kStreaming>(at(P.bq[c], xj), s.off);
            }
            sh[buf][0][s.row + R][s.zl] = wxy[CTR];
            sh[buf][1][s.row + R][s.zl] = cur.yy;
            sh[buf][2][s.row + R][s.zl] = cur.yz;
            if (s.yring) {
                sh[buf][0][s.yr_lds][s.zl] = yd[hc][tid];
                sh[buf][1][s.yr_lds][s.zl] = cur.hyy;
                sh[buf][2][s.yr_lds][s.zl] = cur.hyz;
            }
            float w[12];
            zlanes<R, PL>(s.edge ? zd[hc][s.ze] : zero, wxz[CTR], w);
            dz[0] = sdz<R, PL, false>(P, w);
            zlanes<R, PL>(cur.gyz, cur.yz, w);
            dz[1] = sdz<R, PL, false>(P, w);
            zlanes<R, PL>(cur.gzz, cur.zz, w);
            dz[2] = sdz<R, PL, true>(P, w);
        }
        fetch(i + 1, pf);
        if (out) {
            wf::lds_barrier();
            V f3[3];
            f3[0] = sdx<R, PL, true>(P, wxx) + sdy<R, PL, false>(P, sh[buf][0], s) + dz[0];
            f3[1] = sdx<R, PL, false>(P, wxy) + sdy<R, PL, true>(P, sh[buf][1], s) + dz[1];
            f3[2] = sdx<R, PL, false>(P, wxz) + sdy<R, PL, false>(P, sh[buf][2], s) + dz[2];
            const float dxy = P.dx[j] + dyv;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                V v = vo[c];
#pragma unroll
                for (int k = 0; k < PL; k++) {
                    const float d = dxy + dzv[k];
                    const float dd = d * P.hdt;
                    float r = __builtin_fmaf(1.0f - dd, v[k], bq[c][k] * f3[c][k]);
                    if (d != 0.0f) r /= 1.0f + dd;
                    v[k] = r;
                }
                vstore<PL>(at(P.vo[c] ? P.vo[c] : P.v[c], xj), s.off, v);
            }
            tick++;
        }
    }
}

template <int R, int PL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
el_str_s(const ElParams P)
{
    static_assert(R == 2 || R == 4, "streaming passes cover radius 2 and 4");
    using V = vec<PL>;
    constexpr int U = 2 * R + 1, LR = kSY + 2 * R, CTR = R;
    __shared__ V sh[2][3][LR][kSZ];  // vx, vy, vz along y
    // The halo values of vx, vy, vz (y halo rows, outer z values) are loaded
    // with the neighbouring tiles' own loads of the newest plane, while those
    // lines are in L2, and wait R ticks for the centre in thread-private LDS
    // delay lines.
    __shared__ V yd[R + 1][3][2 * R * kSZ];
    __shared__ V zd[R + 1][3][kSY * edge_lanes<R, PL>()];
    SSite s;
    if (!ssite<R, PL>(P, s)) return;
    const int tid = threadIdx.x;
    const float dyv = s.y < P.ny ? P.dy[s.y] : 0.0f;
    float dzv[PL];
#pragma unroll
    for (int k = 0; k < PL; k++) dzv[k] = s.z + k < P.nz ? P.dz[s.z + k] : 0.0f;
    struct In {
        V x, y, z;     // vx, vy, vz at the window plane i
        V hx, hy, hz;  // y halo at plane i
        V gx, gy, gz;  // outer z values at plane i
    };
    const int i0 = s.xa - R, ilast = s.xb - 1 + R;
    auto fetch = [&](int i, In &f) {
        const int j = i - R;
        const bool c = j >= s.xa && j < s.xb, w = i <= ilast;
        const PlaneRef xw = plane(P, i, w), xc = plane(P, j, c);
        f.x = vload<PL>(at(P.v[0], xw), s.off);
        f.y = vload<PL>(at(P.v[1], xw), s.off);
        f.z = vload<PL>(at(P.v[2], xw), s.off);
        const PlaneRef xh = plane(P, i, i >= s.xa && i < s.xb);  // a centre later
        const wf::rsrc_t dvx = at(P.v[0], xh), dvy = at(P.v[1], xh), dvz = at(P.v[2], xh);
        f.hx = vload<PL>(dvx, s.off_yr);
        f.hy = vload<PL>(dvy, s.off_yr);
        f.hz = vload<PL>(dvz, s.off_yr);
        f.gx = vload<PL>(dvx, s.off_rg);
        f.gy = vload<PL>(dvy, s.off_rg);
        f.gz = vload<PL>(dvz, s.off_rg);
    };
    const V zero = V{};
    V wx[U], wy[U], wz[U];
#pragma unroll
    for (int k = 0; k < U; k++) wx[k] = wy[k] = wz[k] = zero;
    In pf;
    fetch(i0, pf);
    int tick = 0, hs = 0;  // hs: delay slot of plane i, (i - i0) mod (R + 1)
    for (int i = i0; i <= ilast; i++) {
        const In cur = pf;
        if (s.yring) {
            yd[hs][0][tid] = cur.hx;
            yd[hs][1][tid] = cur.hy;
            yd[hs][2][tid] = cur.hz;
        }
        if (s.edge) {
            zd[hs][0][s.ze] = cur.gx;
            zd[hs][1][s.ze] = cur.gy;
            zd[hs][2][s.ze] = cur.gz;
        }
        const int hc = hs == R ? 0 : hs + 1;  // slot of plane i - R
        hs = hc;
#pragma unroll
        for (int k = 0; k + 1 < U; k++) {
            wx[k] = wx[k + 1];
            wy[k] = wy[k + 1];
            wz[k] = wz[k + 1];
        }
        wx[U - 1] = cur.x;
        wy[U - 1] = cur.y;
        wz[U - 1] = cur.z;
        const int j = i - R;
        const bool out = j >= s.xa;
        const PlaneRef xj = plane(P, j, true);
        const int buf = tick & 1;
        V lam, mu, ms[3], t[6], ezz, zxz, zyz;
        if (out) {
            const wf::rsrc_t lj = at(P.lam, xj), mj = at(P.mu, xj);
            lam = vload<PL, wf::kStreaming>(lj, s.off);
            mu = vload<PL, wf::kStreaming>(mj, s.off);
#pragma unroll
            for (int c = 0; c < 3; c++) ms[c] = vload<PL, wf::kStreaming>(at(P.ms[c], xj), s.off);
#pragma unroll
            for (int c = 0; c < 6; c++) t[c] = vload<PL, wf::kStreaming>(at(P.t[c], xj), s.off);
            sh[buf][0][s.row + R][s.zl] = wx[CTR];
            sh[buf][1][s.row + R][s.zl] = wy[CTR];
            sh[buf][2][s.row + R][s.zl] = wz[CTR];
            if (s.yring) {
                sh[buf][0][s.yr_lds][s.zl] = yd[hc][0][tid];
                sh[buf][1][s.yr_lds][s.zl] = yd[hc][1][tid];
                sh[buf][2][s.yr_lds][s.zl] = yd[hc][2][tid];
            }
            V gx = zero, gy = zero, gz = zero;
            if (s.edge) {
                gx = zd[hc][0][s.ze];
                gy = zd[hc][1][s.ze];
                gz = zd[hc][2][s.ze];
            }
            float w[12];
            zlanes<R, PL>(gz, wz[CTR], w);
            ezz = sdz<R, PL, false>(P, w);
            zlanes<R, PL>(gx, wx[CTR], w);
            zxz = sdz<R, PL, true>(P, w);
            zlanes<R, PL>(gy, wy[CTR], w);
            zyz = sdz<R, PL, true>(P, w);
        }
        fetch(i + 1, pf);
        if (out) {
            wf::lds_barrier();
            const V exx = sdx<R, PL, false>(P, wx);
            const V eyy = sdy<R, PL, false>(P, sh[buf][1], s);
            const V gxy = sdy<R, PL, true>(P, sh[buf][0], s) + sdx<R, PL, true>(P, wy);
            const V gxz = zxz + sdx<R, PL, true>(P, wz);
            const V gyz = zyz + sdy<R, PL, true>(P, sh[buf][2], s);
            const float dxy = P.dx[j] + dyv;
#pragma unroll
            for (int k = 0; k < PL; k++) {
                const float d = dxy + dzv[k];
                const float dd = d * P.hdt;
                const float beta = 1.0f - dd;
                const float tr = exx[k] + eyy[k] + ezz[k];
                const float mu2 = 2.0f * mu[k];
                float n[6];
                n[0] = __builtin_fmaf(beta, t[0][k], __builtin_fmaf(lam[k], tr, mu2 * exx[k]));
                n[1] = __builtin_fmaf(beta, t[1][k], __builtin_fmaf(lam[k], tr, mu2 * eyy[k]));
                n[2] = __builtin_fmaf(beta, t[2][k], __builtin_fmaf(lam[k], tr, mu2 * ezz[k]));
                n[3] = __builtin_fmaf(beta, t[3][k], ms[0][k] * gxy[k]);
                n[4] = __builtin_fmaf(beta, t[4][k], ms[1][k] * gxz[k]);
                n[5] = __builtin_fmaf(beta, t[5][k], ms[2][k] * gyz[k]);
                if (d != 0.0f) {
#pragma unroll
                    for (int c = 0; c < 6; c++) n[c] /= 1.0f + dd;
                }
#pragma unroll
                for (int c = 0; c < 6; c++) t[c][k] = n[c];
            }
#pragma unroll
            for (int c = 0; c < 6; c++)
                vstore<PL>(at(P.to[c] ? P.to[c] : P.t[c], xj), s.off, t[c]);
            tick++;
        }
    }
}

__global__ void el_src(float *__restrict__ txx, float *__restrict__ tyy, float *__restrict__ tzz,
                       const float *__restrict__ inc, const long long *__restrict__ soff, int npts,
                       long long plane, int xlo, int xhi)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    const long long o = soff[i], x = o / plane;
    if (x < xlo || x >= xhi) return;
    txx[o] += inc[i];
    tyy[o] += inc[i];
    tzz[o] += inc[i];
}

__global__ void el_rec(const float *__restrict__ txx, const float *__restrict__ tyy,
                       const float *__restrict__ tzz, const float *__restrict__ vz,
                       float *__restrict__ row_p, const long long *__restrict__ roff, int nrid,
                       float *__restrict__ row_v, const long long *__restrict__ roff2, int nrid2,
                       long long plane, int xlo, int xhi)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nrid) {
        const long long o = roff[i], x = o / plane;
        if (x >= xlo && x < xhi) row_p[i] = (txx[o] + tyy[o] + tzz[o]) / 3.0f;
    } else if (i < nrid + nrid2) {
        const int j = i - nrid;
        const long long o = roff2[j], x = o / plane;
        if (x >= xlo && x < xhi) row_v[j] = vz[o];
    }
}

// ---- Adjoint (multipliers vh in P.v, th in P.t; six scratch fields S). ----
// Stress-pass adjoint, pointwise part: S = C (th / alpha) with C = dt
// (lambda, mu, the averaged mu), then th = (beta / alpha) th.
__global__ void __launch_bounds__(256) el_adj_pre_str(const ElParams P, ElScratch S)
{
    Site q;
    if (!locate4(P, q)) return;
    f4 t[6];
#pragma unroll
    for (int c = 0; c < 6; c++) t[c] = ld4(P.t[c], q.off, true);
    const f4 lam = ld4(P.lam, q.off, true), mu = ld4(P.mu, q.off, true);
    const f4 m0 = ld4(P.ms[0], q.off, true), m1 = ld4(P.ms[1], q.off, true),
             m2 = ld4(P.ms[2], q.off, true);
    f4 o[6];
    const float dxy = P.dx[q.x] + P.dy[q.y];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int z = q.z4 + k;
        const float d = dxy + (z < P.nz ? P.dz[z] : 0.0f);
        const float dd = d * P.hdt;
        const float ia = d != 0.0f ? 1.0f / (1.0f + dd) : 1.0f;
        const float a = t[0][k] * ia, b = t[1][k] * ia, c = t[2][k] * ia;
        const float tr = a + b + c;
        o[0][k] = __builtin_fmaf(lam[k], tr, 2.0f * mu[k] * a);
        o[1][k] = __builtin_fmaf(lam[k], tr, 2.0f * mu[k] * b);
        o[2][k] = __builtin_fmaf(lam[k], tr, 2.0f * mu[k] * c);
        o[3][k] = m0[k] * (t[3][k] * ia);
        o[4][k] = m1[k] * (t[4][k] * ia);
        o[5][k] = m2[k] * (t[5][k] * ia);
        const float g = (1.0f - dd) * ia;
#pragma unroll
        for (int f = 0; f < 6; f++) t[f][k] *= g;
    }
#pragma unroll
    for (int c = 0; c < 6; c++) {
        *(f4 *)(S.f[c] + q.off) = o[c];
        *(f4 *)(P.t[c] + q.off) = t[c];
    }
}

// vh -= div S (the divergence of the velocity pass).
template <int R>
__global__ void __launch_bounds__(256) el_adj_vel(const ElParams P, ElScratch S)
{
    Site q;
    if (!locate4(P, q)) return;
    const f4 fx = dstg<R, 0, true>(S.f[0], P, q) + dstg<R, 1, false>(S.f[3], P, q) +
                  dstg<R, 2, false>(S.f[4], P, q);
    const f4 fy = dstg<R, 0, false>(S.f[3], P, q) + dstg<R, 1, true>(S.f[1], P, q) +
                  dstg<R, 2, false>(S.f[5], P, q);
    const f4 fz = dstg<R, 0, false>(S.f[4], P, q) + dstg<R, 1, false>(S.f[5], P, q) +
                  dstg<R, 2, true>(S.f[2], P, q);
    const f4 f3[3] = {fx, fy, fz};
#pragma unroll
    for (int c = 0; c < 3; c++) *(f4 *)(P.v[c] + q.off) = ld4(P.v[c], q.off, true) - f3[c];
}

// Velocity-pass adjoint, pointwise part: S[0..2] = (dt b / alpha) vh, then
// vh = (beta / alpha) vh.
__global__ void __launch_bounds__(256) el_adj_pre_vel(const ElParams P, ElScratch S)
{
    Site q;
    if (!locate4(P, q)) return;
    const float dxy = P.dx[q.x] + P.dy[q.y];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        f4 v = ld4(P.v[c], q.off, true);
        const f4 b = ld4(P.bq[c], q.off, true);
        f4 u;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int z = q.z4 + k;
            const float d = dxy + (z < P.nz ? P.dz[z] : 0.0f);
            const float dd = d * P.hdt;
            const float ia = d != 0.0f ? 1.0f / (1.0f + dd) : 1.0f;
            u[k] = b[k] * (v[k] * ia);
            v[k] *= (1.0f - dd) * ia;
        }
        *(f4 *)(S.f[c] + q.off) = u;
        *(f4 *)((P.vo[c] ? P.vo[c] : P.v[c]) + q.off) = v;
    }
}

// th -= strain(S[0..2]) (the strain operator of the stress pass).
template <int R>
__global__ void __launch_bounds__(256) el_adj_str(const ElParams P, ElScratch S)
{
    Site q;
    if (!locate4(P, q)) return;
    const f4 e[6] = {dstg<R, 0, false>(S.f[0], P, q), dstg<R, 1, false>(S.f[1], P, q),
                     dstg<R, 2, false>(S.f[2], P, q),
                     dstg<R, 1, true>(S.f[0], P, q) + dstg<R, 0, true>(S.f[1], P, q),
                     dstg<R, 2, true>(S.f[0], P, q) + dstg<R, 0, true>(S.f[2], P, q),
                     dstg<R, 2, true>(S.f[1], P, q) + dstg<R, 1, true>(S.f[2], P, q)};
#pragma unroll
    for (int c = 0; c < 6; c++) *(f4 *)(P.t[c] + q.off) = ld4(P.t[c], q.off, true) - e[c];
}

// Receiver adjoint of one step: th_ii += inc_p / 3 at the node points, vh_z
// += inc_v at the vz points.
__global__ void el_adj_inject(float *__restrict__ txx, float *__restrict__ tyy,
                              float *__restrict__ tzz, float *__restrict__ vz,
                              const float *__restrict__ inc_p, const long long *__restrict__ roff,
                              int nrid, const float *__restrict__ inc_v,
                              const long long *__restrict__ roff2, int nrid2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nrid) {
        const long long o = roff[i];
        const float a = inc_p[i] / 3.0f;
        txx[o] += a;
        tyy[o] += a;
        tzz[o] += a;
    } else if (i < nrid + nrid2) {
        const int j = i - nrid;
        vz[roff2[j]] += inc_v[j];
    }
}

// dt (thxx + thyy + thzz) / alpha at the source points.
__global__ void el_adj_record(const float *__restrict__ txx, const float *__restrict__ tyy,
                              const float *__restrict__ tzz, const long long *__restrict__ off,
                              const double *__restrict__ alpha, double dt, int n,
                              float *__restrict__ row)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const long long o = off[i];
        row[i] = (float)(dt * ((double)txx[o] + (double)tyy[o] + (double)tzz[o]) / alpha[i]);
    }
}

// ---- Gradient w.r.t. (lambda, mu, b) at the nodes (FP64 accumulators,
// padded layout; z < nz only). ----
// Stress-pass terms of one step: with s = th / alpha (th the multiplier of
// t^{t+1}) and e the strain of the forward v^{t+1/2} (fv),
//   glam += dt tr(s) tr(e),  gmu += 2 dt sum_i s_ii e_ii,
//   sh[c] += dt s_c e_c at the shear points (spread onto the nodes at the end).
template <int R>
__global__ void __launch_bounds__(256) el_img_str(const ElParams P, ElGradAcc G, ElScratch fv,
                                                  double dt)
{
    Site q;
    if (!locate4(P, q)) return;
    const f4 e[6] = {dstg<R, 0, false>(fv.f[0], P, q), dstg<R, 1, false>(fv.f[1], P, q),
                     dstg<R, 2, false>(fv.f[2], P, q),
                     dstg<R, 1, true>(fv.f[0], P, q) + dstg<R, 0, true>(fv.f[1], P, q),
                     dstg<R, 2, true>(fv.f[0], P, q) + dstg<R, 0, true>(fv.f[2], P, q),
                     dstg<R, 2, true>(fv.f[1], P, q) + dstg<R, 1, true>(fv.f[2], P, q)};
    f4 t[6];
#pragma unroll
    for (int c = 0; c < 6; c++) t[c] = ld4(P.t[c], q.off, true);
    const float dxy = P.dx[q.x] + P.dy[q.y];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int z = q.z4 + k;
        if (z >= P.nz) continue;
        const double ia = 1.0 / (1.0 + (double)((dxy + P.dz[z]) * P.hdt));
        const long long o = q.off + k;
        const double sxx = t[0][k] * ia, syy = t[1][k] * ia, szz = t[2][k] * ia;
        const double exx = e[0][k], eyy = e[1][k], ezz = e[2][k];
        G.lam[o] += dt * (sxx + syy + szz) * (exx + eyy + ezz);
        G.mu[o] += 2.0 * dt * (sxx * exx + syy * eyy + szz * ezz);
#pragma unroll
        for (int c = 0; c < 3; c++) G.sh[c][o] += dt * (t[3 + c][k] * ia) * (double)e[3 + c][k];
    }
}

// Velocity-pass terms: bv[a] += dt vh_a (div t^t)_a / alpha at the velocity
// points (vh the complete multiplier of v^{t+1/2}, ft the forward t^t).
template <int R>
__global__ void __launch_bounds__(256) el_img_vel(const ElParams P, ElGradAcc G, ElScratch ft,
                                                  double dt)
{
    Site q;
    if (!locate4(P, q)) return;
    const f4 fx = dstg<R, 0, true>(ft.f[0], P, q) + dstg<R, 1, false>(ft.f[3], P, q) +
                  dstg<R, 2, false>(ft.f[4], P, q);
    const f4 fy = dstg<R, 0, false>(ft.f[3], P, q) + dstg<R, 1, true>(ft.f[1], P, q) +
                  dstg<R, 2, false>(ft.f[5], P, q);
    const f4 fz = dstg<R, 0, false>(ft.f[4], P, q) + dstg<R, 1, false>(ft.f[5], P, q) +
                  dstg<R, 2, true>(ft.f[2], P, q);
    const f4 f3[3] = {fx, fy, fz};
    const float dxy = P.dx[q.x] + P.dy[q.y];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const f4 v = ld4(P.v[c], q.off, true);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int z = q.z4 + k;
            if (z >= P.nz) continue;
            const double ia = 1.0 / (1.0 + (double)((dxy + P.dz[z]) * P.hdt));
            G.bv[c][q.off + k] += dt * (double)v[k] * ia * (double)f3[c][k];
        }
    }
}

// Spreads the per-element terms onto the nodes (the transposes of the
// means): gmu gets 1/4 of each shear point's term at its four nodes, gb 1/2
// of each velocity point's term at its two nodes; a node index beyond the
// grid is the last node inside (so the last node collects that share too).
// Then out[0..2] = (glam, gmu, gb) unpadded.
__global__ void el_grad_finish(const ElParams P, ElGradAcc G, float *__restrict__ out)
{
    const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long N = (long long)P.nx * P.ny * P.nz;
    if (gid >= N) return;
    const int z = (int)(gid % P.nz);
    const long long xy = gid / P.nz;
    const int y = (int)(xy % P.ny), x = (int)(xy / P.ny);
    const int n3[3] = {P.nx, P.ny, P.nz};
    const int c3[3] = {x, y, z};
    auto at = [&](const double *f, int i, int j, int k) {
        return f[((long long)i * P.ny + j) * P.nzp + k];
    };
    // Weights of the element indices a = c and a = c - 1 along an axis.
    auto w0 = [&](int ax) { return c3[ax] == n3[ax] - 1 ? 2.0 : 1.0; };
    auto w1 = [&](int ax) { return c3[ax] >= 1 ? 1.0 : 0.0; };
    auto shifted = [&](int ax, int d, int *ijk) {
        ijk[0] = x;
        ijk[1] = y;
        ijk[2] = z;
        ijk[ax] -= d;
    };
    double gmu = at(G.mu, x, y, z);
    const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int c = 0; c < 3; c++) {
        const int a1 = pairs[c][0], a2 = pairs[c][1];
        for (int d1 = 0; d1 < 2; d1++)
            for (int d2 = 0; d2 < 2; d2++) {
                const double w = (d1 ? w1(a1) : w0(a1)) * (d2 ? w1(a2) : w0(a2));
                if (w == 0.0) continue;
                int ijk[3];
                shifted(a1, d1, ijk);
                ijk[a2] -= d2;
                gmu += 0.25 * w * at(G.sh[c], ijk[0], ijk[1], ijk[2]);
            }
    }
    double gb = 0.0;
    for (int a = 0; a < 3; a++)
        for (int d = 0; d < 2; d++) {
            const double w = d ? w1(a) : w0(a);
            if (w == 0.0) continue;
            int ijk[3];
            shifted(a, d, ijk);
            gb += 0.5 * w * at(G.bv[a], ijk[0], ijk[1], ijk[2]);
        }
    out[gid] = (float)at(G.lam, x, y, z);
    out[N + gid] = (float)gmu;
    out[2 * N + gid] = (float)gb;
}

unsigned nblocks(long long n) { return (unsigned)((n + 255) / 256); }

// Grid of a tiled launch over `planes` x-planes (16 x 64 tiles, one per
// workgroup), banded: S = tiles of one plane / 8 (rounded up), whole runs of
// 8S workgroups.
unsigned tiled(int planes, int ny, int nz4, int *band)
{
    const long long tpp = (long long)((ny + kTY - 1) / kTY) * ((nz4 + kTZ - 1) / kTZ);
    const long long S = std::max(1LL, (tpp + 7) / 8);
    const long long run = 8 * S, nb = (long long)planes * tpp;
    *band = (int)S;
    return (unsigned)((nb + run - 1) / run * run);
}

}  // namespace

tb_status launch_elastic_step(const ElParams &P, int r, const float *inc, const long long *soff,
                              int npts, float *row_p, const long long *roff, int nrid,
                              float *row_v, const long long *roff2, int nrid2, int rlo, int rhi,
                              hipStream_t st)
{
    const int xlo = P.xlo, xhi = P.xhi > 0 ? P.xhi : P.nx;
    const long long row = (long long)P.ny * (P.nzp / 4);
    const long long total = (long long)(xhi - xlo) * row;
    if (total <= 0) return TB_OK;
    // The velocity pass feeds the stress pass's x derivatives: r planes more
    // on each side. The stress pass reads the new velocities.
    ElParams V = P;
    V.xlo = std::max(0, xlo - r);
    V.xhi = std::min(P.nx, xhi + r);
    const long long vtotal = (long long)(V.xhi - V.xlo) * row;
    ElParams S = P;
    for (int c = 0; c < 3; c++) S.v[c] = P.vo[c] ? P.vo[c] : P.v[c];
    (void)vtotal;
    if (r == 2 || r == 4) {
        constexpr int VPL = 2, SPL = 2;  // z per lane of the two passes
        const unsigned vs = streamed(V.xhi - V.xlo, P.ny, P.nzp, VPL, P.ncu, &V.chunk, &V.nchunks),
                       ss = streamed(xhi - xlo, P.ny, P.nzp, SPL, P.ncu, &S.chunk, &S.nchunks);
        if (r == 2) {
            hipLaunchKernelGGL((el_vel_s<2, VPL>), dim3(vs), dim3(256), 0, st, V);
            hipLaunchKernelGGL((el_str_s<2, SPL>), dim3(ss), dim3(256), 0, st, S);
        } else {
            hipLaunchKernelGGL((el_vel_s<4, VPL>), dim3(vs), dim3(256), 0, st, V);
            hipLaunchKernelGGL((el_str_s<4, SPL>), dim3(ss), dim3(256), 0, st, S);
        }
    } else if (r == 6) {
        const unsigned vgrid = tiled(V.xhi - V.xlo, P.ny, P.nzp / 4, &V.band),
                       sgrid = tiled(xhi - xlo, P.ny, P.nzp / 4, &S.band);
        hipLaunchKernelGGL(el_vel<6>, dim3(vgrid), dim3(256), 0, st, V);
        hipLaunchKernelGGL(el_str<6>, dim3(sgrid), dim3(256), 0, st, S);
    } else {
        set_error("elastic radius %d not built", r);
        return TB_EUNSUPPORTED;
    }
    TB_HIP(hipGetLastError());
    float *const *tout = P.to[0] ? P.to : P.t;
    const long long plane = (long long)P.ny * P.nzp;
    if (npts > 0) {
        hipLaunchKernelGGL(el_src, dim3(nblocks(npts)), dim3(256), 0, st, tout[0], tout[1],
                           tout[2], inc, soff, npts, plane, xlo, xhi);
        TB_HIP(hipGetLastError());
    }
    if (nrid + nrid2 > 0 && rhi > rlo) {
        hipLaunchKernelGGL(el_rec, dim3(nblocks(nrid + nrid2)), dim3(256), 0, st, tout[0], tout[1],
                           tout[2], S.v[2], row_p, roff, nrid, row_v, roff2, nrid2, plane, rlo,
                           rhi);
        TB_HIP(hipGetLastError());
    }
    return TB_OK;
}

tb_status launch_elastic_adjoint_step(const ElParams &P, const ElScratch &S, int r,
                                      const float *inc_p, const long long *roff, int nrid,
                                      const float *inc_v, const long long *roff2, int nrid2,
                                      float *src_row, const long long *soff,
                                      const double *src_alpha, double dt, int npts,
                                      hipStream_t st)
{
    const long long total = (long long)P.nx * P.ny * (P.nzp / 4);
    if (total == 0) return TB_OK;
    if (npts > 0) {
        hipLaunchKernelGGL(el_adj_record, dim3(nblocks(npts)), dim3(256), 0, st, P.t[0], P.t[1],
                           P.t[2], soff, src_alpha, dt, npts, src_row);
        TB_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(el_adj_pre_str, dim3(nblocks(total)), dim3(256), 0, st, P, S);
    if (r == 2) hipLaunchKernelGGL(el_adj_vel<2>, dim3(nblocks(total)), dim3(256), 0, st, P, S);
    else if (r == 4) hipLaunchKernelGGL(el_adj_vel<4>, dim3(nblocks(total)), dim3(256), 0, st, P, S);
    else if (r == 6) hipLaunchKernelGGL(el_adj_vel<6>, dim3(nblocks(total)), dim3(256), 0, st, P, S);
    else {
        set_error("elastic radius %d not built", r);
        return TB_EUNSUPPORTED;
    }
    hipLaunchKernelGGL(el_adj_pre_vel, dim3(nblocks(total)), dim3(256), 0, st, P, S);
    if (r == 2) hipLaunchKernelGGL(el_adj_str<2>, dim3(nblocks(total)), dim3(256), 0, st, P, S);
    else if (r == 4) hipLaunchKernelGGL(el_adj_str<4>, dim3(nblocks(total)), dim3(256), 0, st, P, S);
    else hipLaunchKernelGGL(el_adj_str<6>, dim3(nblocks(total)), dim3(256), 0, st, P, S);
    TB_HIP(hipGetLastError());
    if (nrid + nrid2 > 0) {
        hipLaunchKernelGGL(el_adj_inject, dim3(nblocks(nrid + nrid2)), dim3(256), 0, st, P.t[0],
                           P.t[1], P.t[2], P.v[2], inc_p, roff, nrid, inc_v, roff2, nrid2);
        TB_HIP(hipGetLastError());
    }
    return TB_OK;
}

tb_status launch_elastic_gradient_step(const ElParams &P, const ElScratch &S,
                                       const ElScratch &fv, const ElScratch &ft,
                                       const ElGradAcc &G, int r, const float *inc_p,
                                       const long long *roff, int nrid, const float *inc_v,
                                       const long long *roff2, int nrid2, double dt,
                                       hipStream_t st)
{
    const long long total = (long long)P.nx * P.ny * (P.nzp / 4);
    if (total == 0) return TB_OK;
    const dim3 grid(nblocks(total)), blk(256);
#define TBW_EL_R(KERNEL, ...)                                                    \
    do {                                                                         \
        if (r == 2) hipLaunchKernelGGL(KERNEL<2>, grid, blk, 0, st, __VA_ARGS__); \
        else if (r == 4) hipLaunchKernelGGL(KERNEL<4>, grid, blk, 0, st, __VA_ARGS__); \
        else hipLaunchKernelGGL(KERNEL<6>, grid, blk, 0, st, __VA_ARGS__);       \
    } while (0)
    if (r != 2 && r != 4 && r != 6) {
        set_error("elastic radius %d not built", r);
        return TB_EUNSUPPORTED;
    }
    TBW_EL_R(el_img_str, P, G, fv, dt);
    hipLaunchKernelGGL(el_adj_pre_str, grid, blk, 0, st, P, S);
    TBW_EL_R(el_adj_vel, P, S);
    TBW_EL_R(el_img_vel, P, G, ft, dt);
    hipLaunchKernelGGL(el_adj_pre_vel, grid, blk, 0, st, P, S);
    TBW_EL_R(el_adj_str, P, S);
#undef TBW_EL_R
    TB_HIP(hipGetLastError());
    if (nrid + nrid2 > 0) {
        hipLaunchKernelGGL(el_adj_inject, dim3(nblocks(nrid + nrid2)), dim3(256), 0, st, P.t[0],
                           P.t[1], P.t[2], P.v[2], inc_p, roff, nrid, inc_v, roff2, nrid2);
        TB_HIP(hipGetLastError());
    }
    return TB_OK;
}

tb_status launch_elastic_grad_finish(const ElParams &P, const ElGradAcc &G, float *out,
                                     hipStream_t st)
{
    const long long N = (long long)P.nx * P.ny * P.nz;
    if (N == 0) return TB_OK;
    hipLaunchKernelGGL(el_grad_finish, dim3(nblocks(N)), dim3(256), 0, st, P, G, out);
    TB_HIP(hipGetLastError());
    return TB_OK;
}

}  // namespace tbw
