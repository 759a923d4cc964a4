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
// The forward step at radius 2 and 4 runs the x-streaming forms of the two
// kernels (tti_rot_s, tti_update_s; same per-point operations); radius 6 and
// the adjoint and imaging modes run the tiled ones.
#include <algorithm>

#include "stream_kernel.h"
#include "tti_params.h"

namespace tbw {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
using wf::f4v;

// Each thread takes 4 consecutive z (float4 accesses); neighbours along x and
// y are float4 loads, neighbours along z come from the window [z4-ZB,
// z4+4+ZB) of float4 loads, ZB = 4 up to radius 4 and 8 up to radius 6.
// Reads outside the grid give 0; the z padding holds 0 in every field.
template <int R>
constexpr int zspan()
{
    static_assert(R >= 1 && R <= 6, "radius must be 1..6");
    return R <= 4 ? 4 : 8;
}
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

__device__ __forceinline__ int xend(const TtiParams &P) { return P.xhi > 0 ? P.xhi : P.nx; }

__device__ __forceinline__ bool locate4(const TtiParams &P, Site &q)
{
    const int nz4 = P.nzp / 4;
    const long long gid = block_index(P) * blockDim.x + threadIdx.x;
    if (gid >= (long long)(xend(P) - P.xlo) * P.ny * nz4) return false;
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

template <int ZB>
__device__ __forceinline__ void zwin(const float *f, const Site &q, int nzp, float *w)
{
#pragma unroll
    for (int o = -ZB; o <= ZB; o += 4) {
        const f4 a = ld4(f, q.off + o, q.z4 + o >= 0 && q.z4 + o < nzp);
#pragma unroll
        for (int k = 0; k < 4; k++) w[ZB + o + k] = a[k];
    }
}

// Centred first derivative (unit spacing) of f along x / y at the 4 sites.
template <int R>
__device__ __forceinline__ f4 d1xy(const float *f, const TtiParams &P, const Site &q, int ax)
{
    f4 s = f4{0.f, 0.f, 0.f, 0.f};
    const long long st = ax == 0 ? q.sx : q.sy;
    const int c = ax == 0 ? q.x : q.y, n = ax == 0 ? P.nx : P.ny;
#pragma unroll
    for (int m = 1; m <= R; m++) {
        const f4 up = ld4(f, q.off + m * st, c + m < n), dn = ld4(f, q.off - m * st, c - m >= 0);
#pragma unroll
        for (int k = 0; k < 4; k++) s[k] = __builtin_fmaf(P.w1[m - 1], up[k] - dn[k], s[k]);
    }
    return s;
}

// 2-D tiles of the rotated-gradient and update kernels: a workgroup takes
// 16 y rows x 64 z (16 lanes of 4 z) of one x-plane. The fields (or the
// products of two fields) a kernel differentiates along y or z are staged in
// LDS with R rows and ZB z of halo on each side (zero outside the grid), so
// a y or z neighbour costs an LDS read instead of a vector load; x
// neighbours are read as before. Values and operation order are those of the
// one-point form, so the results are the same bits.
constexpr int kTY = 16, kTZ = 16;

template <int R>
struct TileLds {
    static constexpr int H = zspan<R>() / 4;
    f4 a[kTY + 2 * R][kTZ + 2 * H];
};

struct TileSite {
    Site q;
    int ty, tz, y0, c0;
    bool valid;
};

__device__ __forceinline__ bool tile_site(const TtiParams &P, TileSite &t)
{
    const int nz4 = P.nzp / 4;
    const int nty = (P.ny + kTY - 1) / kTY, ntz = (nz4 + kTZ - 1) / kTZ;
    const long long tpp = (long long)nty * ntz;
    const long long L = block_index(P);
    if (L >= (long long)(xend(P) - P.xlo) * tpp) return false;
    const int x = P.xlo + (int)(L / tpp);
    const int tl = (int)(L % tpp);
    t.ty = threadIdx.x / kTZ;
    t.tz = threadIdx.x % kTZ;
    t.y0 = (tl / ntz) * kTY;
    t.c0 = (tl % ntz) * kTZ;
    const int y = t.y0 + t.ty, z4 = (t.c0 + t.tz) * 4;
    t.valid = y < P.ny && z4 < P.nzp;
    t.q.x = x;
    t.q.y = y;
    t.q.z4 = z4;
    t.q.sx = (long long)P.ny * P.nzp;
    t.q.sy = P.nzp;
    t.q.off = ((long long)x * P.ny + y) * P.nzp + z4;
    return true;
}

// f (times g when g is set) at this tile's x: its own points, plus (YH) R
// rows above and below and (ZH) ZB z before and after. a[i][j] holds row
// y0 + i - R, float4 column c0 + j - H.
template <int R, bool YH, bool ZH>
__device__ __forceinline__ void stage(TileLds<R> &L, const float *f, const float *g,
                                      const TtiParams &P, const TileSite &t)
{
    constexpr int H = TileLds<R>::H;
    const long long plane = (long long)t.q.x * P.ny;
    auto at = [&](int y, int c) {
        const bool ok = y >= 0 && y < P.ny && c >= 0 && 4 * c < P.nzp;
        const long long o = (plane + y) * P.nzp + 4 * c;
        const f4 a = ld4(f, o, ok);
        if (!g) return a;
        const f4 b = ld4(g, o, ok);
        return f4{a[0] * b[0], a[1] * b[1], a[2] * b[2], a[3] * b[3]};
    };
    const int tid = threadIdx.x;
    L.a[t.ty + R][t.tz + H] = at(t.y0 + t.ty, t.c0 + t.tz);
    if constexpr (YH) {
        if (tid < 2 * R * kTZ) {
            const int hr = tid / kTZ, row = hr < R ? hr : kTY + hr;
            L.a[row][t.tz + H] = at(t.y0 + row - R, t.c0 + t.tz);
        }
    }
    if constexpr (ZH) {
        if (tid < 2 * H * kTY) {
            const int row = tid / (2 * H), hc = tid % (2 * H);
            const int col = hc < H ? hc : kTZ + hc;
            L.a[row + R][col] = at(t.y0 + row, t.c0 + col - H);
        }
    }
}

// Staged row y + m (m in [-R, R]) and the z window of the tile site (the
// values zwin reads).
template <int R>
__device__ __forceinline__ f4 yrow(const TileLds<R> &L, const TileSite &t, int m)
{
    return L.a[t.ty + R + m][t.tz + TileLds<R>::H];
}

template <int R>
__device__ __forceinline__ void zwin_lds(const TileLds<R> &L, const TileSite &t, float *w)
{
    constexpr int H = TileLds<R>::H, ZB = 4 * H;
#pragma unroll
    for (int o = -H; o <= H; o++) {
        const f4 a = L.a[t.ty + R][t.tz + H + o];
#pragma unroll
        for (int k = 0; k < 4; k++) w[ZB + 4 * o + k] = a[k];
    }
}

template <int R>
__global__ void __launch_bounds__(256) tti_rot(const TtiParams P)
{
    __shared__ TileLds<R> L[2];  // p, r along y
    TileSite t;
    if (!tile_site(P, t)) return;
    stage<R, true, false>(L[0], P.p, nullptr, P, t);
    stage<R, true, false>(L[1], P.r, nullptr, P, t);
    __syncthreads();
    if (!t.valid) return;
    const Site &q = t.q;
    constexpr int ZB = zspan<R>();
    float zp[4 + 2 * ZB], zr[4 + 2 * ZB];
    zwin<ZB>(P.p, q, P.nzp, zp);
    zwin<ZB>(P.r, q, P.nzp, zr);
    const f4 gpx = d1xy<R>(P.p, P, q, 0), grx = d1xy<R>(P.r, P, q, 0);
    f4 gpy = f4{0.f, 0.f, 0.f, 0.f}, gry = gpy;
#pragma unroll
    for (int m = 1; m <= R; m++) {
        const f4 pu = yrow<R>(L[0], t, m), pd = yrow<R>(L[0], t, -m);
        const f4 ru = yrow<R>(L[1], t, m), rd = yrow<R>(L[1], t, -m);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            gpy[k] = __builtin_fmaf(P.w1[m - 1], pu[k] - pd[k], gpy[k]);
            gry[k] = __builtin_fmaf(P.w1[m - 1], ru[k] - rd[k], gry[k]);
        }
    }
    const f4 ax = ld4(P.ax, q.off, true), ay = ld4(P.ay, q.off, true), az = ld4(P.az, q.off, true);
    f4 qp, qr;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        float gpz = 0.0f, grz = 0.0f;
#pragma unroll
        for (int m = 1; m <= R; m++) {
            gpz = __builtin_fmaf(P.w1[m - 1], zp[ZB + k + m] - zp[ZB + k - m], gpz);
            grz = __builtin_fmaf(P.w1[m - 1], zr[ZB + k + m] - zr[ZB + k - m], grz);
        }
        qp[k] = ax[k] * (gpx[k] * P.ih[0]) + ay[k] * (gpy[k] * P.ih[1]) + az[k] * (gpz * P.ih[2]);
        qr[k] = ax[k] * (grx[k] * P.ih[0]) + ay[k] * (gry[k] * P.ih[1]) + az[k] * (grz * P.ih[2]);
    }
    *(f4 *)(P.qp + q.off) = qp;
    *(f4 *)(P.qr + q.off) = qr;
}

// Modes: kForward, the update above; kAdjoint, the adjoint update, whose
// operator input (p, r) is the mixed field z, with rates psi = (H0 z_p,
// Hz z_r) + (beta/alpha) psi and levels advancing from lambda^{k+1} (lp,
// lr); kImage, the gradient's imaging term of a forward level w = (p, r):
// g += sum_f y_f c (A w)_f with y = (c/alpha) lambda^{k+1} (lp, lr), in FP64.
enum { kForward = 0, kAdjoint = 1, kImage = 2 };

template <int R, int MODE>
__global__ void __launch_bounds__(256) tti_update(const TtiParams P, double *__restrict__ g)
{
    constexpr bool ADJ = MODE == kAdjoint;
    // p, a_y q_p and a_y q_r along y.
    __shared__ TileLds<R> L[3];
    TileSite t;
    if (!tile_site(P, t)) return;
    stage<R, true, false>(L[0], P.p, nullptr, P, t);
    stage<R, true, false>(L[1], P.ay, P.qp, P, t);
    stage<R, true, false>(L[2], P.ay, P.qr, P, t);
    __syncthreads();
    if (!t.valid) return;
    const Site &q = t.q;
    constexpr int ZB = zspan<R>();
    float zp[4 + 2 * ZB], zaz[4 + 2 * ZB], zqp[4 + 2 * ZB], zqr[4 + 2 * ZB];
    zwin<ZB>(P.p, q, P.nzp, zp);
    zwin<ZB>(P.az, q, P.nzp, zaz);
    zwin<ZB>(P.qp, q, P.nzp, zqp);
    zwin<ZB>(P.qr, q, P.nzp, zqr);
    f4 lx = f4{0.f, 0.f, 0.f, 0.f}, ly = lx, hpx = lx, hpy = lx, hrx = lx, hry = lx;
    const f4 pc = ld4(P.p, q.off, true);
    // x neighbours from memory, one offset per iteration (rolled, the kernel
    // keeps 3 waves per SIMD); y neighbours from LDS.
#pragma unroll 1
    for (int m = 1; m <= R; m++) {
        const bool xp = q.x + m < P.nx, xm = q.x - m >= 0;
        const long long ox = m * q.sx;
        const f4 pxp = ld4(P.p, q.off + ox, xp), pxm = ld4(P.p, q.off - ox, xm);
        const f4 axp = ld4(P.ax, q.off + ox, xp), axm = ld4(P.ax, q.off - ox, xm);
        const f4 qpxp = ld4(P.qp, q.off + ox, xp), qpxm = ld4(P.qp, q.off - ox, xm);
        const f4 qrxp = ld4(P.qr, q.off + ox, xp), qrxm = ld4(P.qr, q.off - ox, xm);
        const float w1 = P.w1[m - 1], w2 = P.w2[m];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const float p2 = 2.0f * pc[k];
            lx[k] = __builtin_fmaf(w2, (pxp[k] + pxm[k]) - p2, lx[k]);
            hpx[k] = __builtin_fmaf(w1, axp[k] * qpxp[k] - axm[k] * qpxm[k], hpx[k]);
            hrx[k] = __builtin_fmaf(w1, axp[k] * qrxp[k] - axm[k] * qrxm[k], hrx[k]);
        }
    }
#pragma unroll 2
    for (int m = 1; m <= R; m++) {
        const f4 pyp = yrow<R>(L[0], t, m), pym = yrow<R>(L[0], t, -m);
        const f4 tpp = yrow<R>(L[1], t, m), tpm = yrow<R>(L[1], t, -m);
        const f4 trp = yrow<R>(L[2], t, m), trm = yrow<R>(L[2], t, -m);
        const float w1 = P.w1[m - 1], w2 = P.w2[m];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const float p2 = 2.0f * pc[k];
            ly[k] = __builtin_fmaf(w2, (pyp[k] + pym[k]) - p2, ly[k]);
            hpy[k] = __builtin_fmaf(w1, tpp[k] - tpm[k], hpy[k]);
            hry[k] = __builtin_fmaf(w1, trp[k] - trm[k], hry[k]);
        }
    }
    const f4 zero = f4{0.f, 0.f, 0.f, 0.f};
    const f4 rc = MODE != kForward ? ld4(P.lr, q.off, true) : ld4(P.r, q.off, true);
    const f4 lpc = MODE != kForward ? ld4(P.lp, q.off, true) : pc;
    const f4 e1 = ADJ ? zero : ld4(P.e1, q.off, true), sd = ADJ ? zero : ld4(P.sd, q.off, true),
             cc = ADJ ? zero : ld4(P.c, q.off, true);
    (void)zero;
    f4 vp = ld4(P.vp, q.off, true), vr = ld4(P.vr, q.off, true), pn, rn;
    const float dxy = P.dx[q.x] + P.dy[q.y];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const float p2 = 2.0f * pc[k];
        float lz = 0.0f, hpz = 0.0f, hrz = 0.0f;
#pragma unroll
        for (int m = 1; m <= R; m++) {
            lz = __builtin_fmaf(P.w2[m], (zp[ZB + k + m] + zp[ZB + k - m]) - p2, lz);
            hpz = __builtin_fmaf(P.w1[m - 1], zaz[ZB + k + m] * zqp[ZB + k + m] -
                                                  zaz[ZB + k - m] * zqp[ZB + k - m], hpz);
            hrz = __builtin_fmaf(P.w1[m - 1], zaz[ZB + k + m] * zqr[ZB + k + m] -
                                                  zaz[ZB + k - m] * zqr[ZB + k - m], hrz);
        }
        const float lap = lx[k] * P.ih2[0] + ly[k] * P.ih2[1] + lz * P.ih2[2];
        const float hzp = hpx[k] * P.ih[0] + hpy[k] * P.ih[1] + hpz * P.ih[2];
        const float hzr = hrx[k] * P.ih[0] + hry[k] * P.ih[1] + hrz * P.ih[2];
        const float h0p = lap - hzp;
        const int z = q.z4 + k;
        const float d = dxy + (z < P.nz ? P.dz[z] : 0.0f);
        const float dd = d * P.hdt;
        const float beta = 1.0f - dd;
        float wp, wr;
        if constexpr (MODE == kImage) {
            if (z < P.nz) {
                const float rhs_p = __builtin_fmaf(e1[k], h0p, sd[k] * hzr);
                const float rhs_r = __builtin_fmaf(sd[k], h0p, hzr);
                const double ca = (double)cc[k] / (1.0 + (double)dd);
                g[q.off + k] += ca * ((double)lpc[k] * ((double)cc[k] * rhs_p) +
                                      (double)rc[k] * ((double)cc[k] * rhs_r));
            }
            continue;
        } else if constexpr (ADJ) {
            wp = d != 0.0f ? __builtin_fmaf(beta / (1.0f + dd), vp[k], h0p) : h0p + vp[k];
            wr = d != 0.0f ? __builtin_fmaf(beta / (1.0f + dd), vr[k], hzr) : hzr + vr[k];
        } else {
            const float rhs_p = __builtin_fmaf(e1[k], h0p, sd[k] * hzr);
            const float rhs_r = __builtin_fmaf(sd[k], h0p, hzr);
            wp = __builtin_fmaf(cc[k], rhs_p, beta * vp[k]);
            wr = __builtin_fmaf(cc[k], rhs_r, beta * vr[k]);
            if (d != 0.0f) {
                wp = wp / (1.0f + dd);
                wr = wr / (1.0f + dd);
            }
        }
        vp[k] = wp;
        vr[k] = wr;
        pn[k] = lpc[k] + wp;
        rn[k] = rc[k] + wr;
    }
    if constexpr (MODE != kImage) {
        *(f4 *)((P.vpo ? P.vpo : P.vp) + q.off) = vp;
        *(f4 *)((P.vro ? P.vro : P.vr) + q.off) = vr;
        *(f4 *)(P.pn + q.off) = pn;
        *(f4 *)(P.rn + q.off) = rn;
    }
}

// ---------------------------------------------------------------------------
// Streaming forward kernels (radius 2 and 4; building blocks in
// stream_kernel.h). Slot k of an x window holds plane j - R + k for the
// centre plane j, shifted by one slot per tick. The inputs a tick starts
// with are loaded during the previous tick. Per point the operations and
// their order are those of tti_rot / tti_update above (with contraction off,
// a product formed once and reused rounds the same), so the streaming and
// tiled kernels give the same bits.
using namespace st;

// Centred first derivative (unit weights w1) of the PL points along z.
template <int R, int PL>
__device__ __forceinline__ vec<PL> d1z(const TtiParams &P, const float *w)
{
    vec<PL> g;
#pragma unroll
    for (int k = 0; k < PL; k++) {
        float a = 0.0f;
#pragma unroll
        for (int m = 1; m <= R; m++) a = __builtin_fmaf(P.w1[m - 1], w[4 + k + m] - w[4 + k - m], a);
        g[k] = a;
    }
    return g;
}

template <int R, int PL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
tti_rot_s(const TtiParams P)
{
    static_assert(R == 2 || R == 4, "streaming kernels cover radius 2 and 4");
    using V = vec<PL>;
    constexpr int U = 2 * R + 1, LR = kSY + 2 * R, CTR = R;
    __shared__ V sh[2][2][LR][kSZ];  // p, r along y
    SSite s;
    if (!ssite<R, PL>(P, s)) return;
    struct In {
        V p, r;            // window plane i
        V ax, ay, az;      // centre plane j = i - R
        V yp, yr, gp, gr;  // halo values at j
    };
    const int i0 = s.xa - R, ilast = s.xb - 1 + R;
    auto fetch = [&](int i, In &f) {
        const int j = i - R;
        const bool c = j >= s.xa && j < s.xb, w = i <= ilast;
        const PlaneRef xw = plane(P, i, w), xc = plane(P, j, c);
        f.p = vload<PL>(at(P.p, xw), s.off);
        f.r = vload<PL>(at(P.r, xw), s.off);
        f.ax = vload<PL, wf::kStreaming>(at(P.ax, xc), s.off);
        f.ay = vload<PL, wf::kStreaming>(at(P.ay, xc), s.off);
        f.az = vload<PL, wf::kStreaming>(at(P.az, xc), s.off);
        const wf::rsrc_t pj = at(P.p, xc), rj = at(P.r, xc);
        f.yp = vload<PL>(pj, s.off_yr);
        f.yr = vload<PL>(rj, s.off_yr);
        f.gp = vload<PL>(pj, s.off_rg);
        f.gr = vload<PL>(rj, s.off_rg);
    };
    const V zero = V{};
    V wp[U], wr[U];  // x windows, slot k = plane j - R + k
#pragma unroll
    for (int k = 0; k < U; k++) wp[k] = wr[k] = zero;
    In pf;
    fetch(i0, pf);
    int tick = 0;
    for (int i = i0; i <= ilast; i++) {
        const In cur = pf;
#pragma unroll
        for (int k = 0; k + 1 < U; k++) {
            wp[k] = wp[k + 1];
            wr[k] = wr[k + 1];
        }
        wp[U - 1] = cur.p;
        wr[U - 1] = cur.r;
        const int j = i - R;
        const bool out = j >= s.xa;
        const PlaneRef xj = plane(P, j, true);
        const int buf = tick & 1;
        V gpz, grz;
        if (out) {
            sh[buf][0][s.row + R][s.zl] = wp[CTR];
            sh[buf][1][s.row + R][s.zl] = wr[CTR];
            if (s.yring) {
                sh[buf][0][s.yr_lds][s.zl] = cur.yp;
                sh[buf][1][s.yr_lds][s.zl] = cur.yr;
            }
            float zp[12], zr[12];
            zlanes<R, PL>(cur.gp, wp[CTR], zp);
            zlanes<R, PL>(cur.gr, wr[CTR], zr);
            gpz = d1z<R, PL>(P, zp);
            grz = d1z<R, PL>(P, zr);
        }
        const V ax = cur.ax, ay = cur.ay, az = cur.az;
        fetch(i + 1, pf);
        if (out) {
            wf::lds_barrier();
            V gpx = zero, grx = zero, gpy = zero, gry = zero;
#pragma unroll
            for (int m = 1; m <= R; m++) {
#pragma unroll
                for (int k = 0; k < PL; k++) {
                    gpx[k] = __builtin_fmaf(P.w1[m - 1], wp[CTR + m][k] - wp[CTR - m][k], gpx[k]);
                    grx[k] = __builtin_fmaf(P.w1[m - 1], wr[CTR + m][k] - wr[CTR - m][k], grx[k]);
                }
            }
#pragma unroll
            for (int m = 1; m <= R; m++) {
                const V pu = sh[buf][0][s.row + R + m][s.zl], pd = sh[buf][0][s.row + R - m][s.zl];
                const V ru = sh[buf][1][s.row + R + m][s.zl], rd = sh[buf][1][s.row + R - m][s.zl];
#pragma unroll
                for (int k = 0; k < PL; k++) {
                    gpy[k] = __builtin_fmaf(P.w1[m - 1], pu[k] - pd[k], gpy[k]);
                    gry[k] = __builtin_fmaf(P.w1[m - 1], ru[k] - rd[k], gry[k]);
                }
            }
            V qp, qr;
#pragma unroll
            for (int k = 0; k < PL; k++) {
                qp[k] = ax[k] * (gpx[k] * P.ih[0]) + ay[k] * (gpy[k] * P.ih[1]) + az[k] * (gpz[k] * P.ih[2]);
                qr[k] = ax[k] * (grx[k] * P.ih[0]) + ay[k] * (gry[k] * P.ih[1]) + az[k] * (grz[k] * P.ih[2]);
            }
            vstore<PL>(at(P.qp, xj), s.off, qp);
            vstore<PL>(at(P.qr, xj), s.off, qr);
            tick++;
        }
    }
}

template <int R, int PL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
tti_update_s(const TtiParams P)
{
    static_assert(R == 2 || R == 4, "streaming kernels cover radius 2 and 4");
    using V = vec<PL>;
    constexpr int U = 2 * R + 1, LR = kSY + 2 * R, CTR = R;
    __shared__ V sh[2][3][LR][kSZ];  // p, a_y q_p, a_y q_r along y
    // q_p, q_r of the newest plane wait R ticks for their turn as the centre
    // plane in a thread-private LDS delay line (each thread reads back only
    // its own values): re-reading them from memory would miss L2 by then.
    __shared__ V qd[R + 1][2][kSY * kSZ];
    // The same for the halo values of p, q_p, q_r (the y halo rows and the
    // tile's outer z values): they are loaded with the neighbouring tiles'
    // own loads of the newest plane, while those lines are in L2, and wait R
    // ticks for the centre.
    __shared__ V yd[R + 1][3][2 * R * kSZ];
    __shared__ V zd[R + 1][3][kSY * edge_lanes<R, PL>()];
    SSite s;
    if (!ssite<R, PL>(P, s)) return;
    const bool edge = s.edge;
    const int ze = s.ze;
    const bool yin = s.y < P.ny;
    const float dyv = yin ? P.dy[s.y] : 0.0f;
    float dzv[PL];
#pragma unroll
    for (int k = 0; k < PL; k++) dzv[k] = s.z + k < P.nz ? P.dz[s.z + k] : 0.0f;
    // Inputs loaded a tick ahead (those the tick starts with); the update's
    // own centre inputs (r, w_p, w_r, 1+2e, s, c) are loaded as the tick
    // starts, for use at its end.
    struct In {
        V p, ax, qp, qr;       // window plane i
        V ay, az;              // centre plane j = i - R
        V yp, yqp, yqr;        // y halo at i
        V gp, gqp, gqr;        // outer z values at i
        V yay, gaz;            // y halo and outer z values at j
    };
    float *const vpo = P.vpo ? P.vpo : P.vp;
    float *const vro = P.vro ? P.vro : P.vr;
    const int i0 = s.xa - R, ilast = s.xb - 1 + R;
    auto fetch = [&](int i, In &f) {
        const int j = i - R;
        const bool c = j >= s.xa && j < s.xb, w = i <= ilast;
        const PlaneRef xw = plane(P, i, w), xc = plane(P, j, c);
        f.p = vload<PL>(at(P.p, xw), s.off);
        f.ax = vload<PL>(at(P.ax, xw), s.off);
        f.qp = vload<PL>(at(P.qp, xw), s.off);
        f.qr = vload<PL>(at(P.qr, xw), s.off);
        const bool h = i >= s.xa && i < s.xb;  // plane i is a centre later
        const PlaneRef xh = plane(P, i, h);
        const wf::rsrc_t pi = at(P.p, xh), qpi = at(P.qp, xh),
                         qri = at(P.qr, xh), ayj = at(P.ay, xc),
                         azj = at(P.az, xc);
        f.ay = vload<PL>(ayj, s.off);
        f.az = vload<PL>(azj, s.off);
        f.yp = vload<PL>(pi, s.off_yr);
        f.yqp = vload<PL>(qpi, s.off_yr);
        f.yqr = vload<PL>(qri, s.off_yr);
        f.gp = vload<PL>(pi, s.off_rg);
        f.gqp = vload<PL>(qpi, s.off_rg);
        f.gqr = vload<PL>(qri, s.off_rg);
        f.yay = vload<PL>(ayj, s.off_yr);
        f.gaz = vload<PL>(azj, s.off_rg);
    };
    const V zero = V{};
    V wp[U], wpx[U], wrx[U];  // p, a_x q_p, a_x q_r along x
#pragma unroll
    for (int k = 0; k < U; k++) wp[k] = wpx[k] = wrx[k] = zero;
    In pf;
    fetch(i0, pf);
    const int tid = threadIdx.x;
    int tick = 0, qs = 0;  // qs: delay-line slot of plane i, (i - i0) mod (R + 1)
    for (int i = i0; i <= ilast; i++) {
        const In cur = pf;
        qd[qs][0][tid] = cur.qp;
        qd[qs][1][tid] = cur.qr;
        if (s.yring) {
            yd[qs][0][tid] = cur.yp;
            yd[qs][1][tid] = cur.yqp;
            yd[qs][2][tid] = cur.yqr;
        }
        if (edge) {
            zd[qs][0][ze] = cur.gp;
            zd[qs][1][ze] = cur.gqp;
            zd[qs][2][ze] = cur.gqr;
        }
        const int qc = qs == R ? 0 : qs + 1;  // slot of plane i - R
        qs = qc;
#pragma unroll
        for (int k = 0; k + 1 < U; k++) {
            wp[k] = wp[k + 1];
            wpx[k] = wpx[k + 1];
            wrx[k] = wrx[k + 1];
        }
        wp[U - 1] = cur.p;
        wpx[U - 1] = vmul(cur.ax, cur.qp);
        wrx[U - 1] = vmul(cur.ax, cur.qr);
        const int j = i - R;
        const bool out = j >= s.xa;
        const PlaneRef xj = plane(P, j, true);
        // First half (no LDS reads): publish the centre plane and take the z
        // terms from the adjacent lanes; the next tick's inputs are requested
        // once this tick's are consumed.
        V rc, vpc, vrc, e1, sd, cc, lz, hpz, hrz;
        const int buf = tick & 1;
        const V pc = wp[CTR];
        if (out) {
            const V cqp = qd[qc][0][tid], cqr = qd[qc][1][tid];
            rc = vload<PL, wf::kStreaming>(at(P.r, xj), s.off);
            vpc = vload<PL, wf::kStreaming>(at(P.vp, xj), s.off);
            vrc = vload<PL, wf::kStreaming>(at(P.vr, xj), s.off);
            e1 = vload<PL, wf::kStreaming>(at(P.e1, xj), s.off);
            sd = vload<PL, wf::kStreaming>(at(P.sd, xj), s.off);
            cc = vload<PL, wf::kStreaming>(at(P.c, xj), s.off);
            sh[buf][0][s.row + R][s.zl] = pc;
            sh[buf][1][s.row + R][s.zl] = vmul(cur.ay, cqp);
            sh[buf][2][s.row + R][s.zl] = vmul(cur.ay, cqr);
            if (s.yring) {
                sh[buf][0][s.yr_lds][s.zl] = yd[qc][0][tid];
                sh[buf][1][s.yr_lds][s.zl] = vmul(cur.yay, yd[qc][1][tid]);
                sh[buf][2][s.yr_lds][s.zl] = vmul(cur.yay, yd[qc][2][tid]);
            }
            V gp = zero, gqp = zero, gqr = zero;
            if (edge) {
                gp = zd[qc][0][ze];
                gqp = zd[qc][1][ze];
                gqr = zd[qc][2][ze];
            }
            float zp[12], zqp[12], zqr[12];
            zlanes<R, PL>(gp, pc, zp);
            zlanes<R, PL>(vmul(cur.gaz, gqp), vmul(cur.az, cqp), zqp);
            zlanes<R, PL>(vmul(cur.gaz, gqr), vmul(cur.az, cqr), zqr);
#pragma unroll
            for (int k = 0; k < PL; k++) {
                const float p2 = 2.0f * pc[k];
                float l = 0.0f;
#pragma unroll
                for (int m = 1; m <= R; m++)
                    l = __builtin_fmaf(P.w2[m], (zp[4 + k + m] + zp[4 + k - m]) - p2, l);
                lz[k] = l;
            }
            hpz = d1z<R, PL>(P, zqp);
            hrz = d1z<R, PL>(P, zqr);
        }
        fetch(i + 1, pf);
        if (out) {
            wf::lds_barrier();
            V lx = zero, ly = zero, hpx = zero, hpy = zero, hrx = zero, hry = zero;
#pragma unroll
            for (int m = 1; m <= R; m++) {
                const float w1 = P.w1[m - 1], w2 = P.w2[m];
#pragma unroll
                for (int k = 0; k < PL; k++) {
                    const float p2 = 2.0f * pc[k];
                    lx[k] = __builtin_fmaf(w2, (wp[CTR + m][k] + wp[CTR - m][k]) - p2, lx[k]);
                    hpx[k] = __builtin_fmaf(w1, wpx[CTR + m][k] - wpx[CTR - m][k], hpx[k]);
                    hrx[k] = __builtin_fmaf(w1, wrx[CTR + m][k] - wrx[CTR - m][k], hrx[k]);
                }
            }
#pragma unroll
            for (int m = 1; m <= R; m++) {
                const V pyp = sh[buf][0][s.row + R + m][s.zl], pym = sh[buf][0][s.row + R - m][s.zl];
                const V tpp = sh[buf][1][s.row + R + m][s.zl], tpm = sh[buf][1][s.row + R - m][s.zl];
                const V trp = sh[buf][2][s.row + R + m][s.zl], trm = sh[buf][2][s.row + R - m][s.zl];
                const float w1 = P.w1[m - 1], w2 = P.w2[m];
#pragma unroll
                for (int k = 0; k < PL; k++) {
                    const float p2 = 2.0f * pc[k];
                    ly[k] = __builtin_fmaf(w2, (pyp[k] + pym[k]) - p2, ly[k]);
                    hpy[k] = __builtin_fmaf(w1, tpp[k] - tpm[k], hpy[k]);
                    hry[k] = __builtin_fmaf(w1, trp[k] - trm[k], hry[k]);
                }
            }
            const float dxy = P.dx[j] + dyv;
            V vp = vpc, vr = vrc, pn, rn;
#pragma unroll
            for (int k = 0; k < PL; k++) {
                const float lap = lx[k] * P.ih2[0] + ly[k] * P.ih2[1] + lz[k] * P.ih2[2];
                const float hzp = hpx[k] * P.ih[0] + hpy[k] * P.ih[1] + hpz[k] * P.ih[2];
                const float hzr = hrx[k] * P.ih[0] + hry[k] * P.ih[1] + hrz[k] * P.ih[2];
                const float h0p = lap - hzp;
                const float d = dxy + dzv[k];
                const float dd = d * P.hdt;
                const float beta = 1.0f - dd;
                const float rhs_p = __builtin_fmaf(e1[k], h0p, sd[k] * hzr);
                const float rhs_r = __builtin_fmaf(sd[k], h0p, hzr);
                float wpn = __builtin_fmaf(cc[k], rhs_p, beta * vp[k]);
                float wrn = __builtin_fmaf(cc[k], rhs_r, beta * vr[k]);
                if (d != 0.0f) {
                    wpn = wpn / (1.0f + dd);
                    wrn = wrn / (1.0f + dd);
                }
                vp[k] = wpn;
                vr[k] = wrn;
                pn[k] = pc[k] + wpn;
                rn[k] = rc[k] + wrn;
            }
            vstore<PL>(at(vpo, xj), s.off, vp);
            vstore<PL>(at(vro, xj), s.off, vr);
            vstore<PL>(at(P.pn, xj), s.off, pn);
            vstore<PL>(at(P.rn, xj), s.off, rn);
            tick++;
        }
    }
}

// Points of planes [xlo, xhi) only (plane = ny * nzp elements).
__global__ void tti_sparse(float *__restrict__ p, float *__restrict__ r, float *__restrict__ vp,
                           float *__restrict__ vr, const float *__restrict__ inc,
                           const long long *__restrict__ soff, int npts, long long plane, int xlo,
                           int xhi)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npts) {
        const long long o = soff[i];
        const long long x = o / plane;
        if (x < xlo || x >= xhi) return;
        p[o] += inc[i];
        r[o] += inc[i];
        vp[o] += inc[i];
        vr[o] += inc[i];
    }
}

__global__ void tti_record(const float *__restrict__ p, float *__restrict__ rec_row,
                           const long long *__restrict__ roff, int nrid, long long plane, int xlo,
                           int xhi)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nrid) {
        const long long o = roff[i], x = o / plane;
        if (x >= xlo && x < xhi) rec_row[i] = p[o];
    }
}

// z = (c/alpha) D lambda with D = [[1+2 eps, s], [s, 1]] per node.
__global__ void __launch_bounds__(256) tti_adj_mix(const TtiParams P)
{
    Site q;
    if (!locate4(P, q)) return;
    const f4 lp = ld4(P.lp, q.off, true), lr = ld4(P.lr, q.off, true);
    const f4 cc = ld4(P.c, q.off, true), e1 = ld4(P.e1, q.off, true), sd = ld4(P.sd, q.off, true);
    const float dxy = P.dx[q.x] + P.dy[q.y];
    f4 zp, zr;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int z = q.z4 + k;
        const float d = dxy + (z < P.nz ? P.dz[z] : 0.0f);
        const float ca = d != 0.0f ? cc[k] / (1.0f + d * P.hdt) : cc[k];
        const float yp = ca * lp[k], yr = ca * lr[k];
        zp[k] = __builtin_fmaf(e1[k], yp, sd[k] * yr);
        zr[k] = __builtin_fmaf(sd[k], yp, yr);
    }
    *(f4 *)(P.zp + q.off) = zp;
    *(f4 *)(P.zr + q.off) = zr;
}

// The residual enters the p component of lambda and of its rate.
__global__ void tti_adj_inject(float *__restrict__ lam, float *__restrict__ rate,
                               const float *__restrict__ inc, const long long *__restrict__ off,
                               int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const long long o = off[i];
        lam[o] += inc[i];
        rate[o] += inc[i];
    }
}

// Source-point imaging term: gs[i] += row[i] alpha[i] s[i], with row the
// samples c (lambda_p + lambda_r)^{k+1} / alpha and s the injected increment.
__global__ void tti_image_sparse(const float *__restrict__ row, const double *__restrict__ alpha,
                                 const float *__restrict__ inc, int n, double *__restrict__ gs)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) gs[i] += (double)row[i] * (alpha[i] * (double)inc[i]);
}

// c (lambda_p + lambda_r) / alpha at the source points.
__global__ void tti_adj_record(const float *__restrict__ lp, const float *__restrict__ lr,
                               const float *__restrict__ c, const long long *__restrict__ off,
                               const double *__restrict__ alpha, int n, float *__restrict__ row)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const long long o = off[i];
        row[i] = (float)((double)c[o] * ((double)lp[o] + (double)lr[o]) / alpha[i]);
    }
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

tb_status launch_tti_step(const TtiParams &P, int r, const float *inc, const long long *soff,
                          int npts, float *rec_row, const long long *roff, int nrid, int rlo,
                          int rhi, hipStream_t st)
{
    const int xlo = P.xlo, xhi = P.xhi > 0 ? P.xhi : P.nx;
    const long long row = (long long)P.ny * (P.nzp / 4);
    const long long total = (long long)(xhi - xlo) * row;
    if (total <= 0) return TB_OK;
    // The rotated gradients feed the update's x derivatives: r planes more
    // on each side.
    TtiParams G = P;
    G.xlo = std::max(0, xlo - r);
    G.xhi = std::min(P.nx, xhi + r);
    TtiParams U = P;
    if (r == 2 || r == 4) {
        // The rotated gradient takes 4 z per lane, the update 2 (its three x
        // windows and the next tick's inputs then fit three waves per SIMD).
        const unsigned gs = streamed(G.xhi - G.xlo, P.ny, P.nzp, 4, P.ncu, &G.chunk, &G.nchunks),
                       us = streamed(xhi - xlo, P.ny, P.nzp, 2, P.ncu, &U.chunk, &U.nchunks);
        if (r == 2) {
            hipLaunchKernelGGL((tti_rot_s<2, 4>), dim3(gs), dim3(256), 0, st, G);
            hipLaunchKernelGGL((tti_update_s<2, 2>), dim3(us), dim3(256), 0, st, U);
        } else {
            hipLaunchKernelGGL((tti_rot_s<4, 4>), dim3(gs), dim3(256), 0, st, G);
            hipLaunchKernelGGL((tti_update_s<4, 2>), dim3(us), dim3(256), 0, st, U);
        }
    } else if (r == 6) {
        const unsigned ggrid = tiled(G.xhi - G.xlo, P.ny, P.nzp / 4, &G.band),
                       ugrid = tiled(xhi - xlo, P.ny, P.nzp / 4, &U.band);
        hipLaunchKernelGGL(tti_rot<6>, dim3(ggrid), dim3(256), 0, st, G);
        hipLaunchKernelGGL((tti_update<6, kForward>), dim3(ugrid), dim3(256), 0, st, U, nullptr);
    } else {
        set_error("TTI radius %d not built", r);
        return TB_EUNSUPPORTED;
    }
    TB_HIP(hipGetLastError());
    const long long plane = (long long)P.ny * P.nzp;
    if (npts > 0) {
        hipLaunchKernelGGL(tti_sparse, dim3(nblocks(npts)), dim3(256), 0, st, P.pn, P.rn,
                           P.vpo ? P.vpo : P.vp, P.vro ? P.vro : P.vr, inc, soff, npts, plane,
                           xlo, xhi);
        TB_HIP(hipGetLastError());
    }
    if (nrid > 0 && rhi > rlo) {
        hipLaunchKernelGGL(tti_record, dim3(nblocks(nrid)), dim3(256), 0, st, P.pn, rec_row, roff,
                           nrid, plane, rlo, rhi);
        TB_HIP(hipGetLastError());
    }
    return TB_OK;
}

tb_status launch_tti_adjoint_step(const TtiParams &P, int r, const float *inc,
                                  const long long *roff, int nrid, float *src_row,
                                  const long long *soff, const double *src_alpha, int npts,
                                  hipStream_t st)
{
    const long long total = (long long)P.nx * P.ny * (P.nzp / 4);
    if (total == 0) return TB_OK;
    if (npts > 0) {
        hipLaunchKernelGGL(tti_adj_record, dim3(nblocks(npts)), dim3(256), 0, st, P.lp, P.lr, P.c,
                           soff, src_alpha, npts, src_row);
        TB_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(tti_adj_mix, dim3(nblocks(total)), dim3(256), 0, st, P);
    TtiParams Q = P;
    const unsigned tgrid = tiled(P.nx, P.ny, P.nzp / 4, &Q.band);
    if (r == 2) {
        hipLaunchKernelGGL(tti_rot<2>, dim3(tgrid), dim3(256), 0, st, Q);
        hipLaunchKernelGGL((tti_update<2, kAdjoint>), dim3(tgrid), dim3(256), 0, st, Q,
                           nullptr);
    } else if (r == 4) {
        hipLaunchKernelGGL(tti_rot<4>, dim3(tgrid), dim3(256), 0, st, Q);
        hipLaunchKernelGGL((tti_update<4, kAdjoint>), dim3(tgrid), dim3(256), 0, st, Q,
                           nullptr);
    } else if (r == 6) {
        hipLaunchKernelGGL(tti_rot<6>, dim3(tgrid), dim3(256), 0, st, Q);
        hipLaunchKernelGGL((tti_update<6, kAdjoint>), dim3(tgrid), dim3(256), 0, st, Q,
                           nullptr);
    } else {
        set_error("TTI radius %d not built", r);
        return TB_EUNSUPPORTED;
    }
    TB_HIP(hipGetLastError());
    if (nrid > 0) {
        hipLaunchKernelGGL(tti_adj_inject, dim3(nblocks(nrid)), dim3(256), 0, st, P.pn, P.vp, inc,
                           roff, nrid);
        TB_HIP(hipGetLastError());
    }
    return TB_OK;
}

tb_status launch_tti_image(const TtiParams &P, int r, double *g, hipStream_t st)
{
    const long long total = (long long)P.nx * P.ny * (P.nzp / 4);
    if (total == 0) return TB_OK;
    TtiParams Q = P;
    const unsigned tgrid = tiled(P.nx, P.ny, P.nzp / 4, &Q.band);
    if (r == 2) {
        hipLaunchKernelGGL(tti_rot<2>, dim3(tgrid), dim3(256), 0, st, Q);
        hipLaunchKernelGGL((tti_update<2, kImage>), dim3(tgrid), dim3(256), 0, st, Q, g);
    } else if (r == 4) {
        hipLaunchKernelGGL(tti_rot<4>, dim3(tgrid), dim3(256), 0, st, Q);
        hipLaunchKernelGGL((tti_update<4, kImage>), dim3(tgrid), dim3(256), 0, st, Q, g);
    } else if (r == 6) {
        hipLaunchKernelGGL(tti_rot<6>, dim3(tgrid), dim3(256), 0, st, Q);
        hipLaunchKernelGGL((tti_update<6, kImage>), dim3(tgrid), dim3(256), 0, st, Q, g);
    } else {
        set_error("TTI radius %d not built", r);
        return TB_EUNSUPPORTED;
    }
    TB_HIP(hipGetLastError());
    return TB_OK;
}

tb_status launch_tti_image_sparse(const float *row, const double *alpha, const float *inc,
                                  int npts, double *gs, hipStream_t st)
{
    if (npts == 0) return TB_OK;
    hipLaunchKernelGGL(tti_image_sparse, dim3(nblocks(npts)), dim3(256), 0, st, row, alpha, inc,
                       npts, gs);
    TB_HIP(hipGetLastError());
    return TB_OK;
}

}  // namespace tbw
