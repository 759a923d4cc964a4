// Building blocks of the x-streaming forward kernels (TTI and elastic).
//
// A workgroup of 256 threads owns a 16-row tile of 16 lanes per row, each
// lane PL consecutive z (PL = 2 or 4), and streams a chunk of x planes. Each
// thread keeps the x windows of its column in registers, publishes the
// centre plane's y-differentiated values to double-buffered LDS together
// with R halo rows on each side loaded from memory, and takes z neighbours
// from the adjacent lanes of its 16-lane row by DPP, the row's edge lanes
// supplying the tile's outer z values. All field traffic uses buffer
// instructions with per-plane descriptors built on the scalar unit: lanes
// outside the grid carry an offset past the plane (loads give 0, stores are
// dropped), and planes outside [0, nx), or outside the chunk for the
// centre-plane inputs, get an empty descriptor.
#pragma once

#include <algorithm>

#include "acoustic_kernel.h"  // buffer, DPP and barrier helpers (tbw::wf)

namespace tbw {
namespace st {

constexpr int kSY = 16, kSZ = 16;  // tile rows, lanes per row

// PL consecutive z per lane (2 or 4) as one vector.
template <int PL>
struct VecOf;
template <>
struct VecOf<2> {
    typedef float type __attribute__((ext_vector_type(2)));
    typedef unsigned bits __attribute__((ext_vector_type(2)));
};
template <>
struct VecOf<4> {
    typedef float type __attribute__((ext_vector_type(4)));
    typedef unsigned bits __attribute__((ext_vector_type(4)));
};
template <int PL>
using vec = typename VecOf<PL>::type;

template <int PL, int POLICY = wf::kTemporal>
__device__ __forceinline__ vec<PL> vload(wf::rsrc_t r, unsigned off)
{
    if constexpr (PL == 2)
        return __builtin_bit_cast(vec<2>, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, POLICY));
    else
        return __builtin_bit_cast(vec<4>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, POLICY));
}
template <int PL>
__device__ __forceinline__ void vstore(wf::rsrc_t r, unsigned off, vec<PL> v)
{
    if constexpr (PL == 2)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(typename VecOf<2>::bits, v), r,
                                              (int)off, 0, wf::kStreaming);
    else
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(typename VecOf<4>::bits, v), r,
                                               (int)off, 0, wf::kStreaming);
}
// Lane l takes lane l -+ 1 or 2 of its 16-lane row; lanes whose source lies
// outside the row keep `edge` (vshift) or take 0 (vshift0). One DPP move per
// component, written out (as the acoustic kernel's row_shift): moves over
// vector elements indexed in a loop have been merged into one by the
// compiler.
template <int CTRL, int PL>
__device__ __forceinline__ vec<PL> vshift(vec<PL> edge, vec<PL> v)
{
    if constexpr (PL == 4)
        return wf::row_shift<CTRL>(edge, v);
    else
        return vec<2>{wf::lane_shift<CTRL>(edge.x, v.x), wf::lane_shift<CTRL>(edge.y, v.y)};
}
template <int CTRL, int PL>
__device__ __forceinline__ vec<PL> vshift0(vec<PL> v)
{
    if constexpr (PL == 4)
        return wf::row_shift0<CTRL>(v);
    else
        return vec<2>{wf::lane_shift0<CTRL>(v.x), wf::lane_shift0<CTRL>(v.y)};
}

// z neighbours of the PL own points: w[4 + k + m] is point k's neighbour at
// offset m (|m| <= R <= 4). With 4 z per lane the float4s of lanes l-1, l,
// l+1 cover that; with 2 z per lane the pairs of lanes l-2 .. l+2 (l-1 ..
// l+1 at radius 2). rg: the tile's outer values held by the edge lanes (4 z
// per lane: lane 0 the float4 before the tile, lane 15 the one after; 2 z
// per lane: lanes 0 and 1 the pair 4 z before their own, lanes 14 and 15 the
// pair 4 after, or lanes 0 and 15 the pair 2 away at radius 2).
template <int R, int PL>
__device__ __forceinline__ void zlanes(vec<PL> rg, vec<PL> v, float *w)
{
    if constexpr (PL == 4) {
        const vec<4> l1 = vshift<wf::kDppRowShr1, 4>(rg, v), r1 = vshift<wf::kDppRowShl1, 4>(rg, v);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            w[k] = l1[k];
            w[4 + k] = v[k];
            w[8 + k] = r1[k];
        }
    } else {
        vec<2> l1, r1;
        if constexpr (R <= 2) {
            l1 = vshift<wf::kDppRowShr1, 2>(rg, v);
            r1 = vshift<wf::kDppRowShl1, 2>(rg, v);
        } else {
            // Lane 0's left pair is lane 1's outer pair, lane 15's right
            // pair lane 14's.
            l1 = vshift<wf::kDppRowShr1, 2>(vshift0<wf::kDppRowShl1, 2>(rg), v);
            r1 = vshift<wf::kDppRowShl1, 2>(vshift0<wf::kDppRowShr1, 2>(rg), v);
            const vec<2> l2 = vshift<wf::kDppRowShr2, 2>(rg, v), r2 = vshift<wf::kDppRowShl2, 2>(rg, v);
            w[0] = l2[0];
            w[1] = l2[1];
            w[8] = r2[0];
            w[9] = r2[1];
        }
        w[2] = l1[0];
        w[3] = l1[1];
        w[4] = v[0];
        w[5] = v[1];
        w[6] = r1[0];
        w[7] = r1[1];
    }
}

// Work item and lane geometry of a streaming launch (tiles of 16 rows x
// 16 PL z).
struct SSite {
    int xa, xb;        // chunk planes [xa, xb)
    int row, zl, y, z;
    unsigned off;      // own points in the plane (kNoLane outside the grid)
    unsigned off_yr;   // y halo row of threads < 2R*16 (whole waves)
    unsigned off_rg;   // outer z values of the edge lanes
    int yr_lds;        // LDS row of the y halo value
    bool yring;
    bool edge;         // lane holds outer z values
    int ze;            // its index among the tile's edge lanes (row-major)
};

// Edge lanes per row: lanes 0 and 15, or lanes 0, 1, 14 and 15 (2 z per lane
// beyond radius 2).
template <int R, int PL>
constexpr int edge_lanes()
{
    return PL == 4 || R <= 2 ? 2 : 4;
}

template <int R, int PL, class Params>
__device__ __forceinline__ bool ssite(const Params &P, SSite &s)
{
    constexpr int ZW = PL * kSZ;
    const int ntz = (P.nzp + ZW - 1) / ZW;
    const int ntiles = ((P.ny + kSY - 1) / kSY) * ntz;
    const int nwg = ntiles * P.nchunks;
    // XCD-aware order: the hardware deals consecutive workgroups to the 8
    // XCDs round-robin; XCD k takes the k-th contiguous run of the
    // chunk-major work list, so each XCD streams whole x ranges of
    // neighbouring tiles in step and their halo rows meet in its L2.
    const int b = blockIdx.x, q8 = nwg >> 3, r8 = nwg & 7, xcd = b & 7;
    const int wi = xcd * q8 + min(xcd, r8) + (b >> 3);
    const int chunk = wi / ntiles, tile = wi % ntiles;
    s.xa = P.xlo + chunk * P.chunk;
    s.xb = min(s.xa + P.chunk, P.xhi > 0 ? P.xhi : P.nx);
    const int tid = threadIdx.x;
    s.row = tid / kSZ;
    s.zl = tid % kSZ;
    const int y0 = (tile / ntz) * kSY, z0 = (tile % ntz) * ZW;
    s.y = y0 + s.row;
    s.z = z0 + PL * s.zl;
    const bool yin = s.y < P.ny, zin = s.z < P.nzp;
    s.off = (yin && zin) ? (unsigned)((s.y * P.nzp + s.z) * 4) : wf::kNoLane;
    s.yring = tid < 2 * R * kSZ;
    const int yr = s.row < R ? y0 - R + s.row : y0 + kSY + s.row - R;
    const bool yrok = s.yring && yr >= 0 && yr < P.ny && zin;
    s.off_yr = yrok ? (unsigned)((yr * P.nzp + s.z) * 4) : wf::kNoLane;
    s.yr_lds = s.row < R ? s.row : kSY + s.row;
    constexpr int ZO = PL == 4 || R <= 2 ? PL : 4;  // distance of the outer values
    constexpr int NE = edge_lanes<R, PL>();
    s.edge = s.zl < NE / 2 || s.zl >= kSZ - NE / 2;
    s.ze = s.row * NE + (s.zl < kSZ / 2 ? s.zl : s.zl - kSZ + NE);
    const int zr = s.zl < kSZ / 2 ? s.z - ZO : s.z + ZO;
    const bool rgok = s.edge && yin && zr >= 0 && zr < P.nzp;
    s.off_rg = rgok ? (unsigned)((s.y * P.nzp + zr) * 4) : wf::kNoLane;
    return s.xa < s.xb;
}

template <class V>
__device__ __forceinline__ V vmul(V a, V b)
{
    return a * b;  // elementwise, rounded per element (contraction is off)
}

// Byte offset of plane x and its size (0 unless ok and 0 <= x < nx),
// computed once per plane and tick; at() forms a field's descriptor from it
// with one 64-bit add, so that empty planes read 0 without a branch.
struct PlaneRef {
    long long off;
    unsigned bytes;
};
template <class Params>
__device__ __forceinline__ PlaneRef plane(const Params &P, int x, bool ok)
{
    const bool in = ok && x >= 0 && x < P.nx;
    const long long pb = (long long)P.ny * P.nzp * 4;
    return PlaneRef{in ? (long long)x * pb : 0, in ? (unsigned)pb : 0u};
}
__device__ __forceinline__ wf::rsrc_t at(const float *f, PlaneRef r)
{
    return wf::make_rsrc((const char *)f + r.off, r.bytes);
}

// Grid of a streaming launch over `planes` planes: the tiles of a plane
// times the chunks of x, about two workgroups per CU (ncu compute units)
// with at least 16 planes per chunk (each chunk re-reads 2R planes of halo).
inline unsigned streamed(int planes, int ny, int nzp, int pl, int ncu, int *chunk, int *nchunks)
{
    const int zw = pl * kSZ;
    const int ntiles = ((ny + kSY - 1) / kSY) * ((nzp + zw - 1) / zw);
    const int want = std::max(1, 2 * std::max(1, ncu) / ntiles);
    const int ch = std::min(planes, std::max(16, (planes + want - 1) / want));
    *chunk = ch;
    *nchunks = (planes + ch - 1) / ch;
    return (unsigned)(ntiles * *nchunks);
}

}  // namespace st
}  // namespace tbw
