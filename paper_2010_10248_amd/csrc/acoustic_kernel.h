// Isotropic acoustic propagator kernel for gfx950 (CDNA4).
//
// One kernel template covers both schedules of the paper:
//   T == 1  spatial blocking (Fig. 4a): one time step per pass over memory;
//   T >= 2  wave-front temporal blocking (Section II-B, Fig. 7/8a and the
//           final loop-nest listing): T steps per pass.
//
// A workgroup owns a y-z tile (BYE rows x 64 z; each lane holds 4
// consecutive z as one float4) and streams along x. Stage s of the pipeline
// holds the (2R+1)-plane window of time level n+s in registers (the x
// neighbours) and publishes its centre plane to LDS, from where the y and z
// neighbours are read. Stage s lags stage s-1 by R planes: the wave-front
// angle the stencil radius imposes (Section II-B). The y-z tile carries an
// overlapped halo of R(T-1), so the T stages need no exchange between
// workgroups; an x-chunk carries the same halo along x.
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
//
// Throughput notes (the kernel is VALU-issue bound unless the per-point
// instruction count is kept near the arithmetic of the stencil):
//  * all field traffic uses buffer instructions whose descriptor is rebuilt
//    per plane on the scalar unit; lanes outside the grid carry an offset
//    past the end of the buffer, so their loads return 0 and their stores are
//    dropped — no per-lane address arithmetic or masking;
//  * inputs are loaded PD ticks ahead into a register ring, and the barrier
//    fences LDS only, so the loads of later ticks stay in flight across it;
//  * c = dt^2 vp^2 is zero outside the grid, so points outside the domain
//    evaluate to +0 without masking.
#pragma once

#include <type_traits>

#include "acoustic_params.h"

namespace tbw {
namespace wf {

typedef float f4v __attribute__((ext_vector_type(4)));
using rsrc_t = __amdgpu_buffer_rsrc_t;

// Raw-buffer descriptor word 3 for gfx9-class parts (32-bit data format).
constexpr int kRsrcWord3 = 0x00020000;
// Byte offset beyond any buffer: loads return 0, stores are discarded.
constexpr unsigned kNoLane = 0x80000000u;

// DPP controls (16-lane rows): lane l takes lane l-1 / l+1 of its row; the
// lane at the row's end keeps the value passed as `old`.
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShl1 = 0x101;
constexpr int kDppRowShr2 = 0x112;
constexpr int kDppRowShl2 = 0x102;
// Damping values of the chunk's x range (chunk plus halo) staged in LDS.
constexpr int kDxCap = kMaxChunk + 32;

// z neighbours from the adjacent lanes of the same tile row (a tile row is
// one 16-lane DPP row), with `edge` supplying the lane at the row's end.
// The operands are passed as named scalars: with vector-element operands
// indexed in a loop the compiler merged the four moves into one.
template <int CTRL>
__device__ __forceinline__ float lane_shift(float edge, float v)
{
    const int e = __builtin_bit_cast(int, edge);
    const int x = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(e, x, CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ f4v row_shift(f4v edge, f4v v)
{
    return f4v{lane_shift<CTRL>(edge.x, v.x), lane_shift<CTRL>(edge.y, v.y),
               lane_shift<CTRL>(edge.z, v.z), lane_shift<CTRL>(edge.w, v.w)};
}
// The same with 0 at the row's end (no edge operand to set up).
template <int CTRL>
__device__ __forceinline__ float lane_shift0(float v)
{
    const int x = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ f4v row_shift0(f4v v)
{
    return f4v{lane_shift0<CTRL>(v.x), lane_shift0<CTRL>(v.y), lane_shift0<CTRL>(v.z),
               lane_shift0<CTRL>(v.w)};
}

__device__ __forceinline__ float uniform(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             kRsrcWord3);
}

// Cache policy of the buffer instructions: 2 marks the access streaming
// (non-temporal), so it does not displace lines other workgroups reuse.
constexpr int kTemporal = 0, kStreaming = 2;

template <int POLICY = kTemporal>
__device__ __forceinline__ f4v bload(rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, POLICY));
}

__device__ __forceinline__ void bstore(rsrc_t r, unsigned off, f4v v)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v),
                                           r, (int)off, 0, kStreaming);
}

// Workgroup barrier that orders LDS only. __syncthreads() also fences global
// memory, which makes the compiler wait for every outstanding global load
// (the prefetches of later ticks included) at each barrier; the kernels here
// never exchange global data inside a launch, so an LDS-scoped fence suffices.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// The per-point update shared by every schedule (fixed operation order), in
// the velocity form of the leapfrog recursion, v^n = u^n - u^{n-1}:
//   lap = sum_j wx_j ((x-j + x+j) - 2u) + (same in z) + (same in y)
//   v'  = (c lap + beta v) / alpha
// and then u' = u + v' (after the injection into v'). With differences from
// the centre the Laplacian of a constant is exactly zero whatever the FP32
// rounding of the weights, and carrying v instead of u^{n-1} keeps the
// rounding of u' from entering as a velocity error; in FP32 over a thousand
// steps each of the two changes removes most of the drift from the FP64
// definition. Without damping (d == 0, beta == 1) the fast path evaluates
// the same expression with identical rounding.
//
// With equal spacing on all axes (ISO) the three axes share one weight per
// offset and the Laplacian is sum_j w_j (((x-j + x+j) + (z-j + z+j)) +
// (y-j + y+j) - 6u): seven operations per offset instead of nine, still
// exactly zero on a constant field (the neighbour sum and 6u round the same
// exact value 6u). The Laplacian is evaluated in the kernel body, the
// velocity update here.
template <bool DAMP>
__device__ __forceinline__ float vel_update(const AcParams &p, float lap, float vold, float cc,
                                            float d)
{
    if constexpr (DAMP) {
        // 1/alpha by the hardware reciprocal (exact for alpha == 1, so an
        // undamped point gives the fast path's bits).
        const float dd = d * p.hdt;
        const float beta = 1.0f - dd;
        const float r = __builtin_fmaf(cc, lap, beta * vold);
        return r * __builtin_amdgcn_rcpf(1.0f + dd);
    } else {
        return __builtin_fmaf(cc, lap, vold);
    }
}

// Thread-private LDS rings (each lane reads back only its own points, so
// they need no barrier): stage 0 keeps its c planes for the later stages
// (stage s reads the one of R*s ticks earlier; written after the tick's
// reads, R*(T-1) slots), and stage s hands v to stage s+1, which reads it R
// ticks later (R+1 slots: the writer runs first within a tick).
constexpr int cring_slots(int R, int T) { return T > 1 ? R * (T - 1) : 0; }
constexpr int vring_slots(int R, int T) { return T > 1 ? R + 1 : 0; }


// Side inputs of one tick, loaded PD ticks ahead into a register ring: the
// newest u^n plane, and v^n and c at the stage-0 centre plane.
struct FarIn {
    f4v u;
    f4v v;
    f4v c;
};
// Halo rings of stage 0 (z ring: lanes 0 and 15; y ring: threads < 2R*16),
// mostly served by the caches: loaded right after a tick's barrier for the
// next tick, a full tick ahead of their use, in a single register set.
struct RingIn {
    f4v rg;
    f4v yr;
};

// LDS of one workgroup (one instance shared by the body's variants). The
// 16-byte arrays come first, so the struct has no padding inside.
template <int R, int T, int LZ, int BYE, bool GL>
struct WfLds {
    static constexpr int LR = BYE + 2 * R;  // LDS rows per stage (with the y ring)
    static constexpr int NTH = LZ * BYE;
    static constexpr int NSC = cring_slots(R, T), NSV = vring_slots(R, T);
    static constexpr int SC = GL ? 1 : kSrcCap;
    f4v sh[2][T][LR][LZ];
    f4v s_c[NSC ? NSC : 1][NSC ? NTH : 1];
    f4v s_v[T > 1 ? T - 1 : 1][NSV ? NSV : 1][NSV ? NTH : 1];
    int s_src[SC];  // injection-list keys (the point IDs stay in global memory)
    float s_val[SC][T];
    float s_dx[kDxCap];
};

// LDS bytes of one workgroup of acoustic_wavefront<R, T, LZ, BYE> (GL: the
// sparse lists are read from global memory instead of being staged).
template <int R, int T, int LZ, int BYE, bool GL = false>
constexpr int wavefront_lds()
{
    return (int)sizeof(WfLds<R, T, LZ, BYE, GL>);
}

// The kernel body for one job: b is the workgroup's index within the job's
// grid of p.nwg workgroups.
// GL selects where the segment's sparse lists are walked: staged in LDS
// (the common case), or read in place from global memory when a segment
// holds more entries than the LDS lists (dense sources or receivers).
template <int R, int T, int LZ, int BYE, int PD, bool GL, bool ISO>
__device__ __forceinline__ void wavefront_body(const AcParams &p, const int b,
                                               WfLds<R, T, LZ, BYE, GL> &lds)
{
    constexpr int U = 2 * R + 1;  // window slots: the 2R+1 live planes
    static_assert(U % PD == 0, "prefetch ring must divide the window");
    constexpr int HY = R * (T - 1);
    constexpr int HZ = ((R * (T - 1) + 3) / 4) * 4;
    constexpr int OY = BYE - 2 * HY;
    constexpr int OZ = 4 * LZ - 2 * HZ;
    constexpr int LR = BYE + 2 * R;  // LDS rows per stage (with the y ring)
    // LDS row: the LZ lane columns (z neighbours move between lanes by DPP).
    constexpr int LC = LZ;
    constexpr int NTH = LZ * BYE;
    static_assert(OY > 0 && OZ > 0, "tile too small for this depth");
    static_assert(R >= 1 && R <= 6, "radius must be 1..6");
    // z neighbours span one float4 on each side (R <= 4) or two (R <= 6).
    constexpr int ZB = R <= 4 ? 4 : 8;
    static_assert(NTH <= kMaxThreads && LZ == 16 && BYE <= 32, "workgroup shape");
    constexpr int NSC = cring_slots(R, T);
    constexpr int NSV = vring_slots(R, T);

    auto &sh = lds.sh;
    auto &s_src = lds.s_src;
    auto &s_val = lds.s_val;
    auto &s_dx = lds.s_dx;
    auto &s_c = lds.s_c;
    auto &s_v = lds.s_v;

    const int tid = threadIdx.x;
    const int zl = tid % LZ;
    const int row = tid / LZ;
    // Lanes that load the tile's outer z values for stage 0: the first and
    // last ZB/4 lanes of a row, each the float4 ZB before / after its own.
    const bool has_rg = zl < ZB / 4 || zl >= LZ - ZB / 4;
    const bool has_yr = tid < 2 * R * LZ;
    const int yr_lds = row < R ? row : BYE + row;
    const bool own_rc = row >= HY && row < HY + OY && zl >= HZ / 4 && zl < (HZ + OZ) / 4;
    const unsigned plane_bytes = (unsigned)(p.sx * 4);
    const int mykey = row * 32 + zl;

    // XCD-aware order: hardware hands consecutive workgroups to the 8 XCDs
    // round-robin; give each XCD a contiguous run of work (neighbouring
    // tiles or x ranges) so halo re-reads hit the same L2.
    const int nb = p.nwg;
    const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7;
    const int wg = xcd * q8 + min(xcd, r8) + (b >> 3);

    for (int sg = p.seg_off[wg]; sg < p.seg_off[wg + 1]; sg++) {
    const SegDesc sd = p.segs[sg];
    const int tz = sd.tile % p.tiles_z;
    const int tyi = sd.tile / p.tiles_z;
    const int y0 = tyi * OY - HY, z0 = tz * OZ - HZ;
    const int xc0 = sd.xs, xc1 = sd.xe;
    const int y = y0 + row, z = z0 + 4 * zl;
    const bool yin = (unsigned)y < (unsigned)p.ny;
    const bool zin = z >= 0 && z < p.nzp;
    // In-plane byte offsets (kNoLane for lanes outside the grid).
    const unsigned off_c = (yin && zin) ? (unsigned)((y * p.nzp + z) * 4) : kNoLane;
    const unsigned off_own = own_rc ? off_c : kNoLane;
    // z ring of stage 0: lane 0 of each row loads z0-4..z0-1, lane LZ-1 loads
    // the float4 after the tile (one float4 covers the radius).
    const int zr = zl < LZ / 2 ? z - ZB : z + ZB;
    const bool rgok = yin && has_rg && zr >= 0 && zr < p.nzp;
    const unsigned off_rg = rgok ? (unsigned)((y * p.nzp + zr) * 4) : kNoLane;
    // y ring of stage 0: rows y0-R..y0-1 and y0+BYE..y0+BYE+R-1.
    const int yr = row < R ? y0 - R + row : y0 + BYE + row - R;
    const bool yrok = has_yr && (unsigned)yr < (unsigned)p.ny && zin;
    const unsigned off_yr = yrok ? (unsigned)((yr * p.nzp + z) * 4) : kNoLane;

    // Damping of this thread's points along y and z (zero outside the grid).
    float dyz[4];
    bool any_dyz = false;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const bool in = yin && z + k >= 0 && z + k < p.nz;
        dyz[k] = in ? p.dy[y] + p.dz[z + k] : 0.0f;
        any_dyz |= dyz[k] != 0.0f;
    }
    const bool wave_dyz = __builtin_amdgcn_ballot_w64(any_dyz) != 0;

    // The previous segment's readers are done with LDS before it is reused.
    lds_barrier();
    // Clear the LDS planes so the unused ring rows/columns stay zero.
    for (int k = tid; k < 2 * T * LR * LC; k += NTH)
        (&sh[0][0][0][0])[k] = f4v{0.f, 0.f, 0.f, 0.f};

    // Per-stage x ranges; damping d_x over [xlo, xlo + nxd) staged in LDS.
    int lo[T], hi[T];
#pragma unroll
    for (int s = 0; s < T; s++) {
        lo[s] = max(0, xc0 - R * (T - 1 - s));
        hi[s] = min(p.nx, xc1 + R * (T - 1 - s));
    }
    const int xlo = lo[0];
    const int nxd = hi[0] - lo[0];
    for (int k = tid; k < nxd; k += NTH) s_dx[k] = p.dx[xlo + k];

    // Stage the segment's injection list (with the decomposed wavelet values
    // of this pass's T steps) in LDS; the GL variant reads the list and the
    // values from global memory instead.
    const int sbeg = sd.sbeg, nsl = sd.sn;
    const int rbeg = sd.rbeg, nrl = sd.rn;
    const int2 *gsrc = p.src + sbeg, *grec = p.rec + rbeg;
    if constexpr (!GL) {
        // The host launches this variant only for segments within the LDS
        // capacities; the bounds keep LDS writes inside the arrays regardless.
        for (int k = tid; k < nsl && k < kSrcCap; k += NTH) {
            const int2 e = gsrc[k];
            s_src[k] = e.x;
#pragma unroll
            for (int s = 0; s < T; s++)
                s_val[k][s] = p.dcmp[(long long)(p.n0 + s) * p.npts + e.y];
        }
    }
    // List accessors (one address space per instantiation).
    auto skey = [&](int k) -> int {
        if constexpr (GL) return gsrc[k].x;
        else return s_src[k];
    };
    lds_barrier();
    // Each lane walks its own entries (sorted by x) with one cursor per stage,
    // so a tick costs one compare per stage unless this lane has a point on
    // the stage's plane.
    auto first_at = [&](auto key, int n, int x) {
        const int want = tile_key(row, zl, x, 0);  // first entry of this lane at >= x
        int a = 0, b2 = n;
        while (a < b2) {
            const int mid = (a + b2) >> 1;
            if (key(mid) < want) a = mid + 1;
            else b2 = mid;
        }
        return a;
    };
    auto next_x = [&](auto key, int n, int k) {
        if (k >= n) return 0x7fffffff;
        const int e = key(k);
        return (e >> 18) == mykey ? ((e >> 2) & 0xffff) : 0x7fffffff;
    };
    int scur[T], snx[T];
#pragma unroll
    for (int s = 0; s < T; s++) {
        scur[s] = nsl ? first_at(skey, nsl, lo[s]) : 0;
        snx[s] = next_x(skey, nsl, scur[s]);
    }
    // Receivers record from the owned copy. Stage s publishes level n0 + s
    // of plane i - R(s+1) to LDS in tick i, so wave 0 records levels
    // n0+1 .. n0+T-1 from there. The segment's entries are sorted by x; for
    // each such level wave 0 holds two batches of 64 in registers (the next
    // batch is read when the current one is used up, 64 entries ahead of
    // its use). Level n0+T is read back from this segment's own stores of
    // out_u when the segment ends.
    constexpr int TG = T > 1 ? T - 1 : 1;
    const bool wave0 = tid < 64;
    int gbase[TG];    // list index of batch A's first entry (uniform)
    int goff[TG];     // entries of batch A already recorded (uniform)
    int2 gA[TG], gB[TG];  // entries gbase + lane and gbase + 64 + lane
    auto gload = [&](int at) {
        const int k = at + tid;
        return k < nrl ? grec[k] : make_int2(0x7fffffff, 0);
    };
#pragma unroll
    for (int g = 0; g < TG; g++) {
        gbase[g] = 0;
        goff[g] = 0;
        if (T > 1 && wave0) {
            gA[g] = gload(0);
            gB[g] = gload(64);
        }
    }

    f4v q[T][U];
#pragma unroll
    for (int s = 0; s < T; s++)
#pragma unroll
        for (int k = 0; k < U; k++) q[s][k] = f4v{0.f, 0.f, 0.f, 0.f};

    const int i0 = max(0, xc0 - R * T);
    const int ilast = xc1 - 1 + R * T;

    // Descriptor of plane x of a field (zero records outside [0, nx): every
    // lane then reads 0).
    auto plane = [&](const float *f, int x) {
        const bool in = x >= 0 && x < p.nx;
        return make_rsrc(f + (in ? (long long)x * p.sx : 0), in ? plane_bytes : 0u);
    };
    // Inputs of tick i: the newest plane i of u^n, and v^n and c at the
    // stage-0 centre plane (later stages take c and v from the LDS rings).
    // v and c are read once per point in a pass except where tiles overlap
    // (T > 1), whose neighbours then find them in L2; with T == 1 they
    // stream past L2.
    constexpr int VC = T > 1 ? kTemporal : kStreaming;
    auto fetch_far = [&](int i, FarIn &f) {
        const int c0 = i - R;
        f.u = bload(plane(p.u, i), off_c);
        f.v = bload<VC>(plane(p.v, c0), off_c);
        f.c = bload<VC>(plane(p.c, (c0 >= lo[0] && c0 < hi[0]) ? c0 : -1), off_c);
    };
    auto fetch_ring = [&](int i, RingIn &f) {
        const rsrc_t ru = plane(p.u, i - R);
        f.rg = bload(ru, off_rg);
        f.yr = bload(ru, off_yr);
    };
    FarIn pf[PD];
    RingIn rgn;
    static_for<0, PD>([&](auto KC) {
        constexpr int k = decltype(KC)::value;
        fetch_far(i0 + k, pf[k]);
    });
    fetch_ring(i0, rgn);
    lds_barrier();

    int i = i0;
    int tick = 0;
    int cslot = 0;  // tick mod NSC
    int vslot = 0;  // tick mod NSV
    while (i <= ilast) {
        static_for<0, U>([&](auto PC) {
            constexpr int P = PC.value;
            constexpr int SLOT = P % PD;
            constexpr int CTR = (P + R) % U;
            constexpr int NEW = (P + 2 * R) % U;
            if (i > ilast) return;
            const FarIn &in = pf[SLOT];
            q[0][NEW] = in.u;
            const int buf = tick & 1;
#pragma unroll
            for (int s = 0; s < T; s++) sh[buf][s][row + R][zl] = q[s][CTR];
            const f4v rg_now = rgn.rg;
            if (has_yr) sh[buf][0][yr_lds][zl] = rgn.yr;
            lds_barrier();
            fetch_ring(i + 1, rgn);

            static_for<0, T>([&](auto SC) {
                constexpr int s = SC.value;
                const int cs = i - R * (s + 1);
                if constexpr (s > 0) {
                    // Level n0+s at plane cs, from this tick's LDS plane.
                    constexpr int g = s - 1;
                    if (wave0) {
                        // Past the list end the entries hold x = 2^20 - 1.
                        while ((__builtin_amdgcn_readlane(gA[g].x, goff[g]) >> 11) == cs) {
                            const int e = gA[g].x;
                            const bool hit = tid >= goff[g] && (e >> 11) == cs;
                            if (hit) {
                                const float *cell =
                                    (const float *)&sh[buf][s][((e >> 6) & 31) + R][(e >> 2) & 15];
                                p.rec_dcmp[(long long)(p.n0 + s) * p.nrid + gA[g].y] = cell[e & 3];
                            }
                            goff[g] += __builtin_popcountll(__builtin_amdgcn_ballot_w64(hit));
                            if (goff[g] == 64) {
                                gA[g] = gB[g];
                                gbase[g] += 64;
                                goff[g] = 0;
                                gB[g] = gload(gbase[g] + 64);
                            }
                        }
                    }
                }
                f4v v = f4v{0.f, 0.f, 0.f, 0.f};   // v^{n+s+1}
                f4v un = f4v{0.f, 0.f, 0.f, 0.f};  // u^{n+s+1}
                if (cs >= lo[s] && cs < hi[s]) {
                    const f4v ctr = q[s][CTR];
                    f4v vold, cf;
                    if constexpr (s == 0) {
                        vold = in.v;
                        cf = in.c;
                    } else {
                        const int vs = vslot + 1 == NSV ? 0 : vslot + 1;  // tick - R
                        vold = s_v[s - 1][vs][tid];
                        const int sl = cslot - R * s;                      // tick - R s
                        cf = s_c[sl < 0 ? sl + NSC : sl][tid];
                    }
                    // Stage 0 takes the tile's outer z values from the ring;
                    // later stages do not need them (their edge lanes lie
                    // in the halo, which they need not compute correctly).
                    // zw: the float4s of lanes l-2 (ZB == 8), l-1, l, l+1,
                    // l+2 (ZB == 8), i.e. z - ZB .. z + 4 + ZB.
                    float zw[4 + 2 * ZB];
                    f4v zl4, zr4;
                    if constexpr (s == 0 && ZB == 4) {
                        zl4 = row_shift<kDppRowShr1>(rg_now, ctr);
                        zr4 = row_shift<kDppRowShl1>(rg_now, ctr);
                    } else if constexpr (s == 0) {
                        // Lane 0's left float4 is lane 1's ring value, lane
                        // 15's right float4 lane 14's.
                        zl4 = row_shift<kDppRowShr1>(row_shift0<kDppRowShl1>(rg_now), ctr);
                        zr4 = row_shift<kDppRowShl1>(row_shift0<kDppRowShr1>(rg_now), ctr);
                    } else {
                        zl4 = row_shift0<kDppRowShr1>(ctr);
                        zr4 = row_shift0<kDppRowShl1>(ctr);
                    }
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        zw[ZB - 4 + k] = zl4[k];
                        zw[ZB + k] = ctr[k];
                        zw[ZB + 4 + k] = zr4[k];
                    }
                    if constexpr (ZB == 8) {
                        f4v zl8, zr8;
                        if constexpr (s == 0) {
                            zl8 = row_shift<kDppRowShr2>(rg_now, ctr);
                            zr8 = row_shift<kDppRowShl2>(rg_now, ctr);
                        } else {
                            zl8 = row_shift0<kDppRowShr2>(ctr);
                            zr8 = row_shift0<kDppRowShl2>(ctr);
                        }
#pragma unroll
                        for (int k = 0; k < 4; k++) {
                            zw[k] = zl8[k];
                            zw[16 + k] = zr8[k];
                        }
                    }
                    // Laplacian of the 4 points, one offset at a time; per
                    // point the operations are those of the per-point
                    // definition above, in the same order.
                    float lap[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                    // y rows of each offset: read together up front (their LDS
                    // latency overlaps) up to radius 4; at radius 6, where
                    // registers are short, where they are used.
                    constexpr bool YPRE = R <= 4;
                    f4v yrow[YPRE ? 2 * R : 1];
                    if constexpr (YPRE) {
#pragma unroll
                        for (int j = 1; j <= R; j++) {
                            yrow[2 * j - 2] = sh[buf][s][row + R - j][zl];
                            yrow[2 * j - 1] = sh[buf][s][row + R + j][zl];
                        }
                    }
                    auto yrows = [&](int j, f4v &ym_, f4v &yp_) {
                        if constexpr (YPRE) {
                            ym_ = yrow[2 * j - 2];
                            yp_ = yrow[2 * j - 1];
                        } else {
                            ym_ = sh[buf][s][row + R - j][zl];
                            yp_ = sh[buf][s][row + R + j][zl];
                        }
                    };
                    if constexpr (ISO) {
                        float t6[4];
#pragma unroll
                        for (int k = 0; k < 4; k++) t6[k] = 6.0f * ctr[k];
#pragma unroll
                        for (int j = 1; j <= R; j++) {
                            const f4v xmj = q[s][(P + R - j) % U], xpj = q[s][(P + R + j) % U];
                            f4v ymj, ypj;
                            yrows(j, ymj, ypj);
#pragma unroll
                            for (int k = 0; k < 4; k++)
                                lap[k] = __builtin_fmaf(
                                    p.wx[j - 1],
                                    (((xmj[k] + xpj[k]) + (zw[ZB + k - j] + zw[ZB + k + j])) +
                                     (ymj[k] + ypj[k])) - t6[k],
                                    lap[k]);
                        }
                    } else {
                        float t2[4];
#pragma unroll
                        for (int k = 0; k < 4; k++) t2[k] = 2.0f * ctr[k];
#pragma unroll
                        for (int j = 1; j <= R; j++) {
                            const f4v xmj = q[s][(P + R - j) % U], xpj = q[s][(P + R + j) % U];
#pragma unroll
                            for (int k = 0; k < 4; k++)
                                lap[k] = __builtin_fmaf(p.wx[j - 1], (xmj[k] + xpj[k]) - t2[k],
                                                        lap[k]);
                        }
#pragma unroll
                        for (int j = 1; j <= R; j++)
#pragma unroll
                            for (int k = 0; k < 4; k++)
                                lap[k] = __builtin_fmaf(
                                    p.wz[j - 1], (zw[ZB + k - j] + zw[ZB + k + j]) - t2[k], lap[k]);
#pragma unroll
                        for (int j = 1; j <= R; j++) {
                            f4v ymj, ypj;
                            yrows(j, ymj, ypj);
#pragma unroll
                            for (int k = 0; k < 4; k++)
                                lap[k] = __builtin_fmaf(p.wy[j - 1], (ymj[k] + ypj[k]) - t2[k],
                                                        lap[k]);
                        }
                    }
                    const float dxs = uniform(s_dx[cs - xlo]);
                    auto compute = [&](auto DC) {
                        constexpr bool DAMP = decltype(DC)::value;
#pragma unroll
                        for (int k = 0; k < 4; k++)
                            v[k] = vel_update<DAMP>(p, lap[k], vold[k], cf[k], dxs + dyz[k]);
                    };
                    if (dxs != 0.0f || wave_dyz) compute(std::true_type{});
                    else compute(std::false_type{});
                    // Fused injection at every computed copy (per-tile list).
                    if (__builtin_amdgcn_ballot_w64(snx[s] == cs) && snx[s] == cs) {
                        int kk = scur[s];
                        for (; kk < nsl && (skey(kk) >> 18) == mykey &&
                               ((skey(kk) >> 2) & 0xffff) == cs;
                             kk++) {
                            const int k = skey(kk) & 3;
                            float add;
                            if constexpr (GL)
                                add = p.dcmp[(long long)(p.n0 + s) * p.npts + gsrc[kk].y];
                            else
                                add = s_val[kk][s];
                            v[0] = k == 0 ? v[0] + add : v[0];
                            v[1] = k == 1 ? v[1] + add : v[1];
                            v[2] = k == 2 ? v[2] + add : v[2];
                            v[3] = k == 3 ? v[3] + add : v[3];
                        }
                        scur[s] = kk;
                        snx[s] = next_x(skey, nsl, kk);
                    }
#pragma unroll
                    for (int k = 0; k < 4; k++) un[k] = ctr[k] + v[k];
                }
                if constexpr (s + 1 < T) {
                    q[s + 1 < T ? s + 1 : 0][NEW] = un;
                    s_v[s + 1 < T ? s : 0][vslot][tid] = v;
                } else {
                    const bool st_in = cs >= xc0 && cs < xc1;
                    bstore(plane(p.out_u, st_in ? cs : -1), off_own, un);
                    bstore(plane(p.out_v, st_in ? cs : -1), off_own, v);
                    if constexpr (T > 1)
                        if (p.out_mid) bstore(plane(p.out_mid, st_in ? cs : -1), off_own, q[s][CTR]);
                }
            });
            // Stage 0's c plane for the later stages, after this tick's reads.
            if constexpr (NSC > 0) {
                s_c[cslot][tid] = in.c;
                cslot = cslot + 1 == NSC ? 0 : cslot + 1;
            }
            if constexpr (NSV > 0) vslot = vslot + 1 == NSV ? 0 : vslot + 1;
            // Loads for tick i + PD.
            fetch_far(i + PD, pf[SLOT]);
            i++;
            tick++;
        });
    }
    if (nrl > 0) {
        // Level n0+T: this segment stored every owned point of its planes;
        // the barrier makes those stores visible to the whole workgroup.
        __syncthreads();
        for (int k = tid; k < nrl; k += NTH) {
            const int2 e = grec[k];
            const int y = y0 + ((e.x >> 6) & 31), z = z0 + 4 * ((e.x >> 2) & 15) + (e.x & 3);
            const long long at = (long long)(e.x >> 11) * p.sx + (long long)y * p.nzp + z;
            p.rec_dcmp[(long long)(p.n0 + T) * p.nrid + e.y] = p.out_u[at];
        }
    }
    }  // segments
}

template <int R, int T, int LZ, int BYE, int PD, bool GL>
__global__ void __launch_bounds__(LZ *BYE) acoustic_wavefront(const AcParams p)
{
    __shared__ WfLds<R, T, LZ, BYE, GL> lds;
    if (p.iso) wavefront_body<R, T, LZ, BYE, PD, GL, true>(p, blockIdx.x, lds);
    else wavefront_body<R, T, LZ, BYE, PD, GL, false>(p, blockIdx.x, lds);
}

// Several jobs (different grids, sparse sets and time levels) in one launch:
// job j owns workgroups [wg_off[j], wg_off[j] + jobs[j].nwg); every wg_off[j]
// is a multiple of 8, so a job's local index keeps the hardware's XCD
// round-robin, and workgroups of the padding exit at once. Each job
// evaluates exactly the arithmetic of a launch of its own.
template <int R, int T, int LZ, int BYE, int PD>
__global__ void __launch_bounds__(LZ *BYE)
    acoustic_wavefront_batch(const AcParams *__restrict__ jobs, const int *__restrict__ wg_off,
                             int njobs)
{
    const int bx = blockIdx.x;
    int j = 0;
    while (j + 1 < njobs && wg_off[j + 1] <= bx) j++;
    const AcParams &p = jobs[j];
    const int b = bx - wg_off[j];
    if (b >= p.nwg) return;
    __shared__ WfLds<R, T, LZ, BYE, false> lds;
    if (p.iso) wavefront_body<R, T, LZ, BYE, PD, false, true>(p, b, lds);
    else wavefront_body<R, T, LZ, BYE, PD, false, false>(p, b, lds);
}

// Prefetch depth (ticks of loads in flight): it must divide the window 2R+1,
// and the deeper pipelines keep fewer ticks in flight so their register
// windows still fit.
template <int R, int T>
constexpr int prefetch_depth()
{
    if constexpr (R == 4) return 3;
    else if constexpr (R == 2) return T <= 2 ? 5 : 1;
    else return 1;  // R = 6: the window of 13 planes is prime
}
static_assert((2 * 4 + 1) % 3 == 0 && (2 * 2 + 1) % 5 == 0, "depth must divide the window");

// Instantiated shapes: 16-lane tiles of 16 or 32 rows whose LDS fits one
// workgroup, at least without the staged lists (GL).
template <int R, int T, int LZ, int BYE, bool GL = true>
constexpr bool wavefront_fits()
{
    return BYE - 2 * R * (T - 1) > 0 && wavefront_lds<R, T, LZ, BYE, GL>() <= kLdsBytes &&
           LZ * BYE <= kMaxThreads;
}
// Whether the shape also fits with the injection list staged in LDS (the
// common variant and the batched entry); otherwise only GL runs it.
template <int R, int T, int LZ, int BYE>
constexpr bool lists_in_lds()
{
    return wavefront_fits<R, T, LZ, BYE, false>();
}

// Calls f.template operator()<T, LZ, BYE>() for an instantiated shape.
template <int R, class F>
hipError_t dispatch_shape(int T, int LZ, int BYE, F &&f)
{
    auto rt = [&]<int TT>() -> hipError_t {
        if (LZ == 16 && BYE == 16) {
            if constexpr (wavefront_fits<R, TT, 16, 16>()) return f.template operator()<TT, 16, 16>();
        } else if (LZ == 16 && BYE == 32) {
            if constexpr (wavefront_fits<R, TT, 16, 32>()) return f.template operator()<TT, 16, 32>();
        }
        return hipErrorInvalidValue;
    };
    switch (T) {
    case 1: return rt.template operator()<1>();
    case 2: return rt.template operator()<2>();
    case 3: return rt.template operator()<3>();
    case 4: return rt.template operator()<4>();
    }
    return hipErrorInvalidValue;
}

template <int R>
hipError_t launch_r(const AcParams &p, int T, int LZ, int BYE, bool gl, hipStream_t st)
{
    return dispatch_shape<R>(T, LZ, BYE, [&]<int TT, int L, int B>() {
        if constexpr (lists_in_lds<R, TT, L, B>()) {
            if (!gl) {
                hipLaunchKernelGGL(
                    (acoustic_wavefront<R, TT, L, B, prefetch_depth<R, TT>(), false>),
                    dim3(p.nwg), dim3(L * B), 0, st, p);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL((acoustic_wavefront<R, TT, L, B, prefetch_depth<R, TT>(), true>),
                           dim3(p.nwg), dim3(L * B), 0, st, p);
        return hipGetLastError();
    });
}

template <int R>
hipError_t launch_batch_r(const AcParams *jobs, const int *wg_off, int njobs, int total_wg, int T,
                          int LZ, int BYE, hipStream_t st)
{
    return dispatch_shape<R>(T, LZ, BYE, [&]<int TT, int L, int B>() {
        if constexpr (lists_in_lds<R, TT, L, B>()) {
            hipLaunchKernelGGL((acoustic_wavefront_batch<R, TT, L, B, prefetch_depth<R, TT>()>),
                               dim3(total_wg), dim3(L * B), 0, st, jobs, wg_off, njobs);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    });
}

}  // namespace wf
}  // namespace tbw
