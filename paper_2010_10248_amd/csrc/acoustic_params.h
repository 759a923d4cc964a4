// Kernel argument block of the acoustic wave-front kernels.
#pragma once

#include "tb_internal.h"

namespace tbw {

struct AcParams {
    const float *__restrict__ u;   // u^n      [nx][ny][nzp]
    const float *__restrict__ v;   // v^n = u^n - u^{n-1}
    const float *__restrict__ c;   // dt^2 vp^2
    const float *zero;             // 16 zeroed bytes (target of masked-off loads)
    float *out_u;                  // u^{n+T}
    float *out_v;                  // v^{n+T}
    float *out_mid;                // u^{n+T-1} (T >= 2), or NULL
    const float *__restrict__ dx;  // damping per axis
    const float *__restrict__ dy;
    const float *__restrict__ dz;
    float hdt;  // dt / 2
    float wx[6], wy[6], wz[6];  // off-centre weights per axis (h^-2 scaled)
    int iso;                    // wx == wy == wz (equal spacing on all axes)
    int nx, ny, nz, nzp;
    long long sx;  // plane stride ny * nzp
    int tiles_z, nwg;
    const SegDesc *__restrict__ segs;
    const int *__restrict__ seg_off;
    const int2 *__restrict__ src;
    const float *__restrict__ dcmp;
    int npts, n0;
    const int2 *__restrict__ rec;
    float *rec_dcmp;
    int nrid;
};

// Launchers of the wave-front kernel for one stencil radius (one translation
// unit per radius so the instantiations compile in parallel).
// gl: the variant that walks the sparse lists in global memory (segments with
// more entries than the LDS lists hold).
hipError_t launch_acoustic_r2(const AcParams &p, int T, int LZ, int BYE, bool gl,
                              hipStream_t st);
hipError_t launch_acoustic_r4(const AcParams &p, int T, int LZ, int BYE, bool gl,
                              hipStream_t st);
hipError_t launch_acoustic_r6(const AcParams &p, int T, int LZ, int BYE, bool gl,
                              hipStream_t st);
// Batched launch: jobs[njobs] in device memory, wg_off[njobs] (device) the
// first workgroup of each job (multiples of 8), total_wg the grid size.
hipError_t launch_acoustic_batch_r2(const AcParams *jobs, const int *wg_off, int njobs,
                                    int total_wg, int T, int LZ, int BYE, hipStream_t st);
hipError_t launch_acoustic_batch_r4(const AcParams *jobs, const int *wg_off, int njobs,
                                    int total_wg, int T, int LZ, int BYE, hipStream_t st);
hipError_t launch_acoustic_batch_r6(const AcParams *jobs, const int *wg_off, int njobs,
                                    int total_wg, int T, int LZ, int BYE, hipStream_t st);

bool acoustic_shape_ok_r2(int T, int LZ, int BYE);
bool acoustic_shape_ok_r4(int T, int LZ, int BYE);
bool acoustic_shape_ok_r6(int T, int LZ, int BYE);
// Whether a shape also runs with its injection list staged in LDS (and so
// has a batched entry); a shape without is run by the global-list variant
// alone.
bool acoustic_lists_in_lds(int R, int T, int LZ, int BYE);
bool acoustic_lists_in_lds_r2(int T, int LZ, int BYE);
bool acoustic_lists_in_lds_r4(int T, int LZ, int BYE);
bool acoustic_lists_in_lds_r6(int T, int LZ, int BYE);

// Kernel parameters of one pass of one job.
AcParams make_params(const tb_model *m, const TileLists &tl, const AcLaunch &a);
// One batched launch over several jobs of the same radius and kernel shape
// (device tables; see launch_acoustic_batch_r*).
tb_status launch_acoustic_batch(int r, const AcParams *d_jobs, const int *d_wgoff, int njobs,
                                int total_wg, int T, int LZ, int BYE, hipStream_t st,
                                bool allow_timing);

// Optional per-launch event timing of the propagation kernels.
bool timing_enabled();
void timing_begin(hipStream_t st, hipEvent_t *a, hipEvent_t *b);
void timing_end(hipStream_t st, hipEvent_t a, hipEvent_t b);

}  // namespace tbw
