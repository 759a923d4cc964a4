// Wave-front kernel instantiations for stencil radius 4 (space order 8).
#include "acoustic_kernel.h"

namespace tbw {

hipError_t launch_acoustic_r4(const AcParams &p, int T, int LZ, int BYE, bool gl,
                              hipStream_t st)
{
    return wf::launch_r<4>(p, T, LZ, BYE, gl, st);
}

hipError_t launch_acoustic_batch_r4(const AcParams *jobs, const int *wg_off, int njobs,
                                    int total_wg, int T, int LZ, int BYE, hipStream_t st)
{
    return wf::launch_batch_r<4>(jobs, wg_off, njobs, total_wg, T, LZ, BYE, st);
}

bool acoustic_shape_ok_r4(int T, int LZ, int BYE)
{
    return wf::dispatch_shape<4>(T, LZ, BYE, []<int TT, int L, int B>() { return hipSuccess; }) ==
           hipSuccess;
}

bool acoustic_lists_in_lds_r4(int T, int LZ, int BYE)
{
    return wf::dispatch_shape<4>(T, LZ, BYE, []<int TT, int L, int B>() {
               return wf::lists_in_lds<4, TT, L, B>() ? hipSuccess : hipErrorInvalidValue;
           }) == hipSuccess;
}

}  // namespace tbw
