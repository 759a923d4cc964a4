// Wave-front kernel instantiations for stencil radius 2 (space order 4).
#include "acoustic_kernel.h"

namespace tbw {

hipError_t launch_acoustic_r2(const AcParams &p, int T, int LZ, int BYE, hipStream_t st)
{
    return wf::launch_r<2>(p, T, LZ, BYE, st);
}

}  // namespace tbw
