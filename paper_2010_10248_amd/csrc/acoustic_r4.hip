// Wave-front kernel instantiations for stencil radius 4 (space order 8).
#include "acoustic_kernel.h"

namespace tbw {

hipError_t launch_acoustic_r4(const AcParams &p, int T, int LZ, int BYE, hipStream_t st)
{
    return wf::launch_r<4>(p, T, LZ, BYE, st);
}

}  // namespace tbw
