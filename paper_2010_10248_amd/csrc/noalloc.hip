// Forward run that allocates nothing: its workspace is a fixed device array
// of the library instead of caller memory, for callers that cannot allocate
// (code under stream capture, serving loops that forbid allocation).
#include <mutex>

#include <hip/hip_runtime.h>

#include "plan.h"

namespace {

constexpr size_t kScratchBytes = 64ull << 20;  // 64 MiB on each device used
constexpr int kMaxDevices = 64;

// The workspace: one copy per device, alive until the process ends. Host
// code never uses this name as an address; it takes the per-device address
// from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array, looked up once per
// device with that device current.
tb_status scratch_ptr(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) {
        tbw::set_error("device %d beyond the %d the library tracks", dev, kMaxDevices);
        return TB_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            tbw::set_error("hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            return TB_EHIP;
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return TB_OK;
}

}  // namespace

extern "C" tb_status tb_forward_noalloc(const tb_model *m, const tb_sparse *s_,
                                        const tb_schedule *sched, float *rec_out,
                                        float *field_out, float *field_prev_out, void *stream)
{
    using namespace tbw;
    tb_sparse *s = const_cast<tb_sparse *>(s_);
    if (!m || !s || s->m != m) {
        set_error("tb_forward_noalloc: invalid argument");
        return TB_EINVAL;
    }
    if (timing_enabled()) {
        set_error("tb_forward_noalloc: per-launch timing (tb_kernel_timing) creates events; "
                  "switch it off");
        return TB_EINVAL;
    }
    int dev = -1;
    TB_HIP(hipGetDevice(&dev));
    if (dev != m->device) {
        set_error("tb_forward_noalloc: the model lives on device %d, device %d is current",
                  m->device, dev);
        return TB_EINVAL;
    }
    SchedChoice sc;
    tb_status st = resolve_schedule(m, sched, &sc);
    if (st) return st;
    const size_t need = forward_ws_bytes(m, s, sc);
    if (need > kScratchBytes) {
        set_error("tb_forward_noalloc: the run needs %zu bytes of workspace, above the fixed "
                  "%zu", need, kScratchBytes);
        return TB_EWORKSPACE;
    }
    void *ws = nullptr;
    if ((st = scratch_ptr(dev, &ws))) return st;
    Plan plan;
    if ((st = plan_forward(m, s, sc, ws, rec_out, field_out, field_prev_out, &plan))) return st;
    if (!plan_lists_cached(m, s, sc, plan)) {
        set_error("tb_forward_noalloc: the tile lists of this schedule are not built yet (the "
                  "first tb_forward with the schedule builds and uploads them)");
        return TB_EINVAL;
    }
    return run_plan(m, s, sc, plan, (hipStream_t)stream);
}
