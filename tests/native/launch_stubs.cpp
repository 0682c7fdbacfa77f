// Host-only stand-ins for the kernel launchers, so the library's host code
// (validation, lowering, translation, scheduling, GP breeding) can be built
// with the address and undefined-behaviour sanitizers, without device code.
// Every launch reports that there is no device.
#include <hip/hip_runtime_api.h>

#include "blockgp.h"
#include "core_kernels.h"
#include "gp.h"

namespace gpx {
hipError_t core_launch(int, const CoreArgs&, uint32_t, hipStream_t) { return hipErrorNoDevice; }
int core_blocks_per_cu(int) { return 1; }
hipError_t core_zero_counter(uint32_t*, hipStream_t) { return hipErrorNoDevice; }
hipError_t core_reduce_jobs(const ReduceArgs*, int32_t, int64_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t core_reduce_one(const ReduceArgs&, hipStream_t) { return hipErrorNoDevice; }
hipError_t blockgp_launch(int, const BgArgs&, int32_t, hipStream_t) { return hipErrorNoDevice; }
}  // namespace gpx

// the device-array evaluation lives with its device code; without it, it reports no device
extern "C" gp_status gp_progset_eval_noalloc(gp_progset*, const float*, int32_t, int64_t, const float*, int32_t,
                                             void*, void*) {
    return GP_E_DEVICE;
}
