// Program-set evaluation that allocates nothing (gp_progset_eval_noalloc).
//
// The evaluation kernels need one scratch buffer beyond the caller's inputs
// and outputs: the binary64 partial sums, one per (program, 256-case block),
// that the fixed-order reduction turns into fitness values.  gp_progset_eval
// keeps them in a per-stream buffer that grows with hipMalloc; this entry
// point keeps them in `scratch`, a file-scope device array of fixed size that
// every GPU the library runs on holds until the process ends.  Programs and
// their group layout were uploaded when the set was created, so a call
// launches the evaluation and reduction kernels and nothing else: no
// hipMalloc, hipFree, host-to-device copy or allocating library routine.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/gp.h"
#include "runtime.h"

// Host code may not use this name as a device address: its address on each
// device comes from hipGetSymbolAddress (below).  No element needs to start
// at zero: the evaluation kernel writes every partial sum the reduction
// reads.
static __device__ __align__(256) double scratch[GP_NOALLOC_MAX_PARTIALS];

namespace {

constexpr size_t kScratchDoubles = GP_NOALLOC_MAX_PARTIALS;

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices];   // scratch's address on each device, once looked up

// scratch's address on the current device: looked up on the first call on
// that device, with the device current.
gp_status scratch_ptr(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return gpx::fail(GP_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return gpx::fail(GP_E_DEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return gpx::fail(GP_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_ptr[dev] = (double*)p;
    }
    *out = g_ptr[dev];
    return GP_OK;
}

}  // namespace

extern "C" gp_status gp_progset_eval_noalloc(gp_progset* ps, const float* X, int32_t n_feat, int64_t n_cases,
                                             const float* y, int32_t kind, void* out, void* stream) {
    gpx::clear_error();
    double* p = nullptr;
    gp_status st = scratch_ptr(&p);
    if (st != GP_OK) return st;
    return gpx::progset_eval_no_alloc(ps, X, n_feat, n_cases, y, kind, out, (hipStream_t)stream, p,
                                      kScratchDoubles * sizeof(double));
}
