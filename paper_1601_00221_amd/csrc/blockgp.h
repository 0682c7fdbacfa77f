// The one-dimensional-stack comparator (gp_eval_tree_1d): kernel arguments
// shared by blockgp.cpp and blockgp_kernels.hip.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace gpx {

// Stack values per thread; equal to GP_1D_MAX_STACK.
enum : int { GP_BG_MAX_STACK = 64 };

struct BgArgs {
    const uint32_t* code;   // two words per instruction, all programs back to back
    const uint32_t* poff;   // first instruction of program p
    const uint32_t* plen;   // instructions of program p
    const float* X;         // feature-major cases
    const float* y;         // targets (null for GP_OUT_CASES)
    void* out;              // fitness per program, or n_prog x N outputs
    int64_t N;
    int32_t kind;
    uint32_t max_len;       // longest program (sizes the LDS copy)
};

hipError_t blockgp_launch(int form, const BgArgs& a, int32_t n_prog, hipStream_t s);

}  // namespace gpx
