// Host runtime internals shared by the evaluation, batching and serving code.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include <map>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/gp.h"
#include "gp_internal.h"

namespace gpx {

gp_status fail(gp_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
const char* last_error();

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    gp_status reserve(size_t n);
    void release();
};

// Pinned host staging for host-to-device copies.  begin() waits until the
// copies of the previous use have left the buffer.
struct Staging {
    void* host = nullptr;
    size_t cap = 0;
    size_t used = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
    gp_status begin(size_t n);
    gp_status put(const void* src, size_t n, void* dst, hipStream_t s);
    gp_status end(hipStream_t s);
};

// Lowered programs on the host.
struct ProgData {
    int form = 0;
    int opset = OPSET_REAL;  // function set of trees (OPSET_BOOL: Boolean, 32 cases per slot)
    int32_t n_prog = 0;
    int32_t n_feat = 0;     // declared feature count (register initialisation wraps around it)
    int32_t n_reg = 0;
    int32_t n_load = 1;     // features the programs actually read (max index + 1)
    int32_t max_depth = 0;
    int64_t n_instr = 0;
    int64_t n_gpop = 0;     // GP operations per case: tree nodes or linear instructions
    int64_t n_transc = 0;   // sin/cos/exp/log instructions (evaluated in binary64 by compiled code)
    std::vector<uint32_t> code;
    std::vector<DevProg> progs;
    std::vector<uint32_t> cost;
};

// Device copies of programs translated for one core variant, plus cached
// group layouts.
struct DevProgs {
    bool uploaded = false;
    DevBuf code;
    DevBuf progs;
    std::map<int32_t, std::pair<int64_t, std::unique_ptr<DevBuf>>> groups_by_G;
    void release() {
        uploaded = false;
        code.release();
        progs.release();
        for (auto& kv : groups_by_G) kv.second.second->release();
        groups_by_G.clear();
    }
};

// Per-stream scratch: partial sums, staging and the one-shot program buffers.
struct Workspace {
    std::mutex mu;
    DevBuf partials;
    Staging staging;
    std::map<int, DevProgs> oneshot;   // by core variant
    DevBuf bg_code, bg_meta;           // programs of the one-dimensional-stack comparator
};

struct EvalOptions {
    int variant = -1;            // core variant index, -1 = chosen from the programs
    int32_t group_instr = 0;     // core instructions per program group, 0 = automatic
    int32_t tiles_per_wave = 0;  // tiles each wave walks per group, 0 = automatic
    int32_t target_blocks = 0;   // blocks the launch should have at least, 0 = automatic
};

Workspace& workspace(hipStream_t s);
int32_t code_prefetch();

// Kernel timing brackets (active only while gp_timing_enable(1)).
hipError_t timed_launch_begin(hipStream_t s, int* slot);
hipError_t timed_launch_end(hipStream_t s, int slot);

gp_status build_tree(const int32_t* tok, const float* cst, const int64_t* off, int32_t P, int32_t n_feat,
                     ProgData& pd, int opset = OPSET_REAL);
gp_status build_linear(const uint32_t* code, const int64_t* off, const float* cst, const int64_t* cst_off,
                       int32_t P, int32_t n_reg, int32_t n_feat, ProgData& pd);
// Evaluate lowered programs on one case matrix.  dps caches the programs
// translated per core variant; fresh forces a new translation and upload.
// Boolean programs (pd.opset == OPSET_BOOL) take X and y as 32-bit words, N
// words per row, and n_bits > 0 cases; every other call passes n_bits = 0.
gp_status eval_core(const ProgData& pd, std::map<int, DevProgs>& dps, bool fresh, const float* X, int32_t n_feat,
                    int64_t N, const float* y, int32_t kind, void* out, hipStream_t s, Workspace& w,
                    const EvalOptions* opt, int64_t n_bits = 0);

}  // namespace gpx
