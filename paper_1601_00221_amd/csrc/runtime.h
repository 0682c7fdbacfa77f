// Host runtime internals shared by the evaluation, batching and serving code.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include <functional>
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

// Grow-only device buffer.  It owns its allocation: moving hands it over,
// destruction frees it.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), cap(o.cap) { o.p = nullptr; o.cap = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            cap = o.cap;
            o.p = nullptr;
            o.cap = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    gp_status reserve(size_t n);
    void release();
};

// Pinned host staging for host-to-device copies, in two halves used in
// turn: begin() takes the other half and waits only until the copies of
// that half's previous use (two uses ago) have left it, so a call does not
// wait for its own copies or for the kernels queued before them.
struct Staging {
    struct Half {
        void* host = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
        bool pending = false;
    };
    Half half[2];
    int cur = 0;
    size_t used = 0;
    gp_status begin(size_t n);
    gp_status put(const void* src, size_t n, void* dst, hipStream_t s);
    gp_status end(hipStream_t s);
    void release();
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

// Device copies of programs translated for one core variant, plus their
// group layouts (program order and group offsets) by group count.  `ready`
// is recorded on the stream of the last upload into these buffers; a launch
// on any stream waits for it.
struct DevProgs {
    bool uploaded = false;
    DevBuf code;
    DevBuf progs;
    std::map<int32_t, std::pair<int64_t, DevBuf>> groups_by_G;
    DevBuf groups_once;        // one-shot calls: the group layout of the current programs
    hipEvent_t ready = nullptr;
    DevProgs() = default;
    DevProgs(const DevProgs&) = delete;
    DevProgs& operator=(const DevProgs&) = delete;
    ~DevProgs() { release(); }
    void release() {
        uploaded = false;
        code.release();
        progs.release();
        groups_by_G.clear();
        groups_once.release();
        if (ready) (void)hipEventDestroy(ready);
        ready = nullptr;
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
    // Evaluation without any allocation or upload: the programs and the group
    // layout for `groups` groups are already on the device (a program set),
    // and the partial sums go to `partials` (at most `partials_bytes`).
    bool no_alloc = false;
    int32_t groups = 0;
    double* partials = nullptr;
    size_t partials_bytes = 0;
};

Workspace& workspace(hipStream_t s);
// Run fn over [0, n) split into chunks on a pool of host threads (the caller
// takes part); small ranges run on the calling thread.  Calls take turns.
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& fn);
int32_t code_prefetch();

// Kernel timing brackets (active only while gp_timing_enable(1)).
hipError_t timed_launch_begin(hipStream_t s, int* slot);
hipError_t timed_launch_end(hipStream_t s, int slot);

gp_status build_tree(const int32_t* tok, const float* cst, const int64_t* off, int32_t P, int32_t n_feat,
                     ProgData& pd, int opset = OPSET_REAL);
gp_status build_linear(const uint32_t* code, const int64_t* off, const float* cst, const int64_t* cst_off,
                       int32_t P, int32_t n_reg, int32_t n_feat, ProgData& pd);
// The kernel variant an evaluation of these programs uses by default.
int default_variant(const ProgData& pd);
// Evaluate lowered programs on one case matrix.  dps caches the programs
// translated per core variant; fresh forces a new translation and upload.
// Boolean programs (pd.opset == OPSET_BOOL) take X and y as 32-bit words, N
// words per row, and n_bits > 0 cases; every other call passes n_bits = 0.
gp_status eval_core(const ProgData& pd, std::map<int, DevProgs>& dps, bool fresh, const float* X, int32_t n_feat,
                    int64_t N, const float* y, int32_t kind, void* out, hipStream_t s, Workspace* w,
                    const EvalOptions* opt, int64_t n_bits = 0);
}  // namespace gpx

struct gp_progset;

namespace gpx {
// Evaluate a program set as gp_progset_eval does, with nothing allocated or
// uploaded: the partial sums go to `partials` (device memory of
// `partials_bytes`); the set's programs and group layout were uploaded when
// it was created.
gp_status progset_eval_no_alloc(gp_progset* ps, const float* X, int32_t n_feat, int64_t n_cases, const float* y,
                                int32_t kind, void* out, hipStream_t s, double* partials, size_t partials_bytes);
// Program groups of a launch over plentiful case tiles (the layout a program
// set uploads when it is created).
int32_t base_groups(const ProgData& pd);

}  // namespace gpx
