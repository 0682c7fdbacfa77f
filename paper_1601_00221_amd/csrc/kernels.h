// Launch interface between the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "gp_internal.h"

namespace gpx {

// Arguments of one evaluation launch over one case matrix.
struct EvalArgs {
    const uint32_t* code;       // lowered program words
    const DevProg* progs;       // per-program records
    const uint32_t* order;      // program indices, grouped
    const uint32_t* group_off;  // group g is order[group_off[g] .. group_off[g+1])
    const float* X;             // feature-major cases
    const float* y;             // targets (null for per-case output)
    double* partials;           // one partial sum per (program, tile)
    float* cases_out;           // per-case output rows (GP_OUT_CASES)
    int64_t N;                  // cases
    int32_t n_load;             // features loaded into the tile (programs read f < n_load)
    int32_t n_feat_prog;        // feature count that register initialisation wraps around
    int32_t tiles;              // ceil(N / (64 * T))
    int32_t n_units;            // tiles * groups
    int32_t kind;               // gp_fitness_kind
    int32_t pad;
};

struct ReduceArgs {
    const double* partials;
    uint64_t part_base;
    int64_t stride;             // distance between consecutive blocks of one program
    int64_t n_prog;
    int64_t N;
    void* out;
    int32_t blocks;             // ceil(N / 256)
    int32_t kind;
};

// Batched evaluation (several jobs over several datasets in one launch).
struct DatasetDesc {
    const float* X;
    const float* y;
    int64_t N;
};

struct JobDesc {
    int32_t ds;                 // dataset index
    int32_t kind;
    int32_t n_load;             // features the job's programs read
    int32_t n_feat_prog;        // feature count register initialisation wraps around
};

struct UnitDesc {
    uint32_t job;
    uint32_t tile;
    uint32_t q0, q1;            // programs order[q0 .. q1)
};

struct BatchArgs {
    const uint32_t* code;
    const DevProg* progs;
    const uint32_t* order;
    const UnitDesc* units;
    const JobDesc* jobs;
    const DatasetDesc* datasets;
    double* partials;
    uint32_t* counter;          // next unit (persistent form)
    int32_t n_units;
    int32_t persistent;
};

struct VariantDesc {
    int t;   // case slots per lane
    int d;   // stack levels held in registers
    int fv;  // feature slots per case held in registers
};

int n_variants();
const VariantDesc& variant(int i);
// Smallest-footprint compiled variant able to hold n_feat_load features and
// `depth` stack levels, or -1.
int pick_variant(int n_feat_load, int depth);

hipError_t launch_eval(int variant, const EvalArgs& a, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& r, hipStream_t s);
hipError_t launch_batch(int variant, const BatchArgs& a, uint32_t grid_blocks, hipStream_t s);
hipError_t launch_reduce_jobs(const ReduceArgs* jobs_dev, int32_t n_jobs, int64_t max_prog, hipStream_t s);
int batch_blocks_per_cu(int variant);

}  // namespace gpx
