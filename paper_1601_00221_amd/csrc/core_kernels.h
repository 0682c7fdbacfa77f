// Launch interface of the core-based evaluation kernel.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "gp_internal.h"

namespace gpx {

enum : uint32_t { CORE_OP_END = 15 };   // exit operation that ends a program

struct DatasetDesc {
    const float* X;
    const float* y;
    int64_t N;
};

struct JobDesc {
    int32_t ds;                 // dataset index
    int32_t kind;
    int32_t n_load;             // features the job's programs read
    int32_t pad;
    uint64_t part_base;         // the job's partial sums start here (see ReduceArgs)
};

struct UnitDesc {
    uint32_t job;
    uint32_t tile;
    uint32_t q0, q1;            // programs order[q0 .. q1)
};

// Partial sums are program-major: block b of program p (its row in the
// job) is partials[part_base + p * blocks + b], so one wave's blocks of one
// program are adjacent.
struct ReduceArgs {
    const double* partials;
    uint64_t part_base;
    int64_t n_prog;
    int64_t N;
    void* out;
    int32_t blocks;             // ceil(N / 256)
    int32_t kind;
};

struct CoreArgs {
    const uint32_t* code;       // core instructions, 16 bytes each
    const DevProg* progs;
    const uint32_t* order;      // program indices grouped by unit
    // table of units (batched launches); null: implicit units over one dataset
    const UnitDesc* units;
    const JobDesc* jobs;
    const DatasetDesc* datasets;
    uint32_t* counter;          // next unit, persistent form
    // implicit units: block unit b = (group quad b div chunks, chunk b mod
    // chunks); a chunk is tiles_per_wave consecutive tiles
    const uint32_t* group_off;
    const float* X;
    const float* y;
    int64_t N;
    int32_t n_load;
    int32_t kind;
    int32_t tiles;
    int32_t n_units;            // table units, or implicit block units
    int32_t persistent;
    int32_t tiles_per_wave;
    int32_t chunks;
    int32_t prefetch;           // scalar loads in flight when a program's code is burst-loaded into the
                                // scalar cache before it runs (1-15), or 0: no burst load
    int32_t n_groups;           // program groups (implicit units)
    int32_t same_group;         // implicit units: the four waves of a block run one group on four chunks
    int64_t n_bits;             // Boolean kernels: cases (bits) in the N words of each row
    uint32_t probe;             // nonzero: write the handler table address and return
    double* partials;
    float* cases_out;
    uint64_t* probe_out;
};

hipError_t core_launch(int variant, const CoreArgs& a, uint32_t blocks, hipStream_t s);
int core_blocks_per_cu(int variant);
hipError_t core_zero_counter(uint32_t* counter, hipStream_t s);
hipError_t core_reduce_jobs(const ReduceArgs* jobs_dev, int32_t n_jobs, int64_t max_prog, hipStream_t s);
hipError_t core_reduce_one(const ReduceArgs& r, hipStream_t s);

}  // namespace gpx
