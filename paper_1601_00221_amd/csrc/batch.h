// Batched evaluation internals shared by the batch API and the server.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "../../include/gp.h"
#include "core_kernels.h"
#include "runtime.h"

namespace gpx {

// One population of lowered programs to evaluate on one dataset.
struct BatchJobRef {
    const ProgData* pd;
    int32_t ds;
    int32_t kind;
    void* out;
};

// Host image of one batched launch.
struct BatchPlan {
    int vi = -1;
    bool persistent = true;
    std::vector<uint32_t> code;
    std::vector<DevProg> progs;
    std::vector<uint32_t> order;
    std::vector<UnitDesc> units;
    std::vector<JobDesc> jobs;
    std::vector<DatasetDesc> datasets;
    std::vector<ReduceArgs> reduce;
    int64_t partial_doubles = 0;
    int64_t max_prog = 0;
    int64_t gpop = 0;            // GP operations of the whole batch
};

// Device buffers of one stream's batched launches.
struct BatchScratch {
    std::mutex mu;
    DevBuf code, progs, order, units, jobs, datasets, reduce, partials, counter;
    Staging staging;
};

gp_status plan_batch(const std::vector<BatchJobRef>& jobs, const std::vector<gp_dataset>& ds,
                     const gp_batch_config& cfg, BatchPlan& plan);
size_t plan_device_bytes(const BatchPlan& p);
gp_status upload_plan(BatchPlan& p, BatchScratch& sc, hipStream_t s);
gp_status launch_plan(const BatchPlan& p, BatchScratch& sc, hipStream_t s);
gp_status tune_batch(const std::vector<BatchJobRef>& jobs, const std::vector<gp_dataset>& ds, int reps,
                     BatchScratch& sc, hipStream_t s, gp_batch_config* best, double* best_ms);
bool tuned_config(const std::vector<BatchJobRef>& jobs, const std::vector<gp_dataset>& ds, gp_batch_config* c);
gp_batch_config default_config(const std::vector<BatchJobRef>& jobs);
gp_status check_datasets(const gp_dataset* ds, int32_t n_ds);
gp_status build_job(const gp_job& j, const gp_dataset* ds, int32_t n_ds, ProgData& pd);

}  // namespace gpx
