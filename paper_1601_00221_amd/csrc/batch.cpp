// Batched evaluation: several program populations (tree and linear) over
// several resident case matrices in one persistent launch, plus the
// autotuner that picks tile width, stack depth variant, unit size and
// schedule for a batch shape.
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/gp.h"
#include "batch.h"
#include "core_host.h"
#include "core_kernels.h"
#include "runtime.h"

namespace gpx {

static int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

static double transc_fraction(const std::vector<BatchJobRef>& jobs) {
    int64_t e = 0, n = 0;
    for (const BatchJobRef& j : jobs) {
        e += j.pd->n_transc;
        n += j.pd->n_instr;
    }
    return n ? (double)e / (double)n : 0.0;
}

gp_status plan_batch(const std::vector<BatchJobRef>& jobs, const std::vector<gp_dataset>& ds,
                     const gp_batch_config& cfg, BatchPlan& plan) {
    plan = BatchPlan();
    int n_load = 1, depth = 0;
    bool any_transc = false;
    for (const BatchJobRef& j : jobs) {
        n_load = std::max(n_load, j.pd->n_load);
        depth = std::max(depth, j.pd->max_depth);
        any_transc = any_transc || j.pd->n_transc > 0;
    }
    const int vi = cfg.variant;
    if (vi < 0 || vi >= core_variants()) return fail(GP_E_INVAL, "kernel variant %d does not exist", vi);
    const int vt = core_variant_t(vi);
    if (core_variant_nf(vi) < n_load || core_variant_d(vi) < depth)
        return fail(GP_E_INVAL, "variant %d (%d features, depth %d) cannot hold %d features / depth %d", vi,
                    core_variant_nf(vi), core_variant_d(vi), n_load, depth);
    if (core_variant_arith(vi) && any_transc)
        return fail(GP_E_INVAL, "variant %d has no sin/cos/exp/log code", vi);
    if (core_variant_bool(vi)) return fail(GP_E_INVAL, "variant %d is a Boolean kernel", vi);
    if (core_variant_trees_only(vi))
        for (const BatchJobRef& j : jobs)
            if (j.pd->form != FORM_TREE) return fail(GP_E_INVAL, "variant %d runs trees only", vi);
    plan.vi = vi;
    const int32_t unit_prog = std::max(1, cfg.unit_programs);
    int64_t n_prog = 0;
    for (const BatchJobRef& j : jobs) n_prog += j.pd->n_prog;
    if (n_prog > 0x7FFFFFFFll) return fail(GP_E_INVAL, "batch too large");
    plan.progs.reserve((size_t)n_prog);
    plan.order.reserve((size_t)n_prog);
    uint64_t part_base = 0;
    std::vector<std::pair<double, UnitDesc>> units;
    for (size_t ji = 0; ji < jobs.size(); ji++) {
        const BatchJobRef& j = jobs[ji];
        const ProgData& pd = *j.pd;
        const gp_dataset& d = ds[j.ds];
        const int64_t N = d.n_cases;
        const int64_t blocks = (N + 255) / 256;
        const int64_t tiles = (N + 64LL * vt - 1) / (64LL * vt);
        std::vector<uint32_t> jcode;
        std::vector<DevProg> jprogs;
        gp_status st = core_translate(pd, vi, jcode, jprogs);
        if (st != GP_OK) return st;
        if ((plan.code.size() + jcode.size()) * 4 > 0xFFFFFFF0ull) return fail(GP_E_INVAL, "batch code exceeds 4 GiB");
        const uint32_t code_base = (uint32_t)plan.code.size();
        const uint32_t prog_base = (uint32_t)plan.progs.size();
        plan.code.insert(plan.code.end(), jcode.begin(), jcode.end());
        for (int32_t p = 0; p < pd.n_prog; p++) {
            DevProg dp = jprogs[p];
            dp.code_off += code_base;
            dp.row = (uint64_t)p;
            plan.progs.push_back(dp);
        }
        // programs of this job, longest first, dealt to groups in snake order
        std::vector<uint32_t> idx(pd.n_prog);
        std::iota(idx.begin(), idx.end(), 0u);
        std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) { return pd.cost[a] > pd.cost[b]; });
        const int32_t G = std::max<int32_t>(1, (pd.n_prog + unit_prog - 1) / unit_prog);
        std::vector<std::vector<uint32_t>> groups(G);
        std::vector<double> gcost(G, 0.0);
        for (int32_t i = 0; i < pd.n_prog; i++) {
            const int32_t r = i / G, k = i % G;
            const int32_t g = (r & 1) ? G - 1 - k : k;
            groups[g].push_back(prog_base + idx[i]);
            gcost[g] += pd.cost[idx[i]];
        }
        std::vector<std::pair<uint32_t, uint32_t>> qr(G);
        for (int32_t g = 0; g < G; g++) {
            qr[g].first = (uint32_t)plan.order.size();
            plan.order.insert(plan.order.end(), groups[g].begin(), groups[g].end());
            qr[g].second = (uint32_t)plan.order.size();
        }
        for (int64_t t = 0; t < tiles; t++) {
            for (int32_t g = 0; g < G; g++) {
                if (qr[g].first == qr[g].second) continue;
                UnitDesc u{(uint32_t)ji, (uint32_t)t, qr[g].first, qr[g].second};
                // every slot of a tile is interpreted, ragged or not; add the tile load
                units.push_back({gcost[g] + 8.0 * pd.n_load, u});
            }
        }
        JobDesc jd;
        memset(&jd, 0, sizeof jd);
        jd.ds = j.ds;
        jd.kind = j.kind;
        jd.n_load = pd.n_load;
        jd.part_base = part_base;
        plan.jobs.push_back(jd);
        ReduceArgs r;
        memset(&r, 0, sizeof r);
        r.part_base = part_base;
        r.n_prog = pd.n_prog;
        r.N = N;
        r.out = j.out;
        r.blocks = (int32_t)blocks;
        r.kind = j.kind;
        plan.reduce.push_back(r);
        plan.max_prog = std::max<int64_t>(plan.max_prog, pd.n_prog);
        plan.gpop += pd.n_gpop * N;
        part_base += (uint64_t)blocks * (uint64_t)pd.n_prog;
    }
    if (units.size() > 0x7FFFFFF0ull) return fail(GP_E_INVAL, "batch has too many work units");
    if (cfg.persistent)
        std::stable_sort(units.begin(), units.end(),
                         [](const std::pair<double, UnitDesc>& a, const std::pair<double, UnitDesc>& b) {
                             return a.first > b.first;
                         });
    plan.units.reserve(units.size());
    for (auto& u : units) plan.units.push_back(u.second);
    plan.partial_doubles = (int64_t)part_base;
    plan.persistent = cfg.persistent != 0;
    for (const gp_dataset& d : ds) {
        DatasetDesc dd;
        dd.X = d.X;
        dd.y = d.y;
        dd.N = d.n_cases;
        plan.datasets.push_back(dd);
    }
    return GP_OK;
}

size_t plan_device_bytes(const BatchPlan& p) {
    return p.code.size() * 4 + p.progs.size() * sizeof(DevProg) + p.order.size() * 4 +
           p.units.size() * sizeof(UnitDesc) + p.jobs.size() * sizeof(JobDesc) +
           p.datasets.size() * sizeof(DatasetDesc) + p.reduce.size() * sizeof(ReduceArgs) +
           (size_t)p.partial_doubles * sizeof(double) + 4096;
}

gp_status upload_plan(BatchPlan& p, BatchScratch& sc, hipStream_t s) {
    gp_status st;
    if ((st = sc.code.reserve(std::max<size_t>(4, p.code.size() * 4))) != GP_OK) return st;
    if ((st = sc.progs.reserve(std::max<size_t>(1, p.progs.size()) * sizeof(DevProg))) != GP_OK) return st;
    if ((st = sc.order.reserve(std::max<size_t>(1, p.order.size()) * 4)) != GP_OK) return st;
    if ((st = sc.units.reserve(std::max<size_t>(1, p.units.size()) * sizeof(UnitDesc))) != GP_OK) return st;
    if ((st = sc.jobs.reserve(std::max<size_t>(1, p.jobs.size()) * sizeof(JobDesc))) != GP_OK) return st;
    if ((st = sc.datasets.reserve(std::max<size_t>(1, p.datasets.size()) * sizeof(DatasetDesc))) != GP_OK) return st;
    if ((st = sc.reduce.reserve(std::max<size_t>(1, p.reduce.size()) * sizeof(ReduceArgs))) != GP_OK) return st;
    if ((st = sc.partials.reserve(std::max<size_t>(1, (size_t)p.partial_doubles) * sizeof(double))) != GP_OK) return st;
    if ((st = sc.counter.reserve(256)) != GP_OK) return st;
    for (ReduceArgs& r : p.reduce) r.partials = (const double*)sc.partials.p;
    const size_t total = plan_device_bytes(p) - (size_t)p.partial_doubles * sizeof(double) + 8 * 256;
    if ((st = sc.staging.begin(total)) != GP_OK) return st;
    if ((st = sc.staging.put(p.code.data(), p.code.size() * 4, sc.code.p, s)) != GP_OK) return st;
    if ((st = sc.staging.put(p.progs.data(), p.progs.size() * sizeof(DevProg), sc.progs.p, s)) != GP_OK) return st;
    if ((st = sc.staging.put(p.order.data(), p.order.size() * 4, sc.order.p, s)) != GP_OK) return st;
    if ((st = sc.staging.put(p.units.data(), p.units.size() * sizeof(UnitDesc), sc.units.p, s)) != GP_OK) return st;
    if ((st = sc.staging.put(p.jobs.data(), p.jobs.size() * sizeof(JobDesc), sc.jobs.p, s)) != GP_OK) return st;
    if ((st = sc.staging.put(p.datasets.data(), p.datasets.size() * sizeof(DatasetDesc), sc.datasets.p, s)) != GP_OK)
        return st;
    if ((st = sc.staging.put(p.reduce.data(), p.reduce.size() * sizeof(ReduceArgs), sc.reduce.p, s)) != GP_OK)
        return st;
    return sc.staging.end(s);
}

gp_status launch_plan(const BatchPlan& p, BatchScratch& sc, hipStream_t s) {
    if (p.units.empty()) return GP_OK;
    CoreArgs a;
    memset(&a, 0, sizeof a);
    a.code = (const uint32_t*)sc.code.p;
    a.progs = (const DevProg*)sc.progs.p;
    a.order = (const uint32_t*)sc.order.p;
    a.units = (const UnitDesc*)sc.units.p;
    a.jobs = (const JobDesc*)sc.jobs.p;
    a.datasets = (const DatasetDesc*)sc.datasets.p;
    a.partials = (double*)sc.partials.p;
    a.counter = (uint32_t*)sc.counter.p;
    a.n_units = (int32_t)p.units.size();
    a.persistent = p.persistent ? 1 : 0;
    a.prefetch = code_prefetch();
    const uint32_t grid = p.persistent ? (uint32_t)(device_cus() * core_blocks_per_cu(p.vi))
                                       : (uint32_t)((p.units.size() + 3) / 4);
    int slot;
    hipError_t e = hipSuccess;
    if (p.persistent) e = core_zero_counter(a.counter, s);
    if (e == hipSuccess) e = timed_launch_begin(s, &slot);
    if (e == hipSuccess) e = core_launch(p.vi, a, grid, s);
    if (e == hipSuccess) e = timed_launch_end(s, slot);
    if (e != hipSuccess) return fail(GP_E_DEVICE, "batch launch: %s", hipGetErrorString(e));
    e = core_reduce_jobs((const ReduceArgs*)sc.reduce.p, (int32_t)p.reduce.size(), p.max_prog, s);
    if (e != hipSuccess) return fail(GP_E_DEVICE, "batch reduction launch: %s", hipGetErrorString(e));
    return GP_OK;
}

// ---------------------------------------------------------------------------
// Autotuning
// ---------------------------------------------------------------------------
static std::mutex g_tune_mu;
static std::map<std::string, gp_batch_config> g_tune_cache;
static bool g_tune_loaded = false;

static const char* tune_cache_path() { return getenv("GP2D_TUNE_CACHE"); }

static void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = tune_cache_path();
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    // one entry per line: "key": [variant, unit_programs, persistent]
    char line[4096];
    while (fgets(line, sizeof line, f)) {
        char* q1 = strchr(line, '"');
        if (!q1) continue;
        char* q2 = strchr(q1 + 1, '"');
        if (!q2) continue;
        std::string key(q1 + 1, q2);
        gp_batch_config c;
        memset(&c, 0, sizeof c);
        if (sscanf(q2 + 1, " : [ %d , %d , %d ]", &c.variant, &c.unit_programs, &c.persistent) == 3)
            g_tune_cache[key] = c;
    }
    fclose(f);
}

static void tune_save_locked() {
    const char* path = tune_cache_path();
    if (!path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n");
    size_t i = 0;
    for (auto& kv : g_tune_cache) {
        fprintf(f, "\"%s\": [%d, %d, %d]%s\n", kv.first.c_str(), kv.second.variant, kv.second.unit_programs,
                kv.second.persistent, ++i < g_tune_cache.size() ? "," : "");
    }
    fprintf(f, "}\n");
    fclose(f);
    rename(tmp.c_str(), path);
}

// Shape signature of a batch: what the best configuration depends on.
static std::string batch_key(const std::vector<BatchJobRef>& jobs, const std::vector<gp_dataset>& ds) {
    std::string k;
    char buf[128];
    for (const gp_dataset& d : ds) {
        snprintf(buf, sizeof buf, "d%lldx%d;", (long long)d.n_cases, d.n_feat);
        k += buf;
    }
    for (const BatchJobRef& j : jobs) {
        // program counts and mean lengths rounded to powers of two
        const int64_t P = j.pd->n_prog;
        const int64_t mean = P ? j.pd->n_instr / P : 0;
        int lp = 0, lm = 0;
        while ((1LL << lp) < P) lp++;
        while ((1LL << lm) < mean) lm++;
        snprintf(buf, sizeof buf, "j%d,%d,%d,%d,%d,%d;", j.pd->form, j.ds, lp, lm, j.pd->n_load, j.pd->max_depth);
        k += buf;
    }
    return k;
}

static gp_status time_config(const std::vector<BatchJobRef>& jobs, const std::vector<gp_dataset>& ds,
                             const gp_batch_config& c, int reps, BatchScratch& sc, hipStream_t s, double* ms) {
    gp_status st = core_ready(c.variant, s);
    if (st != GP_OK) return st;
    BatchPlan plan;
    st = plan_batch(jobs, ds, c, plan);
    if (st != GP_OK) return st;
    if ((st = upload_plan(plan, sc, s)) != GP_OK) return st;
    if ((st = launch_plan(plan, sc, s)) != GP_OK) return st;  // warm-up
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(GP_E_DEVICE, "hipEventCreate failed");
    std::vector<float> t;
    for (int r = 0; r < reps; r++) {
        hipError_t e = hipEventRecord(e0, s);
        st = launch_plan(plan, sc, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (st != GP_OK) break;
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e != hipSuccess) {
            st = fail(GP_E_DEVICE, "hipEventSynchronize: %s", hipGetErrorString(e));
            break;
        }
        float x = 0;
        e = hipEventElapsedTime(&x, e0, e1);
        if (e != hipSuccess) {
            st = fail(GP_E_DEVICE, "hipEventElapsedTime: %s", hipGetErrorString(e));
            break;
        }
        t.push_back(x);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != GP_OK) return st;
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return GP_OK;
}

gp_status tune_batch(const std::vector<BatchJobRef>& jobs, const std::vector<gp_dataset>& ds, int reps,
                     BatchScratch& sc, hipStream_t s, gp_batch_config* best, double* best_ms) {
    int n_load = 1, depth = 0;
    bool any_transc = false;
    for (const BatchJobRef& j : jobs) {
        n_load = std::max(n_load, j.pd->n_load);
        depth = std::max(depth, j.pd->max_depth);
        any_transc = any_transc || j.pd->n_transc > 0;
    }
    double best_t = 1e300;
    gp_batch_config b;
    memset(&b, 0, sizeof b);
    b.variant = -1;
    const int unit_sizes[] = {8, 32, 128};
    for (int vi = 0; vi < core_variants(); vi++) {
        if (core_variant_nf(vi) < n_load || core_variant_d(vi) < depth) continue;
        if (core_variant_arith(vi) && any_transc) continue;
        if (core_variant_bool(vi) || core_variant_trees_only(vi)) continue;
        for (int us : unit_sizes) {
            for (int pers = 1; pers >= 0; pers--) {
                gp_batch_config c;
                memset(&c, 0, sizeof c);
                c.variant = vi;
                c.unit_programs = us;
                c.persistent = pers;
                double ms = 0;
                gp_status st = time_config(jobs, ds, c, reps, sc, s, &ms);
                if (st != GP_OK) return st;
                if (ms < best_t) {
                    best_t = ms;
                    b = c;
                }
            }
        }
    }
    if (b.variant < 0) return fail(GP_E_DEPTH, "no kernel variant holds %d features and depth %d", n_load, depth);
    *best = b;
    if (best_ms) *best_ms = best_t;
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_load_locked();
    g_tune_cache[batch_key(jobs, ds)] = b;
    tune_save_locked();
    return GP_OK;
}

bool tuned_config(const std::vector<BatchJobRef>& jobs, const std::vector<gp_dataset>& ds, gp_batch_config* c) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_load_locked();
    auto it = g_tune_cache.find(batch_key(jobs, ds));
    if (it == g_tune_cache.end()) return false;
    *c = it->second;
    return true;
}

gp_batch_config default_config(const std::vector<BatchJobRef>& jobs) {
    int n_load = 1, depth = 0;
    for (const BatchJobRef& j : jobs) {
        n_load = std::max(n_load, j.pd->n_load);
        depth = std::max(depth, j.pd->max_depth);
    }
    gp_batch_config c;
    memset(&c, 0, sizeof c);
    bool any_transc = false;
    for (const BatchJobRef& j : jobs) any_transc = any_transc || j.pd->n_transc > 0;
    c.variant = pick_core_variant(n_load, depth, transc_fraction(jobs), any_transc);
    c.unit_programs = 32;
    c.persistent = 1;
    return c;
}

// ---------------------------------------------------------------------------
// Job intake shared by the batch API and the server
// ---------------------------------------------------------------------------
gp_status check_datasets(const gp_dataset* ds, int32_t n_ds) {
    if (n_ds < 1 || !ds) return fail(GP_E_INVAL, "no datasets");
    for (int32_t i = 0; i < n_ds; i++) {
        if (!ds[i].X) return fail(GP_E_INVAL, "dataset %d: X is null", i);
        if (ds[i].n_cases < 1) return fail(GP_E_INVAL, "dataset %d: n_cases < 1", i);
        if (ds[i].n_feat < 1) return fail(GP_E_INVAL, "dataset %d: n_feat < 1", i);
    }
    return GP_OK;
}

gp_status build_job(const gp_job& j, const gp_dataset* ds, int32_t n_ds, ProgData& pd) {
    if (j.dataset < 0 || j.dataset >= n_ds) return fail(GP_E_NOTFOUND, "dataset %d does not exist", j.dataset);
    if (j.kind != GP_FIT_SUM_ABS && j.kind != GP_FIT_MSE && j.kind != GP_FIT_HITS && j.kind != GP_FIT_CLASS_ERR)
        return fail(GP_E_INVAL, "batched jobs take GP_FIT_SUM_ABS, GP_FIT_MSE, GP_FIT_HITS or GP_FIT_CLASS_ERR (got %d)",
                    j.kind);
    if (!j.out && j.n_prog > 0) return fail(GP_E_INVAL, "job output is null");
    if (!ds[j.dataset].y) return fail(GP_E_INVAL, "dataset %d has no targets", j.dataset);
    const int32_t F = ds[j.dataset].n_feat;
    gp_status st;
    if (j.form == FORM_TREE) st = build_tree(j.tok, j.tcst, j.toff, j.n_prog, F, pd);
    else if (j.form == FORM_LINEAR)
        st = build_linear(j.code, j.loff, j.lcst, j.lcst_off, j.n_prog, j.n_reg, F, pd);
    else return fail(GP_E_INVAL, "unknown program form %d", j.form);
    if (st != GP_OK) return st;
    if (pd.n_load > GP_MAX_FEAT)
        return fail(GP_E_INVAL, "programs read feature %d; at most %d features are supported", pd.n_load - 1,
                    GP_MAX_FEAT);
    return GP_OK;
}

}  // namespace gpx

// ===========================================================================
// C ABI
// ===========================================================================
using namespace gpx;

namespace {
std::mutex g_batch_mu;
std::map<hipStream_t, BatchScratch*> g_batch_scratch;

BatchScratch& batch_scratch(hipStream_t s) {
    std::lock_guard<std::mutex> g(g_batch_mu);
    auto it = g_batch_scratch.find(s);
    if (it != g_batch_scratch.end()) return *it->second;
    BatchScratch* sc = new BatchScratch();  // lives until process exit
    g_batch_scratch[s] = sc;
    return *sc;
}

gp_status intake(const gp_dataset* ds, int32_t n_ds, const gp_job* jobs, int32_t n_jobs,
                 std::vector<ProgData>& pds, std::vector<BatchJobRef>& refs, std::vector<gp_dataset>& dv) {
    gp_status st = check_datasets(ds, n_ds);
    if (st != GP_OK) return st;
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(GP_E_INVAL, "bad job array");
    pds.resize(n_jobs);
    for (int32_t i = 0; i < n_jobs; i++) {
        if ((st = build_job(jobs[i], ds, n_ds, pds[i])) != GP_OK) {
            char msg[512];
            snprintf(msg, sizeof msg, "%s", last_error());
            return fail(st, "job %d: %s", i, msg);
        }
    }
    for (int32_t i = 0; i < n_jobs; i++) {
        if (pds[i].n_prog == 0) continue;
        refs.push_back(BatchJobRef{&pds[i], jobs[i].dataset, jobs[i].kind, jobs[i].out});
    }
    dv.assign(ds, ds + n_ds);
    return GP_OK;
}
}  // namespace

extern "C" {

gp_status gp_eval_batch(const gp_dataset* ds, int32_t n_ds, const gp_job* jobs, int32_t n_jobs,
                        const gp_batch_config* cfg, void* stream) {
    clear_error();
    std::vector<ProgData> pds;
    std::vector<BatchJobRef> refs;
    std::vector<gp_dataset> dv;
    gp_status st = intake(ds, n_ds, jobs, n_jobs, pds, refs, dv);
    if (st != GP_OK || refs.empty()) return st;
    hipStream_t s = (hipStream_t)stream;
    BatchScratch& sc = batch_scratch(s);
    std::lock_guard<std::mutex> g(sc.mu);
    gp_batch_config c;
    if (cfg) c = *cfg;
    else if (!tuned_config(refs, dv, &c)) c = default_config(refs);
    if (c.variant < 0) return fail(GP_E_DEPTH, "no kernel variant can hold these programs");
    if ((st = core_ready(c.variant, s)) != GP_OK) return st;
    BatchPlan plan;
    if ((st = plan_batch(refs, dv, c, plan)) != GP_OK) return st;
    if ((st = upload_plan(plan, sc, s)) != GP_OK) return st;
    return launch_plan(plan, sc, s);
}

gp_status gp_tune_batch(const gp_dataset* ds, int32_t n_ds, const gp_job* jobs, int32_t n_jobs, int32_t reps,
                        gp_batch_config* best, double* best_ms, void* stream) {
    clear_error();
    if (!best) return fail(GP_E_INVAL, "best is null");
    std::vector<ProgData> pds;
    std::vector<BatchJobRef> refs;
    std::vector<gp_dataset> dv;
    gp_status st = intake(ds, n_ds, jobs, n_jobs, pds, refs, dv);
    if (st != GP_OK) return st;
    if (refs.empty()) return fail(GP_E_INVAL, "nothing to tune");
    hipStream_t s = (hipStream_t)stream;
    BatchScratch& sc = batch_scratch(s);
    std::lock_guard<std::mutex> g(sc.mu);
    return tune_batch(refs, dv, reps < 1 ? 3 : reps, sc, s, best, best_ms);
}

int32_t gp_num_variants(void) { return core_variants(); }

gp_status gp_variant_info(int32_t i, int32_t* t, int32_t* depth, int32_t* n_feat, int32_t* vgprs,
                          int32_t* flags) {
    clear_error();
    if (i < 0 || i >= core_variants()) return fail(GP_E_INVAL, "variant %d does not exist", i);
    if (t) *t = core_variant_t(i);
    if (depth) *depth = core_variant_d(i);
    if (n_feat) *n_feat = core_variant_nf(i);
    if (vgprs) *vgprs = core_variant_ncv(i);
    if (flags)
        *flags = (core_variant_arith(i) ? GP_VARIANT_NO_TRANSC : 0) | (core_variant_bool(i) ? GP_VARIANT_BOOLEAN : 0) |
                 (core_variant_trees_only(i) && !core_variant_bool(i) ? GP_VARIANT_TREES_ONLY : 0);
    return GP_OK;
}

}  // extern "C"
