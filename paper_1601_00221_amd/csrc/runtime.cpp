// Host runtime of the GP population evaluator: argument checks, program
// lowering and upload, scheduling of (case tile, program group) units, and
// the C ABI declared in include/gp.h.
#include <hip/hip_runtime_api.h>
#include <stdarg.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/gp.h"
#include "core_host.h"
#include "core_kernels.h"
#include "gp_internal.h"
#include "runtime.h"

namespace gpx {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local char t_err[512] = "";

gp_status fail(gp_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_err, sizeof t_err, fmt, ap);
    va_end(ap);
    return s;
}
void clear_error() { t_err[0] = 0; }
const char* last_error() { return t_err; }

// ---------------------------------------------------------------------------
// Buffers
// ---------------------------------------------------------------------------
gp_status DevBuf::reserve(size_t n) {
    if (n <= cap) return GP_OK;
    if (p) {
        hipError_t e = hipFree(p);  // waits for the device before releasing
        p = nullptr;
        cap = 0;
        if (e != hipSuccess) return fail(GP_E_DEVICE, "hipFree: %s", hipGetErrorString(e));
    }
    size_t want = n < 4096 ? 4096 : n + n / 4;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        p = nullptr;
        return fail(e == hipErrorOutOfMemory ? GP_E_NOMEM : GP_E_DEVICE, "hipMalloc(%zu): %s", want,
                    hipGetErrorString(e));
    }
    cap = want;
    return GP_OK;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
}

gp_status Staging::begin(size_t n) {
    cur ^= 1;
    Half& h = half[cur];
    if (h.pending) {
        hipError_t e = hipEventSynchronize(h.ev);
        if (e != hipSuccess) return fail(GP_E_DEVICE, "hipEventSynchronize: %s", hipGetErrorString(e));
        h.pending = false;
    }
    if (!h.ev) {
        hipError_t e = hipEventCreateWithFlags(&h.ev, hipEventDisableTiming);
        if (e != hipSuccess) return fail(GP_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
    if (n > h.cap) {
        if (h.host) (void)hipHostFree(h.host);
        h.host = nullptr;
        h.cap = 0;
        size_t want = n < 65536 ? 65536 : n + n / 4;
        hipError_t e = hipHostMalloc(&h.host, want, hipHostMallocDefault);
        if (e != hipSuccess) {
            h.host = nullptr;
            return fail(GP_E_NOMEM, "hipHostMalloc(%zu): %s", want, hipGetErrorString(e));
        }
        h.cap = want;
    }
    used = 0;
    return GP_OK;
}

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& fn);

gp_status Staging::put(const void* src, size_t n, void* dst, hipStream_t s) {
    if (n == 0) return GP_OK;
    Half& h = half[cur];
    if (used + n > h.cap) return fail(GP_E_INVAL, "internal: staging overflow (%zu + %zu > %zu)", used, n, h.cap);
    char* to = (char*)h.host + used;
    if (n >= ((size_t)1 << 22)) {
        // a large program set: copy into the pinned buffer on the host threads, 64 KiB apiece
        const int64_t pieces = (int64_t)((n + ((size_t)1 << 16) - 1) >> 16);
        parallel_for(pieces, [&](int64_t i0, int64_t i1) {
            const size_t a = (size_t)i0 << 16, b = std::min(n, (size_t)i1 << 16);
            memcpy(to + a, (const char*)src + a, b - a);
        });
    } else {
        memcpy(to, src, n);
    }
    hipError_t e = hipMemcpyAsync(dst, to, n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail(GP_E_DEVICE, "hipMemcpyAsync: %s", hipGetErrorString(e));
    used += (n + 255) & ~(size_t)255;
    return GP_OK;
}

gp_status Staging::end(hipStream_t s) {
    Half& h = half[cur];
    hipError_t e = hipEventRecord(h.ev, s);
    if (e != hipSuccess) return fail(GP_E_DEVICE, "hipEventRecord: %s", hipGetErrorString(e));
    h.pending = true;
    return GP_OK;
}

void Staging::release() {
    for (Half& h : half) {
        if (h.pending && h.ev) (void)hipEventSynchronize(h.ev);
        if (h.host) (void)hipHostFree(h.host);
        if (h.ev) (void)hipEventDestroy(h.ev);
        h = Half();
    }
    used = 0;
}

static std::mutex g_ws_mu;
static std::unordered_map<hipStream_t, Workspace*> g_ws;

Workspace& workspace(hipStream_t s) {
    std::lock_guard<std::mutex> g(g_ws_mu);
    auto it = g_ws.find(s);
    if (it != g_ws.end()) return *it->second;
    Workspace* w = new Workspace();  // lives until process exit
    g_ws[s] = w;
    return *w;
}

// ---------------------------------------------------------------------------
// Host threads: a fixed pool that splits a range of programs
// ---------------------------------------------------------------------------
namespace {
struct Pool {
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::vector<std::thread> th;
    const std::function<void(int64_t, int64_t)>* fn = nullptr;
    int64_t n = 0, chunk = 1;
    std::atomic<int64_t> next{0};
    int active = 0;
    uint64_t gen = 0;
    bool stop = false;

    explicit Pool(int k) {
        for (int i = 0; i < k; i++) th.emplace_back([this] { worker(); });
    }
    ~Pool() {
        {
            std::lock_guard<std::mutex> g(mu);
            stop = true;
        }
        cv.notify_all();
        for (auto& t : th) t.join();
    }
    void take() {
        for (;;) {
            const int64_t lo = next.fetch_add(chunk);
            if (lo >= n) return;
            (*fn)(lo, std::min(n, lo + chunk));
        }
    }
    void worker() {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv.wait(lk, [&] { return stop || gen != seen; });
            if (stop) return;
            seen = gen;
            lk.unlock();
            take();
            lk.lock();
            if (--active == 0) done_cv.notify_all();
        }
    }
    void run(int64_t count, const std::function<void(int64_t, int64_t)>& f) {
        std::unique_lock<std::mutex> lk(mu);
        fn = &f;
        n = count;
        chunk = std::max<int64_t>(1, count / (8 * (int64_t)(th.size() + 1)));
        next = 0;
        active = (int)th.size();
        gen++;
        cv.notify_all();
        lk.unlock();
        take();
        lk.lock();
        done_cv.wait(lk, [&] { return active == 0; });
        fn = nullptr;
    }
};

std::mutex g_pool_mu;   // one parallel_for at a time (calls from several host threads take turns)
}  // namespace

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& fn) {
    if (n <= 0) return;
    if (n < 64) {
        fn(0, n);
        return;
    }
    static Pool* pool = [] {
        const unsigned hc = std::thread::hardware_concurrency();
        return new Pool((int)std::max(1u, std::min(16u, hc ? hc : 1u)) - 1);   // the caller is the last thread
    }();
    std::lock_guard<std::mutex> g(g_pool_mu);
    pool->run(n, fn);
}

// ---------------------------------------------------------------------------
// Program building
// ---------------------------------------------------------------------------
// Relative cost of one instruction, used only to balance program groups:
// the vector instructions it issues per slot, plus one for its dispatch.
// Protected division (about 15 per slot), the compares, IF and AND/OR (a
// compare or two and a select) run in the core; sin/cos/exp/log are exits to
// binary64 code of some 34 (sin, cos) or 24 (exp, log) per value.  Every
// Boolean function is one bitwise instruction per slot.
static uint32_t op_cost(uint32_t op, int opset) {
    if (opset == OPSET_BOOL) return 2;
    switch (op) {
        case GP_PDIV: return 16;
        case GP_GT: case GP_LT: case GP_EQ: case OP_IF: return 3;
        case GP_AND: case GP_OR: return 4;
        case GP_SIN: case GP_COS: return 35;
        case GP_EXPC: case GP_PLOG: return 25;
        default: return 2;
    }
}

gp_status build_tree(const int32_t* tok, const float* cst, const int64_t* off, int32_t P,
                     int32_t n_feat, ProgData& pd, int opset) {
    if (P < 0) return fail(GP_E_INVAL, "n_prog < 0");
    if (P > 0 && (!tok || (!cst && opset != OPSET_BOOL) || !off)) return fail(GP_E_INVAL, "null program array");
    if (n_feat < 1) return fail(GP_E_INVAL, "n_feat < 1");
    pd = ProgData();
    pd.form = FORM_TREE;
    pd.opset = opset;
    pd.n_prog = P;
    pd.n_feat = n_feat;
    if (P == 0) return GP_OK;
    if (off[0] != 0) return fail(GP_E_INVAL, "off[0] must be 0");
    int64_t total = 0;
    for (int32_t p = 0; p < P; p++) {
        const int64_t n = off[p + 1] - off[p];
        if (n < 1) return fail(GP_E_INVAL, "program %d is empty", p);
        if (n > GP_MAX_LEN) return fail(GP_E_DEPTH, "program %d: %lld nodes exceeds %d", p, (long long)n, GP_MAX_LEN);
        total += n;
    }
    if (total > 0x7FFFFFFFll) return fail(GP_E_INVAL, "programs exceed 2^31 nodes");
    // Program p is lowered at word 2 * off[p] (at most one instruction per
    // node), so the programs are independent: they are lowered in parallel.
    pd.code.resize((size_t)total * 2);
    pd.progs.resize(P);
    pd.cost.resize(P);
    std::vector<TreeLowering> lst(P);
    std::vector<int32_t> pfeat(P, -1), prc(P, GP_OK), ptransc(P, 0);
    parallel_for(P, [&](int64_t p0, int64_t p1) {
        char err[256];
        for (int64_t p = p0; p < p1; p++) {
            const int64_t n = off[p + 1] - off[p];
            uint32_t* words = pd.code.data() + 2 * off[p];
            const int rc = lower_tree(tok + off[p], cst ? cst + off[p] : nullptr, n, n_feat, words, &lst[p], err, opset);
            if (rc != GP_OK) {
                prc[p] = rc;
                return;
            }
            int32_t mf = -1;
            for (int64_t i = 0; i < n; i++) {
                const int32_t t = tok[off[p] + i];
                if ((t & 0xFF) == GP_VAR) mf = std::max<int32_t>(mf, (int32_t)((uint32_t)t >> 8));
            }
            pfeat[p] = mf;
            uint32_t cost = 0;
            int32_t nt = 0;
            for (int32_t i = 0; i < lst[p].n_instr; i++) {
                const uint32_t op = words[2 * i] & 15u;
                cost += op_cost(op, opset);
                nt += opset != OPSET_BOOL && op >= GP_SIN && op <= GP_PLOG;
            }
            ptransc[p] = nt;
            pd.cost[p] = cost + 16;
        }
    });
    int32_t max_feat = -1;
    for (int32_t p = 0; p < P; p++) {
        if (prc[p] != GP_OK) {
            // lower the first failing program again on this thread for its message
            char err[256];
            TreeLowering st;
            lower_tree(tok + off[p], cst ? cst + off[p] : nullptr, off[p + 1] - off[p], n_feat, nullptr, &st, err,
                       opset);
            return fail((gp_status)prc[p], "program %d: %s", p, err);
        }
        const TreeLowering& st = lst[p];
        DevProg& d = pd.progs[p];
        d.code_off = (uint32_t)(2 * off[p]);
        d.len = (uint32_t)st.n_instr;
        d.meta = FORM_TREE | ((uint32_t)st.max_depth << 8);
        d.reserved0 = 0;
        d.reserved1 = 0;
        d.row = (uint64_t)p;
        max_feat = std::max(max_feat, pfeat[p]);
        pd.n_transc += ptransc[p];
        pd.max_depth = std::max(pd.max_depth, st.max_depth);
        pd.n_instr += st.n_instr;
        pd.n_gpop += st.n_nodes;
    }
    pd.n_load = max_feat + 1 > 0 ? max_feat + 1 : 1;
    return GP_OK;
}

gp_status build_linear(const uint32_t* code, const int64_t* off, const float* cst, const int64_t* cst_off,
                       int32_t P, int32_t n_reg, int32_t n_feat, ProgData& pd) {
    if (P < 0) return fail(GP_E_INVAL, "n_prog < 0");
    if (P > 0 && (!code || !off)) return fail(GP_E_INVAL, "null program array");
    if (n_reg < 1 || n_reg > GP_MAX_REG) return fail(GP_E_INVAL, "n_reg %d outside [1, %d]", n_reg, GP_MAX_REG);
    if (n_feat < 1 || n_reg + n_feat > GP_SRC_CONST)
        return fail(GP_E_INVAL, "n_feat %d: registers plus features must stay below %d", n_feat, GP_SRC_CONST);
    pd = ProgData();
    pd.form = FORM_LINEAR;
    pd.n_prog = P;
    pd.n_feat = n_feat;
    pd.n_reg = n_reg;
    if (P == 0) return GP_OK;
    if (off[0] != 0) return fail(GP_E_INVAL, "off[0] must be 0");
    if (cst_off && cst_off[0] != 0) return fail(GP_E_INVAL, "cst_off[0] must be 0");
    int64_t total = 0;
    for (int32_t p = 0; p < P; p++) {
        const int64_t n = off[p + 1] - off[p];
        const int64_t nc = cst_off ? cst_off[p + 1] - cst_off[p] : 0;
        if (n < 1) return fail(GP_E_INVAL, "program %d is empty", p);
        if (n > GP_MAX_LEN) return fail(GP_E_DEPTH, "program %d: %lld instructions exceeds %d", p, (long long)n, GP_MAX_LEN);
        if (nc < 0 || nc > 256 - GP_SRC_CONST) return fail(GP_E_INVAL, "program %d: %lld constants", p, (long long)nc);
        if (nc > 0 && !cst) return fail(GP_E_INVAL, "null constant array");
        total += n + nc;
    }
    if (total > 0xFFFFFFFFll) return fail(GP_E_INVAL, "programs exceed 2^32 device words");
    pd.code.resize((size_t)total);
    pd.progs.resize(P);
    pd.cost.resize(P);
    int64_t w = 0;
    int32_t max_feat = std::min(n_feat, n_reg) - 1;  // registers start from these features
    char err[256];
    for (int32_t p = 0; p < P; p++) {
        const int64_t n = off[p + 1] - off[p];
        const int64_t nc = cst_off ? cst_off[p + 1] - cst_off[p] : 0;
        const uint32_t* src = code + off[p];
        int rc = check_linear(src, n, nc, n_reg, n_feat, err);
        if (rc != GP_OK) return fail((gp_status)rc, "program %d: %s", p, err);
        uint32_t cost = 0;
        for (int64_t i = 0; i < n; i++) {
            const uint32_t wd = src[i];
            const int op = wd & 0xFF;
            cost += op_cost(op, OPSET_REAL);
            const bool unary = op >= GP_SIN && op <= GP_PLOG;
            pd.n_transc += unary;
            const int na = unary ? 1 : 2;
            for (int q = 0; q < na; q++) {
                const int id = (int)((wd >> (16 + 8 * q)) & 0xFF);
                if (id >= n_reg && id < GP_SRC_CONST) max_feat = std::max(max_feat, id - n_reg);
            }
        }
        memcpy(pd.code.data() + w, src, sizeof(uint32_t) * (size_t)n);
        if (nc) memcpy(pd.code.data() + w + n, cst + cst_off[p], sizeof(float) * (size_t)nc);
        DevProg& d = pd.progs[p];
        d.code_off = (uint32_t)w;
        d.len = (uint32_t)n;
        d.meta = FORM_LINEAR | ((uint32_t)n_reg << 8);
        d.reserved0 = 0;
        d.reserved1 = 0;
        d.row = (uint64_t)p;
        pd.cost[p] = cost + 16;
        pd.n_instr += n;
        pd.n_gpop += n;
        w += n + nc;
    }
    pd.n_load = max_feat + 1;
    return GP_OK;
}

// Programs sorted by cost (longest first) and dealt to G groups in snake
// order, so every group carries about the same work.
static void make_groups(const ProgData& pd, int32_t G, std::vector<uint32_t>& order,
                        std::vector<uint32_t>& goff) {
    const int32_t P = pd.n_prog;
    std::vector<uint32_t> idx(P);
    std::iota(idx.begin(), idx.end(), 0u);
    std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) { return pd.cost[a] > pd.cost[b]; });
    std::vector<std::vector<uint32_t>> g(G);
    for (int32_t i = 0; i < P; i++) {
        const int32_t r = i / G, k = i % G;
        g[(r & 1) ? G - 1 - k : k].push_back(idx[i]);
    }
    order.clear();
    goff.assign(1, 0);
    for (int32_t k = 0; k < G; k++) {
        order.insert(order.end(), g[k].begin(), g[k].end());
        goff.push_back((uint32_t)order.size());
    }
}

// Translate and upload the programs for variant vi (when `fresh` or not yet
// uploaded) and the group layout for G groups (when not cached), all in one
// staging pass on stream s, then record dp.ready on s.  One-shot calls
// (`fresh`) keep a single group layout, replaced on every call.  G <= 0:
// programs only.
static gp_status prepare_programs(const ProgData& pd, int vi, DevProgs& dp, bool fresh, int32_t G, hipStream_t s,
                                  Workspace& w, const uint32_t** order, const uint32_t** goff) {
    std::vector<uint32_t> code, o, g;
    std::vector<DevProg> progs;
    gp_status st;
    const bool upload = fresh || !dp.uploaded;
    if (!upload && dp.ready) {
        // uploaded earlier, possibly on another stream: order this launch after it
        hipError_t e = hipStreamWaitEvent(s, dp.ready, 0);
        if (e != hipSuccess) return fail(GP_E_DEVICE, "hipStreamWaitEvent: %s", hipGetErrorString(e));
    }
    if (upload && (st = core_translate(pd, vi, code, progs)) != GP_OK) return st;
    DevBuf* gb = nullptr;
    int64_t n_order = 0;
    if (fresh) {
        gb = &dp.groups_once;
    } else {
        auto it = dp.groups_by_G.find(G);
        if (it != dp.groups_by_G.end()) {
            gb = &it->second.second;
            n_order = it->second.first;
        }
    }
    const bool new_groups = G > 0 && (fresh || gb == nullptr);
    if (new_groups) {
        make_groups(pd, G, o, g);
        n_order = (int64_t)o.size();
        if (!fresh) gb = &dp.groups_by_G.emplace(G, std::make_pair(n_order, DevBuf())).first->second.second;
        if ((st = gb->reserve((o.size() + g.size()) * 4)) != GP_OK) return st;
    }
    if (upload || new_groups) {
        if (upload) {
            if ((st = dp.code.reserve(std::max<size_t>(16, code.size() * 4))) != GP_OK) return st;
            if ((st = dp.progs.reserve(std::max<size_t>(1, progs.size()) * sizeof(DevProg))) != GP_OK) return st;
        }
        const size_t bytes = code.size() * 4 + progs.size() * sizeof(DevProg) + (o.size() + g.size()) * 4 + 1024;
        if ((st = w.staging.begin(bytes)) != GP_OK) return st;
        if (upload) {
            if ((st = w.staging.put(code.data(), code.size() * 4, dp.code.p, s)) != GP_OK) return st;
            if ((st = w.staging.put(progs.data(), progs.size() * sizeof(DevProg), dp.progs.p, s)) != GP_OK) return st;
        }
        if (new_groups) {
            if ((st = w.staging.put(o.data(), o.size() * 4, gb->p, s)) != GP_OK) return st;
            if ((st = w.staging.put(g.data(), g.size() * 4, (uint32_t*)gb->p + o.size(), s)) != GP_OK) return st;
        }
        if ((st = w.staging.end(s)) != GP_OK) return st;
        if (!dp.ready) {
            hipError_t e = hipEventCreateWithFlags(&dp.ready, hipEventDisableTiming);
            if (e != hipSuccess) return fail(GP_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
        }
        hipError_t e = hipEventRecord(dp.ready, s);
        if (e != hipSuccess) return fail(GP_E_DEVICE, "hipEventRecord: %s", hipGetErrorString(e));
        dp.uploaded = true;
    }
    if (order) *order = gb ? (const uint32_t*)gb->p : nullptr;
    if (goff) *goff = gb ? (const uint32_t*)gb->p + n_order : nullptr;
    return GP_OK;
}

// Launch shape of one evaluation.  Programs are dealt into G groups of
// about `group_instr` core instructions; each block runs four groups (one
// per wave) on a chunk of tiles_per_wave tiles.  Chunks lengthen only while
// four times `target_blocks` blocks remain; with few tiles, groups are made
// smaller instead, down to one program, so the chip still fills.  (Group
// size and chunk length were chosen by sweeps on the 4096-program tree and
// linear workloads.)
struct LaunchShape {
    int32_t G, tiles_per_wave, chunks;
};

static int32_t env_int(const char* name, int32_t dflt) {
    const char* v = getenv(name);
    if (!v || !*v) return dflt;
    const long x = strtol(v, nullptr, 10);
    return x > 0 && x < (1L << 30) ? (int32_t)x : dflt;
}

int32_t code_prefetch() {
    // GP2D_CODE_PREFETCH: 0 = no burst load, n = n loads in flight (at most 15, the scalar
    // memory counter's limit), unset = 15 (measured best: 2-3 % faster than 8 on the
    // interpreter-bound workloads)
    const char* v = getenv("GP2D_CODE_PREFETCH");
    if (!v || !*v) return 15;
    const long n = strtol(v, nullptr, 10);
    return n <= 0 ? 0 : (n > 15 ? 15 : (int32_t)n);
}

static LaunchShape launch_shape(const ProgData& pd, int32_t tiles, const EvalOptions* opt, int32_t force_G = 0) {
    // Program groups of about 1024 core instructions when the programs read at most 12 features, else
    // 4096: every wave loads the features of its tile before it runs its group, and a longer group
    // spreads those loads over more instructions.  Measured on the 4096-program workloads (kernel
    // time, 4096 against 1024): 8-feature trees 7 % (sin/cos/exp/log) and 1.5 % (+, -, *) slower,
    // 9-feature classification trees 2.7 % slower; 16-feature linear programs 2 %, 20-input
    // multiplexer trees 2.4 % and 41-feature classification trees 6 % faster.
    const bool few_feat = pd.n_load <= 12;
    const int32_t group_instr =
        opt && opt->group_instr > 0 ? opt->group_instr : env_int("GP2D_GROUP_INSTR", few_feat ? 1024 : 4096);
    const int32_t target_blocks = opt && opt->target_blocks > 0 ? opt->target_blocks : env_int("GP2D_TARGET_BLOCKS", 4096);
    int64_t G = (pd.n_instr + group_instr - 1) / group_instr;
    if (((G + 3) / 4) * tiles < target_blocks) G = 4 * ((target_blocks + tiles - 1) / tiles);
    G = std::max<int64_t>(1, std::min<int64_t>(G, pd.n_prog));
    if (force_G > 0) G = force_G;
    const int64_t quads = (G + 3) / 4;
    int32_t tpw = opt && opt->tiles_per_wave > 0 ? opt->tiles_per_wave : env_int("GP2D_TILES_PER_WAVE", 0);
    if (tpw <= 0) {
        tpw = 1;
        while (tpw < 16 && quads * ((tiles + 2 * tpw - 1) / (2 * tpw)) >= 4 * (int64_t)target_blocks) tpw *= 2;
    }
    LaunchShape L;
    L.G = (int32_t)G;
    L.tiles_per_wave = tpw;
    L.chunks = (int32_t)((tiles + tpw - 1) / tpw);
    return L;
}

// ---------------------------------------------------------------------------
// Kernel timing
// ---------------------------------------------------------------------------
static std::mutex g_tm_mu;
static bool g_tm_on = false;
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_tm_events;
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_tm_free;

hipError_t timed_launch_begin(hipStream_t s, int* slot) {
    *slot = -1;
    std::lock_guard<std::mutex> g(g_tm_mu);
    if (!g_tm_on) return hipSuccess;
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (!g_tm_free.empty()) {
        ev = g_tm_free.back();
        g_tm_free.pop_back();
    } else {
        hipError_t e = hipEventCreate(&ev.first);
        if (e != hipSuccess) return e;
        e = hipEventCreate(&ev.second);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(ev.first, s);
    if (e != hipSuccess) return e;
    g_tm_events.push_back(ev);
    *slot = (int)g_tm_events.size() - 1;
    return hipSuccess;
}

hipError_t timed_launch_end(hipStream_t s, int slot) {
    if (slot < 0) return hipSuccess;
    std::lock_guard<std::mutex> g(g_tm_mu);
    return hipEventRecord(g_tm_events[slot].second, s);
}

int32_t base_groups(const ProgData& pd) { return launch_shape(pd, 1 << 30, nullptr).G; }

int default_variant(const ProgData& pd) {
    return pick_core_variant(pd.n_load, pd.max_depth, pd.n_instr ? (double)pd.n_transc / pd.n_instr : 0.0,
                             pd.n_transc > 0, pd.opset == OPSET_BOOL, pd.form == FORM_TREE);
}

// The variant an evaluation without an explicit one launches: GP2D_VARIANT
// (tuning: a kernel variant index + 1) when that variant can hold the
// programs, else the default.
static int tuned_variant(const ProgData& pd) {
    const int32_t ev = env_int("GP2D_VARIANT", 0) - 1;
    if (ev >= 0 && ev < core_variants() && core_variant_nf(ev) >= pd.n_load && core_variant_d(ev) >= pd.max_depth &&
        !(core_variant_arith(ev) && pd.n_transc > 0) && core_variant_bool(ev) == (pd.opset == OPSET_BOOL) &&
        !(core_variant_trees_only(ev) && pd.form != FORM_TREE))
        return ev;
    return default_variant(pd);
}

gp_status eval_core(const ProgData& pd, std::map<int, DevProgs>& dps, bool fresh, const float* X, int32_t n_feat,
                    int64_t N, const float* y, int32_t kind, void* out, hipStream_t s, Workspace* w,
                    const EvalOptions* opt, int64_t n_bits) {
    if (!X) return fail(GP_E_INVAL, "X is null");
    if (!out) return fail(GP_E_INVAL, "out is null");
    if (N < 1) return fail(GP_E_INVAL, "n_cases must be >= 1");
    if (kind < GP_FIT_SUM_ABS || kind > GP_FIT_CLASS_ERR) return fail(GP_E_INVAL, "unknown fitness kind %d", kind);
    if (kind != GP_OUT_CASES && !y) return fail(GP_E_INVAL, "y is null");
    if (n_feat < pd.n_feat) return fail(GP_E_INVAL, "case matrix has %d features, programs need %d", n_feat, pd.n_feat);
    if (pd.n_prog == 0) return GP_OK;
    if (pd.n_load > GP_MAX_FEAT)
        return fail(GP_E_INVAL, "programs read feature %d; at most %d features are supported", pd.n_load - 1, GP_MAX_FEAT);
    const bool boolean = pd.opset == OPSET_BOOL;
    if (boolean != (n_bits > 0)) return fail(GP_E_INVAL, "internal: Boolean programs need a bit count");
    if (boolean && kind != GP_FIT_HITS && kind != GP_OUT_CASES)
        return fail(GP_E_INVAL, "Boolean programs take GP_FIT_HITS or GP_OUT_CASES, not kind %d", kind);
    const int vi = opt && opt->variant >= 0 ? opt->variant
                   : opt && opt->no_alloc   ? default_variant(pd)
                                            : tuned_variant(pd);
    if (vi < 0 || vi >= core_variants())
        return fail(GP_E_DEPTH, "no kernel variant for %d features and depth %d", pd.n_load, pd.max_depth);
    if (core_variant_nf(vi) < pd.n_load || core_variant_d(vi) < pd.max_depth ||
        (core_variant_arith(vi) && pd.n_transc > 0) || core_variant_bool(vi) != boolean ||
        (core_variant_trees_only(vi) && pd.form != FORM_TREE))
        return fail(GP_E_INVAL, "variant %d cannot hold these programs", vi);
    const bool no_alloc = opt && opt->no_alloc;
    gp_status st;
    if (no_alloc) {
        if (!core_is_ready(vi)) return fail(GP_E_DEVICE, "kernel variant %d is not set up on this device", vi);
    } else if ((st = core_ready(vi, s)) != GP_OK) {
        return st;
    }
    auto dit = dps.find(vi);
    if (no_alloc && dit == dps.end()) return fail(GP_E_INVAL, "programs are not on the device for variant %d", vi);
    DevProgs& dp = no_alloc ? dit->second : dps[vi];
    const int T = core_variant_t(vi);
    const int64_t tiles64 = (N + 64LL * T - 1) / (64LL * T);
    if (tiles64 > (1LL << 30)) return fail(GP_E_INVAL, "n_cases too large");
    const int32_t tiles = (int32_t)tiles64;
    const LaunchShape L = launch_shape(pd, tiles, opt, no_alloc ? opt->groups : 0);
    const int32_t G = L.G;
    const int32_t same_group = env_int("GP2D_SAME_GROUP", 0) > 0 ? 1 : 0;
    const int64_t units = same_group ? (int64_t)G * ((L.chunks + 3) / 4) : (int64_t)L.chunks * ((G + 3) / 4);
    if (units > (1LL << 31) - 64) return fail(GP_E_INVAL, "too many work units");
    const int64_t n_blocks = (N + 255) / 256;
    const size_t part_bytes = kind == GP_OUT_CASES ? 0 : (size_t)n_blocks * pd.n_prog * sizeof(double);
    const uint32_t *order, *goff;
    double* partials = nullptr;
    if (no_alloc) {
        auto git = dp.groups_by_G.find(G);
        if (!dp.uploaded || git == dp.groups_by_G.end() || !dp.ready)
            return fail(GP_E_INVAL, "programs or their group layout are not on the device");
        if (part_bytes > opt->partials_bytes)
            return fail(GP_E_NOMEM, "%lld programs x %lld blocks of 256 cases need %zu bytes of partial sums; "
                        "this entry point has %zu", (long long)pd.n_prog, (long long)n_blocks, part_bytes,
                        opt->partials_bytes);
        hipError_t e = hipStreamWaitEvent(s, dp.ready, 0);
        if (e != hipSuccess) return fail(GP_E_DEVICE, "hipStreamWaitEvent: %s", hipGetErrorString(e));
        order = (const uint32_t*)git->second.second.p;
        goff = order + git->second.first;
        partials = opt->partials;
    } else {
        if (!w) return fail(GP_E_INVAL, "internal: no workspace");
        if ((st = prepare_programs(pd, vi, dp, fresh, G, s, *w, &order, &goff)) != GP_OK) return st;
        if (part_bytes && (st = w->partials.reserve(part_bytes)) != GP_OK) return st;
        partials = (double*)w->partials.p;
    }
    CoreArgs a;
    memset(&a, 0, sizeof a);
    a.code = (const uint32_t*)dp.code.p;
    a.progs = (const DevProg*)dp.progs.p;
    a.order = order;
    a.group_off = goff;
    a.X = X;
    a.y = kind == GP_OUT_CASES ? nullptr : y;
    a.N = N;
    a.n_load = pd.n_load;
    a.kind = kind;
    a.tiles = tiles;
    a.n_units = (int32_t)units;
    a.tiles_per_wave = L.tiles_per_wave;
    a.chunks = L.chunks;
    a.prefetch = code_prefetch();
    a.n_groups = G;
    a.same_group = same_group;
    a.n_bits = n_bits;
    a.partials = partials;
    a.cases_out = kind == GP_OUT_CASES ? (float*)out : nullptr;
    uint32_t blocks = (uint32_t)units;
    blocks = (blocks + 7u) & ~7u;
    int slot = -1;
    hipError_t e = no_alloc ? hipSuccess : timed_launch_begin(s, &slot);
    if (e == hipSuccess) e = core_launch(vi, a, blocks, s);
    if (e == hipSuccess) e = timed_launch_end(s, slot);
    if (e != hipSuccess) return fail(GP_E_DEVICE, "evaluation launch: %s", hipGetErrorString(e));
    if (kind == GP_OUT_CASES) return GP_OK;
    ReduceArgs r;
    memset(&r, 0, sizeof r);
    r.partials = partials;
    r.part_base = 0;
    r.n_prog = pd.n_prog;
    r.N = N;
    r.out = out;
    r.blocks = (int32_t)n_blocks;
    r.kind = kind;
    e = core_reduce_one(r, s);
    if (e != hipSuccess) return fail(GP_E_DEVICE, "reduction launch: %s", hipGetErrorString(e));
    return GP_OK;
}

}  // namespace gpx

// ===========================================================================
// C ABI
// ===========================================================================
using namespace gpx;

struct gp_progset {
    ProgData pd;
    std::map<int, DevProgs> dps;   // translated per core variant
    int32_t groups = 0;            // the group layout uploaded at creation
    std::mutex mu;
};

// Evaluate a program set with nothing allocated or uploaded (see runtime.h).
gp_status gpx::progset_eval_no_alloc(gp_progset* ps, const float* X, int32_t n_feat, int64_t n_cases, const float* y,
                                int32_t kind, void* out, hipStream_t s, double* partials, size_t partials_bytes) {
    if (!ps) return fail(GP_E_INVAL, "ps is null");
    std::lock_guard<std::mutex> g(ps->mu);
    EvalOptions o;
    o.no_alloc = true;
    o.groups = ps->groups;
    o.partials = partials;
    o.partials_bytes = partials_bytes;
    if (ps->pd.opset == OPSET_BOOL) {
        if (n_cases < 1) return fail(GP_E_INVAL, "n_cases must be >= 1");
        if (n_cases > 0x7FFFFFFF) return fail(GP_E_INVAL, "n_cases above 2^31 - 1 (hit counts are int32)");
        return eval_core(ps->pd, ps->dps, false, X, n_feat, (n_cases + 31) / 32, y, kind, out, s, nullptr, &o,
                         n_cases);
    }
    return eval_core(ps->pd, ps->dps, false, X, n_feat, n_cases, y, kind, out, s, nullptr, &o);
}

extern "C" {

const char* gp_last_error(void) { return last_error(); }

const char* gp_version(void) { return "gp2d 0.1 (gfx950)"; }

gp_status gp_eval_tree(const int32_t* tok, const float* cst, const int64_t* off, int32_t n_prog,
                       const float* X, int32_t n_feat, int64_t n_cases, const float* y, int32_t kind,
                       void* out, void* stream) {
    clear_error();
    ProgData pd;
    gp_status st = build_tree(tok, cst, off, n_prog, n_feat, pd);
    if (st != GP_OK || n_prog == 0) return st;
    hipStream_t s = (hipStream_t)stream;
    Workspace& w = workspace(s);
    std::lock_guard<std::mutex> g(w.mu);
    return eval_core(pd, w.oneshot, true, X, n_feat, n_cases, y, kind, out, s, &w, nullptr);
}

gp_status gp_eval_linear(const uint32_t* code, const int64_t* off, const float* cst, const int64_t* cst_off,
                         int32_t n_prog, int32_t n_reg, const float* X, int32_t n_feat, int64_t n_cases,
                         const float* y, int32_t kind, void* out, void* stream) {
    clear_error();
    ProgData pd;
    gp_status st = build_linear(code, off, cst, cst_off, n_prog, n_reg, n_feat, pd);
    if (st != GP_OK || n_prog == 0) return st;
    hipStream_t s = (hipStream_t)stream;
    Workspace& w = workspace(s);
    std::lock_guard<std::mutex> g(w.mu);
    return eval_core(pd, w.oneshot, true, X, n_feat, n_cases, y, kind, out, s, &w, nullptr);
}

gp_status gp_eval_bool(const int32_t* tok, const int64_t* off, int32_t n_prog, const uint32_t* X, int32_t n_feat,
                       int64_t n_cases, const uint32_t* y, int32_t kind, void* out, void* stream) {
    clear_error();
    if (n_cases < 1) return fail(GP_E_INVAL, "n_cases must be >= 1");
    if (n_cases > 0x7FFFFFFF) return fail(GP_E_INVAL, "n_cases above 2^31 - 1 (hit counts are int32)");
    if (kind != GP_FIT_HITS && kind != GP_OUT_CASES)
        return fail(GP_E_INVAL, "Boolean programs take GP_FIT_HITS or GP_OUT_CASES, not kind %d", kind);
    ProgData pd;
    gp_status st = build_tree(tok, nullptr, off, n_prog, n_feat, pd, OPSET_BOOL);
    if (st != GP_OK || n_prog == 0) return st;
    hipStream_t s = (hipStream_t)stream;
    Workspace& w = workspace(s);
    std::lock_guard<std::mutex> g(w.mu);
    // one slot per 32-bit word: the kernel sees n_words "cases"
    const int64_t n_words = (n_cases + 31) / 32;
    return eval_core(pd, w.oneshot, true, (const float*)X, n_feat, n_words, (const float*)y, kind, out, s, &w,
                     nullptr, n_cases);
}

static gp_status progset_finish(ProgData&& pd, void* stream, gp_progset** ps) {
    // Translate the programs for the kernel variant evaluations will use and
    // upload them on `stream` now; an evaluation on any stream waits for it.
    std::unique_ptr<gp_progset> p(new gp_progset());
    p->pd = std::move(pd);
    if (p->pd.n_prog > 0) {
        const int vi = default_variant(p->pd);
        if (vi < 0) return fail(GP_E_DEPTH, "no kernel variant for %d features and depth %d", p->pd.n_load,
                                p->pd.max_depth);
        hipStream_t s = (hipStream_t)stream;
        gp_status st;
        if ((st = core_ready(vi, s)) != GP_OK) return st;
        Workspace& w = workspace(s);
        std::lock_guard<std::mutex> g(w.mu);
        p->groups = base_groups(p->pd);
        if ((st = prepare_programs(p->pd, vi, p->dps[vi], false, p->groups, s, w, nullptr, nullptr)) != GP_OK)
            return st;
    }
    *ps = p.release();
    return GP_OK;
}

gp_status gp_progset_tree(const int32_t* tok, const float* cst, const int64_t* off, int32_t n_prog,
                          int32_t n_feat, void* stream, gp_progset** ps) {
    clear_error();
    if (!ps) return fail(GP_E_INVAL, "ps is null");
    ProgData pd;
    gp_status st = build_tree(tok, cst, off, n_prog, n_feat, pd);
    if (st != GP_OK) return st;
    return progset_finish(std::move(pd), stream, ps);
}

gp_status gp_progset_bool(const int32_t* tok, const int64_t* off, int32_t n_prog, int32_t n_feat, void* stream,
                          gp_progset** ps) {
    clear_error();
    if (!ps) return fail(GP_E_INVAL, "ps is null");
    ProgData pd;
    gp_status st = build_tree(tok, nullptr, off, n_prog, n_feat, pd, OPSET_BOOL);
    if (st != GP_OK) return st;
    return progset_finish(std::move(pd), stream, ps);
}

gp_status gp_progset_linear(const uint32_t* code, const int64_t* off, const float* cst,
                            const int64_t* cst_off, int32_t n_prog, int32_t n_reg, int32_t n_feat,
                            void* stream, gp_progset** ps) {
    clear_error();
    if (!ps) return fail(GP_E_INVAL, "ps is null");
    ProgData pd;
    gp_status st = build_linear(code, off, cst, cst_off, n_prog, n_reg, n_feat, pd);
    if (st != GP_OK) return st;
    return progset_finish(std::move(pd), stream, ps);
}

gp_status gp_progset_eval(gp_progset* ps, const float* X, int32_t n_feat, int64_t n_cases, const float* y,
                          int32_t kind, void* out, void* stream) {
    clear_error();
    if (!ps) return fail(GP_E_INVAL, "ps is null");
    hipStream_t s = (hipStream_t)stream;
    Workspace& w = workspace(s);
    std::lock_guard<std::mutex> g(w.mu);
    std::lock_guard<std::mutex> g2(ps->mu);
    if (ps->pd.opset == OPSET_BOOL) {
        // Boolean set: X and y are 32-bit words, n_cases counts bits
        if (n_cases < 1) return fail(GP_E_INVAL, "n_cases must be >= 1");
        if (n_cases > 0x7FFFFFFF) return fail(GP_E_INVAL, "n_cases above 2^31 - 1 (hit counts are int32)");
        return eval_core(ps->pd, ps->dps, false, X, n_feat, (n_cases + 31) / 32, y, kind, out, s, &w, nullptr,
                         n_cases);
    }
    return eval_core(ps->pd, ps->dps, false, X, n_feat, n_cases, y, kind, out, s, &w, nullptr);
}

gp_status gp_progset_get_info(const gp_progset* ps, gp_progset_info* info) {
    clear_error();
    if (!ps || !info) return fail(GP_E_INVAL, "null argument");
    info->n_prog = ps->pd.n_prog;
    info->form = ps->pd.form;
    info->n_feat = ps->pd.n_feat;
    info->max_depth = ps->pd.max_depth;
    info->n_instr = ps->pd.n_instr;
    info->n_gpop = ps->pd.n_gpop;
    info->variant = tuned_variant(ps->pd);
    info->pad = 0;
    return GP_OK;
}

gp_status gp_progset_destroy(gp_progset* ps) {
    clear_error();
    if (!ps) return GP_OK;
    for (auto& kv : ps->dps) kv.second.release();
    delete ps;
    return GP_OK;
}

static gp_status core_lower_common(ProgData& pd, int32_t variant, uint64_t table_base, uint32_t* words,
                                   int64_t max_words, int64_t* prog_off, int64_t* n_words) {
    std::vector<uint32_t> code;
    std::vector<DevProg> progs;
    gp_status st = core_translate_at(pd, variant, table_base, code, progs);
    if (st != GP_OK) return st;
    if (n_words) *n_words = (int64_t)code.size();
    if (words) {
        if (max_words < (int64_t)code.size()) return fail(GP_E_INVAL, "words buffer too small");
        memcpy(words, code.data(), code.size() * 4);
    }
    if (prog_off) {
        for (int32_t p = 0; p < pd.n_prog; p++) prog_off[p] = progs[p].code_off;
        prog_off[pd.n_prog] = (int64_t)code.size();
    }
    return GP_OK;
}

gp_status gp_core_lower_tree(const int32_t* tok, const float* cst, const int64_t* off, int32_t n_prog, int32_t n_feat,
                             int32_t variant, uint64_t table_base, uint32_t* words, int64_t max_words,
                             int64_t* prog_off, int64_t* n_words) {
    clear_error();
    if (variant < 0 || variant >= core_variants()) return fail(GP_E_INVAL, "variant %d does not exist", variant);
    // a Boolean kernel takes trees of the Boolean function set
    ProgData pd;
    gp_status st = build_tree(tok, cst, off, n_prog, n_feat, pd, core_variant_bool(variant) ? OPSET_BOOL : OPSET_REAL);
    if (st != GP_OK) return st;
    return core_lower_common(pd, variant, table_base, words, max_words, prog_off, n_words);
}

gp_status gp_core_lower_linear(const uint32_t* code, const int64_t* off, const float* cst, const int64_t* cst_off,
                               int32_t n_prog, int32_t n_reg, int32_t n_feat, int32_t variant, uint64_t table_base,
                               uint32_t* words, int64_t max_words, int64_t* prog_off, int64_t* n_words) {
    clear_error();
    if (variant < 0 || variant >= core_variants()) return fail(GP_E_INVAL, "variant %d does not exist", variant);
    if (core_variant_trees_only(variant)) return fail(GP_E_INVAL, "variant %d runs trees only", variant);
    ProgData pd;
    gp_status st = build_linear(code, off, cst, cst_off, n_prog, n_reg, n_feat, pd);
    if (st != GP_OK) return st;
    return core_lower_common(pd, variant, table_base, words, max_words, prog_off, n_words);
}

gp_status gp_timing_enable(int on) {
    clear_error();
    std::lock_guard<std::mutex> g(g_tm_mu);
    g_tm_on = on != 0;
    return GP_OK;
}

gp_status gp_timing_read(int64_t* launches, double* total_ms, int reset) {
    clear_error();
    std::lock_guard<std::mutex> g(g_tm_mu);
    double ms = 0.0;
    for (auto& ev : g_tm_events) {
        hipError_t e = hipEventSynchronize(ev.second);
        if (e != hipSuccess) return fail(GP_E_DEVICE, "hipEventSynchronize: %s", hipGetErrorString(e));
        float t = 0.0f;
        e = hipEventElapsedTime(&t, ev.first, ev.second);
        if (e != hipSuccess) return fail(GP_E_DEVICE, "hipEventElapsedTime: %s", hipGetErrorString(e));
        ms += t;
    }
    if (launches) *launches = (int64_t)g_tm_events.size();
    if (total_ms) *total_ms = ms;
    if (reset) {
        g_tm_free.insert(g_tm_free.end(), g_tm_events.begin(), g_tm_events.end());
        g_tm_events.clear();
    }
    return GP_OK;
}

gp_status gp_lower_tree(const int32_t* tok, const float* cst, int64_t n, int32_t n_feat, uint32_t* words,
                        int64_t max_words, gp_lower_stats* stats) {
    clear_error();
    if (!tok || !cst) return fail(GP_E_INVAL, "null program");
    if (n_feat < 1) return fail(GP_E_INVAL, "n_feat < 1");
    if (n > GP_MAX_LEN) return fail(GP_E_DEPTH, "program of %lld nodes exceeds %d", (long long)n, GP_MAX_LEN);
    std::vector<uint32_t> buf(2 * (size_t)std::max<int64_t>(n, 1));
    TreeLowering st;
    char err[256];
    int rc = lower_tree(tok, cst, n, n_feat, buf.data(), &st, err);
    if (rc != GP_OK) return fail((gp_status)rc, "%s", err);
    if (words) {
        if (max_words < 2 * (int64_t)st.n_instr) return fail(GP_E_INVAL, "words buffer too small");
        memcpy(words, buf.data(), sizeof(uint32_t) * 2 * (size_t)st.n_instr);
    }
    if (stats) {
        stats->n_nodes = st.n_nodes;
        stats->n_instr = st.n_instr;
        stats->max_depth = st.max_depth;
        stats->stack_fetches = st.stack_fetches;
        stats->n_values = st.n_values;
        stats->n_reversed = st.n_reversed;
    }
    return GP_OK;
}

}  // extern "C"
