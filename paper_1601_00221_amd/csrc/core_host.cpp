// Host side of the interpreter core: find each kernel variant's handler
// table on the device, and translate lowered programs into core
// instructions (handler address, operand offsets, constant).
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/gp.h"
#include "core_host.h"
#include "core_kernels.h"
#include "gp_internal.h"
#include "runtime.h"

namespace gpx {
#include "core_gen.inc"

namespace {

// Handler slot by key: an open-addressing table (a few thousand keys, one
// lookup per translated instruction).
struct SlotTable {
    std::vector<uint32_t> keys;   // 0xFFFFFFFF = empty (no handler key has it)
    std::vector<uint16_t> slots;
    uint32_t mask = 0;
    static uint32_t hash(uint32_t k) { return (k * 0x9E3779B1u) ^ (k >> 15); }
    void build(const std::vector<std::pair<uint32_t, uint16_t>>& kv) {
        uint32_t cap = 16;
        while (cap < 2 * kv.size()) cap <<= 1;
        keys.assign(cap, 0xFFFFFFFFu);
        slots.assign(cap, 0);
        mask = cap - 1;
        for (auto& e : kv) {
            uint32_t i = hash(e.first) & mask;
            while (keys[i] != 0xFFFFFFFFu && keys[i] != e.first) i = (i + 1) & mask;
            keys[i] = e.first;
            slots[i] = e.second;
        }
    }
    bool find(uint32_t k, uint16_t* out) const {
        if (keys.empty()) return false;
        for (uint32_t i = hash(k) & mask;; i = (i + 1) & mask) {
            if (keys[i] == k) {
                *out = slots[i];
                return true;
            }
            if (keys[i] == 0xFFFFFFFFu) return false;
        }
    }
};

struct VariantMap {
    bool ready = false;
    int device = -1;
    uint64_t base = 0;
    SlotTable slot;
};

std::mutex g_mu;
std::vector<VariantMap> g_maps;

uint32_t key_of(int kind, int op, int p1, int p2) {
    return (uint32_t)kind | ((uint32_t)op << 8) | ((uint32_t)(uint8_t)(int8_t)p1 << 16) |
           ((uint32_t)(uint8_t)(int8_t)p2 << 24);
}

}  // namespace

static SlotTable variant_slots(int vi) {
    const CoreVariantDesc& v = kCoreVariants[vi];
    std::vector<std::pair<uint32_t, uint16_t>> kv;
    kv.reserve(v.n);
    for (int i = 0; i < v.n; i++)
        kv.push_back({key_of(v.keys[i].kind, v.keys[i].op, v.keys[i].p1, v.keys[i].p2), v.slots[i]});
    SlotTable t;
    t.build(kv);
    return t;
}

const CoreVariantDesc& core_desc(int vi) { return kCoreVariants[vi]; }
int core_variants() { return (int)(sizeof(kCoreVariants) / sizeof(kCoreVariants[0])); }
int core_reg_levels(int vi) {
    // Boolean kernels run trees only: no linear registers before the features
    const CoreVariantDesc& v = kCoreVariants[vi];
    return v.arith >= 2 || v.d > GPX_LIN_REGS ? v.d : GPX_LIN_REGS;
}

// Kernel modes (gen_core.py): 0 full, 1 without sin/cos/exp/log code, 2 Boolean, 3 trees only without
// sin/cos/exp/log code, 4 trees only with it.
static bool mode_no_transc(int mode) { return mode == 1 || mode == 2 || mode == 3; }

static constexpr int kShallowDepth = 12;

int pick_core_variant(int n_load, int depth, double transc_frac, bool has_transc, bool boolean, bool trees_only) {
    // Programs rich in sin/cos/exp/log (binary64, evaluated by compiled code
    // outside the core) run best with room for that code (no spills) and as
    // many waves per SIMD as that leaves, to hide its latency; the others with
    // the widest tile, on a kernel without that code if they use none of it.  Ties go to the fewest feature slots, then the fewest
    // handlers (least code).  (Measured on the 4096 x 65,536 tree workloads.)
    const bool heavy = transc_frac > 0.2;
    int best = -1;
    auto waves = [](const CoreVariantDesc& v) {
        const int lv = v.arith >= 2 || v.d > GPX_LIN_REGS ? v.d : GPX_LIN_REGS;
        const int vg = (v.ncv + lv * v.t + v.nf * v.t + 7) / 8 * 8;
        return 512 / vg;
    };
    auto score = [&](const CoreVariantDesc& v) {
        if (heavy) return (v.ncv >= 64) * 100000000 + waves(v) * 1000000 + v.t * 10000 - v.nf * 100 - v.n / 100;
        // trees-only kernels first (the smallest handler tables), then those without sin/cos/exp/log code, the
        // widest tile, then the most waves per SIMD (4 against 3 at T = 4: 13-16 % on the linear and Shuttle-shaped
        // workloads)
        return (v.arith == 3) * 400000000 + mode_no_transc(v.arith) * 200000000 + (v.ncv <= 64) * 100000000 + v.t * 10000 +
               waves(v) * 1000 - v.nf * 100 - v.n / 100;
    };
    // Boolean programs: the most slots in flight per SIMD (waves x tile width); ties go to more waves (they
    // hide the dispatch chain of the one-instruction handlers: measured 5 % on the 20-multiplexer), then to
    // more VGPRs for the compiled code, then to fewer feature slots
    auto score_bool = [&](const CoreVariantDesc& v) {
        return waves(v) * v.t * 100000 + waves(v) * 1000 + v.ncv * 10 - v.nf;
    };
    for (int i = 0; i < core_variants(); i++) {
        const CoreVariantDesc& v = kCoreVariants[i];
        if ((v.arith == 2) != boolean) continue;
        if (v.arith >= 3 && !trees_only) continue;
        if (v.nf < n_load || v.d < depth || (mode_no_transc(v.arith) && has_transc)) continue;
        // the deep variants (fewer waves per SIMD) serve only programs that need them
        if (v.d > kShallowDepth && depth <= kShallowDepth) continue;
        if (best < 0) { best = i; continue; }
        const bool better = boolean ? score_bool(v) > score_bool(kCoreVariants[best])
                                    : score(v) > score(kCoreVariants[best]);
        if (better) best = i;
    }
    return best;
}

gp_status core_ready(int vi, hipStream_t s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(GP_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> g(g_mu);
    if ((int)g_maps.size() < core_variants()) g_maps.resize(core_variants());
    VariantMap& m = g_maps[vi];
    if (m.ready && m.device == dev) return GP_OK;
    uint64_t* d = nullptr;
    e = hipMalloc(&d, 256);
    if (e != hipSuccess) return fail(GP_E_DEVICE, "hipMalloc: %s", hipGetErrorString(e));
    CoreArgs a;
    memset(&a, 0, sizeof a);
    a.probe = 1;
    a.probe_out = d;
    e = core_launch(vi, a, 1, s);
    uint64_t base = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&base, d, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(GP_E_DEVICE, "handler table probe: %s", hipGetErrorString(e));
    if (base == 0 || (base & (GPX_SLOT - 1)) != 0) return fail(GP_E_DEVICE, "handler table probe returned %llx",
                                                               (unsigned long long)base);
    m.slot = variant_slots(vi);
    m.base = base;
    m.device = dev;
    m.ready = true;
    return GP_OK;
}

bool core_is_ready(int vi) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> g(g_mu);
    return vi >= 0 && vi < (int)g_maps.size() && g_maps[vi].ready && g_maps[vi].device == dev;
}

namespace {

// Handlers come in two phases (records are fetched two at a time, see
// gen_core.py): instructions alternate A, B, A, ... and every entry into the
// core -- a program's start, the return from an exit -- begins with A.
constexpr int kPhaseB = 0x80;

// Writes core instructions (4 words each) to `out`, at most `cap` of them.
struct Emitter {
    const VariantMap& m;
    uint32_t* out;
    int64_t cap;
    char* err;
    int64_t n = 0;
    bool ok = true;
    int phase = 0;

    void put(int kind, int op, int p1, int p2, uint32_t pay, uint32_t cst) {
        uint16_t slot = 0;
        const bool have = m.slot.find(key_of(kind | phase, op, p1, p2), &slot);
        phase ^= kPhaseB;
        if (!have) {
            snprintf(err, 256, "no core handler for kind %d op %d (%d, %d)", kind, op, p1, p2);
            ok = false;
            return;
        }
        if (n >= cap) {
            snprintf(err, 256, "internal: core code longer than counted");
            ok = false;
            return;
        }
        const uint64_t addr = m.base + (uint64_t)slot * GPX_SLOT;
        uint32_t* o = out + 4 * n++;
        o[0] = (uint32_t)addr;
        o[1] = (uint32_t)(addr >> 32);
        o[2] = pay;
        o[3] = cst;
    }
    // leave the core: operation op on A (offset or constant), B, into D
    void exit(uint32_t op, int oa, int ob, int od, bool a_const, bool b_const, uint32_t cst) {
        const uint32_t fl = (a_const ? 1u : 0u) | (b_const ? 2u : 0u);
        put(CK_EXIT, 0, 0, 0,
            (uint32_t)(oa & 255) | ((uint32_t)(ob & 255) << 8) | ((uint32_t)(od & 255) << 16) |
                ((op | (fl << 4)) << 24),
            cst);
        phase = 0;   // the core is entered again after an exit
    }
    // protected division, in the core (every arithmetic kernel has its
    // handlers): the exit's payload layout, without leaving
    void fail_two_constants() {
        // lowering pushes one of two constant operands first, and register programs move one into the
        // destination: no function of two constants reaches the handlers
        snprintf(err, 256, "internal: a function of two constants reached core translation");
        ok = false;
    }
    void div(int oa, int ob, int od, bool a_const, bool b_const, uint32_t cst) {
        if (a_const && b_const) return fail_two_constants();
        const int kind = a_const ? CK_DCV : b_const ? CK_DVC : CK_DVV;
        put(kind, GP_PDIV, 0, 0,
            (uint32_t)(oa & 255) | ((uint32_t)(ob & 255) << 8) | ((uint32_t)(od & 255) << 16), cst);
    }
    // >, <, ==, logical AND and OR in the core: 1 or 0 per slot
    void cmp(uint32_t op, int oa, int ob, int od, bool a_const, bool b_const, uint32_t cst) {
        if (a_const && b_const) return fail_two_constants();
        const int kind = a_const ? CK_CCV : b_const ? CK_CVC : CK_CVV;
        put(kind, (int)op, 0, 0,
            (uint32_t)(oa & 255) | ((uint32_t)(ob & 255) << 8) | ((uint32_t)(od & 255) << 16), cst);
    }
    // the binary functions the arithmetic kernels apply in their own handlers: protected division and the
    // classification functions (sin/cos/exp/log are unary and leave the core)
    void apply(uint32_t op, bool boolean, int oa, int ob, int od, bool a_const, bool b_const, uint32_t cst) {
        if (!boolean && op == GP_PDIV) {
            div(oa, ob, od, a_const, b_const, cst);
        } else if (!boolean && (op == GP_GT || op == GP_LT || op == GP_EQ || op == GP_AND || op == GP_OR)) {
            cmp(op, oa, ob, od, a_const, b_const, cst);
        } else {
            snprintf(err, 256, "no core handler for binary function %u", op);
            ok = false;
        }
    }
};

// Functions the core applies itself: + - * and, in Boolean kernels, the four
// bitwise functions; the others leave the core (in arithmetic trees opcodes 8
// and 9 are the logical AND and OR, which are exits).
bool is_core_op(uint32_t op, bool boolean) {
    return op == GP_ADD || op == GP_SUB || op == GP_MUL || (boolean && op >= GP_AND && op <= GP_NOR);
}

}  // namespace

static int translate_tree(const uint32_t* w, int64_t n_instr, int vi, const VariantMap& m, uint32_t* out,
                          int64_t cap, int64_t* n_out, char* err) {
    const CoreVariantDesc& v = kCoreVariants[vi];
    const int T = v.t, FO = core_reg_levels(vi) * T;
    Emitter e{m, out, cap, err};
    for (int64_t i = 0; i < n_instr && e.ok; i++) {
        const uint32_t w0 = w[2 * i], c = w[2 * i + 1];
        const uint32_t op = w0 & 15u, mode = (w0 >> 4) & 15u;
        const int fa = (int)((w0 >> 8) & 255u), fb = (int)((w0 >> 16) & 255u), ha = (int)(w0 >> 24);
        int h;  // stack height before the instruction
        switch (mode) {
            case M_SS: case M_SSR: h = ha + 1; break;
            case M_S3: h = ha + 2; break;
            case M_XX: case M_XC: case M_CX: case M_X: case M_C: h = ha - 1; break;
            default: h = ha; break;
        }
        const int xa = FO + fa * T, xb = FO + fb * T;
        if (op == OP_PUSH) {
            if (mode == M_X) {
                // Boolean kernels push a variable only as a whole program, at the bottom
                if (v.arith == 2 && h != 0) {
                    snprintf(err, 256, "push of a variable above the stack bottom");
                    return GP_E_INVAL;
                }
                e.put(CK_PUSHX, 0, h, 0, (uint32_t)xa, 0);
            } else {
                e.put(CK_PUSHC, 0, 0, 0, (uint32_t)(h * T), c);
            }
            continue;
        }
        if (mode == M_S3) {
            // IF: operands at positions fa, fb and the third of s[h-3 .. h-1]; the exit writes
            // the lowest of the three offsets
            const int pc = 3 - fa - fb;
            if (op != OP_IF || fa > 2 || fb > 2 || pc < 0 || pc > 2 || fa == fb || h < 3) {
                snprintf(err, 256, "malformed three-operand instruction");
                return GP_E_INVAL;
            }
            // IF runs in the core: operands at three offsets, the result to the lowest, s[h-3]
            e.put(CK_IF3, GP_IF, 0, 0,
                  (uint32_t)((h - 3 + fa) * T) | ((uint32_t)((h - 3 + fb) * T) << 8) |
                      ((uint32_t)((h - 3 + pc) * T) << 16) | ((uint32_t)((h - 3) * T) << 24),
                  0);
            continue;
        }
        if (is_core_op(op, v.arith == 2)) {
            const bool comm = op != GP_SUB;
            switch (mode) {
                case M_SS: e.put(CK_SS, op, 0, 0, (uint32_t)((h - 2) * T), 0); break;
                case M_SSR:
                    if (comm) e.put(CK_SS, op, 0, 0, (uint32_t)((h - 2) * T), 0);
                    else e.put(CK_SSR, op, 0, 0, (uint32_t)((h - 2) * T), 0);
                    break;
                case M_SX: e.put(CK_SX, op, h - 1, 0, (uint32_t)xb, 0); break;
                case M_XS:
                    if (comm) e.put(CK_SX, op, h - 1, 0, (uint32_t)xa, 0);
                    else e.put(CK_XS, op, h - 1, 0, (uint32_t)xa, 0);
                    break;
                case M_SC: e.put(CK_SC, op, 0, 0, (uint32_t)((h - 1) * T), c); break;
                case M_CS:
                    if (comm) e.put(CK_SC, op, 0, 0, (uint32_t)((h - 1) * T), c);
                    else e.put(CK_CS, op, 0, 0, (uint32_t)((h - 1) * T), c);
                    break;
                case M_XX:
                    if (v.nf <= 8 && v.arith != 2) {   // (Boolean kernels have no one-pass XX handlers)
                        if (comm) {
                            const int a = fa < fb ? fa : fb, b = fa < fb ? fb : fa;
                            e.put(CK_XX, op, h, b - a, (uint32_t)(a * T), 0);
                        } else {
                            e.put(CK_XX, op, h, fb - fa, (uint32_t)(fa * T), 0);
                        }
                    } else {
                        e.put(CK_XX2, op, h, 0, (uint32_t)xa | ((uint32_t)xb << 8), 0);
                    }
                    break;
                case M_XC: e.put(CK_XC, op, h, 0, (uint32_t)xa, c); break;
                case M_CX:
                    if (comm) e.put(CK_XC, op, h, 0, (uint32_t)xb, c);
                    else e.put(CK_CX, op, h, 0, (uint32_t)xb, c);
                    break;
                default:
                    snprintf(err, 256, "mode %u is not a binary mode", mode);
                    return GP_E_INVAL;
            }
            continue;
        }
        // protected division has handlers of its own; the transcendentals and the classification
        // functions leave the core
        const bool bl = v.arith == 2;
        switch (mode) {
            case M_SS: e.apply(op, bl, (h - 2) * T, (h - 1) * T, (h - 2) * T, false, false, 0); break;
            case M_SSR: e.apply(op, bl, (h - 1) * T, (h - 2) * T, (h - 2) * T, false, false, 0); break;
            case M_SX: e.apply(op, bl, (h - 1) * T, xb, (h - 1) * T, false, false, 0); break;
            case M_XS: e.apply(op, bl, xa, (h - 1) * T, (h - 1) * T, false, false, 0); break;
            case M_SC: e.apply(op, bl, (h - 1) * T, 0, (h - 1) * T, false, true, c); break;
            case M_CS: e.apply(op, bl, 0, (h - 1) * T, (h - 1) * T, true, false, c); break;
            case M_XX: e.apply(op, bl, xa, xb, h * T, false, false, 0); break;
            case M_XC: e.apply(op, bl, xa, 0, h * T, false, true, c); break;
            case M_CX: e.apply(op, bl, 0, xb, h * T, true, false, c); break;
            case M_S: e.exit(op, (h - 1) * T, 0, (h - 1) * T, false, false, 0); break;
            case M_X: e.exit(op, xa, 0, h * T, false, false, 0); break;
            default: e.exit(op, 0, 0, h * T, true, false, c); break;  // M_C
        }
    }
    if (e.ok) e.exit(CORE_OP_END, 0, 0, 0, false, false, 0);
    *n_out = e.n;
    return e.ok ? GP_OK : GP_E_INVAL;
}

// Core instructions of a register program: the register set-up, one or two
// per instruction, and the end.
static int64_t linear_records(const uint32_t* w, int64_t n, int32_t n_reg) {
    int64_t k = n_reg + n + 1;
    for (int64_t i = 0; i < n; i++) {
        const uint32_t op = w[i] & 255u;
        const bool c1 = ((w[i] >> 16) & 255u) >= GP_SRC_CONST, c2 = (w[i] >> 24) >= GP_SRC_CONST;
        k += (c1 && c2 && !(op >= GP_SIN && op <= GP_PLOG));
    }
    return k;
}

static int translate_linear(const uint32_t* w, int64_t n, const uint32_t* cst, int32_t n_reg, int32_t n_feat, int vi,
                            const VariantMap& m, uint32_t* out, int64_t cap, int64_t* n_out, char* err) {
    const CoreVariantDesc& v = kCoreVariants[vi];
    const int T = v.t, FO = core_reg_levels(vi) * T;
    Emitter e{m, out, cap, err};
    auto off = [&](int id) { return id < n_reg ? id * T : FO + (id - n_reg) * T; };
    // registers start as r[k] = x[k mod n_feat]
    for (int k = 0; k < n_reg && e.ok; k++) e.put(CK_MOVX, 0, k, 0, (uint32_t)(FO + (k % n_feat) * T), 0);
    for (int64_t i = 0; i < n && e.ok; i++) {
        const uint32_t wd = w[i];
        const uint32_t op = wd & 255u;
        const int d = (int)((wd >> 8) & 255u), s1 = (int)((wd >> 16) & 255u), s2 = (int)(wd >> 24);
        const bool c1 = s1 >= GP_SRC_CONST, c2 = s2 >= GP_SRC_CONST;
        const uint32_t v1 = c1 ? cst[s1 - GP_SRC_CONST] : 0u, v2 = c2 ? cst[s2 - GP_SRC_CONST] : 0u;
        if (op >= GP_SIN && op <= GP_PLOG) {  // unary: leave the core
            e.exit(op, c1 ? 0 : off(s1), 0, d * T, c1, false, v1);
            continue;
        }
        if (!is_core_op(op, false)) {   // protected division and the classification functions
            if (c1 && c2) {
                e.put(CK_MOVC, 0, d, 0, 0, v1);
                e.apply(op, false, d * T, 0, d * T, false, true, v2);
            } else {
                e.apply(op, false, c1 ? 0 : off(s1), c2 ? 0 : off(s2), d * T, c1, c2, c1 ? v1 : v2);
            }
            continue;
        }
        const bool comm = op != GP_SUB;
        if (c1 && c2) {
            e.put(CK_MOVC, 0, d, 0, 0, v1);
            if (comm) e.put(CK_CR, op, d, 0, (uint32_t)(d * T), v2);
            else e.put(CK_RC, op, d, 0, (uint32_t)(d * T), v2);
        } else if (c1) {
            e.put(CK_CR, op, d, 0, (uint32_t)off(s2), v1);
        } else if (c2) {
            if (comm) e.put(CK_CR, op, d, 0, (uint32_t)off(s1), v2);
            else e.put(CK_RC, op, d, 0, (uint32_t)off(s1), v2);
        } else if (s1 < n_reg) {
            e.put(CK_RR, op, d, s1, (uint32_t)off(s2), 0);
        } else if (s2 < n_reg) {
            if (comm) e.put(CK_RR, op, d, s2, (uint32_t)off(s1), 0);
            else e.put(CK_XR, op, d, s2, (uint32_t)off(s1), 0);
        } else {
            e.put(CK_FF, op, d, 0, (uint32_t)off(s1) | ((uint32_t)off(s2) << 8), 0);
        }
    }
    if (e.ok) e.exit(CORE_OP_END, 0, 0, 0, false, false, 0);
    *n_out = e.n;
    return e.ok ? GP_OK : GP_E_INVAL;
}

static VariantMap map_at(int vi, uint64_t base) {
    VariantMap m;
    m.slot = variant_slots(vi);
    m.base = base;
    m.ready = true;
    return m;
}

// Programs are translated in parallel, each into its own counted range of
// the code: a tree gives one core instruction per lowered instruction plus
// the end; a register program as linear_records counts.
static gp_status translate_with(const ProgData& pd, int vi, const VariantMap& m, std::vector<uint32_t>& code,
                                std::vector<DevProg>& progs) {
    const int32_t P = pd.n_prog;
    progs = pd.progs;
    std::vector<int64_t> start((size_t)P + 1, 0);
    for (int32_t p = 0; p < P; p++) {
        const DevProg& src = pd.progs[p];
        const int64_t k = (src.meta & 1u) == FORM_TREE ? (int64_t)src.len + 1
                                                        : linear_records(pd.code.data() + src.code_off, src.len,
                                                                         pd.n_reg);
        start[p + 1] = start[p] + k;
    }
    if (start[P] * 16 > 0xFFFFFFF0ll) return fail(GP_E_INVAL, "programs exceed 4 GiB of core code");
    // the core reads records two at a time, up to one record past a program's
    // last one: the code ends with padding
    code.assign((size_t)start[P] * 4 + 16, 0u);
    std::vector<int32_t> rc((size_t)P, GP_OK);
    parallel_for(P, [&](int64_t p0, int64_t p1) {
        char err[256];
        for (int64_t p = p0; p < p1; p++) {
            const DevProg& src = pd.progs[p];
            uint32_t* out = code.data() + 4 * start[p];
            const int64_t cap = start[p + 1] - start[p];
            int64_t n = 0;
            if ((src.meta & 1u) == FORM_TREE)
                rc[p] = translate_tree(pd.code.data() + src.code_off, src.len, vi, m, out, cap, &n, err);
            else
                rc[p] = translate_linear(pd.code.data() + src.code_off, src.len,
                                         pd.code.data() + src.code_off + src.len, pd.n_reg, pd.n_feat, vi, m, out,
                                         cap, &n, err);
            if (rc[p] == GP_OK && n != cap) rc[p] = GP_E_INVAL;
        }
    });
    for (int32_t p = 0; p < P; p++) {
        if (rc[p] != GP_OK) {
            // translate the first failing program again on this thread for its message
            const DevProg& src = pd.progs[p];
            std::vector<uint32_t> tmp(4 * (size_t)(start[p + 1] - start[p] + 8));
            char err[256] = "internal: core code length differs from its count";
            int64_t n = 0;
            if ((src.meta & 1u) == FORM_TREE)
                translate_tree(pd.code.data() + src.code_off, src.len, vi, m, tmp.data(), (int64_t)tmp.size() / 4, &n,
                               err);
            else
                translate_linear(pd.code.data() + src.code_off, src.len, pd.code.data() + src.code_off + src.len,
                                 pd.n_reg, pd.n_feat, vi, m, tmp.data(), (int64_t)tmp.size() / 4, &n, err);
            return fail((gp_status)rc[p], "program %d: %s", p, err);
        }
        progs[p].code_off = (uint32_t)(4 * start[p]);   // words
        progs[p].len = (uint32_t)(start[p + 1] - start[p]);
    }
    return GP_OK;
}

gp_status core_translate(const ProgData& pd, int vi, std::vector<uint32_t>& code, std::vector<DevProg>& progs) {
    VariantMap m;
    {
        std::lock_guard<std::mutex> g(g_mu);
        if ((int)g_maps.size() <= vi || !g_maps[vi].ready) return fail(GP_E_DEVICE, "core variant %d not probed", vi);
        m = g_maps[vi];
    }
    return translate_with(pd, vi, m, code, progs);
}

gp_status core_translate_at(const ProgData& pd, int vi, uint64_t base, std::vector<uint32_t>& code,
                            std::vector<DevProg>& progs) {
    if (vi < 0 || vi >= core_variants()) return fail(GP_E_INVAL, "variant %d does not exist", vi);
    if (base & (GPX_SLOT - 1)) return fail(GP_E_INVAL, "table base must be %d-byte aligned", GPX_SLOT);
    return translate_with(pd, vi, map_at(vi, base), code, progs);
}

int core_variant_t(int vi) { return kCoreVariants[vi].t; }
int core_variant_ncv(int vi) { return kCoreVariants[vi].ncv; }
int core_variant_d(int vi) { return kCoreVariants[vi].d; }
int core_variant_nf(int vi) { return kCoreVariants[vi].nf; }
int core_variant_arith(int vi) { return mode_no_transc(kCoreVariants[vi].arith); }
bool core_variant_bool(int vi) { return kCoreVariants[vi].arith == 2; }
bool core_variant_trees_only(int vi) { return kCoreVariants[vi].arith >= 2; }

}  // namespace gpx
