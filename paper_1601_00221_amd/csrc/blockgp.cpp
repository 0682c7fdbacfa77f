// Host side of the one-dimensional-stack comparator (gp_eval_tree_1d): the
// BlockGP design of section 4.2 (postfix code, Table 3) and its linear
// stack-operand form (section 5, Table 7), one workgroup per program.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "blockgp.h"
#include "runtime.h"

namespace gpx {

static int arity(uint32_t op) { return op >= GP_VAR ? 0 : (op >= GP_SIN ? 1 : 2); }

// Postfix code of one validated prefix tree: children first, left to right,
// then the node.  Word 0 is the opcode | feature << 8, word 1 the constant.
// Returns the stack values the postfix evaluation needs.
static int32_t to_postfix(const int32_t* tok, const float* cst, int64_t n, uint32_t* out) {
    // subtree sizes from a backward scan: the top of the size stack is the
    // leftmost pending subtree
    std::vector<int64_t> size((size_t)n), sz;
    for (int64_t i = n - 1; i >= 0; i--) {
        int64_t s = 1;
        for (int k = arity((uint32_t)tok[i] & 255u); k > 0; k--) {
            s += sz.back();
            sz.pop_back();
        }
        size[(size_t)i] = s;
        sz.push_back(s);
    }
    // post-order walk with an explicit stack of (node, children emitted)
    std::vector<std::pair<int64_t, int>> walk;
    walk.emplace_back(0, 0);
    int64_t w = 0;
    int32_t h = 0, depth = 0;
    while (!walk.empty()) {
        auto& top = walk.back();
        const int64_t i = top.first;
        const uint32_t t = (uint32_t)tok[i], op = t & 255u;
        if (top.second < arity(op)) {
            const int64_t child = top.second == 0 ? i + 1 : i + 1 + size[(size_t)(i + 1)];
            top.second++;
            walk.emplace_back(child, 0);
            continue;
        }
        walk.pop_back();
        uint32_t cbits = 0;
        if (op == GP_CONST) memcpy(&cbits, &cst[i], 4);
        out[2 * w] = op == GP_VAR ? (GP_VAR | (t >> 8) << 8) : op;
        out[2 * w + 1] = cbits;
        w++;
        h += 1 - arity(op);
        depth = std::max(depth, h);
    }
    return depth;
}

static gp_status upload(Workspace& w, const std::vector<uint32_t>& code, const std::vector<uint32_t>& meta,
                        hipStream_t s) {
    gp_status st;
    if ((st = w.bg_code.reserve(std::max<size_t>(16, code.size() * 4))) != GP_OK) return st;
    if ((st = w.bg_meta.reserve(meta.size() * 4)) != GP_OK) return st;
    if ((st = w.staging.begin(code.size() * 4 + meta.size() * 4 + 1024)) != GP_OK) return st;
    if ((st = w.staging.put(code.data(), code.size() * 4, w.bg_code.p, s)) != GP_OK) return st;
    if ((st = w.staging.put(meta.data(), meta.size() * 4, w.bg_meta.p, s)) != GP_OK) return st;
    return w.staging.end(s);
}

}  // namespace gpx

using namespace gpx;

extern "C" gp_status gp_eval_tree_1d(const int32_t* tok, const float* cst, const int64_t* off, int32_t n_prog,
                                     const float* X, int32_t n_feat, int64_t n_cases, const float* y,
                                     int32_t kind, int32_t form, void* out, void* stream) {
    clear_error();
    if (form != GP_1D_RPN && form != GP_1D_LGP) return fail(GP_E_INVAL, "unknown 1D form %d", form);
    ProgData pd;
    gp_status st = build_tree(tok, cst, off, n_prog, n_feat, pd);   // validates and lowers
    if (st != GP_OK || n_prog == 0) return st;
    // the comparator reproduces the paper's regression measurements: the arithmetic and
    // transcendental functions only
    for (int64_t i = 0; i < off[n_prog]; i++) {
        const int op = tok[i] & 0xFF;
        if (op >= GP_AND && op <= GP_IF)
            return fail(GP_E_INVAL, "token %lld: the 1D comparator runs {+,-,*,/,sin,cos,exp,log} trees only",
                        (long long)i);
    }
    if (!X) return fail(GP_E_INVAL, "X is null");
    if (!out) return fail(GP_E_INVAL, "out is null");
    if (n_cases < 1) return fail(GP_E_INVAL, "n_cases must be >= 1");
    if (kind < GP_FIT_SUM_ABS || kind > GP_OUT_CASES) return fail(GP_E_INVAL, "unknown fitness kind %d", kind);
    if (kind != GP_OUT_CASES && !y) return fail(GP_E_INVAL, "y is null");
    if (pd.n_load > GP_MAX_FEAT)
        return fail(GP_E_INVAL, "programs read feature %d; at most %d features are supported", pd.n_load - 1,
                    GP_MAX_FEAT);
    if (n_prog > 0x7FFFFFFF / 2) return fail(GP_E_INVAL, "too many programs");

    // code: two words per instruction; meta: n_prog offsets then n_prog lengths
    std::vector<uint32_t> code, meta(2 * (size_t)n_prog);
    uint32_t max_len = 0;
    if (form == GP_1D_LGP) {
        code = pd.code;
        for (int32_t p = 0; p < n_prog; p++) {
            const DevProg& d = pd.progs[p];
            if (d.len > GP_1D_MAX_LEN)
                return fail(GP_E_DEPTH, "program %d: %u instructions exceeds %d", p, d.len, GP_1D_MAX_LEN);
            meta[p] = d.code_off / 2;
            meta[n_prog + p] = d.len;
            max_len = std::max(max_len, d.len);
        }
    } else {
        code.resize((size_t)(off[n_prog] - off[0]) * 2);
        for (int32_t p = 0; p < n_prog; p++) {
            const int64_t n = off[p + 1] - off[p];
            if (n > GP_1D_MAX_LEN)
                return fail(GP_E_DEPTH, "program %d: %lld nodes exceeds %d", p, (long long)n, GP_1D_MAX_LEN);
            const int32_t depth = to_postfix(tok + off[p], cst + off[p], n, code.data() + 2 * off[p]);
            if (depth > GP_BG_MAX_STACK)
                return fail(GP_E_DEPTH, "program %d: postfix needs %d stack values, more than %d", p, depth,
                            GP_BG_MAX_STACK);
            meta[p] = (uint32_t)off[p];
            meta[n_prog + p] = (uint32_t)n;
            max_len = std::max(max_len, (uint32_t)n);
        }
    }
    if (code.size() > 0xFFFFFFFFull) return fail(GP_E_INVAL, "programs exceed 2^32 device words");

    hipStream_t s = (hipStream_t)stream;
    Workspace& w = workspace(s);
    std::lock_guard<std::mutex> g(w.mu);
    if ((st = upload(w, code, meta, s)) != GP_OK) return st;
    BgArgs a;
    a.code = (const uint32_t*)w.bg_code.p;
    a.poff = (const uint32_t*)w.bg_meta.p;
    a.plen = a.poff + n_prog;
    a.X = X;
    a.y = kind == GP_OUT_CASES ? nullptr : y;
    a.out = out;
    a.N = n_cases;
    a.kind = kind;
    a.max_len = max_len;
    int slot = -1;
    hipError_t e = timed_launch_begin(s, &slot);
    if (e == hipSuccess) e = blockgp_launch(form, a, n_prog, s);
    if (e == hipSuccess) e = timed_launch_end(s, slot);
    if (e != hipSuccess) return fail(GP_E_DEVICE, "1D kernel launch: %s", hipGetErrorString(e));
    return GP_OK;
}
