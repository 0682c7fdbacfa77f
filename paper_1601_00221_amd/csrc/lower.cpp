// Host-side validation and lowering of GP programs.
//
// Trees arrive in prefix order.  They are lowered to the stack-operand
// linear form of the paper (section 5): every function becomes one
// instruction whose operands are a case input X, a constant C or the top of
// the stack S, and whose result is pushed.  The paper produces this form
// from the postfix string with a symbolic stack; here it is produced from
// the tree directly, with one change the paper's conclusions point to
// (reduce the stack memory a program needs): of two function operands the
// one needing more stack levels is evaluated first (Sethi-Ullman order).  A
// program's depth is then at most floor(log2(terminals)) levels, so a small
// register-resident stack holds every program of realistic size.  When the
// right operand of a non-commutative function ran first, the instruction is
// marked reversed so the operand order of the tree is kept.
//
// The three-operand IF of the classification function set (section 4.2) has
// no form with X or C operands: its terminal operands are pushed, its
// subtrees run in order of decreasing stack need, and the instruction reads
// the three values from the top of the stack, recording where each operand
// landed.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/gp.h"
#include "gp_internal.h"

namespace gpx {

static int arity_of(int op, int opset = OPSET_REAL) {
    if (opset == OPSET_BOOL) {
        switch (op) {
            case GP_AND: case GP_OR: case GP_NAND: case GP_NOR: return 2;
            case GP_VAR: return 0;
            default: return -1;
        }
    }
    switch (op) {
        case GP_ADD: case GP_SUB: case GP_MUL: case GP_PDIV: return 2;
        case GP_AND: case GP_OR: case GP_GT: case GP_LT: case GP_EQ: return 2;   // logical AND, OR here
        case GP_IF: return 3;
        case GP_SIN: case GP_COS: case GP_EXPC: case GP_PLOG: return 1;
        case GP_VAR: case GP_CONST: return 0;
        default: return -1;
    }
}

// the four Boolean functions are symmetric, like + and *, and so are ==, logical AND and OR
static bool commutative(int op) {
    return op == GP_ADD || op == GP_MUL || (op >= GP_AND && op <= GP_NOR) || op == GP_EQ;
}

static uint32_t fbits(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

namespace {
struct LowerFrame {
    int32_t node;
    int32_t stage;
};
struct LowerScratch {
    std::vector<int32_t> kid, need, open;
    std::vector<int8_t> ar, filled;
    std::vector<LowerFrame> fr;
};
LowerScratch& lower_scratch() {
    thread_local LowerScratch s;
    return s;
}
}  // namespace

int lower_tree(const int32_t* tok, const float* cst, int64_t n, int32_t n_feat, uint32_t* out,
               TreeLowering* st, char* err, int opset) {
    TreeLowering s;
    if (n < 1) {
        snprintf(err, 256, "empty program");
        return GP_E_INVAL;
    }
    if (n > GP_MAX_LEN) {
        snprintf(err, 256, "program of %lld nodes exceeds %d", (long long)n, GP_MAX_LEN);
        return GP_E_DEPTH;
    }
    const int32_t N = (int32_t)n;
    // per-thread work arrays, reused from program to program (host threads lower programs in parallel)
    LowerScratch& S = lower_scratch();
    std::vector<int32_t>&kid = S.kid, &need = S.need, &open = S.open;
    std::vector<int8_t>&ar = S.ar, &filled = S.filled;
    std::vector<LowerFrame>& fr = S.fr;
    kid.assign(3 * (size_t)N, -1);
    ar.resize(N);
    filled.assign(N, 0);
    open.clear();
    for (int32_t i = 0; i < N; i++) {
        const int op = tok[i] & 0xFF;
        const int a = arity_of(op, opset);
        if (a < 0) {
            snprintf(err, 256, "token %d: opcode %d is not in the %s function set", i, op,
                     opset == OPSET_BOOL ? "Boolean" : "arithmetic");
            return GP_E_INVAL;
        }
        if (op == GP_VAR) {
            const uint32_t f = (uint32_t)tok[i] >> 8;
            if ((int64_t)f >= n_feat) {
                snprintf(err, 256, "token %d: feature %u >= n_feat %d", i, f, n_feat);
                return GP_E_INVAL;
            }
        } else if ((uint32_t)tok[i] >> 8) {
            snprintf(err, 256, "token %d: argument bits set on opcode %d", i, op);
            return GP_E_INVAL;
        }
        ar[i] = (int8_t)a;
        if (i > 0) {
            if (open.empty()) {
                snprintf(err, 256, "token %d: tokens after a complete tree", i);
                return GP_E_INVAL;
            }
            const int32_t p = open.back();
            kid[3 * (size_t)p + filled[p]] = i;
            if (++filled[p] == ar[p]) open.pop_back();
        }
        if (a > 0) open.push_back(i);
    }
    if (!open.empty()) {
        snprintf(err, 256, "program ends with %zu unfilled operand slots", open.size());
        return GP_E_INVAL;
    }
    s.n_nodes = N;

    // Stack levels each subtree needs when its terminals are read as operands.
    need.assign(N, 0);
    // IF: its three operands in the order they are evaluated (decreasing need, ties left to right)
    auto if_order = [&](int32_t i, int32_t ord[3]) {
        int32_t nd[3];
        for (int k = 0; k < 3; k++) {
            const int32_t c = kid[3 * (size_t)i + k];
            nd[k] = ar[c] == 0 ? 1 : need[c];
            ord[k] = k;
        }
        for (int x = 1; x < 3; x++)
            for (int y = x; y > 0 && nd[ord[y]] > nd[ord[y - 1]]; y--) std::swap(ord[y], ord[y - 1]);
        int32_t m = 0;
        for (int k = 0; k < 3; k++) m = std::max(m, nd[ord[k]] + k);
        return m;
    };
    for (int32_t i = N - 1; i >= 0; i--) {
        if (ar[i] == 0) continue;
        const int32_t a = kid[3 * (size_t)i];
        if (ar[i] == 3) {
            int32_t ord[3];
            need[i] = if_order(i, ord);
            continue;
        }
        if (ar[i] == 1) {
            need[i] = ar[a] == 0 ? 1 : need[a];
            continue;
        }
        const int32_t b = kid[3 * (size_t)i + 1];
        const bool ta = ar[a] == 0, tb = ar[b] == 0;
        if (ta && tb) need[i] = 1;
        else if (tb) need[i] = need[a];
        else if (ta) need[i] = need[b];
        else if (need[a] >= need[b]) need[i] = need[a] > need[b] + 1 ? need[a] : need[b] + 1;
        else need[i] = need[b] > need[a] + 1 ? need[b] : need[a] + 1;
    }

    int32_t h = 0;
    int32_t w = 0;
    auto emit = [&](uint32_t op, uint32_t mode, uint32_t fa, uint32_t fb, float c, int dh,
                    int fetch, bool is_fun, int n_args) {
        h += dh;
        if (h > s.max_depth) s.max_depth = h;
        if (out) {
            out[2 * (size_t)w] = enc_w0(op, mode, fa, fb, (uint32_t)h);
            out[2 * (size_t)w + 1] = fbits(c);
        }
        w++;
        s.stack_fetches += fetch;
        if (is_fun) s.n_values += 1 + n_args;
    };
    auto feat = [&](int32_t i) -> uint32_t { return (uint32_t)tok[i] >> 8; };
    auto is_var = [&](int32_t i) { return (tok[i] & 0xFF) == GP_VAR; };

    auto push_terminal = [&](int32_t i) {
        if (is_var(i)) emit(OP_PUSH, M_X, feat(i), 0, 0.0f, +1, 0, false, 0);
        else emit(OP_PUSH, M_C, 0, 0, cst[i], +1, 0, false, 0);
    };

    fr.clear();
    if (ar[0] == 0) {
        // A lone terminal: push it.
        push_terminal(0);
    } else {
        fr.push_back(LowerFrame{0, 0});
    }
    while (!fr.empty()) {
        LowerFrame& f = fr.back();
        const int32_t i = f.node;
        const int op = tok[i] & 0xFF;
        const int32_t a = kid[3 * (size_t)i];
        if (ar[i] == 3) {
            int32_t ord[3];
            if_order(i, ord);
            if (f.stage < 3) {
                const int32_t c = kid[3 * (size_t)i + ord[f.stage]];
                f.stage++;
                if (ar[c] == 0) push_terminal(c);
                else fr.push_back(LowerFrame{c, 0});
                continue;
            }
            // operand ord[k] is the k-th of the three values from the bottom
            uint32_t pos[3];
            for (int k = 0; k < 3; k++) pos[ord[k]] = (uint32_t)k;
            emit(OP_IF, M_S3, pos[0], pos[1], 0.0f, -2, 3, true, 3);
            fr.pop_back();
            continue;
        }
        if (ar[i] == 1) {
            if (ar[a] == 0) {
                if (is_var(a)) emit(op, M_X, feat(a), 0, 0.0f, +1, 0, true, 1);
                else emit(op, M_C, 0, 0, cst[a], +1, 0, true, 1);
                fr.pop_back();
            } else if (f.stage == 0) {
                f.stage = 1;
                fr.push_back(LowerFrame{a, 0});
            } else {
                emit(op, M_S, 0, 0, 0.0f, 0, 1, true, 1);
                fr.pop_back();
            }
            continue;
        }
        const int32_t b = kid[3 * (size_t)i + 1];
        const bool ta = ar[a] == 0, tb = ar[b] == 0;
        if (ta && tb) {
            if (is_var(a) && is_var(b)) emit(op, M_XX, feat(a), feat(b), 0.0f, +1, 0, true, 2);
            else if (is_var(a)) emit(op, M_XC, feat(a), 0, cst[b], +1, 0, true, 2);
            else if (is_var(b)) emit(op, M_CX, 0, feat(b), cst[a], +1, 0, true, 2);
            else {
                // two constants: push the left one, then apply with the right one
                emit(OP_PUSH, M_C, 0, 0, cst[a], +1, 0, false, 0);
                emit(op, M_SC, 0, 0, cst[b], 0, 1, true, 2);
            }
            fr.pop_back();
        } else if (tb) {
            if (f.stage == 0) {
                f.stage = 1;
                fr.push_back(LowerFrame{a, 0});
            } else {
                if (is_var(b)) emit(op, M_SX, 0, feat(b), 0.0f, 0, 1, true, 2);
                else emit(op, M_SC, 0, 0, cst[b], 0, 1, true, 2);
                fr.pop_back();
            }
        } else if (ta) {
            if (f.stage == 0) {
                f.stage = 1;
                fr.push_back(LowerFrame{b, 0});
            } else {
                if (is_var(a)) emit(op, M_XS, feat(a), 0, 0.0f, 0, 1, true, 2);
                else emit(op, M_CS, 0, 0, cst[a], 0, 1, true, 2);
                fr.pop_back();
            }
        } else {
            const bool left_first = need[a] >= need[b];
            if (f.stage == 0) {
                f.stage = 1;
                fr.push_back(LowerFrame{left_first ? a : b, 0});
            } else if (f.stage == 1) {
                f.stage = 2;
                fr.push_back(LowerFrame{left_first ? b : a, 0});
            } else {
                const bool rev = !left_first && !commutative(op);
                if (rev) s.n_reversed++;
                emit(op, rev ? M_SSR : M_SS, 0, 0, 0.0f, -1, 2, true, 2);
                fr.pop_back();
            }
        }
    }
    if (h != 1) {
        snprintf(err, 256, "internal: lowered program leaves %d values", h);
        return GP_E_INVAL;
    }
    s.n_instr = w;
    if (s.max_depth > GP_MAX_DEPTH) {
        snprintf(err, 256, "program needs %d stack levels (max %d)", s.max_depth, GP_MAX_DEPTH);
        return GP_E_DEPTH;
    }
    if (st) *st = s;
    return GP_OK;
}

int check_linear(const uint32_t* code, int64_t n, int64_t n_cst, int32_t n_reg, int32_t n_feat,
                 char* err) {
    if (n < 1) {
        snprintf(err, 256, "empty linear program");
        return GP_E_INVAL;
    }
    if (n > GP_MAX_LEN) {
        snprintf(err, 256, "linear program of %lld instructions exceeds %d", (long long)n, GP_MAX_LEN);
        return GP_E_DEPTH;
    }
    for (int64_t i = 0; i < n; i++) {
        const uint32_t wd = code[i];
        const int op = wd & 0xFF;
        const int a = arity_of(op);
        const uint32_t dst = (wd >> 8) & 0xFF;
        if (a < 1 || a > 2) {
            snprintf(err, 256, "instruction %lld: opcode %d is not a function", (long long)i, op);
            return GP_E_INVAL;
        }
        if ((int32_t)dst >= n_reg) {
            snprintf(err, 256, "instruction %lld: dst %u >= n_reg %d", (long long)i, dst, n_reg);
            return GP_E_INVAL;
        }
        for (int q = 0; q < a; q++) {
            const int32_t id = (int32_t)((wd >> (16 + 8 * q)) & 0xFF);
            if (id < n_reg + n_feat) continue;
            if (id >= GP_SRC_CONST && id - GP_SRC_CONST < n_cst) continue;
            snprintf(err, 256, "instruction %lld: source id %d is not a register, feature or constant",
                     (long long)i, id);
            return GP_E_INVAL;
        }
    }
    return GP_OK;
}

}  // namespace gpx
