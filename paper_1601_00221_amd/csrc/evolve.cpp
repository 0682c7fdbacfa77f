// A GP run around the evaluator: the paper measures GPop/s over whole GP
// runs with the parameters of Table 2 (population 1000, 50 generations,
// tournaments of 7, crossover 0.95, mutation 0.2, depth at most 50, size at
// most 1000).  The population lives on the host as prefix trees and is bred
// there; every generation is evaluated on the GPU by gp_eval_tree (or
// gp_eval_bool for the Boolean function set) and its fitness copied back.
//
// Operators (Koza's tree GP):
//   initialisation  ramped half-and-half over [init_min_depth, init_max_depth];
//   selection       tournament: the best of `tournament` uniform draws;
//   crossover       with probability p_crossover: the subtree at a random
//                   point of the first parent is replaced by a random subtree
//                   of the second (points are functions with probability 0.9
//                   when the tree has any); otherwise the first parent is copied;
//   mutation        then, with probability p_mutation, a random subtree is
//                   replaced by a grown tree of depth at most mutation_depth.
// An offspring deeper than max_depth (edges from the root) or larger than
// max_size is replaced by its first parent.  Random numbers come from
// SplitMix64 (Steele, Lea and Flood 2014), so a run is reproducible from its
// seed.
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "../../include/gp.h"
#include "runtime.h"

namespace gpx {
namespace {

struct Rng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uni() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }   // [0, 1)
    uint32_t below(uint32_t n) { return (uint32_t)(((next() >> 32) * (uint64_t)n) >> 32); }
};

struct Tree {
    std::vector<int32_t> tok;
    std::vector<float> cst;
};

bool is_bool_op(int op) { return op >= GP_AND && op <= GP_NOR; }

int arity(int32_t t) {
    const int op = t & 0xFF;
    if (op == GP_VAR || op == GP_CONST) return 0;
    if (op == GP_IF) return 3;
    return (op >= GP_SIN && op <= GP_PLOG) ? 1 : 2;
}

// one past the end of the subtree starting at i
size_t subtree_end(const std::vector<int32_t>& tok, size_t i) {
    int64_t need = 1;
    while (need > 0) need += arity(tok[i++]) - 1;
    return i;
}

// edges on the longest root-to-leaf path
int depth_of(const std::vector<int32_t>& tok) {
    std::vector<int> open;   // remaining children of each open function
    int d = 0;
    for (size_t i = 0; i < tok.size(); i++) {
        d = std::max(d, (int)open.size());
        const int a = arity(tok[i]);
        if (a > 0) {
            open.push_back(a);
            continue;
        }
        while (!open.empty() && --open.back() == 0) open.pop_back();
    }
    return d;
}

struct Ctx {
    const gp_evolve_config& c;
    int32_t n_feat;
    bool boolean;
    std::vector<int> funs;
    Rng rng;

    void terminal(Tree& t) {
        if (!boolean && c.p_const > 0 && rng.uni() < c.p_const) {
            t.tok.push_back(GP_CONST);
            t.cst.push_back((float)(c.const_lo + (c.const_hi - c.const_lo) * rng.uni()));
        } else {
            t.tok.push_back(GP_VAR | (int32_t)(rng.below((uint32_t)n_feat) << 8));
            t.cst.push_back(0.0f);
        }
    }
    // Koza's grow (any primitive below the depth limit) or full method
    void grow(Tree& t, int depth, bool full) {
        const size_t n_term = (size_t)n_feat + (!boolean && c.p_const > 0 ? 1 : 0);
        if (depth == 0 || (!full && rng.uni() < (double)n_term / (double)(n_term + funs.size()))) {
            terminal(t);
            return;
        }
        const int f = funs[rng.below((uint32_t)funs.size())];
        t.tok.push_back(f);
        t.cst.push_back(0.0f);
        for (int k = arity(f); k > 0; k--) grow(t, depth - 1, full);
    }
    size_t pick_point(const std::vector<int32_t>& tok) {
        size_t n_fun = 0;
        for (int32_t t : tok) n_fun += arity(t) > 0;
        const bool want_fun = n_fun > 0 && rng.uni() < 0.9;
        const size_t n = want_fun ? n_fun : tok.size() - n_fun;
        size_t k = rng.below((uint32_t)n);
        for (size_t i = 0; i < tok.size(); i++)
            if ((arity(tok[i]) > 0) == want_fun && k-- == 0) return i;
        return 0;
    }
    bool fits(const Tree& t) const {
        return (int64_t)t.tok.size() <= c.max_size && depth_of(t.tok) <= c.max_depth;
    }
    // t with its subtree at i replaced by src's subtree at j
    static Tree splice(const Tree& t, size_t i, const Tree& src, size_t j) {
        const size_t ie = subtree_end(t.tok, i), je = subtree_end(src.tok, j);
        Tree o;
        o.tok.reserve(t.tok.size() - (ie - i) + (je - j));
        o.tok.insert(o.tok.end(), t.tok.begin(), t.tok.begin() + i);
        o.tok.insert(o.tok.end(), src.tok.begin() + j, src.tok.begin() + je);
        o.tok.insert(o.tok.end(), t.tok.begin() + ie, t.tok.end());
        o.cst.insert(o.cst.end(), t.cst.begin(), t.cst.begin() + i);
        o.cst.insert(o.cst.end(), src.cst.begin() + j, src.cst.begin() + je);
        o.cst.insert(o.cst.end(), t.cst.begin() + ie, t.cst.end());
        return o;
    }
};

gp_status check_config(const gp_evolve_config* c, int32_t n_feat, bool* boolean, std::vector<int>& funs) {
    if (!c) return fail(GP_E_INVAL, "config is null");
    if (c->pop_size < 1 || c->generations < 0 || c->tournament < 1 || c->max_size < 1 || c->max_depth < 0)
        return fail(GP_E_INVAL, "bad population size, generations, tournament or limits");
    if (c->init_min_depth < 0 || c->init_max_depth < c->init_min_depth || c->mutation_depth < 0)
        return fail(GP_E_INVAL, "bad initial or mutation depths");
    if (!(c->p_crossover >= 0 && c->p_crossover <= 1 && c->p_mutation >= 0 && c->p_mutation <= 1 &&
          c->p_const >= 0 && c->p_const <= 1))
        return fail(GP_E_INVAL, "probabilities must lie in [0, 1]");
    if (n_feat < 1) return fail(GP_E_INVAL, "n_feat < 1");
    funs.clear();
    for (int op = 0; op < 32; op++)
        if (c->functions & (1u << op)) {
            if (op > GP_IF) return fail(GP_E_INVAL, "function bit %d is not an opcode", op);
            funs.push_back(op);
        }
    if (funs.empty()) return fail(GP_E_INVAL, "empty function set");
    // a Boolean set holds only the four bitwise functions; an arithmetic set may hold AND and OR
    // (logical there) but not NAND or NOR
    bool b = true;
    for (int op : funs) b = b && is_bool_op(op);
    for (int op : funs)
        if (!b && (op == GP_NAND || op == GP_NOR))
            return fail(GP_E_INVAL, "NAND and NOR belong to the Boolean set; arithmetic functions mixed in");
    if (b && c->kind != GP_FIT_HITS) return fail(GP_E_INVAL, "Boolean runs use GP_FIT_HITS");
    if (!b && c->kind != GP_FIT_MSE && c->kind != GP_FIT_SUM_ABS && c->kind != GP_FIT_HITS &&
        c->kind != GP_FIT_CLASS_ERR)
        return fail(GP_E_INVAL, "unknown fitness kind %d", c->kind);
    *boolean = b;
    return GP_OK;
}

void init_population(Ctx& x, std::vector<Tree>& pop) {
    const int span = x.c.init_max_depth - x.c.init_min_depth + 1;
    pop.assign((size_t)x.c.pop_size, Tree());
    for (int32_t i = 0; i < x.c.pop_size; i++) {
        int d = x.c.init_min_depth + (i / 2) % span;
        // redraw a tree over the size or depth limit; after 8 draws lower its
        // depth (a lone terminal always fits)
        for (int attempt = 1;; attempt++) {
            pop[i].tok.clear();
            pop[i].cst.clear();
            x.grow(pop[i], d, i % 2 == 1);
            if (x.fits(pop[i])) break;
            if (attempt % 8 == 0 && d > 0) d--;
        }
    }
}

// lower score is better
void breed(Ctx& x, const std::vector<Tree>& pop, const std::vector<double>& score, std::vector<Tree>& next) {
    const uint32_t P = (uint32_t)pop.size();
    auto tournament = [&]() {
        uint32_t best = x.rng.below(P);
        for (int k = 1; k < x.c.tournament; k++) {
            const uint32_t o = x.rng.below(P);
            if (score[o] < score[best]) best = o;
        }
        return best;
    };
    next.assign(P, Tree());
    for (uint32_t i = 0; i < P; i++) {
        const Tree& a = pop[tournament()];
        Tree child;
        if (x.rng.uni() < x.c.p_crossover) {
            const Tree& b = pop[tournament()];
            child = Ctx::splice(a, x.pick_point(a.tok), b, x.pick_point(b.tok));
        } else {
            child = a;
        }
        if (x.rng.uni() < x.c.p_mutation) {
            Tree sub;
            x.grow(sub, (int)x.rng.below((uint32_t)x.c.mutation_depth + 1), false);
            child = Ctx::splice(child, x.rng.below((uint32_t)child.tok.size()), sub, 0);
        }
        next[i] = x.fits(child) ? std::move(child) : a;
    }
}

gp_status to_csr(const std::vector<Tree>& pop, int32_t* tok, float* cst, int64_t* off, int64_t max_tokens) {
    int64_t n = 0;
    for (const Tree& t : pop) n += (int64_t)t.tok.size();
    if (n > max_tokens) return fail(GP_E_NOMEM, "population has %lld tokens, buffer holds %lld", (long long)n,
                                    (long long)max_tokens);
    int64_t w = 0;
    off[0] = 0;
    for (size_t p = 0; p < pop.size(); p++) {
        memcpy(tok + w, pop[p].tok.data(), pop[p].tok.size() * 4);
        memcpy(cst + w, pop[p].cst.data(), pop[p].cst.size() * 4);
        w += (int64_t)pop[p].tok.size();
        off[p + 1] = w;
    }
    return GP_OK;
}

}  // namespace
}  // namespace gpx

using namespace gpx;

extern "C" {

gp_status gp_init_population(const gp_evolve_config* cfg, int32_t n_feat, int32_t* tok, float* cst, int64_t* off,
                             int64_t max_tokens) {
    clear_error();
    bool boolean;
    std::vector<int> funs;
    gp_status st = check_config(cfg, n_feat, &boolean, funs);
    if (st != GP_OK) return st;
    if (!tok || !cst || !off) return fail(GP_E_INVAL, "null output array");
    Ctx x{*cfg, n_feat, boolean, funs, Rng{cfg->seed}};
    std::vector<Tree> pop;
    init_population(x, pop);
    return to_csr(pop, tok, cst, off, max_tokens);
}

gp_status gp_breed(const gp_evolve_config* cfg, const int32_t* tok, const float* cst, const int64_t* off,
                   int32_t n_feat, const double* score, uint64_t seed, int32_t* out_tok, float* out_cst,
                   int64_t* out_off, int64_t max_tokens) {
    clear_error();
    bool boolean;
    std::vector<int> funs;
    gp_status st = check_config(cfg, n_feat, &boolean, funs);
    if (st != GP_OK) return st;
    if (!tok || !off || !score || !out_tok || !out_cst || !out_off || (!cst && !boolean))
        return fail(GP_E_INVAL, "null array");
    // the parents must be valid programs of the run's function set
    ProgData pd;
    if ((st = build_tree(tok, cst, off, cfg->pop_size, n_feat, pd, boolean ? OPSET_BOOL : OPSET_REAL)) != GP_OK)
        return st;
    std::vector<Tree> pop((size_t)cfg->pop_size), next;
    std::vector<double> sc((size_t)cfg->pop_size);
    for (int32_t p = 0; p < cfg->pop_size; p++) {
        pop[p].tok.assign(tok + off[p], tok + off[p + 1]);
        if (cst) pop[p].cst.assign(cst + off[p], cst + off[p + 1]);
        else pop[p].cst.assign((size_t)(off[p + 1] - off[p]), 0.0f);
        sc[p] = std::isnan(score[p]) ? INFINITY : score[p];
    }
    Ctx x{*cfg, n_feat, boolean, funs, Rng{seed}};
    breed(x, pop, sc, next);
    return to_csr(next, out_tok, out_cst, out_off, max_tokens);
}

gp_status gp_evolve(const gp_evolve_config* cfg, const void* X, int32_t n_feat, int64_t n_cases, const void* y,
                    double* best_per_gen, int32_t* best_tok, float* best_cst, int32_t best_cap,
                    gp_evolve_result* res, void* stream) {
    clear_error();
    using clk = std::chrono::steady_clock;
    const auto t_start = clk::now();
    bool boolean;
    std::vector<int> funs;
    gp_status st = check_config(cfg, n_feat, &boolean, funs);
    if (st != GP_OK) return st;
    if (!X || !y || !res) return fail(GP_E_INVAL, "null X, y or result");
    if (n_cases < 1) return fail(GP_E_INVAL, "n_cases must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    const bool hits = cfg->kind == GP_FIT_HITS;                       // maximised
    const bool counts = hits || cfg->kind == GP_FIT_CLASS_ERR;        // int32 fitness
    const int32_t P = cfg->pop_size;
    void* d_out = nullptr;
    hipError_t e = hipMalloc(&d_out, (size_t)P * 4);
    if (e != hipSuccess) return fail(GP_E_NOMEM, "hipMalloc: %s", hipGetErrorString(e));
    std::vector<float> fit_f((size_t)P);
    std::vector<int32_t> fit_i((size_t)P);
    std::vector<double> score((size_t)P);
    std::vector<int32_t> tok;
    std::vector<float> cst;
    std::vector<int64_t> off((size_t)P + 1);

    Ctx x{*cfg, n_feat, boolean, funs, Rng{cfg->seed}};
    std::vector<Tree> pop, next;
    init_population(x, pop);
    memset(res, 0, sizeof *res);
    double best = INFINITY;
    Tree best_tree;
    double eval_s = 0, breed_s = 0;
    for (int32_t g = 0; g <= cfg->generations; g++) {
        // evaluate the generation on the GPU
        const auto t0 = clk::now();
        int64_t n_tok = 0;
        for (const Tree& t : pop) n_tok += (int64_t)t.tok.size();
        tok.resize((size_t)n_tok);
        cst.resize((size_t)n_tok);
        if ((st = to_csr(pop, tok.data(), cst.data(), off.data(), n_tok)) != GP_OK) break;
        if (boolean)
            st = gp_eval_bool(tok.data(), off.data(), P, (const uint32_t*)X, n_feat, n_cases, (const uint32_t*)y,
                              GP_FIT_HITS, d_out, stream);
        else
            st = gp_eval_tree(tok.data(), cst.data(), off.data(), P, (const float*)X, n_feat, n_cases,
                              (const float*)y, cfg->kind, d_out, stream);
        if (st != GP_OK) break;
        e = hipMemcpyAsync(counts ? (void*)fit_i.data() : (void*)fit_f.data(), d_out, (size_t)P * 4,
                           hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            st = fail(GP_E_DEVICE, "fitness copy: %s", hipGetErrorString(e));
            break;
        }
        res->gp_ops += n_tok * n_cases;
        const auto t1 = clk::now();
        eval_s += std::chrono::duration<double>(t1 - t0).count();
        // the best program so far (lower score is better: errors, or minus the hits)
        int32_t gbest = 0;
        for (int32_t p = 0; p < P; p++) {
            const double v = hits ? -(double)fit_i[p] : (counts ? (double)fit_i[p] : (double)fit_f[p]);
            score[p] = std::isnan(v) ? INFINITY : v;
            if (score[p] < score[gbest]) gbest = p;
        }
        if (score[gbest] < best) {
            best = score[gbest];
            best_tree = pop[gbest];
            res->best_generation = g;
        }
        if (best_per_gen) best_per_gen[g] = hits ? -best : best;
        res->generations_run = g + 1;
        if (g == cfg->generations) break;
        breed(x, pop, score, next);
        pop.swap(next);
        breed_s += std::chrono::duration<double>(clk::now() - t1).count();
    }
    (void)hipFree(d_out);
    if (st != GP_OK) return st;
    res->best_fitness = hits ? -best : best;
    res->best_size = (int32_t)best_tree.tok.size();
    if (best_tok && best_cst && best_cap >= res->best_size) {
        memcpy(best_tok, best_tree.tok.data(), best_tree.tok.size() * 4);
        memcpy(best_cst, best_tree.cst.data(), best_tree.cst.size() * 4);
    }
    res->eval_seconds = eval_s;
    res->breed_seconds = breed_s;
    res->total_seconds = std::chrono::duration<double>(clk::now() - t_start).count();
    return GP_OK;
}

}  // extern "C"
