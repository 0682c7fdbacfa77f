/*
 * CPU ORACLE for GP population evaluation -- test infrastructure only.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or
 * helper with the HIP evaluator; what the two have in common is the public
 * program/data interchange format, restated here from its definition.
 *
 * What it computes (plain definitions, no blocking, no fusion, no reordering):
 *
 *   o[p][c]   = value of program p on fitness case c          (section 3/4:
 *               every candidate program is run over every fitness case)
 *   fitness[p]= F(o[p][.], y)                                   (Table 2:
 *               regression uses mean squared error; the classification
 *               fitness counts incorrect classifications -- here the
 *               complementary hit count of the sign rule)
 *
 * Program forms:
 *   - prefix trees, evaluated by a recursive interpreter -- the slow
 *     alternative the paper names in section 5 next to the iterative one;
 *   - the postfix (RPN) form and its one-dimensional stack interpreter
 *     (section 5, the classic tree-GP interpreter);
 *   - the paper's stack-operand linear form ("prefix LGP", section 5): a list
 *     of functions whose operands are a case input X, a constant C or the
 *     top of the stack S, with results always pushed; produced from RPN by a
 *     symbolic stack (section 5);
 *   - register linear GP programs (dst, op, src1, src2), the register-based
 *     linear form of Brameier and Banzhaf the paper cites in section 5;
 *   - Boolean trees over {AND, OR, NAND, NOR} on bit-packed cases, 32 per
 *     machine word (sub-machine-code GP, sections 3 and 4.2), with the hit
 *     count checked bit by bit.
 *
 * Operator semantics (IEEE binary32, round to nearest even, no contraction,
 * denormals kept).  The paper names the functions but not their protection;
 * the readings taken here are:
 *   pdiv(a,b) = |b| < 1e-6f ? 1 : a/b        (threshold compared in binary32)
 *   plog(a)   = |a| < 1e-6f ? 0 : log|a|
 *   expc(a)   = exp(a > 88 ? 88 : a)          (NaN passes through the compare)
 *   sin, cos, exp, log are computed in binary64 and rounded once to binary32.
 *
 * Classification functions (section 4.2: the Shuttle and KDD Cup 99 problems
 * add {>, <, ==, AND, OR, IF} to the arithmetic set; the paper names them
 * without defining them).  Readings taken here: a comparison gives 1 or 0;
 * AND, OR and IF take a value as true when it is not zero (so NaN is true);
 * IF(a, b, c) = (a != 0) ? b : c, its three operands all evaluated.  In an
 * arithmetic tree the opcodes 8 and 9 (AND and OR of the Boolean set) are
 * these logical functions.
 *
 * Fitness: d = o - y in binary32; the term is |d| (sum of absolute errors),
 * d*d (mean squared error) or the hit (o > 0) == (y > 0); sums of terms are
 * accumulated in binary64 in case order and rounded to binary32 at the end
 * (MSE divides by N first).  Hits are an exact integer count.  The
 * classification fitness (Table 2: the sum of incorrect classifications)
 * decodes the output to the class rint(o) (binary32, ties to even) and counts
 * the cases where it differs from y, the class index; a NaN or infinite output
 * is never a class.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared -pthread -lm
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* interchange-format opcodes */
enum { O_ADD = 0, O_SUB = 1, O_MUL = 2, O_PDIV = 3, O_SIN = 4, O_COS = 5,
       O_EXPC = 6, O_PLOG = 7, O_LAND = 8, O_LOR = 9, O_GT = 12, O_LT = 13,
       O_EQ = 14, O_IF = 15, O_VAR = 64, O_CONST = 65 };
/* fitness kinds */
enum { K_SUM_ABS = 0, K_MSE = 1, K_HITS = 2, K_CASES = 3, K_CLASS = 4 };

#define ORC_OK 0
#define ORC_BAD (-1)

static int arity_of(int op)
{
    switch (op) {
    case O_ADD: case O_SUB: case O_MUL: case O_PDIV: return 2;
    case O_LAND: case O_LOR: case O_GT: case O_LT: case O_EQ: return 2;
    case O_IF: return 3;
    case O_SIN: case O_COS: case O_EXPC: case O_PLOG: return 1;
    case O_VAR: case O_CONST: return 0;
    default: return -1;
    }
}

/* Move a binary32 value n representable steps towards +inf (n > 0) or -inf
 * (n < 0).  Used only to probe how sensitive a program's fitness is to the
 * last-place error that a binary32 sin/cos/exp/log may carry. */
static float nudge_ulps(float v, int n)
{
    while (n > 0) { v = nextafterf(v, INFINITY); n--; }
    while (n < 0) { v = nextafterf(v, -INFINITY); n++; }
    return v;
}

static float apply_unary(int op, float a, int nudge)
{
    float r;
    switch (op) {
    case O_SIN: r = (float)sin((double)a); break;
    case O_COS: r = (float)cos((double)a); break;
    case O_EXPC: {
        float t = (a > 88.0f) ? 88.0f : a;
        r = (float)exp((double)t);
        break;
    }
    case O_PLOG: {
        float m = fabsf(a);
        if (m < 1e-6f) return 0.0f;
        r = (float)log((double)m);
        break;
    }
    default: return NAN;
    }
    return nudge ? nudge_ulps(r, nudge) : r;
}

static float apply_binary(int op, float a, float b)
{
    switch (op) {
    case O_ADD: return a + b;
    case O_SUB: return a - b;
    case O_MUL: return a * b;
    case O_PDIV: return (fabsf(b) < 1e-6f) ? 1.0f : a / b;
    case O_GT: return (a > b) ? 1.0f : 0.0f;
    case O_LT: return (a < b) ? 1.0f : 0.0f;
    case O_EQ: return (a == b) ? 1.0f : 0.0f;
    case O_LAND: return (a != 0.0f && b != 0.0f) ? 1.0f : 0.0f;
    case O_LOR: return (a != 0.0f || b != 0.0f) ? 1.0f : 0.0f;
    default: return NAN;
    }
}

static float apply_ternary(int op, float a, float b, float c)
{
    return op == O_IF ? ((a != 0.0f) ? b : c) : NAN;
}

/* ------------------------------------------------------------------------ */
/* Prefix trees                                                              */
/* ------------------------------------------------------------------------ */

/* Length of the well-formed prefix subtree starting at i, or -1. */
static int64_t subtree_len(const int32_t* tok, int64_t i, int64_t n)
{
    int64_t need = 1, j = i;
    while (need > 0) {
        if (j >= n) return -1;
        int a = arity_of(tok[j] & 0xFF);
        if (a < 0) return -1;
        need += a - 1;
        j++;
    }
    return j - i;
}

/* Recursive prefix interpreter: evaluates the subtree at *i for case c and
 * advances *i past it.  Operands are evaluated left to right. */
static float eval_prefix(const int32_t* tok, const float* cst, int64_t* i,
                         const float* X, int64_t N, int64_t c, int nudge)
{
    int32_t t = tok[*i];
    int op = t & 0xFF;
    int64_t me = *i;
    (*i)++;
    if (op == O_VAR) return X[(int64_t)((uint32_t)t >> 8) * N + c];
    if (op == O_CONST) return cst[me];
    if (arity_of(op) == 1) {
        float a = eval_prefix(tok, cst, i, X, N, c, nudge);
        return apply_unary(op, a, nudge);
    }
    float a = eval_prefix(tok, cst, i, X, N, c, nudge);
    float b = eval_prefix(tok, cst, i, X, N, c, nudge);
    if (arity_of(op) == 3) {
        float d = eval_prefix(tok, cst, i, X, N, c, nudge);
        return apply_ternary(op, a, b, d);
    }
    return apply_binary(op, a, b);
}

static int check_tree(const int32_t* tok, int64_t n, int32_t F)
{
    if (n <= 0) return ORC_BAD;
    if (subtree_len(tok, 0, n) != n) return ORC_BAD;
    for (int64_t i = 0; i < n; i++)
        if ((tok[i] & 0xFF) == O_VAR && (int64_t)((uint32_t)tok[i] >> 8) >= F) return ORC_BAD;
    return ORC_OK;
}

/* out[p*N + c] = value of tree p on case c */
int orc_tree_outputs(const int32_t* tok, const float* cst, const int64_t* off,
                     int32_t P, const float* X, int32_t F, int64_t N, int nudge,
                     float* out)
{
    for (int32_t p = 0; p < P; p++) {
        const int32_t* t = tok + off[p];
        const float* k = cst + off[p];
        int64_t n = off[p + 1] - off[p];
        if (check_tree(t, n, F) != ORC_OK) return ORC_BAD;
        for (int64_t c = 0; c < N; c++) {
            int64_t i = 0;
            out[(int64_t)p * N + c] = eval_prefix(t, k, &i, X, N, c, nudge);
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Fitness of one program's outputs                                          */
/* ------------------------------------------------------------------------ */
int orc_fitness(const float* o, const float* y, int64_t N, int kind,
                double* sum_out, float* fit_out, int32_t* hits_out)
{
    double s = 0.0;
    int64_t h = 0;
    for (int64_t c = 0; c < N; c++) {
        float d = o[c] - y[c];
        if (kind == K_SUM_ABS) s += (double)fabsf(d);
        else if (kind == K_MSE) { float q = d * d; s += (double)q; }
        else if (kind == K_HITS) h += ((o[c] > 0.0f) == (y[c] > 0.0f));
        else if (kind == K_CLASS) h += !(rintf(o[c]) == y[c]);
        else return ORC_BAD;
    }
    if (sum_out) *sum_out = (kind == K_HITS || kind == K_CLASS) ? (double)h : s;
    if (fit_out) {
        if (kind == K_SUM_ABS) *fit_out = (float)s;
        else if (kind == K_MSE) *fit_out = (float)(s / (double)N);
        else *fit_out = (float)h;
    }
    if (hits_out) *hits_out = (int32_t)h;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Register linear GP                                                        */
/* word = op | dst << 8 | src1 << 16 | src2 << 24;  source ids: [0,R)        */
/* registers, [R,R+F) features, [128,256) the program's constants.          */
/* Registers start as r[k] = x[k mod F]; the output is r[0]; a unary        */
/* function reads src1 only.                                                 */
/* ------------------------------------------------------------------------ */
#define ORC_MAX_REG 64

static int check_linear(const uint32_t* code, int64_t n, int64_t n_cst,
                        int32_t R, int32_t F)
{
    for (int64_t i = 0; i < n; i++) {
        uint32_t w = code[i];
        int op = w & 0xFF, dst = (w >> 8) & 0xFF;
        int s[2] = { (int)((w >> 16) & 0xFF), (int)((w >> 24) & 0xFF) };
        int a = arity_of(op);
        if (a < 1 || a > 2) return ORC_BAD;     /* no ternary function in the register form */
        if (dst >= R) return ORC_BAD;
        for (int q = 0; q < a; q++) {
            int id = s[q];
            if (id < R + F) continue;
            if (id >= 128 && id - 128 < n_cst) continue;
            return ORC_BAD;
        }
    }
    return ORC_OK;
}

static float lin_src(int id, const float* r, const float* X, int64_t N, int64_t c,
                     const float* k, int32_t R)
{
    if (id < R) return r[id];
    if (id < 128) return X[(int64_t)(id - R) * N + c];
    return k[id - 128];
}

int orc_linear_outputs(const uint32_t* code, const int64_t* off, const float* cst,
                       const int64_t* cst_off, int32_t P, int32_t R,
                       const float* X, int32_t F, int64_t N, int nudge, float* out)
{
    if (R < 1 || R > ORC_MAX_REG || F < 1 || R + F > 128) return ORC_BAD;
    for (int32_t p = 0; p < P; p++) {
        const uint32_t* w = code + off[p];
        int64_t n = off[p + 1] - off[p];
        const float* k = cst + cst_off[p];
        if (check_linear(w, n, cst_off[p + 1] - cst_off[p], R, F) != ORC_OK) return ORC_BAD;
        for (int64_t c = 0; c < N; c++) {
            float r[ORC_MAX_REG];
            for (int q = 0; q < R; q++) r[q] = X[(int64_t)(q % F) * N + c];
            for (int64_t i = 0; i < n; i++) {
                uint32_t v = w[i];
                int op = v & 0xFF, dst = (v >> 8) & 0xFF;
                float a = lin_src((v >> 16) & 0xFF, r, X, N, c, k, R);
                if (arity_of(op) == 1) {
                    r[dst] = apply_unary(op, a, nudge);
                } else {
                    float b = lin_src((v >> 24) & 0xFF, r, X, N, c, k, R);
                    r[dst] = apply_binary(op, a, b);
                }
            }
            out[(int64_t)p * N + c] = r[0];
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Whole-population fitness, optionally on several threads (static          */
/* partition of the programs).                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int form;                 /* 0 tree, 1 linear */
    const int32_t* tok; const float* tcst; const int64_t* toff;
    const uint32_t* code; const int64_t* loff; const float* lcst; const int64_t* lcst_off;
    int32_t R;
    const float* X; int32_t F; int64_t N; const float* y; int kind; int nudge;
    int32_t p0, p1;
    void* out; double* sums;
    int status;
} job_t;

static void* run_job(void* arg)
{
    job_t* j = (job_t*)arg;
    float* o = (float*)malloc(sizeof(float) * (size_t)(j->N > 0 ? j->N : 1));
    if (!o) { j->status = ORC_BAD; return NULL; }
    j->status = ORC_OK;
    for (int32_t p = j->p0; p < j->p1 && j->status == ORC_OK; p++) {
        int rc;
        if (j->form == 0) {
            int64_t off1[2] = { 0, j->toff[p + 1] - j->toff[p] };
            rc = orc_tree_outputs(j->tok + j->toff[p], j->tcst + j->toff[p], off1, 1,
                                  j->X, j->F, j->N, j->nudge, o);
        } else {
            int64_t off1[2] = { 0, j->loff[p + 1] - j->loff[p] };
            int64_t coff1[2] = { 0, j->lcst_off[p + 1] - j->lcst_off[p] };
            rc = orc_linear_outputs(j->code + j->loff[p], off1, j->lcst + j->lcst_off[p], coff1, 1,
                                    j->R, j->X, j->F, j->N, j->nudge, o);
        }
        if (rc != ORC_OK) { j->status = rc; break; }
        if (j->kind == K_CASES) {
            memcpy((float*)j->out + (int64_t)p * j->N, o, sizeof(float) * (size_t)j->N);
            continue;
        }
        double s; float f; int32_t h;
        rc = orc_fitness(o, j->y, j->N, j->kind, &s, &f, &h);
        if (rc != ORC_OK) { j->status = rc; break; }
        if (j->kind == K_HITS || j->kind == K_CLASS) ((int32_t*)j->out)[p] = h;
        else ((float*)j->out)[p] = f;
        if (j->sums) j->sums[p] = s;
    }
    free(o);
    return NULL;
}

static int run_population(job_t base, int32_t P, int n_threads)
{
    if (n_threads < 1) n_threads = 1;
    if (n_threads > P) n_threads = P > 0 ? P : 1;
    job_t* jobs = (job_t*)calloc((size_t)n_threads, sizeof(job_t));
    pthread_t* th = (pthread_t*)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return ORC_BAD; }
    for (int t = 0; t < n_threads; t++) {
        jobs[t] = base;
        jobs[t].p0 = (int32_t)((int64_t)P * t / n_threads);
        jobs[t].p1 = (int32_t)((int64_t)P * (t + 1) / n_threads);
    }
    for (int t = 1; t < n_threads; t++) pthread_create(&th[t], NULL, run_job, &jobs[t]);
    run_job(&jobs[0]);
    for (int t = 1; t < n_threads; t++) pthread_join(th[t], NULL);
    int rc = ORC_OK;
    for (int t = 0; t < n_threads; t++) if (jobs[t].status != ORC_OK) rc = jobs[t].status;
    free(jobs); free(th);
    return rc;
}

/* out: float[P] (sum_abs, mse), int32[P] (hits) or float[P*N] (cases).
 * sums (optional): the binary64 sum per program (hit count for hits). */
int orc_eval_tree(const int32_t* tok, const float* cst, const int64_t* off, int32_t P,
                  const float* X, int32_t F, int64_t N, const float* y, int kind,
                  int nudge, int n_threads, void* out, double* sums)
{
    if (P < 0 || N < 1 || F < 1 || kind < 0 || kind > K_CLASS) return ORC_BAD;
    job_t b; memset(&b, 0, sizeof b);
    b.form = 0; b.tok = tok; b.tcst = cst; b.toff = off;
    b.X = X; b.F = F; b.N = N; b.y = y; b.kind = kind; b.nudge = nudge;
    b.out = out; b.sums = sums;
    return run_population(b, P, n_threads);
}

int orc_eval_linear(const uint32_t* code, const int64_t* off, const float* cst,
                    const int64_t* cst_off, int32_t P, int32_t R, const float* X,
                    int32_t F, int64_t N, const float* y, int kind, int nudge,
                    int n_threads, void* out, double* sums)
{
    if (P < 0 || N < 1 || F < 1 || kind < 0 || kind > K_CLASS) return ORC_BAD;
    job_t b; memset(&b, 0, sizeof b);
    b.form = 1; b.code = code; b.loff = off; b.lcst = cst; b.lcst_off = cst_off; b.R = R;
    b.X = X; b.F = F; b.N = N; b.y = y; b.kind = kind; b.nudge = nudge;
    b.out = out; b.sums = sums;
    return run_population(b, P, n_threads);
}

/* ------------------------------------------------------------------------ */
/* The paper's representations (used to pin the oracle against the worked   */
/* example of section 5 and against each other).                            */
/* ------------------------------------------------------------------------ */

/* Prefix -> postfix (RPN): children first, left to right, then the node.    */
static int64_t to_postfix(const int32_t* tok, const float* cst, int64_t i, int64_t n,
                          int32_t* ot, float* oc, int64_t* w)
{
    int a = arity_of(tok[i] & 0xFF);
    int64_t j = i + 1;
    for (int q = 0; q < a; q++) {
        int64_t len = subtree_len(tok, j, n);
        if (len < 0) return -1;
        if (to_postfix(tok, cst, j, n, ot, oc, w) < 0) return -1;
        j += len;
    }
    ot[*w] = tok[i];
    oc[*w] = cst[i];
    (*w)++;
    return j - i;
}

int orc_prefix_to_rpn(const int32_t* tok, const float* cst, int64_t n,
                      int32_t* rpn_tok, float* rpn_cst)
{
    if (check_tree(tok, n, 1 << 23) != ORC_OK) return ORC_BAD;
    int64_t w = 0;
    return to_postfix(tok, cst, 0, n, rpn_tok, rpn_cst, &w) == n ? ORC_OK : ORC_BAD;
}

/* One-dimensional stack RPN interpreter for one case: push terminals; a
 * function pops its operands (the right one is on top) and pushes the
 * result.  Reports the largest stack height and the number of values the
 * functions fetched from the stack. */
int orc_rpn_eval(const int32_t* tok, const float* cst, int64_t n, const float* X,
                 int64_t N, int64_t c, float* result, int32_t* max_depth,
                 int32_t* stack_fetches)
{
    float st[4096];
    int sp = 0, hi = 0, fetch = 0;
    for (int64_t i = 0; i < n; i++) {
        int op = tok[i] & 0xFF;
        int a = arity_of(op);
        if (a < 0) return ORC_BAD;
        if (a == 0) {
            if (sp >= 4096) return ORC_BAD;
            st[sp++] = (op == O_VAR) ? X[(int64_t)((uint32_t)tok[i] >> 8) * N + c] : cst[i];
        } else if (a == 1) {
            if (sp < 1) return ORC_BAD;
            st[sp - 1] = apply_unary(op, st[sp - 1], 0);
            fetch += 1;
        } else if (a == 2) {
            if (sp < 2) return ORC_BAD;
            float b = st[--sp];
            float x = st[sp - 1];
            st[sp - 1] = apply_binary(op, x, b);
            fetch += 2;
        } else {
            if (sp < 3) return ORC_BAD;
            float d = st[--sp];
            float b = st[--sp];
            float x = st[sp - 1];
            st[sp - 1] = apply_ternary(op, x, b, d);
            fetch += 3;
        }
        if (sp > hi) hi = sp;
    }
    if (sp != 1) return ORC_BAD;
    if (result) *result = st[0];
    if (max_depth) *max_depth = hi;
    if (stack_fetches) *stack_fetches = fetch;
    return ORC_OK;
}

/* Paper LGP form produced from RPN with a symbolic stack (section 5).
 * Each instruction: op, n_args, and per argument a kind (0 = S, 1 = X,
 * 2 = C) with a feature index or constant.  Conversion: scan the RPN;
 * a terminal is pushed on the symbolic stack as itself; a function is
 * written out followed by the top `arity` symbols (deepest first, which is
 * the left-to-right operand order), those symbols are popped, and S is
 * pushed to stand for its result. */
typedef struct { int32_t op; int32_t n_args; int32_t kind[2]; int32_t feat[2]; float cval[2]; } orc_lgp_ins;

int orc_rpn_to_lgp(const int32_t* tok, const float* cst, int64_t n, orc_lgp_ins* out,
                   int64_t* n_out)
{
    int32_t sk[4096]; int32_t sf[4096]; float sc[4096];
    int sp = 0;
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++) {
        int op = tok[i] & 0xFF;
        int a = arity_of(op);
        if (a < 0 || a > 2) return ORC_BAD;     /* the record holds at most two operands */
        if (a == 0) {
            if (sp >= 4096) return ORC_BAD;
            sk[sp] = (op == O_VAR) ? 1 : 2;
            sf[sp] = (op == O_VAR) ? (int32_t)((uint32_t)tok[i] >> 8) : 0;
            sc[sp] = (op == O_CONST) ? cst[i] : 0.0f;
            sp++;
            continue;
        }
        if (sp < a) return ORC_BAD;
        orc_lgp_ins* ins = &out[m++];
        ins->op = op; ins->n_args = a;
        for (int q = 0; q < a; q++) {
            int s = sp - a + q;
            ins->kind[q] = sk[s]; ins->feat[q] = sf[s]; ins->cval[q] = sc[s];
        }
        sp -= a;
        sk[sp] = 0; sf[sp] = 0; sc[sp] = 0.0f;
        sp++;
    }
    if (sp != 1) return ORC_BAD;
    *n_out = m;
    return ORC_OK;
}

/* Interpreter of the paper's LGP form for one case: gather the operands
 * (X from the case, C from the instruction, S from the stack -- the S
 * operands of one instruction are the topmost entries, the left operand
 * being the deeper one), apply the function, push the result.  A program
 * that is a lone terminal has no instruction; its value is that terminal
 * and is supplied by the caller. */
int orc_lgp_eval(const orc_lgp_ins* ins, int64_t m, const float* X, int64_t N, int64_t c,
                 float* result, int32_t* max_depth, int32_t* stack_fetches)
{
    float st[4096];
    int sp = 0, hi = 0, fetch = 0;
    for (int64_t i = 0; i < m; i++) {
        const orc_lgp_ins* q = &ins[i];
        int ns = 0;
        for (int k = 0; k < q->n_args; k++) ns += (q->kind[k] == 0);
        if (sp < ns) return ORC_BAD;
        float v[2];
        int s = sp - ns;
        for (int k = 0; k < q->n_args; k++) {
            if (q->kind[k] == 0) v[k] = st[s++];
            else if (q->kind[k] == 1) v[k] = X[(int64_t)q->feat[k] * N + c];
            else v[k] = q->cval[k];
        }
        fetch += ns;
        sp -= ns;
        float r = (q->n_args == 1) ? apply_unary(q->op, v[0], 0) : apply_binary(q->op, v[0], v[1]);
        if (sp >= 4096) return ORC_BAD;
        st[sp++] = r;
        if (sp > hi) hi = sp;
    }
    if (m > 0 && sp != 1) return ORC_BAD;
    if (result && m > 0) *result = st[0];
    if (max_depth) *max_depth = hi;
    if (stack_fetches) *stack_fetches = fetch;
    return ORC_OK;
}

/* Single-operator reference for per-operation sweeps. */
float orc_apply(int op, float a, float b)
{
    return arity_of(op) == 1 ? apply_unary(op, a, 0) : apply_binary(op, a, b);
}

float orc_apply3(int op, float a, float b, float c)
{
    return apply_ternary(op, a, b, c);
}

int orc_sizeof_lgp_ins(void) { return (int)sizeof(orc_lgp_ins); }

/* ------------------------------------------------------------------------ */
/* Boolean trees over bit-packed cases (the multiplexer problem, sections 3  */
/* and 4.2: sub-machine-code GP evaluates 32 cases per machine word)         */
/* ------------------------------------------------------------------------ */
/* Functions AND, OR, NAND, NOR of two inputs; terminals are the inputs.
 * Case c is bit (c mod 32) of word (c div 32): X[f * W + w] holds input f for
 * cases 32w .. 32w + 31.  A bitwise function of two words is the function of
 * the two inputs for each of the 32 cases, so evaluating a tree on a word
 * evaluates it on 32 cases at once. */
enum { O_AND = 8, O_OR = 9, O_NAND = 10, O_NOR = 11 };

static int bool_arity(int op)
{
    switch (op) {
    case O_AND: case O_OR: case O_NAND: case O_NOR: return 2;
    case O_VAR: return 0;
    default: return -1;
    }
}

static int check_bool_tree(const int32_t* tok, int64_t n, int32_t F)
{
    int64_t need = 1;
    if (n <= 0) return ORC_BAD;
    for (int64_t i = 0; i < n; i++) {
        int a = bool_arity(tok[i] & 0xFF);
        if (a < 0 || need <= 0) return ORC_BAD;
        if (a == 0 && (int64_t)((uint32_t)tok[i] >> 8) >= F) return ORC_BAD;
        need += a - 1;
    }
    return need == 0 ? ORC_OK : ORC_BAD;
}

/* Recursive prefix interpreter on one word of 32 cases. */
static uint32_t eval_bool_prefix(const int32_t* tok, int64_t* i, const uint32_t* X, int64_t W, int64_t w)
{
    int32_t t = tok[*i];
    int op = t & 0xFF;
    (*i)++;
    if (op == O_VAR) return X[(int64_t)((uint32_t)t >> 8) * W + w];
    uint32_t a = eval_bool_prefix(tok, i, X, W, w);
    uint32_t b = eval_bool_prefix(tok, i, X, W, w);
    switch (op) {
    case O_AND: return a & b;
    case O_OR: return a | b;
    case O_NAND: return ~(a & b);
    default: return ~(a | b);      /* O_NOR */
    }
}

/* out[p*W + w] = word w of tree p's outputs, W = ceil(n_cases / 32) */
int orc_bool_outputs(const int32_t* tok, const int64_t* off, int32_t P, const uint32_t* X, int32_t F,
                     int64_t W, uint32_t* out)
{
    for (int32_t p = 0; p < P; p++) {
        const int32_t* t = tok + off[p];
        int64_t n = off[p + 1] - off[p];
        if (check_bool_tree(t, n, F) != ORC_OK) return ORC_BAD;
        for (int64_t w = 0; w < W; w++) {
            int64_t i = 0;
            out[(int64_t)p * W + w] = eval_bool_prefix(t, &i, X, W, w);
        }
    }
    return ORC_OK;
}

/* hits[p] = number of cases c < n_cases whose output bit equals y's bit,
 * counted case by case. */
int orc_bool_hits(const int32_t* tok, const int64_t* off, int32_t P, const uint32_t* X, int32_t F,
                  int64_t n_cases, const uint32_t* y, int64_t* hits)
{
    const int64_t W = (n_cases + 31) / 32;
    for (int32_t p = 0; p < P; p++) {
        const int32_t* t = tok + off[p];
        int64_t n = off[p + 1] - off[p];
        if (check_bool_tree(t, n, F) != ORC_OK) return ORC_BAD;
        int64_t h = 0;
        for (int64_t w = 0; w < W; w++) {
            int64_t i = 0;
            uint32_t o = eval_bool_prefix(t, &i, X, W, w);
            for (int b = 0; b < 32; b++) {
                int64_t c = 32 * w + b;
                if (c >= n_cases) break;
                if (((o >> b) & 1u) == ((y[w] >> b) & 1u)) h++;
            }
        }
        hits[p] = h;
    }
    return ORC_OK;
}
