/*
 * gp.h -- C ABI of the MI355X (gfx950) genetic-programming population
 * evaluator.
 *
 * What it computes.  For every candidate program p and every fitness case c
 * the library runs p on row c of a feature-major case matrix and reduces the
 * per-case errors to one fitness value per program.  This is the evaluation
 * phase of GP, the part of a GP run the paper accelerates: every program is
 * interpreted over every fitness case (sections 1, 3 and 4), and the paper's
 * two-dimensional stack applies each decoded instruction to a whole tile of
 * cases at once (section 4, Figure 1).  Trees are lowered on the host to the
 * paper's stack-operand linear form (operands X = case input, C = constant,
 * S = top of stack; section 5); register linear programs (dst, op, src1,
 * src2) are evaluated directly.
 *
 * Conventions shared by every entry point.
 *   - Return value: GP_OK (0) or a negative gp_status; gp_last_error() then
 *     holds a message for the calling thread.
 *   - Case data: X is DEVICE memory, float32, feature-major: the value of
 *     feature f on case c is X[f * n_cases + c].  y (targets or labels) is
 *     DEVICE memory, float32[n_cases].  Neither is copied; the caller keeps
 *     them alive until the stream has passed the call.
 *   - Programs are HOST memory (a GP run breeds them on the host); the
 *     library validates, lowers and copies them into its own buffers before
 *     the call returns, so the caller may reuse them at once.
 *   - out is DEVICE memory: float[n_prog] for GP_FIT_SUM_ABS and GP_FIT_MSE,
 *     int32[n_prog] for GP_FIT_HITS, float[n_prog * n_cases] (row p holds
 *     program p's outputs) for GP_OUT_CASES.
 *   - stream is a hipStream_t (NULL = the null stream).  Calls are stream
 *     ordered and asynchronous: out is valid once the stream has passed the
 *     call.  Library scratch (lowered programs, per-tile partial sums) is
 *     owned by the library and reused in stream order.
 *   - Arithmetic: IEEE binary32, round to nearest even, no contraction,
 *     denormals kept.  pdiv(a,b) = |b| < 1e-6f ? 1 : a/b; plog(a) =
 *     |a| < 1e-6f ? 0 : log|a|; expc(a) = exp(min(a, 88)) with NaN passing
 *     through; sin/cos/exp/log are evaluated in binary64 (the library's own
 *     table-driven range reduction and polynomials, no math-library call)
 *     and rounded once to binary32 (within 2 ulp of the exact value, and
 *     almost always the correctly rounded one).  The paper names these
 *     functions without defining their protection.
 *   - Fitness: d = out - y in binary32; sum of |d|, mean of d*d, or the
 *     number of cases with (out > 0) == (y > 0) (Table 2: mean squared error
 *     for regression, a count of classifications for classification).  Sums
 *     are accumulated in binary64 and rounded to binary32 once.
 *     GP_FIT_CLASS_ERR (Table 2: the sum of incorrect classifications) decodes
 *     each output to the class rint(out) (binary32, ties to even) and counts
 *     the cases where it differs from y, which holds class indices; a NaN or
 *     infinite output is never a class.  out is int32[n_prog], like hits.
 */
#ifndef GP_H_
#define GP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GP_OK = 0,
    GP_E_INVAL = -1,    /* malformed program, index out of range, null pointer, n_cases < 1, bad kind */
    GP_E_NOMEM = -2,    /* allocation failed, or a request can never fit a server's memory budget */
    GP_E_DEPTH = -3,    /* a program needs more stack levels or instructions than supported */
    GP_E_DEVICE = -4,   /* a HIP call failed; its message is in gp_last_error() */
    GP_E_AGAIN = -5,    /* a server queue is full */
    GP_E_NOTFOUND = -6, /* unknown dataset or ticket */
    GP_E_TIMEOUT = -7   /* a wait ran out of time */
} gp_status;

typedef enum {
    GP_FIT_SUM_ABS = 0,
    GP_FIT_MSE = 1,
    GP_FIT_HITS = 2,
    GP_OUT_CASES = 3,
    GP_FIT_CLASS_ERR = 4   /* classification: the number of cases whose decoded class differs from y */
} gp_fitness_kind;

/* Opcodes.  Tree token: low 8 bits = opcode, high 24 bits = feature index
 * for GP_VAR.  Linear word: op | dst << 8 | src1 << 16 | src2 << 24.
 *
 * The classification problems of section 4.2 (Shuttle, KDD Cup 99) add
 * {>, <, ==, AND, OR, IF} to the arithmetic functions.  The paper names them
 * only; the definitions here are: GP_GT, GP_LT, GP_EQ give 1.0f or 0.0f (a
 * NaN operand gives 0); in arithmetic trees GP_AND and GP_OR are the logical
 * functions, true (1.0f) when both / either operand is non-zero (NaN counts
 * as non-zero); GP_IF(a, b, c) = a != 0 ? b : c, the only three-operand
 * function (trees only: register programs reject it).  gp_eval_bool reads
 * GP_AND .. GP_NOR as bitwise functions of packed cases. */
enum {
    GP_ADD = 0, GP_SUB = 1, GP_MUL = 2, GP_PDIV = 3,
    GP_SIN = 4, GP_COS = 5, GP_EXPC = 6, GP_PLOG = 7,
    /* Boolean functions (bitwise on 32 packed cases in gp_eval_bool; logical in arithmetic trees) */
    GP_AND = 8, GP_OR = 9, GP_NAND = 10, GP_NOR = 11,
    /* classification functions */
    GP_GT = 12, GP_LT = 13, GP_EQ = 14, GP_IF = 15,
    GP_VAR = 64, GP_CONST = 65
};

/* Linear source ids: [0, n_reg) registers, [n_reg, n_reg + n_feat) features,
 * [GP_SRC_CONST, 256) the program's constants. */
#define GP_SRC_CONST 128
#define GP_MAX_REG 8          /* registers of a linear program */
#define GP_MAX_FEAT 44        /* features a program may read (the KDD Cup 99 shape has 41) */
/* Stack levels of a lowered tree.  Every tree of at most GP_MAX_LEN nodes
 * needs at most 20 (at most 15 without IF), so this limit never rejects a
 * valid tree; programs needing more than 12 run on deep kernel variants with
 * fewer waves per SIMD.  With more than 32 features read, 12 levels is the
 * most the register file holds beside them: deeper programs get GP_E_DEPTH. */
#define GP_MAX_DEPTH 20
#define GP_MAX_LEN 65536      /* instructions (tree nodes) per program */

/* ------------------------------------------------------------------------ */
/* One-shot evaluation                                                       */
/* ------------------------------------------------------------------------ */

/* Evaluate n_prog prefix trees.  tok/cst/off are HOST arrays in CSR form:
 * program p is tok[off[p] .. off[p+1]) with cst[i] the value of constant
 * token i.  Each tree is validated (arity, feature index < n_feat), lowered
 * to the stack-operand form with the deeper subtree evaluated first
 * (Sethi-Ullman order, which bounds the stack depth by log2 of the leaf
 * count) and run by the two-dimensional-stack kernel. */
gp_status gp_eval_tree(const int32_t* tok, const float* cst, const int64_t* off, int32_t n_prog,
                       const float* X, int32_t n_feat, int64_t n_cases, const float* y,
                       int32_t kind, void* out, void* stream);

/* Evaluate n_prog register linear programs over n_reg registers: the
 * register-machine linear GP form that section 5 compares against the tree
 * form (Table 8), in which each instruction reads two registers, inputs or
 * constants and writes one register.  code/off are HOST arrays in CSR form;
 * cst/cst_off (HOST, may be NULL when no program uses a constant) hold each
 * program's constant table.  Registers start as r[k] = x[k mod n_feat]; the
 * output is r[0]; unary functions read src1 only. */
gp_status gp_eval_linear(const uint32_t* code, const int64_t* off, const float* cst,
                         const int64_t* cst_off, int32_t n_prog, int32_t n_reg,
                         const float* X, int32_t n_feat, int64_t n_cases, const float* y,
                         int32_t kind, void* out, void* stream);

/* One-dimensional-stack comparator (the BlockGP design the paper measures
 * its 2D stack against: section 4.2, Tables 3 and 7).  One workgroup of 256
 * threads per program with the program copied into LDS; thread t evaluates
 * cases t, t + 256, ... one at a time with a stack of its own in private
 * (scratch) memory.  Same program, case, fitness and arithmetic conventions
 * as gp_eval_tree, and the same fitness values up to the order of the
 * binary64 summation.  form selects the interpreted code:
 *   GP_1D_RPN  the tree in postfix order (one instruction per node; operands
 *              popped from the stack, as in the paper's RPN interpreter);
 *   GP_1D_LGP  the tree lowered to the stack-operand linear form that
 *              gp_eval_tree also uses (section 5, Table 7).
 * Limits: at most GP_1D_MAX_LEN instructions per program (the program must
 * fit in LDS) and GP_1D_MAX_STACK stack values; GP_E_DEPTH beyond them.
 * Functions: the arithmetic and transcendental set (the paper's regression
 * problem); the classification functions give GP_E_INVAL.
 * kind GP_OUT_CASES writes the per-case outputs.  Meant for measurement;
 * gp_eval_tree is the evaluator. */
enum { GP_1D_RPN = 0, GP_1D_LGP = 1 };
#define GP_1D_MAX_LEN 4096
#define GP_1D_MAX_STACK 64
gp_status gp_eval_tree_1d(const int32_t* tok, const float* cst, const int64_t* off, int32_t n_prog,
                          const float* X, int32_t n_feat, int64_t n_cases, const float* y,
                          int32_t kind, int32_t form, void* out, void* stream);

/* Sub-machine-code evaluation of Boolean trees (the paper's multiplexer
 * problem: sections 3 and 4.2, Table 2 and the last row of Tables 3-10).
 * Cases are bit-packed: bit b of word w is case 32 * w + b, and every
 * function is applied to 32 cases at once with one bitwise operation, so
 * one interpreted instruction covers 64 lanes x T words x 32 cases.
 *   tok/off  HOST prefix trees in CSR form over GP_AND, GP_OR, GP_NAND,
 *            GP_NOR (binary) and GP_VAR terminals; no constants.
 *   X        DEVICE uint32, feature-major: word w of input f is
 *            X[f * n_words + w], n_words = ceil(n_cases / 32).
 *   y        DEVICE uint32[n_words], the target bits.
 *   kind     GP_FIT_HITS: out is DEVICE int32[n_prog], the number of cases
 *            whose output bit equals the target bit (bits past n_cases in
 *            the last word are ignored); GP_OUT_CASES: out is DEVICE
 *            uint32[n_prog * n_words], the output words (y may be NULL).
 * n_cases is at most 2^31 - 1.  GP_E_INVAL for any other opcode or kind, GP_E_DEPTH for programs deeper
 * than the Boolean kernels' stacks.  GP operations are counted per case:
 * nodes x n_cases. */
gp_status gp_eval_bool(const int32_t* tok, const int64_t* off, int32_t n_prog, const uint32_t* X,
                       int32_t n_feat, int64_t n_cases, const uint32_t* y, int32_t kind, void* out,
                       void* stream);

/* ------------------------------------------------------------------------ */
/* GP runs around the evaluator.  The paper measures GPop/s over whole GP   */
/* runs with the parameters of Table 2; these calls breed tree populations  */
/* on the host (Koza-style tree GP) and evaluate every generation with      */
/* gp_eval_tree, or gp_eval_bool for the Boolean function set.              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t pop_size;          /* Table 2: 1000 */
    int32_t generations;       /* generations bred after the initial one; Table 2: 50 */
    int32_t max_depth;         /* edges from the root; Table 2: 50 */
    int32_t max_size;          /* nodes; Table 2: 1000 */
    int32_t tournament;        /* Table 2: 7 */
    float p_crossover;         /* Table 2: 0.95 */
    float p_mutation;          /* Table 2: 0.2 */
    int32_t init_min_depth;    /* ramped half-and-half range, e.g. 2 .. 6 */
    int32_t init_max_depth;
    int32_t mutation_depth;    /* depth limit of a mutation's new subtree, e.g. 4 */
    uint32_t functions;        /* bit k set: opcode k (GP_ADD .. GP_IF) is in the function set; the
                                  Boolean set is GP_AND .. GP_NOR alone, an arithmetic set may add
                                  the classification functions (GP_AND, GP_OR logical) */
    float p_const;             /* probability that a terminal is a constant (arithmetic sets) */
    float const_lo, const_hi;  /* constants uniform in [const_lo, const_hi) */
    int32_t kind;              /* GP_FIT_MSE, GP_FIT_SUM_ABS or GP_FIT_CLASS_ERR (minimised) or
                                  GP_FIT_HITS (maximised; the only kind for Boolean sets) */
    uint64_t seed;             /* SplitMix64 seed: a run is reproducible from it */
} gp_evolve_config;

typedef struct {
    double best_fitness;       /* of the best program seen: its error, or its hit count */
    int32_t best_generation;
    int32_t best_size;         /* nodes */
    int32_t generations_run;   /* evaluated generations, the initial one included */
    int32_t pad;
    int64_t gp_ops;            /* sum over evaluations of tree nodes x cases */
    double eval_seconds;       /* host lowering, upload, kernels and fitness copy-back */
    double breed_seconds;      /* selection, crossover and mutation on the host */
    double total_seconds;      /* the whole run */
} gp_evolve_result;

/* One GP run on a case matrix: X, y as for gp_eval_tree (arithmetic sets) or
 * gp_eval_bool (Boolean sets, n_cases in bits).  best_per_gen (HOST, may be
 * NULL) receives the best fitness so far after each generation
 * (generations + 1 values); best_tok/best_cst (HOST, may be NULL) receive
 * the best program if best_cap >= its size.  Synchronous on `stream`. */
gp_status gp_evolve(const gp_evolve_config* cfg, const void* X, int32_t n_feat, int64_t n_cases, const void* y,
                    double* best_per_gen, int32_t* best_tok, float* best_cst, int32_t best_cap,
                    gp_evolve_result* res, void* stream);
/* The run's host steps on their own (no device needed), for inspection and
 * tests.  gp_init_population writes cfg->pop_size ramped half-and-half trees
 * in CSR form (off has pop_size + 1 entries).  gp_breed takes a population
 * of cfg->pop_size trees (cst may be NULL for Boolean sets) and each
 * program's score (lower is better; NaN is worst) and writes the next
 * generation, with random numbers from `seed`.  GP_E_NOMEM if the result
 * exceeds max_tokens. */
gp_status gp_init_population(const gp_evolve_config* cfg, int32_t n_feat, int32_t* tok, float* cst, int64_t* off,
                             int64_t max_tokens);
gp_status gp_breed(const gp_evolve_config* cfg, const int32_t* tok, const float* cst, const int64_t* off,
                   int32_t n_feat, const double* score, uint64_t seed, int32_t* out_tok, float* out_cst,
                   int64_t* out_off, int64_t max_tokens);

/* ------------------------------------------------------------------------ */
/* Resident program sets: lower and upload once, evaluate many times        */
/* (a GP generation evaluated on several datasets, or timed repeatedly).    */
/* ------------------------------------------------------------------------ */
typedef struct gp_progset gp_progset;

typedef struct {
    int32_t n_prog;
    int32_t form;              /* 0 = tree, 1 = linear */
    int32_t n_feat;            /* features the programs may read */
    int32_t max_depth;         /* stack levels needed (trees) */
    int64_t n_instr;           /* device instructions over all programs */
    int64_t n_gpop;            /* GP operations per fitness case: tree nodes, or linear instructions */
    int32_t variant;           /* kernel variant gp_progset_eval launches for the set */
    int32_t pad;
} gp_progset_info;

/* Same program arguments as gp_eval_tree / gp_eval_linear.  The upload is
 * stream ordered on `stream`; *ps is owned by the caller until
 * gp_progset_destroy. */
gp_status gp_progset_tree(const int32_t* tok, const float* cst, const int64_t* off, int32_t n_prog,
                          int32_t n_feat, void* stream, gp_progset** ps);
gp_status gp_progset_linear(const uint32_t* code, const int64_t* off, const float* cst,
                            const int64_t* cst_off, int32_t n_prog, int32_t n_reg, int32_t n_feat,
                            void* stream, gp_progset** ps);
/* Boolean trees as in gp_eval_bool.  gp_progset_eval then takes X and y as
 * DEVICE uint32 words (bit-packed cases, as in gp_eval_bool), n_cases counts
 * cases (bits), and kind is GP_FIT_HITS or GP_OUT_CASES. */
gp_status gp_progset_bool(const int32_t* tok, const int64_t* off, int32_t n_prog, int32_t n_feat, void* stream,
                          gp_progset** ps);
/* Evaluate a resident set on a case matrix with n_feat >= the set's n_feat. */
gp_status gp_progset_eval(gp_progset* ps, const float* X, int32_t n_feat, int64_t n_cases,
                          const float* y, int32_t kind, void* out, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as gp_progset_eval, bit for bit, with nothing allocated and
 * nothing copied from the host during the call -- it launches the evaluation
 * and reduction kernels on `stream` and returns.  The programs and their
 * layout were uploaded when the set was created (on this device).  The
 * per-(program, 256-case block) partial sums go to a fixed device array of
 * GP_NOALLOC_MAX_PARTIALS doubles (16 MiB) that each GPU the library runs on
 * holds until the process ends: n_prog * ceil(n_cases / 256) (Boolean sets:
 * ceil(n_cases / 8192)) must not exceed it, else GP_E_NOMEM and nothing is
 * launched; GP_OUT_CASES needs none.  Every call on one GPU shares that
 * array and leaves its partial sums there: calls that overlap on one GPU
 * (different streams or threads without ordering between them) race and may
 * return wrong fitness values.  Calls in order on one stream are safe. */
#define GP_NOALLOC_MAX_PARTIALS 2097152
gp_status gp_progset_eval_noalloc(gp_progset* ps, const float* X, int32_t n_feat, int64_t n_cases,
                                  const float* y, int32_t kind, void* out, void* stream);
gp_status gp_progset_get_info(const gp_progset* ps, gp_progset_info* info);
/* Waits for the device to finish with the set, then frees it. */
gp_status gp_progset_destroy(gp_progset* ps);

/* ------------------------------------------------------------------------ */
/* Batched evaluation: several populations (trees and linear programs) over */
/* several resident case matrices in one persistent launch.  Work is cut   */
/* into (case tile, program group) units, sorted longest first and pulled  */
/* by the chip's resident wavefronts from a global counter.  Fitness values */
/* are the same as from gp_eval_tree / gp_eval_linear, bit for bit.        */
/* ------------------------------------------------------------------------ */
typedef struct {
    const float* X;            /* DEVICE, feature-major float32[n_feat * n_cases] */
    int32_t n_feat;
    int64_t n_cases;
    const float* y;            /* DEVICE, float32[n_cases] */
} gp_dataset;

enum { GP_FORM_TREE = 0, GP_FORM_LINEAR = 1 };

typedef struct {
    int32_t form;              /* GP_FORM_TREE or GP_FORM_LINEAR */
    int32_t n_prog;
    int32_t dataset;           /* index into the dataset array */
    int32_t kind;              /* GP_FIT_SUM_ABS, GP_FIT_MSE or GP_FIT_HITS */
    /* trees (HOST, as in gp_eval_tree) */
    const int32_t* tok;
    const float* tcst;
    const int64_t* toff;
    /* linear programs (HOST, as in gp_eval_linear) */
    const uint32_t* code;
    const int64_t* loff;
    const float* lcst;
    const int64_t* lcst_off;
    int32_t n_reg;
    void* out;                 /* DEVICE: float[n_prog] or int32[n_prog] (hits) */
} gp_job;

typedef struct {
    int32_t variant;           /* kernel variant (tile width, stack depth, feature slots) */
    int32_t unit_programs;     /* programs per work unit */
    int32_t persistent;        /* 1: resident waves pull units longest first; 0: one wave per unit */
    int32_t reserved;
} gp_batch_config;

/* cfg NULL: the configuration the autotuner stored for this batch shape,
 * else a default.  Stream ordered and asynchronous like gp_eval_tree. */
gp_status gp_eval_batch(const gp_dataset* ds, int32_t n_ds, const gp_job* jobs, int32_t n_jobs,
                        const gp_batch_config* cfg, void* stream);
/* Time every candidate configuration `reps` times on this batch (runs on
 * `stream` and synchronizes on it), store the fastest for the batch's shape
 * and return it with its median time.  The store is kept in memory and, when
 * the environment names a file in GP2D_TUNE_CACHE, in that JSON file. */
gp_status gp_tune_batch(const gp_dataset* ds, int32_t n_ds, const gp_job* jobs, int32_t n_jobs, int32_t reps,
                        gp_batch_config* best, double* best_ms, void* stream);
/* Compiled kernel variants: tile width t (case slots per lane), stack levels,
 * feature slots, the VGPRs left to compiled code (the interpreter core owns
 * the VGPRs from that number up) and flags: GP_VARIANT_NO_TRANSC marks a
 * kernel without sin/cos/exp/log code, used for programs without them;
 * GP_VARIANT_BOOLEAN (with GP_VARIANT_NO_TRANSC) a kernel of the Boolean
 * function set for gp_eval_bool, whose slots are 32-bit words;
 * GP_VARIANT_TREES_ONLY (with GP_VARIANT_NO_TRANSC) an arithmetic kernel for
 * trees only (no linear-program handlers), which one-shot and program-set
 * evaluations of trees prefer and batches do not use.  The variant's kernel
 * is named k_core_<t>_<depth>_<n_feat>_<vgprs>, with "_a" appended for an
 * arithmetic-only, "_at" for a trees-only and "_b" for a Boolean kernel.  Any
 * pointer may be NULL. */
enum { GP_VARIANT_NO_TRANSC = 1, GP_VARIANT_BOOLEAN = 2, GP_VARIANT_TREES_ONLY = 4 };
int32_t gp_num_variants(void);
gp_status gp_variant_info(int32_t i, int32_t* t, int32_t* depth, int32_t* n_feat, int32_t* vgprs, int32_t* flags);

/* ------------------------------------------------------------------------ */
/* Serving: concurrent GP runs submit population evaluations against        */
/* datasets resident in device memory.  A scheduler thread admits requests  */
/* while their device memory fits the budget (FIFO), fuses the admitted     */
/* ones into one batched launch and keeps up to n_streams launches in       */
/* flight, so requests arriving while the GPU is busy start as soon as a    */
/* stream frees up (continuous batching).  A request's fitness values are   */
/* bit-identical to evaluating it alone.                                    */
/* ------------------------------------------------------------------------ */
typedef struct gp_server gp_server;

typedef struct {
    size_t memory_budget;      /* device bytes admitted work may hold (lowered programs, unit
                                  tables, partial sums); 0 = 4 GiB */
    int32_t max_queue;         /* requests waiting for admission; beyond it submit returns
                                  GP_E_AGAIN; 0 = 1024 */
    int32_t n_streams;         /* batched launches in flight at once; 0 = 2, at most 8 */
    int32_t max_batch;         /* requests fused into one launch; 0 = 64 */
    int32_t batching;          /* 0: one launch per request on one stream (the comparison
                                  baseline); nonzero: continuous batching */
    int32_t dry_run;           /* nonzero: schedule without a device -- nothing is launched and
                                  outputs are not written; a batch "runs" for its GP operation
                                  count divided by dry_run_gpops seconds (for testing the
                                  scheduler) */
    int32_t hip_streams;       /* HIP streams the in-flight launches go to: launch slot k uses
                                  stream k mod hip_streams; 0 or 1 = one stream, so the next
                                  launch queues behind the running one (the GPU neither idles
                                  while the host prepares it nor splits its CUs between two
                                  batches); n_streams = one stream per slot */
    double dry_run_gpops;
} gp_serve_config;

typedef struct {
    int64_t submitted, admitted, completed, rejected, cancelled, failed;
    int32_t queue_depth;       /* requests waiting for admission */
    int32_t in_flight_batches;
    int64_t bytes_in_flight;   /* admitted, unfinished requests */
    int64_t batches;
    double mean_batch;         /* requests per launch */
    double p50_us, p99_us;     /* submit-to-completion latency over recent requests */
    double gpops_per_s;        /* GP operations completed / (last completion - first submit) */
} gp_serve_stats_t;

gp_status gp_serve_create(const gp_serve_config* cfg, gp_server** s);
/* Register a resident dataset (DEVICE pointers, kept alive by the caller
 * until gp_serve_destroy); *id is its index for requests. */
gp_status gp_serve_add_dataset(gp_server* s, const float* X, int32_t n_feat, int64_t n_cases, const float* y,
                               int32_t* id);
/* Validate and lower the request's programs on the calling thread, then
 * queue it.  req->dataset is a dataset id.  GP_E_NOMEM if it can never fit
 * the budget, GP_E_AGAIN if the queue is full, GP_E_NOTFOUND for an unknown
 * dataset.  Programs are copied; req->out must stay valid until done. */
gp_status gp_serve_submit(gp_server* s, const gp_job* req, uint64_t* ticket);
/* *done = 1 once the request finished (returns its failure status if it failed). */
gp_status gp_serve_poll(gp_server* s, uint64_t ticket, int32_t* done);
/* Wait for completion; timeout_us < 0 waits forever.  GP_E_TIMEOUT if it
 * did not finish in time. */
gp_status gp_serve_wait(gp_server* s, uint64_t ticket, int64_t timeout_us);
/* Cancel a request that has not been admitted yet (GP_E_AGAIN otherwise). */
gp_status gp_serve_cancel(gp_server* s, uint64_t ticket);
/* Forget a finished ticket. */
gp_status gp_serve_release(gp_server* s, uint64_t ticket);
gp_status gp_serve_stats(gp_server* s, gp_serve_stats_t* out);
/* Cancel queued requests, wait for launched ones, free everything. */
gp_status gp_serve_destroy(gp_server* s);

/* ------------------------------------------------------------------------ */
/* Host-side lowering, exposed for inspection and tests (no GPU needed).    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_nodes;           /* tree nodes (GP operations per case) */
    int32_t n_instr;           /* stack-operand instructions after lowering */
    int32_t max_depth;         /* stack levels the lowered program needs */
    int32_t stack_fetches;     /* S operands read from the stack */
    int32_t n_values;          /* functions plus operands in the lowered form */
    int32_t n_reversed;        /* instructions whose right operand was evaluated first */
} gp_lower_stats;

/* Lower one prefix tree (tok/cst HOST, n tokens).  words (HOST, may be NULL)
 * receives 2 * n_instr uint32 words of device code when non-NULL and
 * max_words is large enough. */
gp_status gp_lower_tree(const int32_t* tok, const float* cst, int64_t n, int32_t n_feat,
                        uint32_t* words, int64_t max_words, gp_lower_stats* stats);

/* Translate programs into the instruction stream of kernel variant
 * `variant`'s interpreter core (trees of the Boolean function set for a
 * GP_VARIANT_BOOLEAN variant, cst then unused), taking its handler table to start at
 * table_base (64-byte aligned; the library finds the real address on the
 * device itself).  Host only.  Each core instruction is 4 uint32 words:
 * handler address (2 words), operand offsets, constant.  words (may be
 * NULL) receives n_words words if max_words allows; prog_off (may be NULL)
 * receives n_prog + 1 word offsets. */
gp_status gp_core_lower_tree(const int32_t* tok, const float* cst, const int64_t* off, int32_t n_prog,
                             int32_t n_feat, int32_t variant, uint64_t table_base, uint32_t* words,
                             int64_t max_words, int64_t* prog_off, int64_t* n_words);
gp_status gp_core_lower_linear(const uint32_t* code, const int64_t* off, const float* cst, const int64_t* cst_off,
                               int32_t n_prog, int32_t n_reg, int32_t n_feat, int32_t variant,
                               uint64_t table_base, uint32_t* words, int64_t max_words, int64_t* prog_off,
                               int64_t* n_words);

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                               */
/* ------------------------------------------------------------------------ */
/* Kernel timing.  While enabled, every evaluation-kernel launch is bracketed
 * by two HIP events recorded on its launch stream.  gp_timing_read waits
 * for the recorded launches, returns how many there were and their summed
 * duration in milliseconds, and forgets them when reset != 0.  Timing is a
 * process-wide switch; it is off by default. */
gp_status gp_timing_enable(int on);
gp_status gp_timing_read(int64_t* launches, double* total_ms, int reset);

/* Launch-shape overrides for tuning and tests, read from the environment at
 * every one-shot or program-set evaluation: GP2D_GROUP_INSTR (core
 * instructions per program group), GP2D_TILES_PER_WAVE (case tiles each
 * wavefront walks per group), GP2D_TARGET_BLOCKS (workgroups the launch aims
 * for), GP2D_CODE_PREFETCH=n (scalar loads in flight, 1-15, when each
 * program's code is burst-loaded into the scalar cache; 15 by default, 0
 * for no burst load), GP2D_SAME_GROUP=1 (the four waves of a block run one program
 * group on four chunks of tiles instead of four groups on one chunk),
 * GP2D_VARIANT=i+1 (kernel variant i of gp_variant_info, when it can hold the
 * programs).  They change the schedule only; fitness values never depend on
 * them. */

/* Message of the last failed call on this thread ("" if none). */
const char* gp_last_error(void);
/* Library version string. */
const char* gp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GP_H_ */
