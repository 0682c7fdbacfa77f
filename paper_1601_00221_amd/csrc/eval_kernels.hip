// HIP kernels (gfx950) of the GP population evaluator.
//
// Work decomposition.  One wavefront owns a case tile of 64 lanes x T
// slots: slot j of lane l holds case  tile*64*T + j*64 + l, so every load of
// a feature row is one contiguous 256-byte access (the paper strides the
// cases of one thread by the thread count for the same reason, section 4.1).
// The wave loads its tile's features and targets into VGPRs once and then
// interprets a group of programs on it.  Every lane runs the same program,
// so instruction words are wave-uniform scalar loads and the dispatch branch
// is taken by the whole wave.
//
// Two-dimensional stack (section 4): stack level k of slot j lives in
// register st[j][k]; one decoded instruction updates all T slots of all 64
// lanes, so interpretation cost is paid once per 64*T cases.  The stack
// pointer is wave-uniform, so a level is selected with the gfx9 VGPR index
// mode instead of memory -- the paper keeps the lowest levels in registers
// for the same reason (section 6.2) but needs a switch per access.
//
// Fitness: per-slot error terms in binary32, per-lane binary64 sums, a
// wavefront butterfly reduction, one partial per (program, tile), then a
// fixed-order reduction over tiles -- the result does not depend on how
// programs were grouped or scheduled.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gp.h"
#include "gp_internal.h"
#include "kernels.h"

namespace gpx {

template <int T> using vec_t = float __attribute__((ext_vector_type(T)));
// Register-resident arrays that are indexed by a wave-uniform value.  The
// compiler turns a uniform dynamic index into one s_set_gpr_idx move only
// when the vector has more than 8 elements (smaller ones become a chain of
// compares and selects), so such arrays are at least 9 wide.
template <int N> struct idx_width { static constexpr int value = N < 9 ? 9 : N; };
template <int N> using ivec_t = vec_t<idx_width<N>::value>;

// --------------------------------------------------------------------------
// Operators
//
// sin, cos, exp and log are evaluated in binary64 and rounded once to
// binary32.  Random GP trees chain many of them and most such programs turn
// a last-place difference into a visible fitness difference, so a binary32
// library result (a few units in the last place) would make fitness depend
// on the evaluator; one rounding of an accurate binary64 value gives the
// correctly rounded binary32 result except when the value lies almost
// exactly between two binary32 numbers.
// --------------------------------------------------------------------------
__device__ __forceinline__ float pdiv(float a, float b) {
    return (fabsf(b) < 1e-6f) ? 1.0f : a / b;
}
__device__ __forceinline__ float gsin(float a) { return (float)sin((double)a); }
__device__ __forceinline__ float gcos(float a) { return (float)cos((double)a); }
__device__ __forceinline__ float expc(float a) {
    const float t = (a > 88.0f) ? 88.0f : a;   // a NaN fails the compare and passes through
    return (float)exp((double)t);
}
__device__ __forceinline__ float plog(float a) {
    const float m = fabsf(a);
    return (m < 1e-6f) ? 0.0f : (float)log((double)m);
}

template <int T>
__device__ __forceinline__ ivec_t<T> apply_op(uint32_t op, const ivec_t<T>& A, const ivec_t<T>& B) {
    ivec_t<T> R;
    switch (op) {
        case GP_ADD:
#pragma unroll
            for (int j = 0; j < T; j++) R[j] = A[j] + B[j];
            break;
        case GP_SUB:
#pragma unroll
            for (int j = 0; j < T; j++) R[j] = A[j] - B[j];
            break;
        case GP_MUL:
#pragma unroll
            for (int j = 0; j < T; j++) R[j] = A[j] * B[j];
            break;
        case GP_PDIV:
#pragma unroll
            for (int j = 0; j < T; j++) R[j] = pdiv(A[j], B[j]);
            break;
        // The transcendentals are long; a rolled loop keeps one copy of each.
        case GP_SIN:
#pragma unroll 1
            for (int j = 0; j < T; j++) R[j] = gsin(A[j]);
            break;
        case GP_COS:
#pragma unroll 1
            for (int j = 0; j < T; j++) R[j] = gcos(A[j]);
            break;
        case GP_EXPC:
#pragma unroll 1
            for (int j = 0; j < T; j++) R[j] = expc(A[j]);
            break;
        case GP_PLOG:
#pragma unroll 1
            for (int j = 0; j < T; j++) R[j] = plog(A[j]);
            break;
        default:  // OP_PUSH
            R = A;
            break;
    }
    return R;
}

// --------------------------------------------------------------------------
// Interpreters.  fx[j][f] = feature f of slot j.
// --------------------------------------------------------------------------
template <int T, int D, int FV>
__device__ __forceinline__ vec_t<T> run_tree(const uint32_t* __restrict__ code, uint32_t len,
                                             const ivec_t<FV> (&fx)[T]) {
    ivec_t<D> st[T];
#pragma unroll
    for (int j = 0; j < T; j++) st[j] = ivec_t<D>(0.0f);
    int h = 0;
    for (uint32_t ip = 0; ip < len; ++ip) {
        const uint32_t w0 = code[2 * ip];
        const float c = __uint_as_float(code[2 * ip + 1]);
        const uint32_t op = w0 & 15u, mode = (w0 >> 4) & 15u;
        const uint32_t fa = (w0 >> 8) & 255u, fb = (w0 >> 16) & 255u;
        ivec_t<T> A, B;
        int dst;
        switch (mode) {
            case M_SS:
#pragma unroll
                for (int j = 0; j < T; j++) { A[j] = st[j][h - 2]; B[j] = st[j][h - 1]; }
                dst = h - 2; h -= 1;
                break;
            case M_SSR:
#pragma unroll
                for (int j = 0; j < T; j++) { A[j] = st[j][h - 1]; B[j] = st[j][h - 2]; }
                dst = h - 2; h -= 1;
                break;
            case M_SX:
#pragma unroll
                for (int j = 0; j < T; j++) { A[j] = st[j][h - 1]; B[j] = fx[j][fb]; }
                dst = h - 1;
                break;
            case M_XS:
#pragma unroll
                for (int j = 0; j < T; j++) { A[j] = fx[j][fa]; B[j] = st[j][h - 1]; }
                dst = h - 1;
                break;
            case M_SC:
#pragma unroll
                for (int j = 0; j < T; j++) { A[j] = st[j][h - 1]; B[j] = c; }
                dst = h - 1;
                break;
            case M_CS:
#pragma unroll
                for (int j = 0; j < T; j++) { A[j] = c; B[j] = st[j][h - 1]; }
                dst = h - 1;
                break;
            case M_XX:
#pragma unroll
                for (int j = 0; j < T; j++) { A[j] = fx[j][fa]; B[j] = fx[j][fb]; }
                dst = h; h += 1;
                break;
            case M_XC:
#pragma unroll
                for (int j = 0; j < T; j++) { A[j] = fx[j][fa]; B[j] = c; }
                dst = h; h += 1;
                break;
            case M_CX:
#pragma unroll
                for (int j = 0; j < T; j++) { A[j] = c; B[j] = fx[j][fb]; }
                dst = h; h += 1;
                break;
            case M_S:
#pragma unroll
                for (int j = 0; j < T; j++) A[j] = st[j][h - 1];
                dst = h - 1;
                break;
            case M_X:
#pragma unroll
                for (int j = 0; j < T; j++) A[j] = fx[j][fa];
                dst = h; h += 1;
                break;
            default:  // M_C
#pragma unroll
                for (int j = 0; j < T; j++) A[j] = c;
                dst = h; h += 1;
                break;
        }
        const ivec_t<T> R = apply_op<T>(op, A, B);
#pragma unroll
        for (int j = 0; j < T; j++) st[j][dst] = R[j];
    }
    vec_t<T> o;
#pragma unroll
    for (int j = 0; j < T; j++) o[j] = st[j][0];
    return o;
}

template <int T, int FV>
__device__ __forceinline__ vec_t<T> run_linear(const uint32_t* __restrict__ code, uint32_t len,
                                               int n_reg, int n_feat, const ivec_t<FV> (&fx)[T]) {
    ivec_t<GP_MAX_REG> r[T];
    for (int k = 0; k < n_reg; k++) {
        const int f = k % n_feat;
#pragma unroll
        for (int j = 0; j < T; j++) r[j][k] = fx[j][f];
    }
    const uint32_t* __restrict__ cst = code + len;
    for (uint32_t ip = 0; ip < len; ++ip) {
        const uint32_t w = code[ip];
        const uint32_t op = w & 255u, dst = (w >> 8) & 255u;
        const int s1 = (int)((w >> 16) & 255u), s2 = (int)(w >> 24);
        ivec_t<T> A, B;
        if (s1 < n_reg) {
#pragma unroll
            for (int j = 0; j < T; j++) A[j] = r[j][s1];
        } else if (s1 < GP_SRC_CONST) {
#pragma unroll
            for (int j = 0; j < T; j++) A[j] = fx[j][s1 - n_reg];
        } else {
            const float c = __uint_as_float(cst[s1 - GP_SRC_CONST]);
#pragma unroll
            for (int j = 0; j < T; j++) A[j] = c;
        }
        if (op < GP_SIN) {
            if (s2 < n_reg) {
#pragma unroll
                for (int j = 0; j < T; j++) B[j] = r[j][s2];
            } else if (s2 < GP_SRC_CONST) {
#pragma unroll
                for (int j = 0; j < T; j++) B[j] = fx[j][s2 - n_reg];
            } else {
                const float c = __uint_as_float(cst[s2 - GP_SRC_CONST]);
#pragma unroll
                for (int j = 0; j < T; j++) B[j] = c;
            }
        }
        const ivec_t<T> R = apply_op<T>(op, A, B);
#pragma unroll
        for (int j = 0; j < T; j++) r[j][dst] = R[j];
    }
    vec_t<T> o;
#pragma unroll
    for (int j = 0; j < T; j++) o[j] = r[j][0];
    return o;
}

// --------------------------------------------------------------------------
// One unit of work: a wave's case tile and a range of programs.
//
// Partial sums are formed per block of 256 consecutive cases (4 slots of
// every lane): each lane adds its 4 terms in slot order, the wave adds the
// 64 lane sums with a fixed butterfly, and block b of program p is stored at
// part_base + b * part_stride.  The same blocks arise for any tile width, so
// a program's fitness does not depend on the kernel variant, on how programs
// were grouped, or on what else shared the launch.
// --------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, 64);
    return v;
}

struct UnitCtx {
    const uint32_t* code;
    const DevProg* progs;
    const uint32_t* order;
    const float* X;
    const float* y;
    double* partials;
    float* cases_out;
    int64_t N;
    int32_t n_load;
    int32_t n_feat_prog;
    int32_t kind;
};

template <int T, int D, int FV>
__device__ __forceinline__ void process_unit(const UnitCtx& a, uint32_t tile, uint32_t q0, uint32_t q1) {
    static_assert(T % 4 == 0, "a tile holds whole 256-case blocks");
    const uint32_t lane = threadIdx.x & 63u;
    const int64_t N = a.N;
    const int64_t base = (int64_t)tile * (64 * T) + lane;
    const int64_t n_blocks = (N + 255) / 256;
    ivec_t<FV> fx[T];
    vec_t<T> yv;
    bool valid[T];
#pragma unroll
    for (int j = 0; j < T; j++) {
        const int64_t c = base + 64 * j;
        valid[j] = c < N;
#pragma unroll
        for (int f = 0; f < FV; f++)
            fx[j][f] = (f < a.n_load && valid[j]) ? a.X[(int64_t)f * N + c] : 0.0f;
        yv[j] = (a.y != nullptr && valid[j]) ? a.y[c] : 0.0f;
    }

    for (uint32_t q = q0; q < q1; ++q) {
        const DevProg P = a.progs[a.order[q]];
        vec_t<T> o;
        if ((P.meta & 1u) == FORM_TREE)
            o = run_tree<T, D, FV>(a.code + P.code_off, P.len, fx);
        else
            o = run_linear<T, FV>(a.code + P.code_off, P.len, (int)((P.meta >> 8) & 255u),
                                  a.n_feat_prog, fx);

        if (a.kind == GP_OUT_CASES) {
            float* row = a.cases_out + (int64_t)P.row * N;
#pragma unroll
            for (int j = 0; j < T; j++)
                if (valid[j]) row[base + 64 * j] = o[j];
            continue;
        }
#pragma unroll
        for (int k = 0; k < T / 4; k++) {
            const int64_t blk = (int64_t)tile * (T / 4) + k;
            double v;
            if (a.kind == GP_FIT_HITS) {
                uint32_t hits = 0;
#pragma unroll
                for (int j = 4 * k; j < 4 * k + 4; j++) {
                    const bool hit = valid[j] && ((o[j] > 0.0f) == (yv[j] > 0.0f));
                    hits += (uint32_t)__popcll(__ballot(hit));
                }
                v = (double)hits;
            } else {
                double acc = 0.0;
#pragma unroll
                for (int j = 4 * k; j < 4 * k + 4; j++) {
                    const float d = o[j] - yv[j];
                    const float t = (a.kind == GP_FIT_MSE) ? d * d : fabsf(d);
                    acc += valid[j] ? (double)t : 0.0;
                }
                v = wave_sum(acc);
            }
            if (lane == 0 && blk < n_blocks) a.partials[P.part_base + (uint64_t)blk * P.part_stride] = v;
        }
    }
}

// Plain evaluation: unit u = (tile, group) with tile = u mod tiles.
template <int T, int D, int FV>
__global__ __launch_bounds__(256) void k_eval(EvalArgs a) {
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // Blocks go to the 8 XCDs round robin; give each XCD a contiguous range
    // of units so a program group's code stays in one L2.
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    const uint32_t lb = (b & 7u) * (nb >> 3) + (b >> 3);
    const uint32_t u = lb * 4u + wib;
    if (u >= (uint32_t)a.n_units) return;
    const uint32_t tile = u % (uint32_t)a.tiles;
    const uint32_t grp = u / (uint32_t)a.tiles;
    UnitCtx c{a.code, a.progs, a.order, a.X, a.y, a.partials, a.cases_out, a.N, a.n_load, a.n_feat_prog, a.kind};
    process_unit<T, D, FV>(c, tile, a.group_off[grp], a.group_off[grp + 1]);
}

// Batched evaluation over several jobs and datasets.  Persistent form: each
// wave takes the next unit from a global counter until none is left (units
// are sorted longest first on the host).  Static form: one wave per unit.
template <int T, int D, int FV>
__global__ __launch_bounds__(256) void k_batch(BatchArgs a) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t u = 0;
    if (!a.persistent) {
        const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        u = blockIdx.x * 4u + wib;
    }
    for (;;) {
        if (a.persistent) {
            uint32_t t = 0;
            if (lane == 0) t = atomicAdd(a.counter, 1u);
            u = __builtin_amdgcn_readfirstlane(t);
        }
        if (u >= (uint32_t)a.n_units) return;
        const UnitDesc ud = a.units[u];
        const JobDesc jd = a.jobs[ud.job];
        const DatasetDesc dd = a.datasets[jd.ds];
        UnitCtx c{a.code, a.progs, a.order, dd.X, dd.y, a.partials, nullptr, dd.N, jd.n_load, jd.n_feat_prog,
                  jd.kind};
        process_unit<T, D, FV>(c, ud.tile, ud.q0, ud.q1);
        if (!a.persistent) return;
    }
}

__global__ void k_zero_u32(uint32_t* p) { *p = 0u; }

// Fixed-order reduction over blocks: program p of job j sums
// partial[base_j + b * P_j + p] for b = 0 .. blocks_j - 1.
__device__ __forceinline__ void reduce_one(const double* partials, uint64_t part_base, int64_t stride, int64_t p,
                                           int64_t N, int32_t blocks, int32_t kind, void* out) {
    const double* src = partials + part_base + p;
    double s = 0.0;
    for (int32_t t = 0; t < blocks; t++) s += src[(int64_t)t * stride];
    if (kind == GP_FIT_HITS) ((int32_t*)out)[p] = (int32_t)s;
    else if (kind == GP_FIT_MSE) ((float*)out)[p] = (float)(s / (double)N);
    else ((float*)out)[p] = (float)s;
}

__global__ __launch_bounds__(256) void k_reduce(ReduceArgs r) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= r.n_prog) return;
    reduce_one(r.partials, r.part_base, r.stride, p, r.N, r.blocks, r.kind, r.out);
}

__global__ __launch_bounds__(256) void k_reduce_jobs(const ReduceArgs* jobs) {
    const ReduceArgs r = jobs[blockIdx.y];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= r.n_prog) return;
    reduce_one(r.partials, r.part_base, r.stride, p, r.N, r.blocks, r.kind, r.out);
}

// --------------------------------------------------------------------------
// Variants
// --------------------------------------------------------------------------
#define GPX_VARIANTS(X) \
    X(8, 4, 8)          \
    X(8, 8, 8)          \
    X(8, 12, 8)         \
    X(4, 8, 16)         \
    X(4, 12, 16)        \
    X(4, 8, 32)         \
    X(4, 12, 32)

static const VariantDesc kVariants[] = {
#define GPX_DESC(T, D, FV) {T, D, FV},
    GPX_VARIANTS(GPX_DESC)
#undef GPX_DESC
};

int n_variants() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
const VariantDesc& variant(int i) { return kVariants[i]; }

int pick_variant(int n_feat_load, int depth) {
    int best = -1;
    for (int i = 0; i < n_variants(); i++) {
        const VariantDesc& v = kVariants[i];
        if (v.fv < n_feat_load || v.d < depth) continue;
        if (best < 0) { best = i; continue; }
        const VariantDesc& b = kVariants[best];
        const int cost_v = v.t * (v.d + v.fv), cost_b = b.t * (b.d + b.fv);
        // prefer the wider tile, then the smaller register footprint
        if (v.t > b.t || (v.t == b.t && cost_v < cost_b)) best = i;
    }
    return best;
}

hipError_t launch_eval(int vi, const EvalArgs& a, hipStream_t s) {
    if (a.n_units <= 0) return hipSuccess;
    uint32_t blocks = (uint32_t)((a.n_units + 3) / 4);
    blocks = (blocks + 7u) & ~7u;
    const VariantDesc& v = kVariants[vi];
#define GPX_LAUNCH(T, D, FV)                                                      \
    if (v.t == T && v.d == D && v.fv == FV) {                                     \
        hipLaunchKernelGGL((k_eval<T, D, FV>), dim3(blocks), dim3(256), 0, s, a); \
        return hipGetLastError();                                                 \
    }
    GPX_VARIANTS(GPX_LAUNCH)
#undef GPX_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_batch(int vi, const BatchArgs& a, uint32_t grid_blocks, hipStream_t s) {
    if (a.n_units <= 0) return hipSuccess;
    if (a.persistent) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, a.counter);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    } else {
        grid_blocks = (uint32_t)((a.n_units + 3) / 4);
    }
    const VariantDesc& v = kVariants[vi];
#define GPX_LAUNCH(T, D, FV)                                                                \
    if (v.t == T && v.d == D && v.fv == FV) {                                               \
        hipLaunchKernelGGL((k_batch<T, D, FV>), dim3(grid_blocks), dim3(256), 0, s, a);     \
        return hipGetLastError();                                                           \
    }
    GPX_VARIANTS(GPX_LAUNCH)
#undef GPX_LAUNCH
    return hipErrorInvalidValue;
}

int batch_blocks_per_cu(int vi) {
    const VariantDesc& v = kVariants[vi];
    int n = 0;
#define GPX_OCC(T, D, FV)                                                                        \
    if (v.t == T && v.d == D && v.fv == FV) {                                                    \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<T, D, FV>, 256, 0) != hipSuccess) n = 1; \
    }
    GPX_VARIANTS(GPX_OCC)
#undef GPX_OCC
    return n > 0 ? n : 1;
}

hipError_t launch_reduce(const ReduceArgs& r, hipStream_t s) {
    if (r.n_prog <= 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)((r.n_prog + 255) / 256);
    hipLaunchKernelGGL(k_reduce, dim3(blocks), dim3(256), 0, s, r);
    return hipGetLastError();
}

hipError_t launch_reduce_jobs(const ReduceArgs* jobs_dev, int32_t n_jobs, int64_t max_prog, hipStream_t s) {
    if (n_jobs <= 0 || max_prog <= 0) return hipSuccess;
    const uint32_t bx = (uint32_t)((max_prog + 255) / 256);
    hipLaunchKernelGGL(k_reduce_jobs, dim3(bx, (uint32_t)n_jobs), dim3(256), 0, s, jobs_dev);
    return hipGetLastError();
}

}  // namespace gpx
