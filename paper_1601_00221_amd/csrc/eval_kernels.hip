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
// Evaluation kernel: one wavefront per unit (tile, program group).
// --------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, 64);
    return v;
}

template <int T, int D, int FV>
__global__ __launch_bounds__(256) void k_eval(EvalArgs a) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // Blocks go to the 8 XCDs round robin; give each XCD a contiguous range
    // of units so a program group's code stays in one L2.
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    const uint32_t lb = (b & 7u) * (nb >> 3) + (b >> 3);
    const uint32_t u = lb * 4u + wib;
    if (u >= (uint32_t)a.n_units) return;
    const uint32_t tile = u % (uint32_t)a.tiles;
    const uint32_t grp = u / (uint32_t)a.tiles;

    const int64_t N = a.N;
    const int64_t base = (int64_t)tile * (64 * T) + lane;
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

    const uint32_t q0 = a.group_off[grp], q1 = a.group_off[grp + 1];
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
        } else if (a.kind == GP_FIT_HITS) {
            uint32_t hits = 0;
#pragma unroll
            for (int j = 0; j < T; j++) {
                const bool hit = valid[j] && ((o[j] > 0.0f) == (yv[j] > 0.0f));
                hits += (uint32_t)__popcll(__ballot(hit));
            }
            if (lane == 0) a.partials[P.part_base + (uint64_t)tile * P.part_stride] = (double)hits;
        } else {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < T; j++) {
                const float d = o[j] - yv[j];
                const float t = (a.kind == GP_FIT_MSE) ? d * d : fabsf(d);
                acc += valid[j] ? (double)t : 0.0;
            }
            acc = wave_sum(acc);
            if (lane == 0) a.partials[P.part_base + (uint64_t)tile * P.part_stride] = acc;
        }
    }
}

// Fixed-order reduction over tiles: thread p sums partial[t*P + p], t = 0..tiles-1.
__global__ __launch_bounds__(256) void k_reduce(ReduceArgs r) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= r.n_prog) return;
    const double* src = r.partials + r.part_base + p;
    double s = 0.0;
    for (int32_t t = 0; t < r.tiles; t++) s += src[(int64_t)t * r.stride];
    if (r.kind == GP_FIT_HITS) ((int32_t*)r.out)[p] = (int32_t)s;
    else if (r.kind == GP_FIT_MSE) ((float*)r.out)[p] = (float)(s / (double)r.N);
    else ((float*)r.out)[p] = (float)s;
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
    // smallest register footprint that fits
    int best = -1;
    for (int i = 0; i < n_variants(); i++) {
        const VariantDesc& v = kVariants[i];
        if (v.fv < n_feat_load || v.d < depth) continue;
        if (best < 0) { best = i; continue; }
        const VariantDesc& b = kVariants[best];
        const int cost_v = v.t * (v.d + v.fv), cost_b = b.t * (b.d + b.fv);
        // prefer the wider tile when the register footprint allows it
        if (v.t > b.t || (v.t == b.t && cost_v < cost_b)) best = i;
    }
    return best;
}

hipError_t launch_eval(int vi, const EvalArgs& a, hipStream_t s) {
    if (a.n_units <= 0) return hipSuccess;
    uint32_t blocks = (uint32_t)((a.n_units + 3) / 4);
    blocks = (blocks + 7u) & ~7u;
    const VariantDesc& v = kVariants[vi];
#define GPX_LAUNCH(T, D, FV)                                                   \
    if (v.t == T && v.d == D && v.fv == FV) {                                  \
        hipLaunchKernelGGL((k_eval<T, D, FV>), dim3(blocks), dim3(256), 0, s, a); \
        return hipGetLastError();                                              \
    }
    GPX_VARIANTS(GPX_LAUNCH)
#undef GPX_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_reduce(const ReduceArgs& r, hipStream_t s) {
    if (r.n_prog <= 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)((r.n_prog + 255) / 256);
    hipLaunchKernelGGL(k_reduce, dim3(blocks), dim3(256), 0, s, r);
    return hipGetLastError();
}

}  // namespace gpx
