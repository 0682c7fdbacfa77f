// The paper's baseline for comparison: GP evaluation with a
// one-dimensional stack, BlockGP style (section 4.2, Tables 3 and 7).  One
// workgroup per program, the program in LDS, each thread takes one case per
// pass (cases tid, tid + 256, ...) and interprets the program with its own
// stack in private memory -- the design the 2D stack improves on.  It is
// compiled C++ (a switch per instruction), kept for measuring that
// improvement on this GPU; the evaluator proper is core_body.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gp.h"
#include "blockgp.h"
#include "gp_internal.h"
#include "gp_math.h"

namespace gpx {

__device__ __forceinline__ float bg_apply(uint32_t op, float a, float b, const double* tab, int z) {
    float v[1] = {a};
    switch (op) {
        case GP_ADD: return a + b;
        case GP_SUB: return a - b;
        case GP_MUL: return a * b;
        case GP_PDIV: return (fabsf(b) < 1e-6f) ? 1.0f : a / b;
        case GP_SIN: gmath::sincos_n<1>(v, false, tab, z); return v[0];
        case GP_COS: gmath::sincos_n<1>(v, true, tab, z); return v[0];
        case GP_EXPC: gmath::expc_n<1>(v, tab, z); return v[0];
        default: gmath::plog_n<1>(v, tab, z); return v[0];
    }
}

__device__ __forceinline__ double bg_block_sum(double v, double* red) {
    for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); i++) t += red[i];
    return t;
}

// FORM 0: postfix tokens (word 0: opcode | feature << 8, word 1: constant).
// FORM 1: the stack-operand form of section 5 (the lowered code, two words
// per instruction, see gp_internal.h).
template <int FORM>
__global__ __launch_bounds__(256) void k_blockgp(BgArgs a) {
    extern __shared__ uint32_t lds[];
    __shared__ __attribute__((aligned(16))) double s_tab[gmath::kTabSize];
    __shared__ double red[4];
    gmath::tab_fill(s_tab, (int)threadIdx.x, (int)blockDim.x);
    const int p = blockIdx.x;
    const uint32_t o = a.poff[p], L = a.plen[p];
    for (uint32_t i = threadIdx.x; i < 2 * L; i += blockDim.x) lds[i] = a.code[2 * (uint64_t)o + i];
    __syncthreads();
    int z = 0;
    asm volatile("" : "+s"(z));
    const int64_t N = a.N;
    double acc = 0.0;
    for (int64_t c = threadIdx.x; c < N; c += blockDim.x) {
        float st[GP_BG_MAX_STACK];
        int h = 0;
        for (uint32_t i = 0; i < L; i++) {
            const uint32_t w0 = lds[2 * i];
            const float k = __uint_as_float(lds[2 * i + 1]);
            if (FORM == 0) {
                const uint32_t op = w0 & 255u;
                if (op == GP_VAR) {
                    st[h++] = a.X[(int64_t)(w0 >> 8) * N + c];
                } else if (op == GP_CONST) {
                    st[h++] = k;
                } else if (op >= GP_SIN) {
                    st[h - 1] = bg_apply(op, st[h - 1], 0.0f, s_tab, z);
                } else {
                    const float b = st[--h];
                    st[h - 1] = bg_apply(op, st[h - 1], b, s_tab, z);
                }
            } else {
                const uint32_t op = w0 & 15u, mode = (w0 >> 4) & 15u;
                const float xa = (mode == M_XS || mode == M_XX || mode == M_XC || mode == M_X)
                                     ? a.X[(int64_t)((w0 >> 8) & 255u) * N + c] : 0.0f;
                const float xb = (mode == M_SX || mode == M_XX || mode == M_CX)
                                     ? a.X[(int64_t)((w0 >> 16) & 255u) * N + c] : 0.0f;
                if (op == OP_PUSH) {
                    st[h++] = (mode == M_X) ? xa : k;
                    continue;
                }
                switch (mode) {
                    case M_SS: st[h - 2] = bg_apply(op, st[h - 2], st[h - 1], s_tab, z); h--; break;
                    case M_SSR: st[h - 2] = bg_apply(op, st[h - 1], st[h - 2], s_tab, z); h--; break;
                    case M_SX: st[h - 1] = bg_apply(op, st[h - 1], xb, s_tab, z); break;
                    case M_XS: st[h - 1] = bg_apply(op, xa, st[h - 1], s_tab, z); break;
                    case M_SC: st[h - 1] = bg_apply(op, st[h - 1], k, s_tab, z); break;
                    case M_CS: st[h - 1] = bg_apply(op, k, st[h - 1], s_tab, z); break;
                    case M_XX: st[h] = bg_apply(op, xa, xb, s_tab, z); h++; break;
                    case M_XC: st[h] = bg_apply(op, xa, k, s_tab, z); h++; break;
                    case M_CX: st[h] = bg_apply(op, k, xb, s_tab, z); h++; break;
                    case M_S: st[h - 1] = bg_apply(op, st[h - 1], 0.0f, s_tab, z); break;
                    case M_X: st[h] = bg_apply(op, xa, 0.0f, s_tab, z); h++; break;
                    default: st[h] = bg_apply(op, k, 0.0f, s_tab, z); h++; break;  // M_C
                }
            }
        }
        if (a.kind == GP_OUT_CASES) {
            ((float*)a.out)[(int64_t)p * N + c] = st[0];
            continue;
        }
        const float yc = a.y[c];
        const float d = st[0] - yc;
        if (a.kind == GP_FIT_HITS) acc += ((st[0] > 0.0f) == (yc > 0.0f)) ? 1.0 : 0.0;
        else acc += (a.kind == GP_FIT_MSE) ? (double)(d * d) : (double)fabsf(d);
    }
    if (a.kind == GP_OUT_CASES) return;
    const double s = bg_block_sum(acc, red);
    if (threadIdx.x == 0) {
        if (a.kind == GP_FIT_HITS) ((int32_t*)a.out)[p] = (int32_t)s;
        else if (a.kind == GP_FIT_MSE) ((float*)a.out)[p] = (float)(s / (double)N);
        else ((float*)a.out)[p] = (float)s;
    }
}

hipError_t blockgp_launch(int form, const BgArgs& a, int32_t n_prog, hipStream_t s) {
    const size_t lds = (size_t)a.max_len * 8;
    if (form == 0) hipLaunchKernelGGL(k_blockgp<0>, dim3((uint32_t)n_prog), dim3(256), lds, s, a);
    else hipLaunchKernelGGL(k_blockgp<1>, dim3((uint32_t)n_prog), dim3(256), lds, s, a);
    return hipGetLastError();
}

}  // namespace gpx
