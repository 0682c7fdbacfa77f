// Evaluation kernel built around the hand-written interpreter core
// (gen_core.py).  One wavefront owns a case tile of 64 lanes x T slots
// (slot j of lane l is case tile*64*T + j*64 + l, so every feature row is
// read with contiguous 256-byte accesses, as the paper strides a thread's
// cases by the thread count, section 4.1).  The tile's features are loaded
// once into the core's VGPR range; then the wave interprets its programs on
// it.  The two-dimensional stack (section 4) is that VGPR range: one decoded
// instruction updates T slots of 64 lanes.
//
// Work the asm core leaves to the compiled code: protected division and
// sin/cos/exp/log (an exit carries the operand and destination offsets; the
// kernel moves the T slots out, computes, moves them back) and the end of a
// program.  sin, cos, exp and log are evaluated in binary64 and rounded
// once (gp_math.h): random GP trees chain many of them, and most such
// programs turn a last-place difference into a visible fitness difference,
// so a binary32 library result would make fitness depend on the evaluator.
//
// Fitness: per-slot error terms in binary32, per-lane binary64 sums over the
// 4 slots of each 256-case block, a fixed wavefront butterfly, one partial
// per (program, block), then a fixed-order reduction over blocks -- the
// result does not depend on the tile width, the grouping, or what else
// shared the launch.
//
// Kernel modes: 0 with the sin/cos/exp/log code, 1 without it (arithmetic
// programs), 3 like 1 for trees only, 4 like 0 for trees only, 2 the Boolean
// function set, whose slots are 32-bit words of bit-packed cases (32 cases
// per slot; a 256-slot block holds 8192 cases) and whose fitness is the
// number of output bits equal to the target bits.
//
// The classification functions (>, <, ==, logical AND and OR, IF; section
// 4.2) are exits in every arithmetic kernel; the classification fitness
// decodes an output to the class rint(o) and counts the cases whose class
// differs from y.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gp.h"
#include "core_kernels.h"
#include "gp_internal.h"
#include "gp_math.h"

namespace gpx {
#include "core_gen.inc"

// Exit payload: byte 0 offset of the operand, byte 2 offset of the
// destination, byte 3 = operation (low nibble) | constant flag (bit 4: the
// operand is the constant).  Only sin, cos, exp and log leave the core:
// protected division and the classification functions have handlers.
template <int T, int V0, bool AR>
__device__ __forceinline__ void do_exit(uint32_t pay, uint32_t cbits, const double* tab) {
    const uint32_t oa = pay & 255u, od = (pay >> 16) & 255u;
    const uint32_t op = (pay >> 24) & 15u, fl = pay >> 28;
    // the operand is the instruction's constant (flag set) or T slots of the
    // core's range; one scalar branch inside the helper picks
    float A[T];
    core_gather_or_const<T, V0>(oa, fl & 1u, cbits, A);
    if constexpr (AR) {
        // arithmetic-only kernel: the host never runs sin/cos/exp/log programs on it
        return;
    }
    // z is 0, but the compiler cannot know it: the coefficient tables are then
    // read with scalar loads, once per exit, instead of living in SGPRs
    int z = 0;
    asm volatile("" : "+s"(z));
    // the T slots of each function side by side; the reduction tables are in LDS
    switch (op) {
        case GP_SIN: gmath::sincos_n<T>(A, false, tab, z); break;
        case GP_COS: gmath::sincos_n<T>(A, true, tab, z); break;
        case GP_EXPC: gmath::expc_n<T>(A, tab, z); break;
        default: gmath::plog_n<T>(A, tab, z); break;  // GP_PLOG
    }
    core_scatter<T, V0>(od, A);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, 64);
    return v;
}

// One work unit: a case tile and the programs order[q0 .. q1).  The kernel
// has exactly one call site of the core (its labels are unique); in probe
// mode the core only reports where its handler table starts.
template <int T, int D, int NF, int V0, int MODE>
__device__ __forceinline__ void process_unit(const CoreArgs& a, const float* X, const float* y, int64_t N,
                                             int32_t n_load, int32_t kind, uint64_t pbase, uint32_t tile,
                                             uint32_t q0, uint32_t q1, const double* tab) {
    static_assert(T % 4 == 0, "a tile holds whole 256-case blocks");
    // register/stack levels before the features (Boolean and trees-only kernels: no linear registers)
    constexpr int RB = (MODE >= 2 || D > GPX_LIN_REGS) ? D : GPX_LIN_REGS;
    const uint32_t lane = threadIdx.x & 63u;
    const int64_t tile0 = (int64_t)tile * (64 * T);            // first case of the tile (uniform)
    const int64_t left = N - tile0;                            // cases from the tile start to the end
    const int64_t n_blocks = (N + 255) / 256;
    // slot j of this lane is case tile0 + 64 j + lane; it exists if 64 j + lane < left
    for (int32_t f = 0; f < n_load; f++) {
        const float* row = X + (int64_t)f * N + tile0;         // uniform base, lane offsets
        float x[T];
#pragma unroll
        for (int j = 0; j < T; j++) x[j] = (64 * j + (int64_t)lane < left) ? row[64 * j + lane] : 0.0f;
        core_scatter<T, V0>((uint32_t)(RB * T + f * T), x);
    }
    const uint64_t code = (uint64_t)a.code;
    for (uint32_t q = q0; q < q1; ++q) {
        DevProg P;
        uint32_t off = 0;
        if (!a.probe) {
            P = a.progs[__builtin_amdgcn_readfirstlane(a.order[q])];
            // program records are wave-uniform; keep the core's offset in an SGPR
            off = __builtin_amdgcn_readfirstlane(P.code_off) * 4u;
        }
        // first entry: burst the program's code into the scalar cache
        uint32_t pf_end = (a.probe || !a.prefetch) ? 0u : off + __builtin_amdgcn_readfirstlane(P.len) * 16u;
        // The core's asm (with its handler table and labels) must exist once in
        // the kernel (the assembler rejects a second copy): the probe flag and
        // the prefetch bound are laundered on every pass, so the loop is
        // neither split on them nor peeled, and the call stays out of the loop
        // header, so loop rotation does not copy it.
        bool more = true;
        while (more) {
            uint32_t pay, cst;
            uint64_t table;
            uint32_t probe = a.probe;
            asm volatile("" : "+s"(probe));
            Core<T, D, NF, V0, (MODE == 4 ? 3 : (MODE >= 2 ? MODE : 0))>::run(code, off, pay, cst, probe, pf_end,
                                                            (uint32_t)a.prefetch, table);
            // later passes skip the prefetch; an opaque 0, so the first pass is not peeled off
            pf_end = 0u;
            asm volatile("" : "+s"(pf_end));
            if (probe) {
                if (threadIdx.x == 0) a.probe_out[0] = table;
                return;
            }
            more = ((pay >> 24) & 15u) != CORE_OP_END;
            if (more) {
                // Boolean programs never leave the core before their end
                if constexpr (MODE != 2) do_exit<T, V0, MODE == 1 || MODE == 3>(pay, cst, tab);
                off += 16u;
            }
        }
        float o[T];
        core_gather<T, V0>(0u, o);

        if (kind == GP_OUT_CASES) {
            float* row = a.cases_out + (int64_t)P.row * N + tile0;
#pragma unroll
            for (int j = 0; j < T; j++)
                if (64 * j + (int64_t)lane < left) row[64 * j + lane] = o[j];
            continue;
        }
        const float* yt = y + tile0;
        double mine = 0.0;   // lane k keeps block k's partial
#pragma unroll
        for (int k = 0; k < T / 4; k++) {
            double v;
            if constexpr (MODE == 2) {
                // slot j of this lane is word tile0 + 64 j + lane: count its
                // output bits equal to the target's, up to case n_bits
                uint32_t eq = 0;
#pragma unroll
                for (int j = 4 * k; j < 4 * k + 4; j++) {
                    const int64_t wd = tile0 + 64 * j + (int64_t)lane;
                    const bool ok = 64 * j + (int64_t)lane < left;
                    const uint32_t yw = ok ? __float_as_uint(yt[64 * j + lane]) : 0u;
                    const int64_t bits = a.n_bits - 32 * wd;
                    const uint32_t mask = bits >= 32 ? 0xFFFFFFFFu : (bits > 0 ? (1u << bits) - 1u : 0u);
                    eq += ok ? (uint32_t)__popc(~(__float_as_uint(o[j]) ^ yw) & mask) : 0u;
                }
                v = wave_sum((double)eq);
            } else if (kind == GP_FIT_HITS || kind == GP_FIT_CLASS_ERR) {
                // hits: the sign rule; class errors: rint(o) is not the class y
                const bool cls = kind == GP_FIT_CLASS_ERR;
                uint32_t hits = 0;
#pragma unroll
                for (int j = 4 * k; j < 4 * k + 4; j++) {
                    const bool ok = 64 * j + (int64_t)lane < left;
                    const float yj = ok ? yt[64 * j + lane] : 0.0f;
                    const bool hit = ok && (cls ? !(rintf(o[j]) == yj) : ((o[j] > 0.0f) == (yj > 0.0f)));
                    hits += (uint32_t)__popcll(__ballot(hit));
                }
                v = (double)hits;
            } else {
                double acc = 0.0;
#pragma unroll
                for (int j = 4 * k; j < 4 * k + 4; j++) {
                    const bool ok = 64 * j + (int64_t)lane < left;
                    const float yj = ok ? yt[64 * j + lane] : 0.0f;
                    const float d = o[j] - yj;
                    const float t = (kind == GP_FIT_MSE) ? d * d : fabsf(d);
                    acc += ok ? (double)t : 0.0;
                }
                v = wave_sum(acc);
            }
            if (lane == (uint32_t)k) mine = v;
        }
        // the tile's T/4 blocks of this program are adjacent: one store
        const int64_t blk = (int64_t)tile * (T / 4) + lane;
        if (lane < (uint32_t)(T / 4) && blk < n_blocks) a.partials[pbase + P.row * (uint64_t)n_blocks + blk] = mine;
    }
}

// Units come either from a table (batched launches: persistent waves pull
// them longest first from a counter, or one wave per unit) or implicitly
// over one dataset: block unit b = (group quad b div chunks, chunk b mod
// chunks); wave w of the block runs program group 4 * quad + w on tiles
// chunk * tiles_per_wave + i, i = 0 .. tiles_per_wave - 1.  The four waves of
// a block work on the same tiles with different instruction streams, so
// their scalar-cache misses do not fall on the same cycles.
template <int T, int D, int NF, int V0, int MODE>
__device__ __forceinline__ void k_core_body(const CoreArgs& a) {
    // the transcendentals' reduction tables, copied into LDS by the whole block
    const double* tab = nullptr;
    if constexpr (MODE == 0 || MODE == 4) {
        __shared__ __attribute__((aligned(16))) double s_tab[gmath::kTabSize];
        gmath::tab_fill(s_tab, (int)threadIdx.x, (int)blockDim.x);
        __syncthreads();
        tab = s_tab;
    }
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool table = a.units != nullptr;
    uint32_t u, grp = 0, chunk = 0;
    if (table) {
        u = blockIdx.x * 4u + wib;
    } else {
        // Blocks go to the 8 XCDs round robin; give each XCD a contiguous
        // range of block units so a program group's code stays in one L2.
        const uint32_t nb = gridDim.x, b = blockIdx.x;
        u = (b & 7u) * (nb >> 3) + (b >> 3);
        if (!a.probe) {
            if (u >= (uint32_t)a.n_units) return;
            if (a.same_group) {
                // wave w of the block runs group u div q on chunk 4 (u mod q) + w, q = chunks / 4 rounded up
                const uint32_t q = ((uint32_t)a.chunks + 3u) / 4u;
                grp = u / q;
                chunk = (u % q) * 4u + wib;
                if (chunk >= (uint32_t)a.chunks) return;
            } else {
                grp = (u / (uint32_t)a.chunks) * 4u + wib;
                chunk = u % (uint32_t)a.chunks;
            }
            if (grp >= (uint32_t)a.n_groups) return;
        }
    }
    for (uint32_t it = 0;; ++it) {
        uint32_t tile = 0, q0 = 0, q1 = 1;
        uint64_t pbase = 0;
        const float *X = nullptr, *y = nullptr;
        int64_t N = 1;
        int32_t n_load = 0, kind = 0;
        if (a.probe) {
            if (u != 0 || wib != 0) return;
        } else if (!table) {
            if (it >= (uint32_t)a.tiles_per_wave) return;
            tile = chunk * (uint32_t)a.tiles_per_wave + it;
            if (tile >= (uint32_t)a.tiles) return;
            q0 = a.group_off[grp];
            q1 = a.group_off[grp + 1];
            X = a.X;
            y = a.y;
            N = a.N;
            n_load = a.n_load;
            kind = a.kind;
        } else {
            if (a.persistent) {
                uint32_t t = 0;
                if (lane == 0) t = atomicAdd(a.counter, 1u);
                u = __builtin_amdgcn_readfirstlane(t);
            } else if (it > 0) {
                return;
            }
            if (u >= (uint32_t)a.n_units) return;
            const UnitDesc ud = a.units[u];
            const JobDesc jd = a.jobs[ud.job];
            const DatasetDesc dd = a.datasets[jd.ds];
            tile = ud.tile;
            q0 = ud.q0;
            q1 = ud.q1;
            X = dd.X;
            y = dd.y;
            N = dd.N;
            n_load = jd.n_load;
            kind = jd.kind;
            pbase = jd.part_base;
        }
        process_unit<T, D, NF, V0, MODE>(a, X, y, N, n_load, kind, pbase, __builtin_amdgcn_readfirstlane(tile),
                               __builtin_amdgcn_readfirstlane(q0), __builtin_amdgcn_readfirstlane(q1), tab);
        if (a.probe) return;
    }
}

// One kernel per variant.  amdgpu_num_vgpr(n) lets the compiler allocate 2n
// VGPRs on gfx950 (checked at build time against the compiler's
// reserved-register report); the core owns v[V0 ...].  MODE: 0 full, 1 no
// sin/cos/exp/log code (for programs without them), 2 Boolean, 3 trees only
// without sin/cos/exp/log code, 4 trees only with it.
#define GPX_KERNEL(T, D, NF, V0, MODE, NAME)                                                            \
    __global__ __launch_bounds__(256) __attribute__((amdgpu_num_vgpr((V0) / 2))) void                   \
        k_core_##NAME(CoreArgs a) {                                                                     \
        k_core_body<T, D, NF, V0, (MODE)>(a);                                                           \
    }

}  // namespace gpx
