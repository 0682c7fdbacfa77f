// sin, cos, exp and log of a binary32 argument, evaluated in binary64 and
// rounded once to binary32 -- the evaluator's definition of the four GP
// transcendentals (sin(x), cos(x), exp(min(x, 88)), log|x|).  The binary64
// value is within a few binary64 ulps of the exact one, so its rounding is
// the correctly rounded binary32 result except when the exact value lies
// within that distance of a rounding boundary.
//
// Method (table-driven reduction, written from the mathematics; the tables
// come from gen_math_tables.py):
//   sin/cos: k = nearest integer to x * 64/pi, j = k mod 128, r = x - k pi/64,
//            |r| <= pi/128.  For |x| < 2^44, k comes from one fused
//            multiply-add against 1.5 * 2^52 (k is then the low word of the
//            sum), and r from pi/64 in three binary64 parts: the first
//            product's remainder is exact because it is a small multiple of
//            that part's last bit.  Larger arguments (and inf, NaN) take
//            another branch: x = m 2^e with m an integer of 24 bits, and
//            x * 64/pi mod 128 is summed from the products of x with five
//            28-bit chunks of 64/pi chosen by e (the chunks before them only
//            add multiples of 128), each product exact in binary64.  Then
//            the Taylor series of sin r to r^7 and cos r to r^6 (the next
//            terms are below 2^-58 relative) and sin x = sin(j pi/64) cos r +
//            cos(j pi/64) sin r from a 128-entry table of (sin, cos) pairs;
//            cos x is sin x with j + 32 (a quarter turn) in place of j.  For
//            |x| < 2^-12 the binary32 sine is x itself, which also keeps the
//            sign of a zero.
//   exp:     the argument clamped to [-104, 88] (exp(-104) rounds to +0 in
//            binary32, and a NaN passes through a final select);
//            k = nearest integer to 64 x / ln 2 = 64 e + j (the same fused
//            multiply-add rounding), r = x - k ln2/64 in two parts, |r| <=
//            ln2/128; Taylor series to r^5 (the r^6 term is below 2^-54
//            relative); times 2^(j/64) from a table, scaled by 2^e.
//   log:     from the binary32 encoding of |x|: |x| = f 2^e with f in
//            [sqrt(1/2), sqrt(2)) (integer operations on the encoding); the
//            bucket centre f_k nearest to f with 8 significant bits indexes a
//            table of c = 1/f_k rounded and -log c; r = f c - 1 (one rounding,
//            |r| <= 2^-9); log|x| = e ln 2 + (-log c) + log1p(r) with the
//            series of log1p to r^6 (the r^7 term is below 2^-56 relative).
//            |x| < 1e-6 (compared in binary32) gives 0; inf and NaN give
//            |x|.
//
// Each function takes N values and runs their stages side by side; the
// common path has no branches (special arguments are patched in with
// selects).  Series coefficients live in a table indexed with an offset `z`
// that is always 0: a caller on the device passes a value the compiler
// cannot see through, so they are read with scalar loads rather than pinned
// in scalar registers.  The reduction tables are read per value from `tab`
// (device: a copy in LDS, filled by tab_fill).  The functions compile for
// the device and, for testing, for the host.
#pragma once

#include <math.h>
#include <stdint.h>
#include <string.h>

// Tables are constexpr arrays (not device variables), so device code reaches
// them PC-relative instead of through the global offset table.
#define GPX_TABLE constexpr
#if defined(__HIPCC__)
#define GPX_HD __host__ __device__ __forceinline__
#else
#define GPX_HD static inline
#endif

namespace gpx {
namespace gmath {

#include "gp_math_tables.h"

// Offsets of the tables in one contiguous block of doubles; the (sin, cos)
// and (c, -log c) pairs are 16-byte aligned so one 16-byte load reads a pair.
enum : int {
    kTabSC = 0,
    kTabExp = 256,
    kTabLog = 320,
    kTabPi = kTabLog + 2 * GPX_LOG_N,
    kTabSize = kTabPi + GPX_PI_CHUNKS,
};
static_assert(kTabLog % 2 == 0, "pairs stay 16-byte aligned");

// Series coefficients, one block: sin (r^3 .. r^7), cos (r^2 .. r^6),
// exp (r^2 .. r^5), log1p (r^2 .. r^6).
enum : int { kCoSin = 0, kCoCos = 3, kCoExp = 6, kCoLog = 10, kCoSize = 15 };
GPX_TABLE double kCoef[kCoSize] = {
    // (-1)^k / (2k+1)!, k = 1 .. 3
    -0x1.5555555555555p-3, 0x1.1111111111111p-7, -0x1.a01a01a01a01ap-13,
    // (-1)^k / (2k)!, k = 1 .. 3
    -0x1.0000000000000p-1, 0x1.5555555555555p-5, -0x1.6c16c16c16c17p-10,
    // 1 / k!, k = 2 .. 5
    0x1.0000000000000p-1, 0x1.5555555555555p-3, 0x1.5555555555555p-5, 0x1.1111111111111p-7,
    // (-1)^(k+1) / k, k = 2 .. 6
    -0x1.0000000000000p-1, 0x1.5555555555555p-2, -0x1.0000000000000p-2, 0x1.999999999999ap-3,
    -0x1.5555555555555p-3,
};

// 1.5 * 2^52: adding it to a binary64 value v with |v| < 2^51 rounds v to the
// nearest integer, which the low 32 bits of the sum then hold (two's
// complement).
constexpr double kRound = 0x1.8p52;

GPX_HD uint32_t lo32(double v) {
    uint64_t b;
    memcpy(&b, &v, 8);
    return (uint32_t)b;
}
GPX_HD uint32_t bits_of(float v) {
    uint32_t b;
    memcpy(&b, &v, 4);
    return b;
}
GPX_HD float float_of(uint32_t b) {
    float v;
    memcpy(&v, &b, 4);
    return v;
}

// Copy the tables into one block (the device copies into LDS).
GPX_HD void tab_fill(double* dst, int i0, int step) {
    for (int i = i0; i < kTabSize; i += step) {
        double v;
        if (i < kTabExp) v = kSinCos[i - kTabSC];
        else if (i < kTabLog) v = kExp2J[i - kTabExp];
        else if (i < kTabPi) v = kLogCT[i - kTabLog];
        else v = kPiChunks[i - kTabPi];
        dst[i] = v;
    }
}

GPX_HD double horner(double t, const double* c, int n) {
    double p = c[n - 1];
    for (int i = n - 2; i >= 0; i--) p = fma(p, t, c[i]);
    return p;
}

// x mod 2 pi for |x| >= 2^44 (and inf, NaN): returns r in about
// [-pi/128, pi/128] and k with x = k pi/64 + r (k mod 128 is what matters).
// x = m 2^(E - 150), E the biased exponent; the product of x with chunk i of
// 64/pi is m c_i 2^(E - 173 - 28 i), a multiple of 128 for chunks before
// i0 = (E - 152) div 28; the five chunks from i0 on give x * 64/pi mod 128 as
// v0 + v1 + p2 + p3 + p4, the first two reduced mod 128 exactly.
GPX_HD void reduce_big(float a, const double* tab, double& r, int& k) {
    const uint32_t u = bits_of(a) & 0x7FFFFFFFu;
    uint32_t e = u >> 23;
    e = e < 171u ? 171u : e;              // lanes that are not big: any valid index
    const int i0 = (int)((e - 152u) / 28u);
    const double* c = tab + kTabPi + i0;
    const double xd = (double)float_of(u);
    const double p0 = xd * c[0], p1 = xd * c[1], p2 = xd * c[2], p3 = xd * c[3], p4 = xd * c[4];
    const double v0 = fma(-128.0, floor(p0 * 0x1p-7), p0);    // exact, in [0, 128)
    const double v1 = fma(-128.0, floor(p1 * 0x1p-7), p1);
    const double kd = rint(v0 + v1 + p2);
    // (v0 - kd) + v1 is exact; the later roundings are relative to the sum
    const double s = (((v0 - kd) + v1) + p2 + p3) + p4;
    const double sg = a < 0.0f ? -1.0 : 1.0;
    r = sg * (s * 0x1.921fb54442d18p-5);
    k = kd == kd ? (int)(sg * kd) : 0;   // inf and NaN: r is NaN, any k
}

// sin or cos (want_cos) of N binary32 values, in place, stage by stage
template <int N>
GPX_HD void sincos_n(float (&a)[N], bool want_cos, const double* tab, int z) {
    const double* co = kCoef + z;
    double r[N];
    int k[N];
    bool big[N];
    bool any_big = false;
    for (int i = 0; i < N; i++) {
        const double x = (double)a[i];
        big[i] = !(fabsf(a[i]) < 0x1p44f);                            // also inf and NaN
        any_big = any_big || big[i];
        const double v = fma(x, 0x1.45f306dc9c883p+4, kRound);         // x * 64/pi + 1.5 * 2^52
        const double kd = v - kRound;
        double t = fma(-kd, 0x1.921fb54442d18p-5, x);                  // exact
        t = fma(-kd, 0x1.1a62633145c07p-59, t);
        r[i] = fma(-kd, -0x1.f1976b7ed8fbcp-115, t);
        k[i] = (int)lo32(v);
    }
    if (any_big) {
        for (int i = 0; i < N; i++) {
            double rb;
            int kb;
            reduce_big(a[i], tab, rb, kb);
            r[i] = big[i] ? rb : r[i];
            k[i] = big[i] ? kb : k[i];
        }
    }
    const int quarter = want_cos ? 32 : 0;
    for (int i = 0; i < N; i++) {
        const double s = r[i] * r[i];
        const double sp = fma(r[i] * s, horner(s, co + kCoSin, 3), r[i]);      // sin r
        const double cp = fma(s, horner(s, co + kCoCos, 3), 1.0);              // cos r
        const double* sc = tab + kTabSC + 2 * ((k[i] + quarter) & 127);
        const double v = fma(sc[0], cp, sc[1] * sp);
        const float o = (float)v;
        a[i] = (!want_cos && fabsf(a[i]) < 0x1p-12f) ? a[i] : o;
    }
}

// exp(min(a, 88)) of N values in place; a NaN passes through the clamp
template <int N>
GPX_HD void expc_n(float (&a)[N], const double* tab, int z) {
    const double* co = kCoef + z;
    for (int i = 0; i < N; i++) {
        const float t = fminf(fmaxf(a[i], -104.0f), 88.0f);          // a NaN becomes -104
        const double x = (double)t;
        const double v = fma(x, 0x1.71547652b82fep+6, kRound);       // 64 x / ln 2 + 1.5 * 2^52
        const double kd = v - kRound;
        const int k = (int)lo32(v);
        double r = fma(-kd, 0x1.62e42fefa39efp-7, x);                // exact
        r = fma(-kd, 0x1.abc9e3b39803fp-62, r);
        // e^r = 1 + r + r^2 (1/2 + r/6 + r^2/24 + r^3/120)
        const double p = fma(r, fma(r, horner(r, co + kCoExp, 4), 1.0), 1.0);
        const double w = ldexp(tab[kTabExp + (k & 63)] * p, k >> 6);
        // below half the least subnormal the result rounds to +0
        a[i] = (a[i] != a[i]) ? a[i] : (float)w;
    }
}

// log|a| of N values in place, and 0 for |a| < 1e-6 (the comparison is binary32)
template <int N>
GPX_HD void plog_n(float (&a)[N], const double* tab, int z) {
    const double* co = kCoef + z;
    for (int i = 0; i < N; i++) {
        const uint32_t u = bits_of(a[i]) & 0x7FFFFFFFu;
        const float m = float_of(u);
        const bool tiny = m < 1e-6f;
        const bool fin = u < 0x7F800000u;                            // false for inf and NaN
        const uint32_t uu = (fin && !tiny) ? u : 0x3F800000u;        // normal, so the encoding splits
        // |a| = f 2^e, f in [sqrt(1/2), sqrt(2)): the exponent taken relative to sqrt(1/2)
        const uint32_t t = uu - 0x3F3504F3u;
        const int e = (int)t >> 23;
        const uint32_t fb = (t & 0x007FFFFFu) + 0x3F3504F3u;
        const int q = (int)((fb + 0x4000u) >> 15) - GPX_LOG_K0;      // nearest 8-bit bucket centre
        const double* ct = tab + kTabLog + 2 * q;
        const double r = fma((double)float_of(fb), ct[0], -1.0);
        const double lp = fma(r * r, horner(r, co + kCoLog, 5), r);  // log1p r
        const double v = fma((double)e, 0x1.62e42fefa39efp-1, ct[1] + lp);
        const float o = (float)v;
        // log of inf is inf and of NaN is NaN, i.e. |a| itself
        a[i] = tiny ? 0.0f : (fin ? o : m);
    }
}

}  // namespace gmath
}  // namespace gpx
