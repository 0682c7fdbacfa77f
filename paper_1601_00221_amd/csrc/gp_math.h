// sin, cos, exp and log of a binary32 argument, evaluated in binary64 and
// rounded once to binary32 -- the evaluator's definition of the four GP
// transcendentals (sin(x), cos(x), exp(min(x, 88)), log|x|).  The result is
// the binary32 rounding of a binary64 value within about two binary64 ulps
// of the exact one, so it is the correctly rounded binary32 result except
// when the exact value lies within that distance of a rounding boundary.
//
// Method (table-driven reduction, written from the mathematics; the tables
// come from gen_math_tables.py):
//   sin/cos: k = nearest integer to x * 64/pi, j = k mod 128; r = x - k pi/64
//            with pi/64 in three binary64 parts (the first product is exact
//            for |x| < 2^19 since x is a binary32 value), |r| <= pi/128;
//            Taylor series of sin r to r^7 and cos r to r^6 (the next terms
//            are below 2^-60 relative); then sin x = sin(j pi/64) cos r +
//            cos(j pi/64) sin r (and the cosine likewise) from a 128-entry
//            table.  |x| >= 2^19, inf and NaN go to the binary64 library
//            function.
//   exp:     k = nearest integer to 64 x / ln 2 = 64 e + j; r = x - k ln2/64
//            (two parts), |r| <= ln2/128; Taylor series to r^5 (the r^6 term
//            is below 2^-54 relative); times 2^(j/64) from a table, scaled by
//            2^e.  Results below the binary32 range underflow to +0.
//   log:     x = f 2^e with f in [sqrt(1/2), sqrt(2)); j = nearest integer
//            to 128 f; r = f * c - 1 with c = 128/j rounded (|r| <= 1/181);
//            log f = log1p(r) - log c, the series of log1p to r^7 and
//            -log c from a table in two binary64 parts; plus e ln 2 (two
//            parts, the first with 45 significant bits so that e * ln2_hi is
//            exact).  j = 128 gives c = 1 exactly, so log 1 = +0.
//
// The common path has no branches (special arguments are patched in with
// selects), so several values give one straight-line sequence.  Series
// coefficients live in tables indexed with an offset `z` that is always 0:
// a caller on the device passes a value the compiler cannot see through, so
// they are read with scalar loads rather than pinned in scalar registers.
// The reduction tables are read per value from `tab` (device: a copy in
// LDS, filled by tab_fill).  The functions compile for the device and, for
// testing, for the host.
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

// Offsets of the reduction tables in one contiguous block of doubles.
enum : int {
    kTabSin = 0,
    kTabCos = 128,
    kTabExp = 256,
    kTabLogInv = 320,
    kTabLogHi = kTabLogInv + (GPX_LOG_J1 - GPX_LOG_J0 + 1),
    kTabLogLo = kTabLogHi + (GPX_LOG_J1 - GPX_LOG_J0 + 1),
    kTabSize = kTabLogLo + (GPX_LOG_J1 - GPX_LOG_J0 + 1),
};

// Series coefficients, one block: sin (r^3 .. r^7), cos (r^2 .. r^6),
// exp (r^2 .. r^5), log1p (r^2 .. r^7).
enum : int { kCoSin = 0, kCoCos = 3, kCoExp = 6, kCoLog = 10, kCoSize = 16 };
GPX_TABLE double kCoef[kCoSize] = {
    // (-1)^k / (2k+1)!, k = 1 .. 3
    -0x1.5555555555555p-3, 0x1.1111111111111p-7, -0x1.a01a01a01a01ap-13,
    // (-1)^k / (2k)!, k = 1 .. 3
    -0x1.0000000000000p-1, 0x1.5555555555555p-5, -0x1.6c16c16c16c17p-10,
    // 1 / k!, k = 2 .. 5
    0x1.0000000000000p-1, 0x1.5555555555555p-3, 0x1.5555555555555p-5, 0x1.1111111111111p-7,
    // (-1)^(k+1) / k, k = 2 .. 7
    -0x1.0000000000000p-1, 0x1.5555555555555p-2, -0x1.0000000000000p-2, 0x1.999999999999ap-3,
    -0x1.5555555555555p-3, 0x1.2492492492492p-3,
};

// Copy the reduction tables into one block (the device copies into LDS).
GPX_HD void tab_fill(double* dst, int i0, int step) {
    for (int i = i0; i < kTabSize; i += step) {
        double v;
        if (i < kTabCos) v = kSinJ[i - kTabSin];
        else if (i < kTabExp) v = kCosJ[i - kTabCos];
        else if (i < kTabLogInv) v = kExp2J[i - kTabExp];
        else if (i < kTabLogHi) v = kLogInv[i - kTabLogInv];
        else if (i < kTabLogLo) v = kLogHi[i - kTabLogHi];
        else v = kLogLo[i - kTabLogLo];
        dst[i] = v;
    }
}

GPX_HD double horner(double t, const double* c, int n) {
    double p = c[n - 1];
    for (int i = n - 2; i >= 0; i--) p = fma(p, t, c[i]);
    return p;
}

// sin or cos (want_cos) of N binary32 values, in place, stage by stage
template <int N>
GPX_HD void sincos_n(float (&a)[N], bool want_cos, const double* tab, int z) {
    const double* co = kCoef + z;
    double x[N], r[N], s[N];
    int j[N];
    bool big[N];
    for (int i = 0; i < N; i++) {
        x[i] = (double)a[i];
        big[i] = !(fabs(x[i]) < 0x1p19);                        // also inf and NaN
        const double xs = big[i] ? 0.0 : x[i];
        const double kd = rint(xs * 0x1.45f306dc9c883p+4);      // x * 64/pi
        double t = fma(-kd, 0x1.921fb54442d18p-5, xs);           // exact
        t = fma(-kd, 0x1.1a62633145c07p-59, t);
        r[i] = fma(-kd, -0x1.f1976b7ed8fbcp-115, t);
        s[i] = r[i] * r[i];
        j[i] = (int)kd & 127;
    }
    for (int i = 0; i < N; i++) {
        const double sp = fma(r[i] * s[i], horner(s[i], co + kCoSin, 3), r[i]);   // sin r
        const double cp = fma(s[i], horner(s[i], co + kCoCos, 3), 1.0);            // cos r
        const double sj = tab[kTabSin + j[i]], cj = tab[kTabCos + j[i]];
        double v = want_cos ? fma(cj, cp, -(sj * sp)) : fma(sj, cp, cj * sp);
        v = (x[i] == 0.0) ? (want_cos ? 1.0 : x[i]) : v;                           // keeps the sign of a zero
        if (big[i]) v = want_cos ? cos(x[i]) : sin(x[i]);
        a[i] = (float)v;
    }
}

// exp(min(a, 88)) of N values in place; a NaN passes through the clamp
template <int N>
GPX_HD void expc_n(float (&a)[N], const double* tab, int z) {
    const double* co = kCoef + z;
    for (int i = 0; i < N; i++) {
        const float t = (a[i] > 88.0f) ? 88.0f : a[i];
        const bool ok = t >= -104.0f;                            // false for NaN
        const double x = ok ? (double)t : 0.0;
        const double kd = rint(x * 0x1.71547652b82fep+6);        // 64 x / ln 2
        const int k = (int)kd;
        double r = fma(-kd, 0x1.62e42fefa39efp-7, x);            // exact
        r = fma(-kd, 0x1.abc9e3b39803fp-62, r);
        // e^r = 1 + r + r^2 (1/2 + r/6 + r^2/24 + r^3/120)
        const double p = fma(r, fma(r, horner(r, co + kCoExp, 4), 1.0), 1.0);
        const double v = ldexp(tab[kTabExp + (k & 63)] * p, k >> 6);
        // below half the least subnormal the result rounds to +0; NaN stays NaN
        a[i] = ok ? (float)v : (t != t ? t : 0.0f);
    }
}

// log|a| of N values in place, and 0 for |a| < 1e-6 (the comparison is binary32)
template <int N>
GPX_HD void plog_n(float (&a)[N], const double* tab, int z) {
    const double* co = kCoef + z;
    for (int i = 0; i < N; i++) {
        const float m = fabsf(a[i]);
        const bool tiny = m < 1e-6f;
        const bool fin = m <= 0x1.fffffep+127f;                   // false for inf and NaN
        const double x = (fin && !tiny) ? (double)m : 1.0;
        int e;
        const double f0 = frexp(x, &e);                           // x = f0 2^e, f0 in [1/2, 1)
        const bool lo = f0 < 0x1.6a09e667f3bcdp-1;
        const double f = lo ? f0 * 2.0 : f0;
        const double ed = (double)(lo ? e - 1 : e);
        const int q = (int)rint(f * 128.0) - GPX_LOG_J0;
        const double r = fma(f, tab[kTabLogInv + q], -1.0);
        const double lp = fma(r * r, horner(r, co + kCoLog, 6), r);       // log1p r
        const double hi = fma(ed, 0x1.62e42fefa3900p-1, tab[kTabLogHi + q]);
        const double lw = fma(ed, 0x1.de6af278ece60p-46, tab[kTabLogLo + q]) + lp;
        const float v = (float)(hi + lw);
        // log of inf is inf and of NaN is NaN, i.e. m itself
        a[i] = tiny ? 0.0f : (fin ? v : m);
    }
}

}  // namespace gmath
}  // namespace gpx
