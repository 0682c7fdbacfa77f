// sin, cos, exp and log of a binary32 argument, evaluated in binary64 and
// rounded once to binary32 -- the evaluator's definition of the four GP
// transcendentals (sin(x), cos(x), exp(min(x, 88)), log|x|).  The result is
// the binary32 rounding of a binary64 value within about one binary64 ulp
// of the exact one, so it is the correctly rounded binary32 result except
// when the exact value lies within that distance of a rounding boundary.
//
// Method (textbook, written from the mathematics):
//   sin/cos: k = nearest integer to x * 2/pi; r = x - k * pi/2 with pi/2
//            split in three binary64 parts (the first product is exact for
//            |x| < 2^19 since x is a binary32 value); Taylor series of sin
//            and cos on |r| <= pi/4 to the r^17 / r^16 terms; the quadrant
//            k mod 4 picks the series and the sign.  |x| >= 2^19, inf and
//            NaN go to the binary64 library function.
//   exp:     k = nearest integer to x / ln 2; r = x - k ln 2 (ln 2 in two
//            parts), |r| <= ln2/2; Taylor series to r^13; scaled by 2^k.
//            Results below the binary32 range underflow to +0.
//   log:     x = f * 2^e with f in [sqrt(1/2), sqrt(2)); log f = 2 atanh(s),
//            s = (f - 1) / (f + 1), |s| <= 0.1716, odd series to s^21;
//            plus e * ln 2 (ln 2 in two parts, the first with 45 significant
//            bits so that e * ln2_hi is exact).
//
// The common path has no branches (special arguments are patched in with
// selects), so a caller applying a function to several values gets one
// straight-line sequence the compiler can interleave.  Coefficients live in
// tables indexed with an offset `z` that is always 0: a caller on the device
// passes a value the compiler cannot see through, so the tables are read
// with a few wide scalar loads rather than kept as ~40 binary64 constants in
// scalar registers.  The functions compile for the device and, for testing,
// for the host.
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define GPX_HD __host__ __device__ __forceinline__
#define GPX_TABLE __constant__
#else
#define GPX_HD static inline
#define GPX_TABLE static
#endif

namespace gpx {
namespace gmath {

// sin r = r + r s (S1 + s S2 + ... + s^7 S8), s = r^2, Sk = (-1)^k / (2k+1)!
GPX_TABLE const double kSin[8] = {-0x1.5555555555555p-3, 0x1.1111111111111p-7, -0x1.a01a01a01a01ap-13,
                                  0x1.71de3a556c734p-19, -0x1.ae64567f544e4p-26, 0x1.6124613a86d09p-33,
                                  -0x1.ae7f3e733b81fp-41, 0x1.952c77030ad4ap-49};
// cos r = 1 + s (C1 + s C2 + ... + s^7 C8), Ck = (-1)^k / (2k)!
GPX_TABLE const double kCos[8] = {-0x1.0000000000000p-1, 0x1.5555555555555p-5, -0x1.6c16c16c16c17p-10,
                                  0x1.a01a01a01a01ap-16, -0x1.27e4fb7789f5cp-22, 0x1.1eed8eff8d898p-29,
                                  -0x1.93974a8c07c9dp-37, 0x1.ae7f3e733b81fp-45};
// 1/k! for k = 2 .. 13
GPX_TABLE const double kExp[12] = {0x1.0000000000000p-1, 0x1.5555555555555p-3, 0x1.5555555555555p-5,
                                   0x1.1111111111111p-7, 0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13,
                                   0x1.a01a01a01a01ap-16, 0x1.71de3a556c734p-19, 0x1.27e4fb7789f5cp-22,
                                   0x1.ae64567f544e4p-26, 0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33};
// 1/(2k+1) for k = 1 .. 10
GPX_TABLE const double kAtanh[10] = {0x1.5555555555555p-2, 0x1.999999999999ap-3, 0x1.2492492492492p-3,
                                     0x1.c71c71c71c71cp-4, 0x1.745d1745d1746p-4, 0x1.3b13b13b13b14p-4,
                                     0x1.1111111111111p-4, 0x1.e1e1e1e1e1e1ep-5, 0x1.af286bca1af28p-5,
                                     0x1.8618618618618p-5};

GPX_HD double horner(double t, const double* c, int n) {
    double p = c[n - 1];
    for (int i = n - 2; i >= 0; i--) p = fma(p, t, c[i]);
    return p;
}

// sin or cos (want_cos) of a binary32 value, as binary64
GPX_HD double sincos64(float a, bool want_cos, int z) {
    const double x = (double)a;
    const bool big = !(fabs(x) < 0x1p19);                       // also inf and NaN
    const double xs = big ? 0.0 : x;
    const double kd = rint(xs * 0x1.45f306dc9c883p-1);          // x * 2/pi
    double r = fma(-kd, 0x1.921fb54442d18p+0, xs);              // exact
    r = fma(-kd, 0x1.1a62633145c07p-54, r);
    r = fma(-kd, -0x1.f1976b7ed8fbcp-110, r);
    const double s = r * r;
    const double ps = fma(r * s, horner(s, kSin + z, 8), r);
    const double pc = fma(s, horner(s, kCos + z, 8), 1.0);
    const int q = (int)kd + (want_cos ? 1 : 0);
    // sin(r + q pi/2): q mod 4 = 0: sin r, 1: cos r, 2: -sin r, 3: -cos r
    const double v0 = (q & 1) ? pc : ps;
    double v = (q & 2) ? -v0 : v0;
    v = (x == 0.0) ? (want_cos ? 1.0 : x) : v;                  // keeps the sign of a zero
    if (big) v = want_cos ? cos(x) : sin(x);
    return v;
}

GPX_HD float sin32(float a, int z = 0) { return (float)sincos64(a, false, z); }
GPX_HD float cos32(float a, int z = 0) { return (float)sincos64(a, true, z); }

// exp(min(a, 88)); a NaN passes through the clamp
GPX_HD float expc32(float a, int z = 0) {
    const float t = (a > 88.0f) ? 88.0f : a;
    const bool ok = t >= -104.0f;                                // false for NaN
    const double x = ok ? (double)t : 0.0;
    const double kd = rint(x * 0x1.71547652b82fep+0);            // x / ln 2
    double r = fma(-kd, 0x1.62e42fefa39efp-1, x);
    r = fma(-kd, 0x1.abc9e3b39803fp-56, r);
    const double p = fma(r, fma(r, horner(r, kExp + z, 12), 1.0), 1.0);
    const float v = (float)ldexp(p, (int)kd);
    // below half the least subnormal the result rounds to +0; NaN stays NaN
    return ok ? v : (t != t ? t : 0.0f);
}

// log|a|, and 0 for |a| < 1e-6 (the comparison is binary32)
GPX_HD float plog32(float a, int z = 0) {
    const float m = fabsf(a);
    const bool tiny = m < 1e-6f;
    const bool fin = m <= 0x1.fffffep+127f;                       // false for inf and NaN
    const double x = (fin && !tiny) ? (double)m : 1.0;
    int e;
    const double f0 = frexp(x, &e);                               // x = f 2^e, f in [1/2, 1)
    const bool lo = f0 < 0x1.6a09e667f3bcdp-1;
    const double f = lo ? f0 * 2.0 : f0;
    const double ed = (double)(lo ? e - 1 : e);
    const double s = (f - 1.0) / (f + 1.0);
    const double t = s * s;
    const double s2 = s + s;
    const double lf = fma(s2 * t, horner(t, kAtanh + z, 10), s2);  // log f = 2 atanh s
    const float v = (float)fma(ed, 0x1.62e42fefa3900p-1, fma(ed, 0x1.de6af278ece60p-46, lf));
    // log of inf is inf and of NaN is NaN, i.e. m itself
    return tiny ? 0.0f : (fin ? v : m);
}

// The same four functions applied to N values at once, written stage by
// stage across the values (every Horner step issues N independent FMAs), so
// that the dependent binary64 chains of different values overlap.  Results
// are identical to the one-value functions.
template <int N>
GPX_HD void sincos_n(float (&a)[N], bool want_cos, int z) {
    double x[N], r[N], s[N], ps[N], pc[N];
    int q[N];
    bool big[N];
    const double* S = kSin + z;
    const double* C = kCos + z;
    for (int j = 0; j < N; j++) {
        x[j] = (double)a[j];
        big[j] = !(fabs(x[j]) < 0x1p19);
        const double xs = big[j] ? 0.0 : x[j];
        const double kd = rint(xs * 0x1.45f306dc9c883p-1);
        double t = fma(-kd, 0x1.921fb54442d18p+0, xs);
        t = fma(-kd, 0x1.1a62633145c07p-54, t);
        r[j] = fma(-kd, -0x1.f1976b7ed8fbcp-110, t);
        s[j] = r[j] * r[j];
        q[j] = (int)kd + (want_cos ? 1 : 0);
        ps[j] = S[7];
        pc[j] = C[7];
    }
    for (int k = 6; k >= 0; k--)
        for (int j = 0; j < N; j++) {
            ps[j] = fma(ps[j], s[j], S[k]);
            pc[j] = fma(pc[j], s[j], C[k]);
        }
    for (int j = 0; j < N; j++) {
        const double sn = fma(r[j] * s[j], ps[j], r[j]);
        const double cs = fma(s[j], pc[j], 1.0);
        const double v0 = (q[j] & 1) ? cs : sn;
        double v = (q[j] & 2) ? -v0 : v0;
        v = (x[j] == 0.0) ? (want_cos ? 1.0 : x[j]) : v;
        if (big[j]) v = want_cos ? cos(x[j]) : sin(x[j]);
        a[j] = (float)v;
    }
}

template <int N>
GPX_HD void expc_n(float (&a)[N], int z) {
    double r[N], p[N];
    int k[N];
    float t[N];
    bool ok[N];
    const double* E = kExp + z;
    for (int j = 0; j < N; j++) {
        t[j] = (a[j] > 88.0f) ? 88.0f : a[j];
        ok[j] = t[j] >= -104.0f;
        const double x = ok[j] ? (double)t[j] : 0.0;
        const double kd = rint(x * 0x1.71547652b82fep+0);
        const double u = fma(-kd, 0x1.62e42fefa39efp-1, x);
        r[j] = fma(-kd, 0x1.abc9e3b39803fp-56, u);
        k[j] = (int)kd;
        p[j] = E[11];
    }
    for (int i = 10; i >= 0; i--)
        for (int j = 0; j < N; j++) p[j] = fma(p[j], r[j], E[i]);
    for (int j = 0; j < N; j++) {
        const double e = fma(r[j], fma(r[j], p[j], 1.0), 1.0);
        const float v = (float)ldexp(e, k[j]);
        a[j] = ok[j] ? v : (t[j] != t[j] ? t[j] : 0.0f);
    }
}

template <int N>
GPX_HD void plog_n(float (&a)[N], int z) {
    double sv[N], t[N], p[N], ed[N];
    float m[N];
    bool tiny[N], fin[N];
    const double* A = kAtanh + z;
    for (int j = 0; j < N; j++) {
        m[j] = fabsf(a[j]);
        tiny[j] = m[j] < 1e-6f;
        fin[j] = m[j] <= 0x1.fffffep+127f;
        const double x = (fin[j] && !tiny[j]) ? (double)m[j] : 1.0;
        int e;
        const double f0 = frexp(x, &e);
        const bool lo = f0 < 0x1.6a09e667f3bcdp-1;
        const double f = lo ? f0 * 2.0 : f0;
        ed[j] = (double)(lo ? e - 1 : e);
        sv[j] = (f - 1.0) / (f + 1.0);
        t[j] = sv[j] * sv[j];
        p[j] = A[9];
    }
    for (int i = 8; i >= 0; i--)
        for (int j = 0; j < N; j++) p[j] = fma(p[j], t[j], A[i]);
    for (int j = 0; j < N; j++) {
        const double s2 = sv[j] + sv[j];
        const double lf = fma(s2 * t[j], p[j], s2);
        const float v = (float)fma(ed[j], 0x1.62e42fefa3900p-1, fma(ed[j], 0x1.de6af278ece60p-46, lf));
        a[j] = tiny[j] ? 0.0f : (fin[j] ? v : m[j]);
    }
}

}  // namespace gmath
}  // namespace gpx
