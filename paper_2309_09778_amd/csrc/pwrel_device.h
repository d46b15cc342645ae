// Device-side arithmetic of the PW_REL perceptron compressor (gfx950).
//
// Everything here is plain IEEE-754 arithmetic (+, -, *, /, explicit fma,
// rint, ldexp, bit extraction) so that every device result is a fixed
// function of its inputs.  Compile with -ffp-contract=off: an a*b+c that is
// not written as __builtin_fma must round twice.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pwrel.h"

namespace pwrel {

constexpr int kR = 32768;                 // 2^(m-1), m = 16 code bits
constexpr double kGridLimit = 1073741824.0; // grid values stay inside +-2^30

// Status codes shared with the C ABI (pwrel.h).
constexpr int kOk = 0, kEInval = -1, kERange = -2, kENonFinite = -3, kENoSpc = -4,
              kECorrupt = -5;

// Constants of a field (Sec. 3.2, Eq. 8-12), produced on the device.
struct DevConsts {
    double eps, eps0, b_a, w, r, Lp, Ln, d0;
    long long p_zero, b_sign, n_lo, delta;
    double abs_min, abs_max;
    unsigned long long n_zero, n_neg, n_nonfinite;
    int status;
    int pad;
    double fm_p, fm_n;  // fast-path margins of t = (log2|x| + L) r, per sign range
    int w32;            // grid values span < 2^27: prediction errors fit 32-bit arithmetic
    int pad2;
    double vm;          // bound certified when t is this far inside its grid cell (below)
    long long p_max;    // no point's grid value exceeds this (the largest |x| of a negative,
                        // else b_sign, plus one grid step against ulp-level log2 errors)
};

// Running statistics of a field (reduced with integer atomics).
struct DevStats {
    unsigned long long min_bits;  // smallest |x| bit pattern among finite non-zero x
    unsigned long long max_bits;  // largest |x| bit pattern among finite x
    unsigned long long n_zero, n_neg, n_nonfinite;
    unsigned long long pad[3];
};

// ---------------------------------------------------------------------------
// log2 by the atanh series: with x = m 2^e, m in (sqrt(1/2), sqrt(2)],
// ln m = 2 sum_{k>=0} s^(2k+1) / (2k+1), s = (m - 1) / (m + 1), |s| < 0.1716;
// eleven terms leave a truncation error below 1e-18.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double det_log2(double x)
{
    int scale_e = 0;
    if (x < 0x1p-1022) {        // subnormal: bring into the normal range exactly
        x = x * 0x1p54;
        scale_e = -54;
    }
    const unsigned long long bits = (unsigned long long)__double_as_longlong(x);
    int e = (int)((bits >> 52) & 0x7ffULL) - 1023;
    double m = __longlong_as_double((long long)((bits & 0x000fffffffffffffULL) |
                                                0x3ff0000000000000ULL));
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        e += 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double s2 = s * s;
    double acc = 1.0 / 21.0;
    acc = __builtin_fma(acc, s2, 1.0 / 19.0);
    acc = __builtin_fma(acc, s2, 1.0 / 17.0);
    acc = __builtin_fma(acc, s2, 1.0 / 15.0);
    acc = __builtin_fma(acc, s2, 1.0 / 13.0);
    acc = __builtin_fma(acc, s2, 1.0 / 11.0);
    acc = __builtin_fma(acc, s2, 1.0 / 9.0);
    acc = __builtin_fma(acc, s2, 1.0 / 7.0);
    acc = __builtin_fma(acc, s2, 1.0 / 5.0);
    acc = __builtin_fma(acc, s2, 1.0 / 3.0);
    acc = __builtin_fma(acc, s2, 1.0);
    return (double)(e + scale_e) + ((s + s) * acc) * 1.4426950408889634;
}

// ---------------------------------------------------------------------------
// 2^t = 2^k e^a with k = rint(t), a = (t - k) ln 2, |a| <= 0.347, and e^a by
// its Taylor polynomial of degree 13 (truncation below 5e-18).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double det_exp2(double t)
{
    const double k = __builtin_rint(t);
    const double a = (t - k) * 0.6931471805599453;
    double acc = 1.0 / 6227020800.0;
    acc = __builtin_fma(acc, a, 1.0 / 479001600.0);
    acc = __builtin_fma(acc, a, 1.0 / 39916800.0);
    acc = __builtin_fma(acc, a, 1.0 / 3628800.0);
    acc = __builtin_fma(acc, a, 1.0 / 362880.0);
    acc = __builtin_fma(acc, a, 1.0 / 40320.0);
    acc = __builtin_fma(acc, a, 1.0 / 5040.0);
    acc = __builtin_fma(acc, a, 1.0 / 720.0);
    acc = __builtin_fma(acc, a, 1.0 / 120.0);
    acc = __builtin_fma(acc, a, 1.0 / 24.0);
    acc = __builtin_fma(acc, a, 1.0 / 6.0);
    acc = __builtin_fma(acc, a, 1.0 / 2.0);
    acc = __builtin_fma(acc, a, 1.0);
    acc = __builtin_fma(acc, a, 1.0);
    return __builtin_ldexp(acc, (int)k);
}

// ---------------------------------------------------------------------------
// FP32 fast paths (FP32 fields only).  They use the hardware log2 / exp2
// (v_log_f32, v_exp_f32) and decide a result only where an error bound proves
// it equal to the FP64 path's; elsewhere the caller takes the FP64 path.  The
// bounds are properties of the hardware instructions, checked over every
// input they can receive (pwrel_fastmath_check):
//   |fast_log2(a) - det_log2(a)| <= kFastLog2Err   for every normal float a > 0
//   |v_exp_f32(f) - 2^f| <= kFastExp2Err 2^f       for every float |f| <= 1/2
// ---------------------------------------------------------------------------
constexpr double kFastLog2Err = PWREL_FAST_LOG2_ERR;
constexpr double kFastExp2Err = PWREL_FAST_EXP2_ERR;

// log2 of a normal float a > 0: exponent plus v_log_f32 of the significand
// taken into [sqrt(1/2), sqrt(2)), summed in FP64
__device__ __forceinline__ double fast_log2(float a)
{
    const unsigned bits = __float_as_uint(a);
    int e = (int)((bits >> 23) & 0xffu) - 127;
    float m = __uint_as_float((bits & 0x7fffffu) | 0x3f800000u);
    if (m >= 1.41421356f) {
        m = m * 0.5f;
        e += 1;
    }
    return (double)e + (double)__builtin_amdgcn_logf(m);
}

template <typename T> __device__ __forceinline__ double to_dtype(double v);
template <> __device__ __forceinline__ double to_dtype<float>(double v) { return (double)(float)v; }
template <> __device__ __forceinline__ double to_dtype<double>(double v) { return v; }

// Grid value of an input value: Eq. 6 (positive), Eq. 7 (negative, plus the
// integer offset delta), Eq. 12 (zero), clamped so that the zero image, the
// positive range and the negative range stay disjoint.  Written without
// branches on the sign so that a wave holding both signs evaluates one log2.
__device__ __forceinline__ int grid_value(double x, const DevConsts &c, int &err)
{
    const double a = __builtin_fabs(x);
    const bool neg = x < 0.0;
    const double t = (det_log2(a > 0.0 ? a : 1.0) + (neg ? c.Ln : c.Lp)) * c.r;
    if (x != 0.0 && !(__builtin_fabs(t) < kGridLimit))
        err = kERange;
    long long q = (long long)__builtin_rint(t);
    const long long qp = q < c.p_zero + 1 ? c.p_zero + 1 : (q > c.b_sign ? c.b_sign : q);
    long long qn = q + c.delta;
    qn = qn < c.b_sign + 1 ? c.b_sign + 1 : qn;
    if (neg && !(__builtin_fabs((double)qn) < kGridLimit))
        err = kERange;
    q = neg ? qn : qp;
    return x == 0.0 ? (int)c.p_zero : (int)q;
}

// Grid value of an FP32 input by the fast path: returns false when the bound
// cannot decide the rounding, or the input is subnormal, non-finite, or so
// large in the grid that the range checks matter (the FP64 path decides then).
// x = 0 is exact (p_zero).  Written without branches: both sign ranges and
// all checks are evaluated and combined with selects.
//
// sure: the PW_REL bound certainly holds for x^ = (float) inverse(q), so the
// verification can be skipped.  With t the exact (log2|x| + L) r, an
// unclamped q = rint(t) has |q - t| <= 1/2 - d', d' = (distance of the fast t
// to the rounding boundary) - fm; then x^ / |x| lies within
// (1 + eps)^(+-(1 - 2 d')) up to the FP32 rounding of x^ (2^-24 relative for
// 2^-124 <= |x| < 2^126, where x^ stays normal and finite), and
// d' > vm = 2^-21 / ln(1 + eps) leaves more than eight times the room those
// roundings and the FP64 comparison need on either side of the bound.  Same
// sign range as x, never zero.
__device__ __forceinline__ bool grid_value_fast(float x, const DevConsts &c, int &q, bool &sure)
{
    const float a = __builtin_fabsf(x);
    const bool neg = x < 0.0f;
    const double t = (fast_log2(a) + (neg ? c.Ln : c.Lp)) * c.r;
    const double margin = neg ? c.fm_n : c.fm_p;
    const double fr = t - __builtin_floor(t);
    const double dist = __builtin_fabs(fr - 0.5);
    const bool in_range = __builtin_fabs(t) < 0x1p29;
    const bool ok = a >= 0x1p-126f && a <= 0x1.fffffep127f && in_range && dist > margin;
    const int qi = (int)__builtin_rint(in_range ? t : 0.0);
    const int pz = (int)c.p_zero, bs = (int)c.b_sign, dl = (int)c.delta;
    int v;
    bool fits = true, clamped;
    if (neg) {
        // q + delta can reach 2^30 only for fields the FP64 path rejects
        const long long w = (long long)qi + dl;
        fits = w < (long long)kGridLimit;
        clamped = w < bs + 1;
        v = (int)(clamped ? bs + 1 : w);
    } else {
        clamped = qi < pz + 1 || qi > bs;
        v = qi < pz + 1 ? pz + 1 : (qi > bs ? bs : qi);
    }
    q = x == 0.0f ? pz : v;
    sure = x == 0.0f || (ok && fits && !clamped && dist > margin + c.vm && a >= 0x1p-124f &&
                         a < 0x1p126f);
    return x == 0.0f || (ok && fits);
}

// Bound check of an FP32 input against the grid value p by the fast path:
// returns false when the bound cannot decide; else sets ok to the FP64
// path's verdict on x^ = (float) inverse(p).
__device__ __forceinline__ bool within_bound_fast(float x, int p, const DevConsts &c, bool &ok)
{
    const int pz = (int)c.p_zero, bs = (int)c.b_sign, dl = (int)c.delta;
    const bool zero_hat = p <= pz;  // x^ = 0
    const bool neg = p > bs;
    // the operations of grid_inverse: t = q w - L
    const double tq = neg ? (double)(p - dl) * c.w - c.Ln : (double)p * c.w - c.Lp;
    const double k = __builtin_rint(tq);
    const bool k_ok = k >= -125.0 && k <= 127.0;
    const double f = tq - k;  // exact, |f| <= 1/2
    const int ki = (int)(k_ok ? k : 0.0);
    const double y = __builtin_ldexp((double)__builtin_amdgcn_exp2f((float)f), ki);
    // |y - x^| <= y (kFastExp2Err + 2^-26 (rounding of f) + 2^-24 (rounding of x^)
    // + 2^-50), enlarged slightly
    const double slack = y * (kFastExp2Err + 0x1p-23);
    const double ax = __builtin_fabs((double)x);
    const double d = __builtin_fabs(ax - y);
    const double bnd = c.eps * ax;
    const bool yes = d + slack <= bnd, no = d - slack > bnd;
    const bool exact_no = x == 0.0f || __builtin_signbit(x) != neg;  // x^ != 0 here
    ok = zero_hat ? x == 0.0f : (!exact_no && yes);
    return zero_hat || exact_no || (k_ok && (yes || no));
}

// Inverse of the grid map (zero / positive / negative by threshold), rounded
// to the field's dtype; one exp2 per point whatever the range.
template <typename T>
__device__ __forceinline__ double grid_inverse(int p, const DevConsts &c)
{
    const long long q = p;
    const bool neg = q > c.b_sign;
    const double t = neg ? (double)(q - c.delta) * c.w - c.Ln : (double)q * c.w - c.Lp;
    const double e = det_exp2(t);
    const double v = q <= c.p_zero ? 0.0 : (neg ? -e : e);
    return to_dtype<T>(v);
}

// |x - x^| <= eps |x| with sign and zero preserved, in FP64.
__device__ __forceinline__ bool within_bound(double x, double xh, double eps)
{
    if (x == 0.0)
        return xh == 0.0;
    if (xh == 0.0)
        return false;
    if (__builtin_signbit(x) != __builtin_signbit(xh))
        return false;
    return __builtin_fabs(x - xh) <= eps * __builtin_fabs(x);
}

// Quantization code of a prediction (Algorithm 1: error = prediction - actual).
__device__ __forceinline__ unsigned short make_code(long long pred, int p, bool ok)
{
    const long long e = pred - (long long)p;
    return (ok && e > -kR && e < kR) ? (unsigned short)(e + kR) : (unsigned short)0;
}

// Lorenzo coefficient (-1)^(|o|+1) of the one-layer Lorenzo predictor.
__host__ __device__ constexpr int lorenzo_sign(int o)
{
    return (__builtin_popcount((unsigned)o) & 1) ? 1 : -1;
}

}  // namespace pwrel
