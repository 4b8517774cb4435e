// fs_point.hpp -- per-point arithmetic of the long-characteristics formal
// solution, shared by the box and the spherical sweep kernels (gfx950).
//
// Per point (Listing 1 of the paper): optical steps from the voxel opacities
// and path lengths (step 3), interpolation weights with the linear fallback
// (step 4) and the vacuum fix-up (4a), the Lambda* data (4b) and exp(-dtau)
// for the intensity update (5).  Everything here is evaluated in double; the
// results are rounded to the recurrence type T at the end.
#pragma once

#include <hip/hip_runtime.h>

namespace rt3d {

// a b + c by the three-address v_fma_f64 with every operand in a vector
// register: the compiler's two-address v_fmac form would first copy a
// constant addend (a polynomial coefficient held in a register) into the
// destination at every use.
__device__ __forceinline__ double fma3(double a, double b, double c)
{
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

__device__ __forceinline__ double seg_depth(double chi, double s)
{
#pragma clang fp contract(off)
    return chi * s;
}

__device__ __forceinline__ double half_sum(double a, double b)
{
#pragma clang fp contract(off)
    return 0.5 * (a + b);
}

// 1/x from the hardware reciprocal estimate refined by Newton steps
// r <- r + r (1 - x r), each of which doubles the correct bits: two steps for
// double results, one when the weights are rounded to single precision.
template <bool FULL = true>
__device__ __forceinline__ double rcp_f64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    if (!FULL) return r;
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// exp(-D) for 1/4 <= D, double results: the Cody-Waite argument reduction
// x = -D = n ln2 + r, |r| <= ln2/2, where n ln2 is subtracted in two parts
// (ln2 split into a high part with trailing zero bits, so that n times it is
// exact, and the low remainder; the split of the fdlibm exponential), exp(r)
// by its degree-12 Taylor polynomial, scaled by 2^n.  D is clamped at 745,
// where the result is already below the smallest subnormal.
__device__ __forceinline__ double exp_neg(double D)
{
    const double x = -(D < 745.0 ? D : 745.0);
    const double n = __builtin_rint(x * 1.4426950408889634);
    double r = __builtin_fma(-n, 6.93147180369123816490e-01, x);
    r = __builtin_fma(-n, 1.90821492927058770002e-10, r);
    double p = 1.0 / 479001600.0;
    p = __builtin_fma(p, r, 1.0 / 39916800.0);
    p = __builtin_fma(p, r, 1.0 / 3628800.0);
    p = __builtin_fma(p, r, 1.0 / 362880.0);
    p = __builtin_fma(p, r, 1.0 / 40320.0);
    p = __builtin_fma(p, r, 1.0 / 5040.0);
    p = __builtin_fma(p, r, 1.0 / 720.0);
    p = __builtin_fma(p, r, 1.0 / 120.0);
    p = __builtin_fma(p, r, 1.0 / 24.0);
    p = __builtin_fma(p, r, 1.0 / 6.0);
    p = __builtin_fma(p, r, 0.5);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    return __builtin_ldexp(p, (int)n);
}

// exp(-D) for 1/4 <= D and single-precision results (the split moments
// below): the reduction of exp_neg, then exp(r) = exp(r/16)^16 with exp(r/16)
// (|r/16| <= 0.0217) from its degree-6 Taylor polynomial (truncation below
// 1e-14 relative after the squarings, rounding ~3e-15).
__device__ __forceinline__ double exp_neg_single(double D)
{
    const double x = -(D < 745.0 ? D : 745.0);
    const double n = __builtin_rint(x * 1.4426950408889634);
    double r = __builtin_fma(-n, 6.93147180369123816490e-01, x);
    r = __builtin_fma(-n, 1.90821492927058770002e-10, r);
    const double s = __builtin_ldexp(r, -4);
    double p = __builtin_fma(s, 1.0 / 720.0, 1.0 / 120.0);
    p = __builtin_fma(p, s, 1.0 / 24.0);
    p = __builtin_fma(p, s, 1.0 / 6.0);
    p = __builtin_fma(p, s, 0.5);
    p = __builtin_fma(p, s, 1.0);
    p = __builtin_fma(p, s, 1.0);
    p = p * p;
    p = p * p;
    p = p * p;
    p = p * p;
    return __builtin_ldexp(p, (int)n);
}

// Attenuation moments for single-precision results, one polynomial for every
// step D > 0 (see kernel_moments for the definitions).  x = -min(D, 745) =
// n ln2 + r with n = rint(x / ln2) and |r| <= ln2/2; the reduction takes one
// FMA with ln2 rounded to double, whose error (|n| <= 1075 times 2.3e-17)
// stays below 3e-14.  The tail u = e^r - 1 - r = r^2 (1/2 + r P(r)), with
// P(r) = sum_{j>=0} r^j/(j+3)! from its degree-6 interpolant at the Chebyshev
// nodes of |r| <= ln2/2 (relative error 1.6e-11 there).  Where n = 0 (D below ln2/2) r is -D
// exactly and the moments follow from u with no cancellation: e1 = u,
// e0 = D - u, ex = 1 - e0, e2 = D^2 - 2 e1 = -2 r^3 P.  Elsewhere
// ex = 2^n (1 + r + u) and the closed forms below, which lose at most about
// five bits to cancellation from D = ln2/2 up.
__device__ __forceinline__ void moments_single(double D, double &ex, double &e0, double &e1, double &e2)
{
    // x = max(-D, -745) by one instruction (the library minimum would first
    // quiet signalling NaNs, which arithmetic never produces); a NaN step
    // gives a finite x, and e1, e2 keep the NaN
    double x;
    asm("v_max_f64 %0, -%1, %2" : "=v"(x) : "v"(D), "s"(-745.0));
    const double n = __builtin_rint(x * 1.4426950408889634);
    const double r = __builtin_fma(-n, 0.6931471805599453, x);
    // degree-6 Chebyshev interpolant of P on |r| <= ln2/2 (gen_moment_poly.py)
    double P = fma3(2.761004197490652e-06, r, 2.485957814859904e-05);
    P = fma3(P, r, 0.00019841238150245533);
    P = fma3(P, r, 0.0013888854049701165);
    P = fma3(P, r, 0.008333333338101687);
    P = fma3(P, r, 0.0416666667189806);
    P = fma3(P, r, 0.16666666666666652);
    const double r2 = r * r;
    const double h = __builtin_fma(r, P, 0.5);  // u = r^2 h
    if (n == 0.0) {
        const double u = r2 * h;
        e1 = u;
        e0 = D - u;
        ex = 1.0 - e0;
        e2 = (-2.0 * r2) * (r * P);
    } else {
        ex = __builtin_ldexp(__builtin_fma(r2, h, 1.0 + r), (int)n);
        e0 = 1.0 - ex;
        e1 = D - e0;
        e2 = __builtin_fma(D, D, -2.0 * e1);
    }
}

// Attenuation moments over an optical step D > 0:
//   ex = exp(-D), e0 = 1 - ex, e1 = D - e0, e2 = D^2 - 2 e1.
// Double results (FULL): below D = 1/4, e2 comes from its 12-term Taylor
// series 2 D^3 sum_j (-D)^j/(j+3)! and e1, e0, ex follow from it without
// cancellation; from 1/4 up the closed forms are used (separate branches: a
// wave whose steps straddle 1/4 runs both).  Single-precision results take
// moments_single, one path for all D, or with SPLIT the same two branches
// with a 7-term series (first omitted term below 1e-10 of e2 at D = 1/4) and
// exp_neg_single: fewer registers, cheaper where the steps of a wave seldom
// straddle 1/4 (the spherical sweep).
template <bool FULL, bool SPLIT = false>
__device__ __forceinline__ void kernel_moments(double D, double &ex, double &e0, double &e1, double &e2)
{
    if constexpr (!FULL && !SPLIT) {
        moments_single(D, ex, e0, e1, e2);
        return;
    }
    double p;
    if constexpr (FULL) {
        p = 1.0 / 87178291200.0;                       // 1/14!
        p = __builtin_fma(-D, p, 1.0 / 6227020800.0);  // 1/13!
        p = __builtin_fma(-D, p, 1.0 / 479001600.0);   // 1/12!
        p = __builtin_fma(-D, p, 1.0 / 39916800.0);    // 1/11!
        p = __builtin_fma(-D, p, 1.0 / 3628800.0);     // 1/10!
        p = __builtin_fma(-D, p, 1.0 / 362880.0);      // 1/9!
    } else {
        p = 1.0 / 362880.0;                            // 1/9!
    }
    p = __builtin_fma(-D, p, 1.0 / 40320.0);       // 1/8!
    p = __builtin_fma(-D, p, 1.0 / 5040.0);        // 1/7!
    p = __builtin_fma(-D, p, 1.0 / 720.0);         // 1/6!
    p = __builtin_fma(-D, p, 1.0 / 120.0);         // 1/5!
    p = __builtin_fma(-D, p, 1.0 / 24.0);          // 1/4!
    p = __builtin_fma(-D, p, 1.0 / 6.0);           // 1/3!
    const double D2 = D * D;
    if (D < 0.25) {
        e2 = 2.0 * D2 * D * p;
        e1 = 0.5 * (D2 - e2);
        e0 = D - e1;
        ex = 1.0 - e0;
        return;
    }
    ex = FULL ? exp_neg(D) : exp_neg_single(D);
    e0 = 1.0 - ex;
    e1 = D - e0;
    e2 = __builtin_fma(D, D, -2.0 * e1);
}

// Smallest optical step used in the arithmetic: a vacuum segment (D = 0,
// Listing 1 step 4a) is evaluated at this step, which leaves the intensity
// unchanged to within 1e-100 of S and keeps the shared reciprocal finite.
constexpr double kMinStep = 1e-100;

// Weights of the segment from the previous point (upwind optical step D) to
// the current one, the downwind step being Dp (ignored when last), in the
// type T of the recurrence:
//   I_m = I_{m-1} ex + a S_{m-1} + b S_m + g S_{m+1}.
// Parabolic: the Lagrange quadratic through the three points integrated
// against exp(-(D-t)); with r = 1/(D Dp (D+Dp)),
//   b = ((D+Dp) e1 - e2) (D+Dp) r,  g = (e2 - D e1) D r,  a = e0 - b - g.
// Linear (the last point of a ray, Dp < D/2, or where the parabolic b would
// reach 1, i.e. Dp e0 <= D e1 - e2):  b = e1/D, a = e0 - b, g = 0.
// dlin = e1/D is the diagonal of the linear-interpolation operator.
template <typename T>
struct PointW {
    T a, b, g, ex, dlin;
};

// FULL: double-accurate moments (the default for double results); false: the
// shorter forms that suffice for single-precision results (SPLIT: their
// two-branch variant).  LIMIT: linear points by the parabolic formulas with
// the downwind step replaced by 2^300, as in point_weights_pos (DLIN: also
// the linear diagonal e1/D, else dlin is left zero).
template <typename T, bool FULL = sizeof(T) == 8, bool SPLIT = false, bool LIMIT = false, bool DLIN = true>
__device__ __forceinline__ PointW<T> point_weights(double D, double Dp, bool last)
{
    const double Dv = D < kMinStep ? kMinStep : D;  // NaN propagates
    double ex, e0, e1, e2;
    kernel_moments<FULL, SPLIT>(Dv, ex, e0, e1, e2);
    const double Dq = Dp < kMinStep ? Dv : Dp;   // keeps r finite on last/vacuum points; NaN propagates
    if constexpr (LIMIT) {
        const double h = __builtin_fma(Dv, e1, -e2);  // D e1 - e2
        const bool lin = last || (Dp < 0.5 * D) || (Dp * e0 <= h);
        const double Dl = lin ? 0x1p300 : Dq;
        const double Ds = Dv + Dl;
        const double r = rcp_f64<FULL>(Dv * Dl * Ds);
        const double b = __builtin_fma(Ds, e1, -e2) * (Ds * r);
        const double g = h * (-Dv * r);
        PointW<T> w;
        w.ex = T(ex);
        w.b = T(b);
        w.g = T(g);
        w.a = T(e0 - b - g);
        w.dlin = T(0);
        if constexpr (DLIN) w.dlin = T(e1 * rcp_f64<FULL>(Dv));
        return w;
    }
    const double Ds = Dv + Dq;
    const double r = rcp_f64<FULL>(Dv * Dq * Ds);
    const double bl = e1 * ((Dq * Ds) * r);      // e1 / D
    const bool lin = last || (Dp < 0.5 * D) || (Dp * e0 <= __builtin_fma(Dv, e1, -e2));
    const double bp = __builtin_fma(Ds, e1, -e2) * (Ds * r);
    const double gp = (e2 - Dv * e1) * (Dv * r);
    PointW<T> w;
    w.ex = T(ex);
    w.dlin = T(bl);
    if (sizeof(T) == 8) {
        w.b = lin ? T(bl) : T(bp);
        w.g = lin ? T(0) : T(gp);
        w.a = lin ? T(e0 - bl) : T(e0 - bp - gp);
    } else {
        const T bl_t = T(bl), al_t = T(e0 - bl), bp_t = T(bp), gp_t = T(gp), ap_t = T(e0 - bp - gp);
        w.b = lin ? bl_t : bp_t;
        w.g = lin ? T(0) : gp_t;
        w.a = lin ? al_t : ap_t;
    }
    return w;
}

// point_weights for optical steps that are already at least kMinStep (formed
// by step_depth): no clamping here.  LAST: the final point of a ray (linear
// weights; Dp is not read).  DLIN: also the linear operator's diagonal e1/D.
// The linear weights are the parabolic ones in the limit of an infinite
// downwind step, so a point that takes them is evaluated with Dp replaced by
// 2^300: beta = e1/D (1 + O(D/2^300)) and gamma = -(D e1 - e2)/(2^300 (D +
// 2^300)), far below the rounding of either for any physical step (gamma is
// then zero in single precision), with one select in place of one per
// weight.  D D'(D + D') stays finite for every D below 2^424.
template <typename T, bool LAST, bool DLIN = true>
__device__ __forceinline__ PointW<T> point_weights_pos(double D, double Dp)
{
    constexpr bool FULL = sizeof(T) == 8;
    double ex, e0, e1, e2;
    kernel_moments<FULL>(D, ex, e0, e1, e2);
    const double h = __builtin_fma(D, e1, -e2);  // D e1 - e2
    const bool lin = LAST || (Dp < 0.5 * D) || (Dp * e0 <= h);
    const double Dq = lin ? 0x1p300 : Dp;
    const double Ds = D + Dq;
    // single-precision results take the hardware estimate as it is: its relative
    // error, at most 4.6e-8 (2^-24.4) over a million random arguments, is below
    // the rounding of the weights to single precision, and a = e0 - b - g keeps
    // the three weights summing to e0 whatever the error of b and g
    const double r = FULL ? rcp_f64<true>(D * Dq * Ds) : __builtin_amdgcn_rcp(D * Dq * Ds);
    const double q = Ds * r;  // 1 / (D Dq)
    const double b = __builtin_fma(Ds, e1, -e2) * q;
    const double g = h * (-D * r);
    PointW<T> w;
    w.ex = T(ex);
    w.b = T(b);
    w.g = T(g);
    w.a = T(e0 - b - g);
    w.dlin = T(0);
    if constexpr (DLIN) w.dlin = T(e1 * (FULL ? rcp_f64<true>(D) : __builtin_amdgcn_rcp(D)));
    return w;
}

// Optical step between two points from their optical depths: D = (ta + tb)/2
// + kMinStep by one FMA (the half sum is exact, so the sum rounds back to it
// for every D above 2^-276; a vacuum step, ta = tb = 0, becomes kMinStep, and
// so the shared reciprocal of the weights stays finite).  NaN and Inf
// propagate.  Depths ta, tb >= 0 (opacities are non-negative).
__device__ __forceinline__ double step_depth(double ta, double tb)
{
    double sum;
    {
#pragma clang fp contract(off)
        sum = ta + tb;
    }
    double d;
    asm("v_fma_f64 %0, %1, 0.5, %2" : "=v"(d) : "v"(sum), "s"(kMinStep));
    return d;
}

// Entry half-segment: constant S from the entry point to the first point.
template <typename T, bool SPLIT = false>
__device__ __forceinline__ void entry_weights(double D0, T &ex_t, T &e0_t)
{
    constexpr bool FULL = sizeof(T) == 8;
    double ex, e0, e1, e2;
    kernel_moments<FULL, SPLIT>(D0 < kMinStep ? kMinStep : D0, ex, e0, e1, e2);
    ex_t = T(ex);
    e0_t = T(e0);
}

}  // namespace rt3d
