// ez_math.h -- FP64 device special functions for the Epstein zeta kernels.
//
// E_p(a) = int_1^inf e^{-a t} t^{-p} dt (generalised exponential integral) carries
// every incomplete gamma of the method: a^{-s} Gamma(s, a) = E_{1-s}(a).
//  * E_1: a < 1 power series (DLMF 6.6.2); a >= 1 the rational fit of
//    x e^x E1(x) in t = 1/x from e1_rational.h (Sanathanan-Koerner least squares).
//  * E_{1/2}(a) = sqrt(pi/a) erfc(sqrt a).
//  * other p by the recurrence p E_{p+1} = e^{-a} - a E_p (DLMF 8.19.12), upward
//    from E_1 / E_{1/2} for p >= 1, downward from E_0 = e^{-a}/a / E_{1/2} below.
#pragma once
#include <hip/hip_runtime.h>
#include "e1_rational.h"
#include "exp2_table.h"
#include "ep_f32_rational.h"
#include "ez_internal.h"

// a*b + c as one three-operand v_fma_f64 whose addend c, a compile-time constant of
// a polynomial or rational table, is read from a scalar register pair: the
// constants of the exponential and of the E_1 / E_{1/2} rationals (about 40
// doubles) then live in SGPRs instead of VGPRs, which the compiler would otherwise
// hoist out of the reciprocal loop (the d = 3 ATM node kernel: 66 VGPRs and seven
// waves per SIMD instead of 124 and four).  c must be uniform over the wave.
__device__ __forceinline__ double ez_fma3(double a, double b, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

// e^{-a} for 0 <= a <= 700.  a = n ln2 + r, n = rint(a / ln2), with ln2 split as
// LN2_HI + LN2_LO (LN2_HI has a 32-bit significand, so n LN2_HI is exact: Cody and
// Waite's argument reduction); e^{-r}, |r| <= ln2/2, by its Taylor series through
// r^13 (truncation < 4e-18); then scaled by 2^{-n}.
__device__ __forceinline__ double ez_expm(double a) {
    const double n = rint(a * 1.4426950408889634);
    double r = fma(-n, 0.6931471803691238, a);
    r = fma(-n, 1.9082149292705877e-10, r);
    const double x = -r;
    double p = 1.0 / 6227020800.0;                       // 1/13!
    p = ez_fma3(p, x, 1.0 / 479001600.0);
    p = ez_fma3(p, x, 1.0 / 39916800.0);
    p = ez_fma3(p, x, 1.0 / 3628800.0);
    p = ez_fma3(p, x, 1.0 / 362880.0);
    p = ez_fma3(p, x, 1.0 / 40320.0);
    p = ez_fma3(p, x, 1.0 / 5040.0);
    p = ez_fma3(p, x, 1.0 / 720.0);
    p = ez_fma3(p, x, 1.0 / 120.0);
    p = ez_fma3(p, x, 1.0 / 24.0);
    p = ez_fma3(p, x, 1.0 / 6.0);
    p = fma(p, x, 0.5);
    p = fma(p, x, 1.0);
    p = fma(p, x, 1.0);
    return ldexp(p, -(int)n);
}

// e^{-a} for 0 <= a <= 700 with a table of 2^{-j/256} in LDS (ez_exp2_tab copied to
// `tab`): a = (n/256) ln2 + r, n = rint(256 a / ln2), |r| <= ln2/512, with ln2/256
// split as the Cody-Waite pair of ez_expm divided by 256 (n LN2_HI/256 exact for
// n < 2^21); e^{-a} = 2^{-floor(n/256)} 2^{-(n mod 256)/256} e^{-r}, e^{-r} by its
// Taylor series through r^4 (truncation < 4e-17 relative).
__device__ __forceinline__ double ez_expm_tab(double a, const double *tab) {
    const double n = rint(a * 369.3299304675746);                 // 256 / ln 2
    double r = fma(-n, 0.6931471803691238 / 256.0, a);
    r = fma(-n, 1.9082149292705877e-10 / 256.0, r);
    const int ni = (int)n;
    const double t = tab[ni & 255];
    const double x = -r;
    double p = 1.0 / 24.0;
    p = ez_fma3(p, x, 1.0 / 6.0);
    p = fma(p, x, 0.5);
    p = fma(p, x, 1.0);
    p = fma(p, x, 1.0);
    return ldexp(p * t, -(ni >> 8));
}

// 1/x: hardware reciprocal estimate refined by two Newton steps (x normal, finite)
__device__ __forceinline__ double ez_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// E1(a) for 0 < a < 1: -gamma - ln a + sum_{k>=1} (-1)^{k+1} a^k / (k k!)
__device__ __forceinline__ double ez_e1_series(double a) {
    // Ein(a) = sum_{k=1}^{19} (-1)^{k+1} a^k/(k k!), Horner in a; terms beyond k = 19 < 1e-19
    double s = 0.0;
#pragma unroll
    for (int k = 19; k >= 1; --k) {
        double fk = 1.0;
        for (int j = 2; j <= k; ++j) fk *= (double)j;          // folded at compile time
        double c = ((k & 1) ? 1.0 : -1.0) / ((double)k * fk);
        s = fma(s, a, c);
    }
    s *= a;
    return -EZ_EULER - log(a) + s;
}

// e^a E1(a) for a >= 1 from the rational fit (relative error < 1e-15)
__device__ __forceinline__ double ez_e1_scaled_large(double a, double inv_a) {
    const double t = inv_a;
    double P = ez_e1r_p[EZ_E1R_DEG], Q = ez_e1r_q[EZ_E1R_DEG];
#pragma unroll
    for (int j = EZ_E1R_DEG - 1; j >= 0; --j) {
        P = fma(P, t, ez_e1r_p[j]);
        Q = fma(Q, t, ez_e1r_q[j]);
    }
    return t * P * ez_rcp(Q);
}

// e^a E1(a) for a >= 1/4 from the wide rational fit, given t = 1/a
__device__ __forceinline__ double ez_e1w_scaled(double t) {
    double P = ez_e1w_p[EZ_E1W_DEG], Q = ez_e1w_q[EZ_E1W_DEG];
#pragma unroll
    for (int j = EZ_E1W_DEG - 1; j >= 0; --j) {
        P = ez_fma3(P, t, ez_e1w_p[j]);
        Q = ez_fma3(Q, t, ez_e1w_q[j]);
    }
    return t * P * ez_rcp(Q);
}

// Far-field bases for a >= 4 from the (7,7) fits with a single reciprocal: with the
// coefficient order reversed, P*(a) = a^7 P(1/a) and Q*(a) = a^7 Q(1/a), so that
//   e^a E1(a)      = t P(t)/Q(t)  = P*(a) / (a Q*(a)),
//   e^a E_{1/2}(a) = t Ph(t)/Qh(t) = Ph*(a) / (a Qh*(a)),
// and 1/a = Q*(a) / (a Q*(a)); all coefficients are positive, so Horner in a keeps
// the relative error at a few units of rounding.  From ex = e^{-a}: E1, E_{1/2}
// (when needed) and inv = 1/a.
__device__ __forceinline__ void ez_far_bases(double a, double ex, bool need_e1, bool need_half, double *E1,
                                             double *Eh, double *inv) {
    double P1 = ez_e1f_p[0], Q1 = ez_e1f_q[0], Ph = ez_ehf_p[0], Qh = ez_ehf_q[0];
#pragma unroll
    for (int j = 1; j <= EZ_E1F_DEG; ++j) {
        if (need_e1) { P1 = ez_fma3(P1, a, ez_e1f_p[j]); Q1 = ez_fma3(Q1, a, ez_e1f_q[j]); }
        if (need_half) { Ph = ez_fma3(Ph, a, ez_ehf_p[j]); Qh = ez_fma3(Qh, a, ez_ehf_q[j]); }
    }
    if (need_e1 && need_half) {
        const double QQ = Q1 * Qh;
        const double R = ez_rcp(a * QQ);
        *E1 = ex * P1 * (R * Qh);
        *Eh = ex * Ph * (R * Q1);
        *inv = R * QQ;
    } else if (need_e1) {
        const double R = ez_rcp(a * Q1);
        *E1 = ex * P1 * R;
        *Eh = 0.0;
        *inv = R * Q1;
    } else if (need_half) {
        const double R = ez_rcp(a * Qh);
        *E1 = 0.0;
        *Eh = ex * Ph * R;
        *inv = R * Qh;
    } else {
        *E1 = 0.0;
        *Eh = 0.0;
        *inv = ez_rcp(a);
    }
}

// ---- FP32 far-field terms of the mixed-precision mode (a >= EZ_EPF_XMIN) ----
// e^{-a} in FP32: x = -a log2 e and n = rint(x) in FP64, the fraction x - n (|.| <= 1/2)
// rounded to FP32, 2^{x-n} by the hardware exponential, scaled by 2^n (exact)
__device__ __forceinline__ float ez_expm_f32(double a) {
    const double x = a * -1.4426950408889634;
    const double n = rint(x);
    return ldexpf(__builtin_amdgcn_exp2f((float)(x - n)), (int)n);
}
// x e^x E_p(x) for x >= EZ_EPF_XMIN, 2p = row + 1, from the (3,3) FP32 fit in t = 1/x
__device__ __forceinline__ float ez_epf(int row, float t) {
    float P = ez_epf_p[row][EZ_EPF_DEG], Q = ez_epf_q[row][EZ_EPF_DEG];
#pragma unroll
    for (int j = EZ_EPF_DEG - 1; j >= 0; --j) {
        P = fmaf(P, t, ez_epf_p[row][j]);
        Q = fmaf(Q, t, ez_epf_q[row][j]);
    }
    return P * __builtin_amdgcn_rcpf(Q);
}

// E1(a) for 0 < a < 1/4 by the series; kept out of line so that its constants
// do not occupy registers in the loops that call it only for a few lanes
__device__ __attribute__((noinline, const)) double ez_e1_small(double a) { return ez_e1_series(a); }

// E1(a), a > 0, given e = e^{-a} and inv_a = 1/a
__device__ __forceinline__ double ez_e1(double a, double e, double inv_a) {
    if (a < 1.0) return ez_e1_series(a);
    return e * ez_e1_scaled_large(a, inv_a);
}

// E_{p}(a) for 2p = p2 (integer), from the bases E1 / E_{1/2}
__device__ __forceinline__ double ez_ep_from(int p2, double a, double e, double inv_a, double E1, double Eh) {
    if ((p2 & 1) == 0) {
        int p = p2 / 2;
        if (p >= 1) {
            double E = E1;
            for (int q = 1; q < p; ++q) E = (e - a * E) * (1.0 / (double)q);
            return E;
        }
        double E = e * inv_a;                      // E_0
        for (int q = -1; q >= p; --q) E = (e - (double)q * E) * inv_a;
        return E;
    }
    // half-integer p = p2/2
    double E = Eh;                                 // E_{1/2}
    if (p2 >= 1) {
        for (int q2 = 1; q2 < p2; q2 += 2) E = (e - a * E) * (2.0 / (double)q2);
        return E;
    }
    for (int q2 = -1; q2 >= p2; q2 -= 2) E = (e - 0.5 * (double)q2 * E) * inv_a;
    return E;
}

// sqrt(pi a) e^a erfc(sqrt a) for a >= 1/4 from the rational fit, given t = 1/a; then
// E_{1/2}(a) = e^{-a} h / a uses the term's e^{-a} and 1/a (no erfc, no second exp)
__device__ __forceinline__ double ez_ehw_scaled(double t) {
    double P = ez_ehw_p[EZ_E1W_DEG], Q = ez_ehw_q[EZ_E1W_DEG];
#pragma unroll
    for (int j = EZ_E1W_DEG - 1; j >= 0; --j) {
        P = ez_fma3(P, t, ez_ehw_p[j]);
        Q = ez_fma3(Q, t, ez_ehw_q[j]);
    }
    return P * ez_rcp(Q);
}

__device__ __forceinline__ double ez_ehalf(double a) {
    double r = sqrt(a);
    return 1.7724538509055160272981674833411452 * erfc(r) / r;   // sqrt(pi) erfc(sqrt a)/sqrt a
}

// 1/Gamma(x), zero at the poles
__device__ __forceinline__ double ez_rgamma(double x) {
    if (x <= 0.0 && x == floor(x)) return 0.0;
    return 1.0 / tgamma(x);
}

// Upper incomplete gamma Gamma(s, a), a > 0, any real s (used off the hot path).
//  2s integer: Gamma(s,a) = a^s E_{1-s}(a) through the E_p recurrences;
//  otherwise, a >= 2 and a >= s + 1: the continued fraction of DLMF 8.9.2 (even
//  part) by Lentz's method;
//  otherwise the series Gamma(s) - a^s sum_k (-a)^k / (k! (s + k)) (DLMF 8.7.1).  Near
//  a pole of Gamma, s = -m + delta (m = rint(-s) >= 0, |delta| < 1/4), Gamma(s) and the
//  k = m term are both ~ 1/delta; with Gamma(-m + delta) = (-1)^m Gamma(1 + delta) /
//  (m! delta prod_{j=1..m} (1 - delta/j)) (DLMF 5.5.1) they combine into
//  (-1)^m [expm1(lgamma(1 + delta) - sum_j log1p(-delta/j)) - expm1(delta ln a)] / (m! delta).
__device__ inline double ez_gamma_upper(double s, double a) {
    const double s2 = 2.0 * s;
    if (s2 == floor(s2) && fabs(s) <= 64.0) {
        int p2 = 2 - (int)s2;                      // 2 (1 - s)
        double e = exp(-a), inv = 1.0 / a;
        double E1 = ((p2 & 1) == 0 && p2 >= 2) ? ez_e1(a, e, inv) : 0.0;
        double Eh = (p2 & 1) ? ez_ehalf(a) : 0.0;
        return pow(a, s) * ez_ep_from(p2, a, e, inv, E1, Eh);
    }
    const double la = log(a);
    if (a >= 2.0 && a >= s + 1.0) {
        const double tiny = 1e-300;
        double F = tiny, C = F, D = 0.0;
        for (int j = 1; j < 4000; ++j) {
            const double aj = (j == 1) ? 1.0 : -(double)(j - 1) * ((double)(j - 1) - s);
            const double bj = a + 2.0 * j - 1.0 - s;
            D = bj + aj * D; if (D == 0.0) D = tiny;
            C = bj + aj / C; if (C == 0.0) C = tiny;
            D = 1.0 / D;
            const double dl = C * D;
            F *= dl;
            if (fabs(dl - 1.0) < 1e-16) break;
        }
        return exp(s * la - a) * F;
    }
    const double mr = rint(-s);
    if (mr >= 0.0 && fabs(s + mr) < 0.25) {
        const int m = (int)mr;
        const double dlt = s + mr;
        double lr = lgamma(1.0 + dlt), mf = 1.0;
        for (int j = 1; j <= m; ++j) {
            lr -= log1p(-dlt / (double)j);
            mf *= (double)j;
        }
        const double hd = (expm1(lr) - expm1(dlt * la)) / (mf * dlt);
        double tail = 0.0, pw = 1.0;                  // pw = (-a)^k / k!
        for (int k = 0; k < 500; ++k) {
            if (k > 0) pw *= -a / (double)k;
            if (k == m) continue;
            const double t = pw / (s + (double)k);
            tail += t;
            if (k > m && fabs(t) < 1e-18 * fabs(tail)) break;
        }
        return ((m & 1) ? -hd : hd) - exp(s * la) * tail;
    }
    double term = 1.0 / s, sum = term;
    for (int k = 1; k < 500; ++k) {
        term *= a / (s + (double)k);
        sum += term;
        if (fabs(term) < 1e-17 * fabs(sum)) break;
    }
    return tgamma(s) - exp(s * la - a) * sum;
}

// E_p(a) = a^{p-1} Gamma(1 - p, a) for real p (non-integer exponents of the quadrature);
// out of line, it is called per term and exponent
__device__ __attribute__((noinline)) double ez_ep_real(double p, double a) {
    return exp((p - 1.0) * log(a)) * ez_gamma_upper(1.0 - p, a);
}

// cos(2 pi t) with the argument reduced exactly modulo 1
__device__ __forceinline__ double ez_cos2pi(double t) { return cospi(2.0 * (t - rint(t))); }
__device__ __forceinline__ void ez_sincos2pi(double t, double *s, double *c) {
    double r = 2.0 * (t - rint(t));
    *s = sinpi(r);
    *c = cospi(r);
}

// out of line, reads and writes no memory (so loads around its call stay scalar)
__device__ __attribute__((noinline, const)) double2 ez_sincos2pi_ool(double t) {
    double s, c;
    ez_sincos2pi(t, &s, &c);
    return make_double2(s, c);
}

// ---- double-double accumulation (error-free sums, fixed order) ----
struct ez_dd { double hi, lo; };
__device__ __forceinline__ ez_dd ez_dd_add(ez_dd a, ez_dd b) {
    double s = a.hi + b.hi;
    double bb = s - a.hi;
    double err = (a.hi - (s - bb)) + (b.hi - bb);
    err += a.lo + b.lo;
    double hi = s + err;
    double lo = err - (hi - s);
    return {hi, lo};
}
__device__ __forceinline__ ez_dd ez_dd_add_d(ez_dd a, double b) { return ez_dd_add(a, ez_dd{b, 0.0}); }

__device__ __forceinline__ ez_dd ez_dd_shfl_xor(ez_dd v, int m) {
    return {__shfl_xor(v.hi, m, 64), __shfl_xor(v.lo, m, 64)};
}
// wave64 butterfly: every lane ends with the same, order-independent-of-timing sum
__device__ __forceinline__ ez_dd ez_dd_wave_sum(ez_dd v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = ez_dd_add(v, ez_dd_shfl_xor(v, m));
    return v;
}
