/*
 * oracle/ezo.c -- plain, slow FP64 CPU reference ("oracle") for the Epstein
 * zeta method for many-body lattice sums (Buchheit & Busse, arXiv 2504.11989).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  It shares no
 * code, header, table or constant with the HIP library: it is an independent
 * statement of what the method computes, written for a reader to check
 * against the paper by eye.  OpenMP is used only to evaluate independent
 * directions in parallel; every reduction is a fixed-order compensated sum.
 *
 * What it computes, and where the paper defines it:
 *   - Epstein zeta Z_{Lambda,nu}(x,y)             Sec. 2, Definition (Epstein zeta function)
 *     by the incomplete-gamma (Crandall) split that the paper cites for its
 *     evaluation; the split itself is not printed in the paper, it follows
 *     from the Mellin integral of |r|^-nu and Poisson summation (written out
 *     above ezo_epstein).
 *   - singular / regular decomposition           Sec. 3, decomposition Z = Z^reg + s_hat/|det A|
 *   - n-body zeta by the Epstein representation  Sec. 2, Theorem (Epstein representation)
 *   - Duffy transform of the Brillouin zone      Sec. 3, Corollary (Duffy transformation)
 *   - Gauss-Legendre in v, split of u at eps,    Sec. 3, the paragraphs on the u-integral and
 *     Taylor expansion of Z^reg on (0,eps),      the meromorphic continuation (Taylor series,
 *     multinomial directional derivatives and    multinomial formula, Hadamard integral)
 *     closed-form Hadamard integrals
 *   - ATM recombination                          Sec. 2, Proposition (ATM in three-body zetas)
 *   - direct truncated sums                      Sec. 2, Definitions (ATM, many-body zeta)
 *
 * Readings where the paper is silent:
 *   - the u-integral on (eps, 1/2] uses a fixed composite Gauss-Legendre rule on
 *     geometric panels (the paper uses adaptive bisection there);
 *   - Z(x,y) at y in Lambda* (and nu != d) takes the value of the meromorphic
 *     continuation in nu at that fixed y; x (y) closer than 1e-12 in
 *     fractional coordinates to a lattice point is snapped onto it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define EZO_PI 3.14159265358979323846264338327950288
#define EZO_EULER 0.57721566490153286060651209008240243

/* status codes (oracle-private) */
#define EZO_OK 0
#define EZO_EINVAL 1
#define EZO_ESINGULAR 2
#define EZO_EPOLE 3
#define EZO_EUNSUPPORTED 4
#define EZO_ENOMEM 5
#define EZO_ENOCONV 6

/* ------------------------------------------------------------------------ */
/* Compensated (Neumaier) summation                                          */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } ksum_t;
static void ks_add(ksum_t *k, double x) {
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
    else k->c += (x - t) + k->s;
    k->s = t;
}
static double ks_val(const ksum_t *k) { return k->s + k->c; }

/* ------------------------------------------------------------------------ */
/* Special functions                                                         */
/* ------------------------------------------------------------------------ */

/* 1/Gamma(x); zero at the poles x = 0, -1, -2, ... */
double ezo_rgamma(double x) {
    if (x <= 0.0 && x == floor(x)) return 0.0;
    return 1.0 / tgamma(x);
}

/* Exponential integral E1(a), a > 0.
 * a <= 1: power series  E1(a) = -gamma - ln a - sum_{k>=1} (-a)^k / (k k!)   (DLMF 6.6.2)
 * a >  1: continued fraction E1(a) = e^-a / (a+1 - 1^2/(a+3 - 2^2/(a+5 - ...)))
 *         (even part of DLMF 6.9.1), evaluated by the modified Lentz method.   */
double ezo_e1(double a) {
    if (!(a > 0.0)) return NAN;
    if (a <= 1.0) {
        double term = 1.0, sum = 0.0;
        for (int k = 1; k < 200; ++k) {
            term *= -a / (double)k;         /* (-a)^k / k! */
            double t = term / (double)k;
            sum += t;
            if (fabs(t) <= 1e-18 * fabs(sum)) break;
        }
        return -EZO_EULER - log(a) - sum;
    }
    const double tiny = 1e-300;
    double f = tiny, C = f, D = 0.0;
    for (int j = 1; j < 100000; ++j) {
        double aj = (j == 1) ? 1.0 : -(double)(j - 1) * (double)(j - 1);
        double bj = a + 2.0 * j - 1.0;
        D = bj + aj * D; if (D == 0.0) D = tiny;
        C = bj + aj / C; if (C == 0.0) C = tiny;
        D = 1.0 / D;
        double delta = C * D;
        f *= delta;
        if (fabs(delta - 1.0) < 1e-17) break;
    }
    return exp(-a) * f;
}

/* Upper incomplete gamma Gamma(s, a) for real s and a > 0.
 *  a >= max(1, s+1): continued fraction (DLMF 8.9.2, even part), modified Lentz
 *  otherwise, s = -m, m in N0: DLMF 8.4.15 with E1
 *  otherwise: Gamma(s) - gamma(s,a), where
 *        gamma(s,a) = a^s e^-a sum_k a^k / (s (s+1) ... (s+k))   (DLMF 8.7.1)      */
double ezo_gamma_upper(double s, double a) {
    if (!(a > 0.0)) {
        if (a == 0.0 && s > 0.0) return tgamma(s);
        return NAN;
    }
    if (a >= 1.0 && a >= s + 1.0) {
        const double tiny = 1e-300;
        double f = tiny, C = f, D = 0.0;
        for (int j = 1; j < 100000; ++j) {
            double aj = (j == 1) ? 1.0 : -(double)(j - 1) * ((double)(j - 1) - s);
            double bj = a + 2.0 * j - 1.0 - s;
            D = bj + aj * D; if (D == 0.0) D = tiny;
            C = bj + aj / C; if (C == 0.0) C = tiny;
            D = 1.0 / D;
            double delta = C * D;
            f *= delta;
            if (fabs(delta - 1.0) < 1e-17) break;
        }
        return exp(s * log(a) - a) * f;
    }
    if (s <= 0.0 && s == floor(s)) {
        int m = (int)(-s);
        double sum = 0.0, kfact = 1.0, apow = 1.0 / a;
        for (int k = 0; k < m; ++k) {
            if (k > 0) kfact *= (double)k;
            sum += ((k % 2) ? -1.0 : 1.0) * kfact * apow;
            apow /= a;
        }
        double mfact = 1.0;
        for (int k = 2; k <= m; ++k) mfact *= (double)k;
        double sgn = (m % 2) ? -1.0 : 1.0;
        return sgn / mfact * (ezo_e1(a) - exp(-a) * sum);
    }
    /* Gamma(s, a) = Gamma(s) - gamma(s, a), gamma(s, a) = a^s sum_k (-a)^k / (k! (s + k))
       (DLMF 8.7.1, the series without the factor e^{-a}).  Near a pole of Gamma(s),
       s = -m + delta with m = round(-s) >= 0 and |delta| small, Gamma(s) and the k = m
       term are both of size 1/delta and cancel.  They are taken together:
         Gamma(-m + delta) = (-1)^m Gamma(1 + delta) / (m! delta prod_{j<=m} (1 - delta/j))
       (DLMF 5.5.1 applied m + 1 times), so
         Gamma(s) - a^s (-a)^m / (m! (s + m))
           = (-1)^m / (m! delta) [ (R - 1) - (a^delta - 1) ],
         R = Gamma(1 + delta) / prod_{j<=m} (1 - delta/j),
       with R - 1 and a^delta - 1 from expm1 of their logarithms (lgamma, log1p). */
    const double m_r = floor(-s + 0.5);
    if (m_r >= 0.0 && fabs(s + m_r) < 0.25) {
        const int m = (int)m_r;
        const double delta = s + m_r;
        double lr = lgamma(1.0 + delta), mfact = 1.0;
        for (int j = 1; j <= m; ++j) {
            lr -= log1p(-delta / (double)j);
            mfact *= (double)j;
        }
        const double la = log(a);
        double head = (expm1(lr) - expm1(delta * la)) / (mfact * delta);
        if (m % 2) head = -head;
        double rest = 0.0, term = 1.0;              /* term = (-a)^k / k! */
        for (int k = 0; k < 100000; ++k) {
            if (k > 0) term *= -a / (double)k;
            if (k == m) continue;
            const double t = term / (s + (double)k);
            rest += t;
            if (k > m && fabs(t) <= 1e-18 * fabs(rest)) break;
        }
        return head - exp(s * la) * rest;
    }
    double term = 1.0 / s, sum = term;
    for (int k = 1; k < 100000; ++k) {
        term *= a / (s + (double)k);
        sum += term;
        if (fabs(term) <= 1e-18 * fabs(sum)) break;
    }
    double lower = exp(s * log(a) - a) * sum;
    return tgamma(s) - lower;
}

/* n-point Gauss-Legendre rule on [lo, hi]: Newton iteration on P_n with the
 * three-term recurrence; weights 2 / ((1-x^2) P_n'(x)^2).                 */
int ezo_gauss_legendre(int n, double lo, double hi, double *x, double *w) {
    if (n < 1) return EZO_EINVAL;
    for (int i = 0; i < n; ++i) {
        double t = cos(EZO_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / (double)k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = t; p0 = 1.0; }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (fabs(dt) < 1e-17) break;
        }
        {   /* final derivative at the converged root */
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / (double)k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = t; p0 = 1.0; }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
        }
        /* root t in (-1,1), descending order; map to ascending on [lo,hi] */
        double wt = 2.0 / ((1.0 - t * t) * dp * dp);
        x[n - 1 - i] = 0.5 * (hi + lo) + 0.5 * (hi - lo) * t;
        w[n - 1 - i] = 0.5 * (hi - lo) * wt;
    }
    return EZO_OK;
}

/* ------------------------------------------------------------------------ */
/* Lattice: Lambda = A Z^d (columns of A are the basis), Lambda* = A^-T Z^d  */
/* (Sec. 2, Definition (Lattices)).  Matrices are row-major d x d.           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int d;
    double A[9], Ainv[9];   /* A and A^{-1}        */
    double B[9], Binv[9];   /* B = A^{-T}, B^{-1} = A^T */
    double V;               /* |det A|             */
    double lam;             /* Ewald split parameter (absolute)  */
    double a_cut;           /* cutoff on the incomplete-gamma argument */
} lat_t;

static int mat_inv(int d, const double *M, double *Mi, double *det) {
    if (d == 1) {
        *det = M[0];
        if (M[0] == 0.0) return EZO_ESINGULAR;
        Mi[0] = 1.0 / M[0];
        return EZO_OK;
    }
    if (d == 2) {
        double dt = M[0] * M[3] - M[1] * M[2];
        *det = dt;
        if (dt == 0.0) return EZO_ESINGULAR;
        Mi[0] = M[3] / dt; Mi[1] = -M[1] / dt;
        Mi[2] = -M[2] / dt; Mi[3] = M[0] / dt;
        return EZO_OK;
    }
    /* d == 3: adjugate / determinant */
    double a = M[0], b = M[1], c = M[2], dd = M[3], e = M[4], f = M[5], g = M[6], h = M[7], i = M[8];
    double c00 = e * i - f * h, c01 = -(dd * i - f * g), c02 = dd * h - e * g;
    double c10 = -(b * i - c * h), c11 = a * i - c * g, c12 = -(a * h - b * g);
    double c20 = b * f - c * e, c21 = -(a * f - c * dd), c22 = a * e - b * dd;
    double dt = a * c00 + b * c01 + c * c02;
    *det = dt;
    if (dt == 0.0) return EZO_ESINGULAR;
    Mi[0] = c00 / dt; Mi[1] = c10 / dt; Mi[2] = c20 / dt;
    Mi[3] = c01 / dt; Mi[4] = c11 / dt; Mi[5] = c21 / dt;
    Mi[6] = c02 / dt; Mi[7] = c12 / dt; Mi[8] = c22 / dt;
    return EZO_OK;
}

static int lat_init(lat_t *L, int d, const double *A, double lam_rel, double a_cut) {
    if (d < 1 || d > 3) return EZO_EINVAL;
    memset(L, 0, sizeof(*L));
    L->d = d;
    for (int i = 0; i < d * d; ++i) {
        if (!isfinite(A[i])) return EZO_EINVAL;
        L->A[i] = A[i];
    }
    double det;
    if (mat_inv(d, L->A, L->Ainv, &det) != EZO_OK) return EZO_ESINGULAR;
    L->V = fabs(det);
    if (!(L->V > 1e-300)) return EZO_ESINGULAR;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            L->B[i * d + j] = L->Ainv[j * d + i];   /* A^{-T} */
            L->Binv[i * d + j] = L->A[j * d + i];   /* A^{T}  */
        }
    if (!(lam_rel > 0.0)) lam_rel = 1.0;
    L->lam = lam_rel * pow(L->V, 1.0 / d);
    L->a_cut = (a_cut > 0.0) ? a_cut : 36.0;
    return EZO_OK;
}

static void matvec(int d, const double *M, const double *x, double *y) {
    for (int i = 0; i < d; ++i) {
        double s = 0.0;
        for (int j = 0; j < d; ++j) s += M[i * d + j] * x[j];
        y[i] = s;
    }
}
static double dot(int d, const double *a, const double *b) {
    double s = 0.0;
    for (int i = 0; i < d; ++i) s += a[i] * b[i];
    return s;
}

/* integer points n with |M n - c| <= R, M with columns as basis */
typedef struct { int n, cap; int *p; } ilist_t;
static void il_free(ilist_t *l) { free(l->p); l->p = NULL; l->n = l->cap = 0; }
static int il_push(ilist_t *l, int d, const int *n) {
    if (l->n == l->cap) {
        int nc = l->cap ? 2 * l->cap : 256;
        int *np = (int *)realloc(l->p, sizeof(int) * 3 * (size_t)nc);
        if (!np) return EZO_ENOMEM;
        l->p = np; l->cap = nc;
    }
    for (int i = 0; i < 3; ++i) l->p[3 * l->n + i] = (i < d) ? n[i] : 0;
    l->n++;
    return EZO_OK;
}
static int enum_ball(int d, const double *M, const double *Minv, const double *c, double R, ilist_t *out) {
    double f[3] = {0, 0, 0}, h[3] = {0, 0, 0};
    matvec(d, Minv, c, f);
    for (int i = 0; i < d; ++i) {
        double r = 0.0;
        for (int j = 0; j < d; ++j) r += Minv[i * d + j] * Minv[i * d + j];
        h[i] = R * sqrt(r);
    }
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int i = 0; i < d; ++i) {
        lo[i] = (int)ceil(f[i] - h[i]);
        hi[i] = (int)floor(f[i] + h[i]);
    }
    int n[3];
    for (n[2] = lo[2]; n[2] <= hi[2]; ++n[2])
        for (n[1] = lo[1]; n[1] <= hi[1]; ++n[1])
            for (n[0] = lo[0]; n[0] <= hi[0]; ++n[0]) {
                double nd[3] = {n[0], n[1], n[2]}, z[3];
                matvec(d, M, nd, z);
                double r2 = 0.0;
                for (int i = 0; i < d; ++i) r2 += (z[i] - c[i]) * (z[i] - c[i]);
                if (r2 <= R * R)
                    if (il_push(out, d, n) != EZO_OK) return EZO_ENOMEM;
            }
    return EZO_OK;
}

/* ------------------------------------------------------------------------ */
/* Epstein zeta by the incomplete-gamma split.                               */
/*                                                                           */
/* From |r|^-nu = pi^{nu/2}/Gamma(nu/2) int_0^inf t^{nu/2-1} e^{-pi t r^2} dt,*/
/* split at t = 1/lam^2; Poisson summation on the small-t piece gives, for   */
/* any lam > 0,                                                              */
/*  Z(x,y) = sum_{z in Lambda, z != x} e^{-2 pi i y.z}                       */
/*             Gamma(nu/2, pi|z-x|^2/lam^2) / (Gamma(nu/2) |z-x|^nu)         */
/*         + pi^{nu-d/2}/(Gamma(nu/2) V) sum_{m* in Lambda*}                  */
/*             e^{-2 pi i (m*+y).x} |m*+y|^{nu-d} Gamma((d-nu)/2, pi lam^2|m*+y|^2) */
/*         - [x in Lambda] e^{-2 pi i y.x} (pi/lam^2)^{nu/2} / Gamma(nu/2+1)  */
/* The m*+y = 0 term is its continuation in nu: 2 (pi lam^2)^{(d-nu)/2}/(nu-d).*/
/* Terms whose incomplete-gamma argument exceeds a_cut are dropped.          */
/* ------------------------------------------------------------------------ */
static int snap_int(int d, double *f, int *n) {
    int all = 1;
    for (int i = 0; i < d; ++i) {
        double r = nearbyint(f[i]);
        if (fabs(f[i] - r) >= 1e-12) all = 0;
        n[i] = (int)r;
    }
    return all;
}

int ezo_epstein(int d, const double *A, double nu, const double *x_in, const double *y_in,
                double lam_rel, double a_cut, double *re, double *im) {
    lat_t L;
    int st = lat_init(&L, d, A, lam_rel, a_cut);
    if (st) return st;
    if (!isfinite(nu)) return EZO_EINVAL;
    double x[3] = {0, 0, 0}, y[3] = {0, 0, 0};
    for (int i = 0; i < d; ++i) { x[i] = x_in[i]; y[i] = y_in[i]; }

    /* is x a lattice point? is y a reciprocal lattice point? */
    double fx[3], gy[3];
    int nx[3] = {0, 0, 0}, my[3] = {0, 0, 0};
    matvec(d, L.Ainv, x, fx);
    int x_in_lat = snap_int(d, fx, nx);
    if (x_in_lat) {
        double nd[3] = {nx[0], nx[1], nx[2]};
        matvec(d, L.A, nd, x);
    }
    matvec(d, L.Binv, y, gy);
    int y_in_rec = snap_int(d, gy, my);
    if (y_in_rec) {
        double md[3] = {my[0], my[1], my[2]};
        matvec(d, L.B, md, y);
    }

    const double lam = L.lam, lam2 = lam * lam;
    const double s_real = 0.5 * nu;
    const double s_rec = 0.5 * (d - nu);
    const double rg = ezo_rgamma(0.5 * nu);
    ksum_t sr = {0, 0}, si = {0, 0};

    /* real-space sum */
    ilist_t zl = {0, 0, NULL};
    double Rr = lam * sqrt(L.a_cut / EZO_PI);
    if (enum_ball(d, L.A, L.Ainv, x, Rr, &zl)) return EZO_ENOMEM;
    for (int t = 0; t < zl.n; ++t) {
        int *n = &zl.p[3 * t];
        if (x_in_lat && n[0] == nx[0] && n[1] == nx[1] && n[2] == nx[2]) continue;
        double nd[3] = {n[0], n[1], n[2]}, z[3], r[3];
        matvec(d, L.A, nd, z);
        for (int i = 0; i < d; ++i) r[i] = z[i] - x[i];
        double r2 = dot(d, r, r);
        double a = EZO_PI * r2 / lam2;
        if (a > L.a_cut) continue;
        double mag = ezo_gamma_upper(s_real, a) * rg * pow(r2, -0.5 * nu);
        double ph = -2.0 * EZO_PI * dot(d, y, z);
        ks_add(&sr, mag * cos(ph));
        ks_add(&si, mag * sin(ph));
    }
    il_free(&zl);

    /* reciprocal-space sum */
    ksum_t rr = {0, 0}, ri = {0, 0};
    ilist_t ml = {0, 0, NULL};
    double Rk = sqrt(L.a_cut / EZO_PI) / lam;
    double my_neg[3] = {-y[0], -y[1], -y[2]};
    if (enum_ball(d, L.B, L.Binv, my_neg, Rk, &ml)) return EZO_ENOMEM;
    for (int t = 0; t < ml.n; ++t) {
        int *m = &ml.p[3 * t];
        double md[3] = {m[0], m[1], m[2]}, q[3];
        matvec(d, L.B, md, q);
        for (int i = 0; i < d; ++i) q[i] += y[i];
        double q2 = dot(d, q, q);
        double val;
        if (y_in_rec && m[0] == -my[0] && m[1] == -my[1] && m[2] == -my[2]) {
            if (s_rec == 0.0) { il_free(&ml); return EZO_EPOLE; }
            val = -pow(EZO_PI * lam2, s_rec) / s_rec;
            q2 = 0.0;
        } else {
            double a = EZO_PI * lam2 * q2;
            if (a > L.a_cut) continue;
            val = pow(q2, -s_rec) * ezo_gamma_upper(s_rec, a);
        }
        double ph = -2.0 * EZO_PI * dot(d, q, x);
        ks_add(&rr, val * cos(ph));
        ks_add(&ri, val * sin(ph));
    }
    il_free(&ml);
    double pref = pow(EZO_PI, nu - 0.5 * d) * rg / L.V;

    double out_re = ks_val(&sr) + pref * ks_val(&rr);
    double out_im = ks_val(&si) + pref * ks_val(&ri);
    if (x_in_lat) {
        double self = pow(EZO_PI / lam2, 0.5 * nu) * ezo_rgamma(0.5 * nu + 1.0);
        double ph = -2.0 * EZO_PI * dot(d, y, x);
        out_re -= self * cos(ph);
        out_im -= self * sin(ph);
    }
    *re = out_re;
    *im = out_im;
    return EZO_OK;
}

/* ------------------------------------------------------------------------ */
/* Singular part s_hat_nu(k) / |det A|   (Sec. 3, decomposition of Z)        */
/*   nu not in d+2N0 : pi^{nu-d/2} Gamma((d-nu)/2)/Gamma(nu/2) |k|^{nu-d}    */
/*   nu = d+2m       : pi^{2m+d/2}/Gamma(m+d/2) (-1)^{m+1}/m! |k|^{2m} log(pi k^2) */
/* ------------------------------------------------------------------------ */
static int log_case(int d, double nu, int *m) {
    double t = 0.5 * (nu - d);
    if (t >= 0.0 && t == floor(t)) { *m = (int)t; return 1; }
    return 0;
}
static double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return f;
}

/* coefficient sigma and exponent e of s_hat(u w)/V = sigma u^e L(u)^delta,
 * L(u) = log(pi u^2 |w|^2)                                                  */
static void sing_coef(int d, double V, double nu, double w2, double *sigma, double *e, int *delta) {
    int m;
    if (log_case(d, nu, &m)) {
        *sigma = pow(EZO_PI, 2.0 * m + 0.5 * d) * ezo_rgamma(m + 0.5 * d) *
                 (((m + 1) % 2) ? -1.0 : 1.0) / factorial(m) * pow(w2, (double)m) / V;
        *e = 2.0 * m;
        *delta = 1;
    } else {
        *sigma = pow(EZO_PI, nu - 0.5 * d) * tgamma(0.5 * (d - nu)) * ezo_rgamma(0.5 * nu) *
                 pow(w2, 0.5 * (nu - d)) / V;
        *e = nu - d;
        *delta = 0;
    }
}

double ezo_sing(int d, const double *A, double nu, const double *k) {
    lat_t L;
    if (lat_init(&L, d, A, 1.0, 36.0)) return NAN;
    double k2 = dot(d, k, k);
    double sigma, e; int delta;
    sing_coef(d, L.V, nu, k2, &sigma, &e, &delta);   /* with w = k, u = 1 */
    return delta ? sigma * log(EZO_PI * k2) : sigma;
}

/* ------------------------------------------------------------------------ */
/* Per-lattice, per-nu context for x = 0 evaluations at many k.              */
/* ------------------------------------------------------------------------ */
typedef struct {
    double nu, s_rec, rg, pref, self;
    int nz;
    double *z;      /* nz x 3 */
    double *W;      /* nz: Gamma(nu/2, pi|z|^2/lam^2)/(Gamma(nu/2)|z|^nu) */
} nuctx_t;

static void nuctx_free(nuctx_t *c) { free(c->z); free(c->W); c->z = c->W = NULL; }

static int nuctx_init(nuctx_t *c, const lat_t *L, double nu) {
    memset(c, 0, sizeof(*c));
    const int d = L->d;
    const double lam2 = L->lam * L->lam;
    c->nu = nu;
    c->s_rec = 0.5 * (d - nu);
    c->rg = ezo_rgamma(0.5 * nu);
    c->pref = pow(EZO_PI, nu - 0.5 * d) * c->rg / L->V;
    c->self = pow(EZO_PI / lam2, 0.5 * nu) * ezo_rgamma(0.5 * nu + 1.0);
    ilist_t zl = {0, 0, NULL};
    double zero[3] = {0, 0, 0};
    double Rr = L->lam * sqrt(L->a_cut / EZO_PI);
    if (enum_ball(d, L->A, L->Ainv, zero, Rr, &zl)) return EZO_ENOMEM;
    c->z = (double *)calloc((size_t)zl.n * 3 + 3, sizeof(double));
    c->W = (double *)calloc((size_t)zl.n + 1, sizeof(double));
    if (!c->z || !c->W) { il_free(&zl); return EZO_ENOMEM; }
    int cnt = 0;
    for (int t = 0; t < zl.n; ++t) {
        int *n = &zl.p[3 * t];
        if (n[0] == 0 && n[1] == 0 && n[2] == 0) continue;
        double nd[3] = {n[0], n[1], n[2]}, z[3] = {0, 0, 0};
        matvec(d, L->A, nd, z);
        double r2 = dot(d, z, z);
        double a = EZO_PI * r2 / lam2;
        if (a > L->a_cut) continue;
        for (int i = 0; i < 3; ++i) c->z[3 * cnt + i] = z[i];
        c->W[cnt] = ezo_gamma_upper(0.5 * nu, a) * c->rg * pow(r2, -0.5 * nu);
        cnt++;
    }
    c->nz = cnt;
    il_free(&zl);
    return EZO_OK;
}

/* full Z_{Lambda,nu}(0,k) (real), k not in Lambda*  */
static double z0_full(const lat_t *L, const nuctx_t *c, const double *k, int *err) {
    const int d = L->d;
    const double lam2 = L->lam * L->lam;
    ksum_t sr = {0, 0};
    for (int t = 0; t < c->nz; ++t) {
        double ph = 2.0 * EZO_PI * dot(d, k, &c->z[3 * t]);
        ks_add(&sr, c->W[t] * cos(ph));
    }
    ksum_t rr = {0, 0};
    ilist_t ml = {0, 0, NULL};
    double Rk = sqrt(L->a_cut / EZO_PI) / L->lam;
    double kneg[3] = {-k[0], -k[1], -k[2]};
    if (enum_ball(d, L->B, L->Binv, kneg, Rk, &ml)) { *err = EZO_ENOMEM; return NAN; }
    for (int t = 0; t < ml.n; ++t) {
        int *m = &ml.p[3 * t];
        double md[3] = {m[0], m[1], m[2]}, q[3];
        matvec(d, L->B, md, q);
        for (int i = 0; i < d; ++i) q[i] += k[i];
        double q2 = dot(d, q, q);
        double a = EZO_PI * lam2 * q2;
        if (a > L->a_cut) continue;
        if (q2 == 0.0) { *err = EZO_EPOLE; il_free(&ml); return NAN; }
        ks_add(&rr, pow(q2, -c->s_rec) * ezo_gamma_upper(c->s_rec, a));
    }
    il_free(&ml);
    return ks_val(&sr) + c->pref * ks_val(&rr) - c->self;
}

/* Regular part of the m* = 0 reciprocal term as a power series in rho = |k|^2:
 * returns coefficients r[0..J] with  C' rho^{-s} Gamma(s, alpha rho) - s_hat/V
 *   = sum_j r[j] rho^j,  alpha = pi lam^2, s = (d-nu)/2, C' = pref.
 * non-log (s not in -N0):  -C' alpha^s sum_j (-1)^j alpha^j rho^j / (j! (s+j))
 * log (s = -m): from DLMF 8.4.15 and the series of E1 (DLMF 6.6.2),
 *   C' [ (-1)^{m+1}/m! rho^m ln lam^2
 *      + alpha^{-m} (-1)^m/m! ( a^m(-gamma - sum_{j>=1} (-a)^j/(j j!))
 *                               - e^{-a} sum_{i<m} (-1)^i i! a^{m-i-1} ) ],  a = alpha rho */
static void m0_reg_series(double s, double pref, double lam, int J, double *r) {
    const double alpha = EZO_PI * lam * lam;
    for (int j = 0; j <= J; ++j) r[j] = 0.0;
    if (s <= 0.0 && s == floor(s)) {
        int m = (int)(-s);
        double sg_m = (m % 2) ? -1.0 : 1.0;
        double mf = factorial(m);
        /* (-1)^{m+1}/m! rho^m ln lam^2 */
        if (m <= J) r[m] += -sg_m / mf * log(lam * lam);
        /* alpha^{-m}(-1)^m/m! * a^m * (-gamma) = (-1)^m/m! (-gamma) rho^m */
        if (m <= J) r[m] += sg_m / mf * (-EZO_EULER);
        /* - alpha^{-m}(-1)^m/m! a^m sum_{j>=1} (-a)^j/(j j!)  -> rho^{m+j} */
        for (int j = 1; m + j <= J; ++j) {
            double c = ((j % 2) ? -1.0 : 1.0) * pow(alpha, (double)j) / ((double)j * factorial(j));
            r[m + j] += -sg_m / mf * c;
        }
        /* - alpha^{-m}(-1)^m/m! e^{-a} sum_{i<m} (-1)^i i! a^{m-i-1} */
        for (int i = 0; i < m; ++i) {
            double ci = ((i % 2) ? -1.0 : 1.0) * factorial(i) * pow(alpha, (double)(m - i - 1));
            for (int rr = 0; m - i - 1 + rr <= J; ++rr) {
                double er = ((rr % 2) ? -1.0 : 1.0) * pow(alpha, (double)rr) / factorial(rr);
                r[m - i - 1 + rr] += -pow(alpha, -(double)m) * sg_m / mf * ci * er;
            }
        }
    } else {
        for (int j = 0; j <= J; ++j)
            r[j] = -pow(alpha, s) * ((j % 2) ? -1.0 : 1.0) * pow(alpha, (double)j) /
                   (factorial(j) * (s + j));
    }
    for (int j = 0; j <= J; ++j) r[j] *= pref;
}

/* Z^reg_{Lambda,nu}(k) = Z(0,k) - s_hat(k)/V, valid also at k = 0 */
int ezo_epstein_reg(int d, const double *A, double nu, const double *k_in, double lam_rel,
                    double a_cut, double *out) {
    lat_t L;
    int st = lat_init(&L, d, A, lam_rel, a_cut);
    if (st) return st;
    nuctx_t c;
    if ((st = nuctx_init(&c, &L, nu))) return st;
    double k[3] = {0, 0, 0};
    for (int i = 0; i < d; ++i) k[i] = k_in[i];
    const double lam2 = L.lam * L.lam;
    ksum_t sr = {0, 0};
    for (int t = 0; t < c.nz; ++t) ks_add(&sr, c.W[t] * cos(2.0 * EZO_PI * dot(d, k, &c.z[3 * t])));
    ksum_t rr = {0, 0};
    ilist_t ml = {0, 0, NULL};
    double Rk = sqrt(L.a_cut / EZO_PI) / L.lam;
    double kneg[3] = {-k[0], -k[1], -k[2]};
    if (enum_ball(d, L.B, L.Binv, kneg, Rk, &ml)) { nuctx_free(&c); return EZO_ENOMEM; }
    for (int t = 0; t < ml.n; ++t) {
        int *m = &ml.p[3 * t];
        if (m[0] == 0 && m[1] == 0 && m[2] == 0) continue;
        double md[3] = {m[0], m[1], m[2]}, q[3];
        matvec(d, L.B, md, q);
        for (int i = 0; i < d; ++i) q[i] += k[i];
        double q2 = dot(d, q, q);
        double a = EZO_PI * lam2 * q2;
        if (a > L.a_cut) continue;
        ks_add(&rr, pow(q2, -c.s_rec) * ezo_gamma_upper(c.s_rec, a));
    }
    il_free(&ml);
    /* m* = 0: regular series, summed to convergence */
    double r[80];
    m0_reg_series(c.s_rec, c.pref, L.lam, 79, r);
    double k2 = dot(d, k, k);
    ksum_t s0 = {0, 0};
    double p = 1.0;
    for (int j = 0; j < 80; ++j) { ks_add(&s0, r[j] * p); p *= k2; }
    *out = ks_val(&sr) + c.pref * ks_val(&rr) + ks_val(&s0) - c.self;
    nuctx_free(&c);
    return EZO_OK;
}

/* ------------------------------------------------------------------------ */
/* Taylor coefficients of Z^reg at the origin (Sec. 3, meromorphic           */
/* continuation): all partial derivatives  nabla^alpha Z^reg(0), |alpha|<=2l, */
/* then the directional derivatives by the multinomial formula               */
/*   C_{k,nu}(w) = 1/(2k)! sum_{|alpha|=2k} (2k)!/alpha! w^alpha nabla^alpha Z^reg(0). */
/* Polynomials in k are held densely by exponent triple.                     */
/* ------------------------------------------------------------------------ */
#define PDEG 13
#define PIDX(i, j, l) (((i) * PDEG + (j)) * PDEG + (l))
typedef struct { double c[PDEG * PDEG * PDEG]; } poly_t;

static void poly_zero(poly_t *p) { memset(p->c, 0, sizeof(p->c)); }
static void poly_mul(const poly_t *a, const poly_t *b, poly_t *out, int maxdeg) {
    poly_t r; poly_zero(&r);
    for (int i = 0; i <= maxdeg; ++i)
        for (int j = 0; i + j <= maxdeg; ++j)
            for (int l = 0; i + j + l <= maxdeg; ++l) {
                double av = a->c[PIDX(i, j, l)];
                if (av == 0.0) continue;
                for (int i2 = 0; i + j + l + i2 <= maxdeg; ++i2)
                    for (int j2 = 0; i + j + l + i2 + j2 <= maxdeg; ++j2)
                        for (int l2 = 0; i + j + l + i2 + j2 + l2 <= maxdeg; ++l2) {
                            double bv = b->c[PIDX(i2, j2, l2)];
                            if (bv != 0.0) r.c[PIDX(i + i2, j + j2, l + l2)] += av * bv;
                        }
            }
    *out = r;
}

/* Taylor polynomial t(k) = sum_alpha D_alpha k^alpha / alpha!  of Z^reg_nu at 0 */
static int reg_taylor_poly(const lat_t *L, const nuctx_t *c, int maxdeg, poly_t *T) {
    const int d = L->d;
    const double lam2 = L->lam * L->lam;
    const double alpha = EZO_PI * lam2;
    poly_zero(T);
    /* real space: sum_z W(z) cos(2 pi k.z) = sum_z W sum_j (-1)^j (2pi)^{2j} (k.z)^{2j}/(2j)!
       coefficient of k^alpha (|alpha| = 2j): (-1)^j (2pi)^{2j} z^alpha / alpha!          */
    for (int t = 0; t < c->nz; ++t) {
        const double *z = &c->z[3 * t];
        for (int i = 0; i <= maxdeg; ++i)
            for (int j = 0; i + j <= maxdeg; ++j)
                for (int l = 0; i + j + l <= maxdeg; ++l) {
                    int deg = i + j + l;
                    if (deg % 2) continue;
                    if ((d < 2 && j) || (d < 3 && l)) continue;
                    double zp = pow(z[0], i) * (d > 1 ? pow(z[1], j) : 1.0) * (d > 2 ? pow(z[2], l) : 1.0);
                    double sg = ((deg / 2) % 2) ? -1.0 : 1.0;
                    T->c[PIDX(i, j, l)] += c->W[t] * sg * pow(2.0 * EZO_PI, deg) * zp /
                                          (factorial(i) * factorial(j) * factorial(l));
                }
    }
    /* reciprocal space, m* != 0:  F(|m*+k|^2) with F(rho) = C' rho^{-s} Gamma(s, alpha rho)
       F(rho0 + delta) = sum_n F^(n)(rho0) delta^n / n!,  delta = 2 m*.k + |k|^2,
       F^(n)(rho) = C' (-1)^n rho^{-(s+n)} Gamma(s+n, alpha rho)                         */
    ilist_t ml = {0, 0, NULL};
    double zero[3] = {0, 0, 0};
    double Rk = sqrt(L->a_cut / EZO_PI) / L->lam + 1.0 / L->lam;   /* margin for derivatives */
    if (enum_ball(d, L->B, L->Binv, zero, Rk, &ml)) return EZO_ENOMEM;
    poly_t *acc = (poly_t *)calloc(1, sizeof(poly_t));
    poly_t *delta = (poly_t *)calloc(1, sizeof(poly_t));
    poly_t *dn = (poly_t *)calloc(1, sizeof(poly_t));
    if (!acc || !delta || !dn) { free(acc); free(delta); free(dn); il_free(&ml); return EZO_ENOMEM; }
    for (int t = 0; t < ml.n; ++t) {
        int *m = &ml.p[3 * t];
        if (m[0] == 0 && m[1] == 0 && m[2] == 0) continue;
        double md[3] = {m[0], m[1], m[2]}, ms[3] = {0, 0, 0};
        matvec(d, L->B, md, ms);
        double rho0 = dot(d, ms, ms);
        poly_zero(delta);
        delta->c[PIDX(1, 0, 0)] = 2.0 * ms[0];
        if (d > 1) delta->c[PIDX(0, 1, 0)] = 2.0 * ms[1];
        if (d > 2) delta->c[PIDX(0, 0, 1)] = 2.0 * ms[2];
        delta->c[PIDX(2, 0, 0)] = 1.0;
        if (d > 1) delta->c[PIDX(0, 2, 0)] = 1.0;
        if (d > 2) delta->c[PIDX(0, 0, 2)] = 1.0;
        poly_zero(dn);
        dn->c[PIDX(0, 0, 0)] = 1.0;        /* delta^0 */
        poly_zero(acc);
        for (int n = 0; n <= maxdeg; ++n) {
            if (n > 0) poly_mul(dn, delta, dn, maxdeg);
            double Fn = ((n % 2) ? -1.0 : 1.0) * pow(rho0, -(c->s_rec + n)) *
                        ezo_gamma_upper(c->s_rec + n, alpha * rho0) / factorial(n);
            for (int i = 0; i < PDEG * PDEG * PDEG; ++i) acc->c[i] += Fn * dn->c[i];
        }
        for (int i = 0; i < PDEG * PDEG * PDEG; ++i) T->c[i] += c->pref * acc->c[i];
    }
    il_free(&ml);
    /* m* = 0 regular series: sum_j r_j |k|^{2j} */
    double r[PDEG];
    m0_reg_series(c->s_rec, c->pref, L->lam, maxdeg / 2, r);
    poly_t *k2 = acc;
    poly_zero(k2);
    k2->c[PIDX(2, 0, 0)] = 1.0;
    if (d > 1) k2->c[PIDX(0, 2, 0)] = 1.0;
    if (d > 2) k2->c[PIDX(0, 0, 2)] = 1.0;
    poly_zero(dn);
    dn->c[PIDX(0, 0, 0)] = 1.0;
    for (int j = 0; 2 * j <= maxdeg; ++j) {
        if (j > 0) poly_mul(dn, k2, dn, maxdeg);
        for (int i = 0; i < PDEG * PDEG * PDEG; ++i) T->c[i] += r[j] * dn->c[i];
    }
    /* self term */
    T->c[PIDX(0, 0, 0)] -= c->self;
    free(acc); free(delta); free(dn);
    return EZO_OK;
}

/* C_{k,nu}(w), k = 0..ell, from the derivative tensor via the multinomial formula */
static void directional_coeffs(int d, const poly_t *T, int ell, const double *w, double *C) {
    for (int k = 0; k <= ell; ++k) {
        int deg = 2 * k;
        double s = 0.0;
        for (int i = 0; i <= deg; ++i)
            for (int j = 0; i + j <= deg; ++j) {
                int l = deg - i - j;
                if ((d < 2 && j) || (d < 3 && l)) continue;
                double fi = factorial(i), fj = factorial(j), fl = factorial(l);
                /* nabla^alpha Z^reg(0) = alpha! * t_alpha */
                double D = T->c[PIDX(i, j, l)] * fi * fj * fl;
                double multinom = factorial(deg) / (fi * fj * fl);
                double wa = pow(w[0], i) * (d > 1 ? pow(w[1], j) : 1.0) * (d > 2 ? pow(w[2], l) : 1.0);
                s += multinom * wa * D;
            }
        C[k] = s / factorial(deg);
    }
}

int ezo_reg_taylor(int d, const double *A, double nu, const double *w, int ell, double lam_rel,
                   double a_cut, double *C) {
    if (ell < 0 || 2 * ell >= PDEG) return EZO_EINVAL;
    lat_t L;
    int st = lat_init(&L, d, A, lam_rel, a_cut);
    if (st) return st;
    nuctx_t c;
    if ((st = nuctx_init(&c, &L, nu))) return st;
    poly_t *T = (poly_t *)calloc(1, sizeof(poly_t));
    if (!T) { nuctx_free(&c); return EZO_ENOMEM; }
    st = reg_taylor_poly(&L, &c, 2 * ell, T);
    if (!st) directional_coeffs(d, T, ell, w, C);
    free(T);
    nuctx_free(&c);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Hadamard integrals on (0, eps)  (Sec. 3, closed forms for q = 0..3)        */
/*   I_q(mu) = fp int_0^eps u^{mu-1} L(u)^q du,  L(u) = log(pi u^2 |w|^2)   */
/*   I_0 = eps^mu / mu ;  I_q = eps^mu L(eps)^q / mu - (2q/mu) I_{q-1}       */
/* (integration by parts, dL/du = 2/u), meromorphic in mu, pole at mu = 0.   */
/* ------------------------------------------------------------------------ */
int ezo_hadamard_I(double mu, int q, double eps, double Leps, double *out) {
    if (mu == 0.0) return EZO_EUNSUPPORTED;
    double em = pow(eps, mu);
    double I = em / mu;
    for (int j = 1; j <= q; ++j) I = em * pow(Leps, j) / mu - (2.0 * j / mu) * I;
    *out = I;
    return EZO_OK;
}

/* ------------------------------------------------------------------------ */
/* n-body zeta by the Epstein representation and the Duffy transform.       */
/*                                                                          */
/*  zeta^(n)(nu) = 2 sum_{p in {+-1}^{d-1}} sum_{j=0}^{d-1} int_0^{1/2} u^{d-1}*/
/*                 int_{[0,1]^{d-1}} f(u w(v)) dv du,                        */
/*  w(v) = A^{-T} sigma^j (p1 v1, ..., p_{d-1} v_{d-1}, 1),  f = prod Z_nu_i. */
/* v: n_q-point Gauss-Legendre per dimension.  u: (0,eps) analytically by    */
/* the Taylor expansion of Z^reg and Hadamard integrals; (eps,1/2] by        */
/* n_panels geometric panels, n_g Gauss-Legendre points each.               */
/*                                                                          */
/* Direction numbering: dir = block * n_q^{d-1} + iv,  block = j 2^{d-1} + ip,*/
/* bit b of ip set <=> p_{b+1} = -1;  iv = sum_b iv_b n_q^b.                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n_q, n_panels, n_g, ell;
    double eps, lam_rel, a_cut;
} ezo_spec_t;

typedef struct { double coef, P; int q; } term_t;

static int nb_prepare(const lat_t *L, int n, const double *nu, nuctx_t **ctx_out, poly_t **T_out,
                      int *uniq_idx, int ell) {
    nuctx_t *ctx = (nuctx_t *)calloc((size_t)n, sizeof(nuctx_t));
    poly_t *T = (poly_t *)calloc((size_t)n, sizeof(poly_t));
    if (!ctx || !T) { free(ctx); free(T); return EZO_ENOMEM; }
    for (int i = 0; i < n; ++i) {
        uniq_idx[i] = i;
        for (int j = 0; j < i; ++j)
            if (nu[j] == nu[i]) { uniq_idx[i] = j; break; }
        if (uniq_idx[i] != i) continue;
        int st = nuctx_init(&ctx[i], L, nu[i]);
        if (!st) st = reg_taylor_poly(L, &ctx[i], 2 * ell, &T[i]);
        if (st) {
            for (int j = 0; j <= i; ++j) if (uniq_idx[j] == j) nuctx_free(&ctx[j]);
            free(ctx); free(T);
            return st;
        }
    }
    *ctx_out = ctx;
    *T_out = T;
    return EZO_OK;
}

/* value of one direction: Hadamard part on (0,eps) + panels on (eps,1/2] (without the
   factor 2 prod w_v) ; also returns both parts separately */
static int nb_direction(const lat_t *L, int n, const double *nu, const nuctx_t *ctx, const poly_t *T,
                        const int *uq, const ezo_spec_t *sp, const double *w,
                        const double *ux, const double *uw, int nu_nodes, double *had, double *num) {
    const int d = L->d;
    const int ell = sp->ell;
    double w2 = dot(d, w, w);
    /* --- (0, eps): product of (singular + Taylor) factors, term by term --- */
    /* Terms with equal (P, q) are merged, so the list never holds more than the
       number of distinct pairs: the sums of the singular exponents take at most
       prod over distinct nu of (count + 1) values, the Taylor degree 2K at most
       n ell + 1 values and q at most n + 1; nor more than (ell + 2)^n.  (Counted
       in double: the product overflows an int for large n.) */
    double unmerged = 1.0, merged = (double)(n * ell + 1) * (double)(n + 1);
    for (int i = 0; i < n; ++i) {
        unmerged = fmin(unmerged * (ell + 2), 1e18);
        int first = 1, count = 0;
        for (int j = 0; j < n; ++j) {
            if (nu[j] == nu[i]) {
                if (j < i) first = 0;
                ++count;
            }
        }
        if (first) merged *= (double)(count + 1);
    }
    const double bound = fmin(unmerged, merged);
    if (bound > 4000000.0) return EZO_EUNSUPPORTED;
    const int maxterms = (int)bound;
    term_t *cur = (term_t *)malloc(sizeof(term_t) * (size_t)maxterms);
    term_t *nxt = (term_t *)malloc(sizeof(term_t) * (size_t)maxterms);
    if (!cur || !nxt) { free(cur); free(nxt); return EZO_ENOMEM; }
    int ncur = 1;
    cur[0].coef = 1.0; cur[0].P = 0.0; cur[0].q = 0;
    double Ck[PDEG];
    for (int i = 0; i < n; ++i) {
        double sigma, e; int delta;
        sing_coef(d, L->V, nu[i], w2, &sigma, &e, &delta);
        directional_coeffs(d, &T[uq[i]], ell, w, Ck);
        int nn = 0;
        for (int t = 0; t < ncur; ++t) {
            /* singular part */
            term_t s = cur[t];
            s.coef *= sigma; s.P += e; s.q += delta;
            /* merge equal (P,q) */
            int found = -1;
            for (int u = 0; u < nn; ++u)
                if (nxt[u].q == s.q && fabs(nxt[u].P - s.P) < 1e-9) { found = u; break; }
            if (found >= 0) nxt[found].coef += s.coef; else nxt[nn++] = s;
            for (int k = 0; k <= ell; ++k) {
                term_t r = cur[t];
                r.coef *= Ck[k]; r.P += 2.0 * k;
                found = -1;
                for (int u = 0; u < nn; ++u)
                    if (nxt[u].q == r.q && fabs(nxt[u].P - r.P) < 1e-9) { found = u; break; }
                if (found >= 0) nxt[found].coef += r.coef; else nxt[nn++] = r;
            }
        }
        term_t *tmp = cur; cur = nxt; nxt = tmp;
        ncur = nn;
    }
    double Leps = log(EZO_PI * sp->eps * sp->eps * w2);
    ksum_t hs = {0, 0};
    int st = EZO_OK;
    for (int t = 0; t < ncur; ++t) {
        double I;
        double mu = (double)d + cur[t].P;
        if (fabs(mu) < 1e-12) { st = EZO_EUNSUPPORTED; break; }
        ezo_hadamard_I(mu, cur[t].q, sp->eps, Leps, &I);
        ks_add(&hs, cur[t].coef * I);
    }
    free(cur); free(nxt);
    if (st) return st;
    *had = ks_val(&hs);
    /* --- (eps, 1/2]: Gauss panels --- */
    ksum_t ns = {0, 0};
    double Zv[64];
    for (int a = 0; a < nu_nodes; ++a) {
        double k[3] = {0, 0, 0};
        for (int i = 0; i < d; ++i) k[i] = ux[a] * w[i];
        double f = 1.0;
        for (int i = 0; i < n; ++i) {
            if (uq[i] == i) {
                int err = 0;
                Zv[i] = z0_full(L, &ctx[i], k, &err);
                if (err) return err;
            } else {
                Zv[i] = Zv[uq[i]];
            }
            f *= Zv[i];
        }
        ks_add(&ns, uw[a] * pow(ux[a], d - 1) * f);
    }
    *num = ks_val(&ns);
    return EZO_OK;
}

static void direction_of(int d, int n_q, const double *vx, const double *vw, int dir,
                         const double *B, double *w, double *wv) {
    int nv = 1;
    for (int i = 0; i < d - 1; ++i) nv *= n_q;
    int block = dir / nv, iv = dir % nv;
    int np = 1 << (d - 1);
    int j = block / np, ip = block % np;
    double wh[3] = {0, 0, 0}, x[3] = {0, 0, 0};
    double weight = 1.0;
    int rem = iv;
    for (int b = 0; b < d - 1; ++b) {
        int ib = rem % n_q; rem /= n_q;
        double p = ((ip >> b) & 1) ? -1.0 : 1.0;
        x[b] = p * vx[ib];
        weight *= vw[ib];
    }
    x[d - 1] = 1.0;
    /* sigma^j: (sigma x)_i = x_{i-1 mod d} */
    for (int i = 0; i < d; ++i) wh[i] = x[((i - j) % d + d) % d];
    matvec(d, B, wh, w);
    *wv = weight;
}

int ezo_nbody_dirs(int d, const double *A, int n, const double *nu, int n_q, int n_panels, int n_g,
                   int ell, double eps, double lam_rel, double a_cut, int dir_lo, int dir_hi,
                   double *dir_had, double *dir_num, double *dir_weight) {
    if (n < 1 || n > 60 || n_q < 1 || n_panels < 1 || n_g < 1 || ell < 0 || 2 * ell >= PDEG ||
        !(eps > 0.0 && eps < 0.5))
        return EZO_EINVAL;
    for (int i = 0; i < n; ++i) if (!isfinite(nu[i])) return EZO_EINVAL;
    lat_t L;
    int st = lat_init(&L, d, A, lam_rel, a_cut);
    if (st) return st;
    ezo_spec_t sp = {n_q, n_panels, n_g, ell, eps, lam_rel, a_cut};
    int nv = 1;
    for (int i = 0; i < d - 1; ++i) nv *= n_q;
    int ndir = d * (1 << (d - 1)) * nv;
    if (dir_lo < 0) dir_lo = 0;
    if (dir_hi < 0 || dir_hi > ndir) dir_hi = ndir;
    double vx[64], vw[64];
    if (n_q > 64) return EZO_EINVAL;
    ezo_gauss_legendre(n_q, 0.0, 1.0, vx, vw);
    int nu_nodes = n_panels * n_g;
    double *ux = (double *)malloc(sizeof(double) * nu_nodes);
    double *uw = (double *)malloc(sizeof(double) * nu_nodes);
    double *gx = (double *)malloc(sizeof(double) * n_g);
    double *gw = (double *)malloc(sizeof(double) * n_g);
    if (!ux || !uw || !gx || !gw) { free(ux); free(uw); free(gx); free(gw); return EZO_ENOMEM; }
    double ratio = pow(0.5 / eps, 1.0 / n_panels);
    for (int pnl = 0; pnl < n_panels; ++pnl) {
        double lo = eps * pow(ratio, pnl);
        double hi = (pnl == n_panels - 1) ? 0.5 : eps * pow(ratio, pnl + 1);
        ezo_gauss_legendre(n_g, lo, hi, gx, gw);
        for (int g = 0; g < n_g; ++g) { ux[pnl * n_g + g] = gx[g]; uw[pnl * n_g + g] = gw[g]; }
    }
    free(gx); free(gw);
    nuctx_t *ctx = NULL; poly_t *T = NULL;
    int uq[64];
    if (n > 64) { free(ux); free(uw); return EZO_EINVAL; }
    if ((st = nb_prepare(&L, n, nu, &ctx, &T, uq, ell))) { free(ux); free(uw); return st; }
    int err = EZO_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (int dir = dir_lo; dir < dir_hi; ++dir) {
        double w[3] = {0, 0, 0}, wv;
        direction_of(d, n_q, vx, vw, dir, L.B, w, &wv);
        double h = 0.0, nm = 0.0;
        int e = nb_direction(&L, n, nu, ctx, T, uq, &sp, w, ux, uw, nu_nodes, &h, &nm);
        if (e) {
#pragma omp critical
            err = e;
        }
        dir_had[dir - dir_lo] = h;
        dir_num[dir - dir_lo] = nm;
        dir_weight[dir - dir_lo] = 2.0 * wv;
    }
    for (int i = 0; i < n; ++i) if (uq[i] == i) nuctx_free(&ctx[i]);
    free(ctx); free(T); free(ux); free(uw);
    return err;
}

int ezo_nbody(int d, const double *A, int n, const double *nu, int n_q, int n_panels, int n_g,
              int ell, double eps, double lam_rel, double a_cut, double *out, double *parts) {
    if (n_q < 1 || n_q > 64 || d < 1 || d > 3) return EZO_EINVAL;
    int nv = 1;
    for (int i = 0; i < d - 1; ++i) nv *= n_q;
    int ndir = d * (1 << (d - 1)) * nv;
    double *h = (double *)malloc(sizeof(double) * ndir);
    double *m = (double *)malloc(sizeof(double) * ndir);
    double *w = (double *)malloc(sizeof(double) * ndir);
    if (!h || !m || !w) { free(h); free(m); free(w); return EZO_ENOMEM; }
    int st = ezo_nbody_dirs(d, A, n, nu, n_q, n_panels, n_g, ell, eps, lam_rel, a_cut, 0, ndir, h, m, w);
    if (!st) {
        ksum_t sh = {0, 0}, sn = {0, 0};
        for (int i = 0; i < ndir; ++i) { ks_add(&sh, w[i] * h[i]); ks_add(&sn, w[i] * m[i]); }
        if (parts) { parts[0] = ks_val(&sn); parts[1] = ks_val(&sh); }
        ksum_t t = {0, 0};
        ks_add(&t, ks_val(&sn)); ks_add(&t, ks_val(&sh));
        *out = ks_val(&t);
    }
    free(h); free(m); free(w);
    return st;
}

/* ATM cohesive energy per particle (Sec. 2, Proposition):
 *   E = 1/24 zeta(3,3,3) - 3/16 zeta(-1,5,5) + 3/8 zeta(1,3,5)              */
int ezo_atm(int d, const double *A, int n_q, int n_panels, int n_g, int ell, double eps,
            double lam_rel, double a_cut, double *out, double *zetas) {
    const double nus[3][3] = {{3, 3, 3}, {-1, 5, 5}, {1, 3, 5}};
    const double c[3] = {1.0 / 24.0, -3.0 / 16.0, 3.0 / 8.0};
    double z[3];
    for (int t = 0; t < 3; ++t) {
        int st = ezo_nbody(d, A, 3, nus[t], n_q, n_panels, n_g, ell, eps, lam_rel, a_cut, &z[t], NULL);
        if (st) return st;
    }
    if (zetas) for (int t = 0; t < 3; ++t) zetas[t] = z[t];
    ksum_t s = {0, 0};
    for (int t = 0; t < 3; ++t) ks_add(&s, c[t] * z[t]);
    *out = ks_val(&s);
    return EZO_OK;
}

/* ------------------------------------------------------------------------ */
/* Direct truncated sums over the box A{-L..L}^d (Sec. 2, Definitions),     */
/* primed: every summand with some |.|^-nu evaluated at 0 is dropped.        */
/* ------------------------------------------------------------------------ */
typedef struct { int d, np; double *z; } box_t;

static int box_init(box_t *b, int d, const double *A, int L) {
    b->d = d;
    int side = 2 * L + 1;
    int np = side;
    for (int i = 1; i < d; ++i) np *= side;
    b->np = np;
    b->z = (double *)malloc(sizeof(double) * 3 * (size_t)np);
    if (!b->z) return EZO_ENOMEM;
    for (int t = 0; t < np; ++t) {
        int rem = t;
        double nd[3] = {0, 0, 0}, z[3] = {0, 0, 0};
        for (int i = 0; i < d; ++i) { nd[i] = (double)(rem % side - L); rem /= side; }
        matvec(d, A, nd, z);
        for (int i = 0; i < 3; ++i) b->z[3 * t + i] = z[i];
    }
    return EZO_OK;
}

static double dist2(const double *a, const double *b) {
    double s = 0.0;
    for (int i = 0; i < 3; ++i) s += (a[i] - b[i]) * (a[i] - b[i]);
    return s;
}

/* recursive chain x^(1..n-1), closing back to x^(0) = x^(n) = 0 */
static void chain_rec(const box_t *b, int n, const double *nu, int level, const double *prev,
                      double prod, ksum_t *acc) {
    const double zero[3] = {0, 0, 0};
    if (level == n) {                       /* closing edge |x^(n) - x^(n-1)| */
        double r2 = dist2(zero, prev);
        if (r2 == 0.0) return;
        ks_add(acc, prod * pow(r2, -0.5 * nu[n - 1]));
        return;
    }
    for (int t = 0; t < b->np; ++t) {
        const double *x = &b->z[3 * t];
        double r2 = dist2(x, prev);
        if (r2 == 0.0) continue;
        chain_rec(b, n, nu, level + 1, x, prod * pow(r2, -0.5 * nu[level - 1]), acc);
    }
}

int ezo_direct_nbody(int d, const double *A, int n, const double *nu, int L, double *out) {
    if (d < 1 || d > 3 || n < 2 || n > 8 || L < 1) return EZO_EINVAL;
    box_t b;
    if (box_init(&b, d, A, L)) return EZO_ENOMEM;
    const double zero[3] = {0, 0, 0};
    ksum_t acc = {0, 0};
    if (n == 3) {
        /* the common case, written as an explicit double loop */
        int np = b.np;
        double *r2o = (double *)malloc(sizeof(double) * np);
        if (!r2o) { free(b.z); return EZO_ENOMEM; }
        for (int t = 0; t < np; ++t) r2o[t] = dist2(&b.z[3 * t], zero);
        ksum_t *part = (ksum_t *)calloc((size_t)np, sizeof(ksum_t));
        if (!part) { free(r2o); free(b.z); return EZO_ENOMEM; }
#pragma omp parallel for schedule(dynamic, 16)
        for (int i = 0; i < np; ++i) {
            if (r2o[i] == 0.0) continue;
            double f1 = pow(r2o[i], -0.5 * nu[0]);
            ksum_t s = {0, 0};
            for (int j = 0; j < np; ++j) {
                if (r2o[j] == 0.0 || j == i) continue;
                double r12 = dist2(&b.z[3 * i], &b.z[3 * j]);
                ks_add(&s, f1 * pow(r12, -0.5 * nu[1]) * pow(r2o[j], -0.5 * nu[2]));
            }
            part[i] = s;
        }
        for (int i = 0; i < np; ++i) { ks_add(&acc, part[i].s); ks_add(&acc, part[i].c); }
        free(part); free(r2o);
    } else {
        chain_rec(&b, n, nu, 1, zero, 1.0, &acc);
    }
    free(b.z);
    *out = ks_val(&acc);
    return EZO_OK;
}

/* ATM potential (Sec. 2, Definition):
 *   U(x,y) = |x|^-3|y|^-3|z|^-3 - 3 (x.y)(y.z)(z.x) / (|x||y||z|)^5,  z = y - x;
 *   E = 1/6 sum'_{x,y} U(x,y)                                              */
int ezo_direct_atm(int d, const double *A, int L, double *out) {
    if (d < 1 || d > 3 || L < 1) return EZO_EINVAL;
    box_t b;
    if (box_init(&b, d, A, L)) return EZO_ENOMEM;
    int np = b.np;
    const double zero[3] = {0, 0, 0};
    ksum_t *part = (ksum_t *)calloc((size_t)np, sizeof(ksum_t));
    if (!part) { free(b.z); return EZO_ENOMEM; }
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < np; ++i) {
        const double *x = &b.z[3 * i];
        double xx = dist2(x, zero);
        if (xx == 0.0) continue;
        ksum_t s = {0, 0};
        for (int j = 0; j < np; ++j) {
            const double *y = &b.z[3 * j];
            double yy = dist2(y, zero);
            if (yy == 0.0 || j == i) continue;
            double z[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
            double zz = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
            double xy = x[0] * y[0] + x[1] * y[1] + x[2] * y[2];
            double yz = y[0] * z[0] + y[1] * z[1] + y[2] * z[2];
            double zx = z[0] * x[0] + z[1] * x[1] + z[2] * x[2];
            double r = sqrt(xx * yy * zz);
            double U = 1.0 / (r * r * r) - 3.0 * xy * yz * zx / (r * r * r * r * r);
            ks_add(&s, U);
        }
        part[i] = s;
    }
    ksum_t acc = {0, 0};
    for (int i = 0; i < np; ++i) { ks_add(&acc, part[i].s); ks_add(&acc, part[i].c); }
    free(part);
    free(b.z);
    *out = ks_val(&acc) / 6.0;
    return EZO_OK;
}

int ezo_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the parallel loops (timing of the oracle as a CPU baseline only) */
void ezo_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
