// ez_quad.hip -- quadrature of products of Epstein zeta functions over the
// Brillouin zone (paper, Sec. 2, Theorem (Epstein representation); Sec. 3,
// Corollary (Duffy transformation) and the meromorphic continuation).
//
//   zeta = 2 sum_{p,j} int_0^{1/2} u^{d-1} int_{[0,1]^{d-1}} f(u w(v)) dv du,
//   w(v) = A^{-T} sigma^j (p1 v1, ..., p_{d-1} v_{d-1}, 1).
//
// ez_node_kernel   : u in (eps, 1/2].  One thread per node k = u w: Z_nu(k) for
//                    the exponent set by the split (real-space table + reciprocal
//                    table), the products of the terms, weight, then a
//                    double-double reduction to one partial per 256-node tile.
// ez_hadamard_kernel: u in (0, eps).  One lane per direction w (64 per workgroup, the
//                    tables split over 4 waves): Taylor
//                    coefficients of Z^reg_nu(u w) in u, expansion of the products
//                    of (singular + Taylor) factors and closed-form Hadamard integrals.
// ez_finalize_kernel: fixed-order double-double sum of tiles and directions.
//
// Direction numbering: dir = block * n_q^{d-1} + iv, block = j 2^{d-1} + ip,
// bit b of ip set <=> p_{b+1} = -1, iv = sum_b iv_b n_q^b; node = dir * n_u + iu.
#include "ez_internal.h"
#include "ez_math.h"
#include "ez_kernels.h"

namespace {

constexpr int EZ_PDEG = 33;   // coefficients kept in the Taylor product polynomials (in u^2)

__device__ __forceinline__ int find_segment(const int *begin, int n, int x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int D>
__device__ __forceinline__ void ez_direction(const EzInstPlan &P, const double *rules, const double *B,
                                             int dir, double *w, double *wv, double *what = nullptr) {
    int nv = 1;
#pragma unroll
    for (int i = 0; i < D - 1; ++i) nv *= P.n_q;
    const int np = 1 << (D - 1);
    const int block = dir / nv;
    int iv = dir - block * nv;
    const int j = block / np, ip = block - j * np;
    double x[3] = {0.0, 0.0, 0.0};
    double weight = 1.0;
#pragma unroll
    for (int b = 0; b < D - 1; ++b) {
        int ib = iv % P.n_q;
        iv /= P.n_q;
        double v = rules[P.vrule + ib];
        weight *= rules[P.vrule + P.n_q + ib];
        x[b] = ((ip >> b) & 1) ? -v : v;
    }
    x[D - 1] = 1.0;
    double wh[3];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        int src = i - j;
        if (src < 0) src += D;
        wh[i] = (src == 0) ? x[0] : (src == 1 ? x[1] : x[2]);
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) s = fma(B[i * D + c], wh[c], s);
        w[i] = s;
        if (what) what[i] = wh[i];
    }
    *wv = weight;
}

// complex multiply (a r + i a i)(b r + i b i)
__device__ __forceinline__ void cmul(double &ar, double &ai, double br, double bi) {
    const double r = fma(ar, br, -ai * bi);
    const double i = fma(ar, bi, ai * br);
    ar = r;
    ai = i;
}

template <int SET>
__device__ __forceinline__ int pset_p2(const EzProgram &prog, int i) {
    if constexpr (SET == 0) return prog.p2[i];
    else return ez_pset(SET).p2[i];
}
template <int SET, int NNU>
__device__ __forceinline__ bool pset_need_e1(const EzProgram &prog) {
    if constexpr (SET == 0) return prog.need_e1 != 0;
    bool r = false;
    for (int i = 0; i < NNU; ++i) r = r || ((ez_pset(SET).p2[i] & 1) == 0 && ez_pset(SET).p2[i] >= 2);
    return r;
}
template <int SET, int NNU>
__device__ __forceinline__ bool pset_need_half(const EzProgram &prog) {
    if constexpr (SET == 0) return prog.need_half != 0;
    bool r = false;
    for (int i = 0; i < NNU; ++i) r = r || (ez_pset(SET).p2[i] & 1);
    return r;
}

template <int D, int NNU, int SET>
__global__ __launch_bounds__(EZ_TILE) void ez_node_kernel(EzQuadArgs args) {
    const int tile = blockIdx.x;
    const int inst = find_segment(args.tile_begin, args.batch, tile);
    const EzInstPlan P = args.plans[inst];
    const EzLatMeta *M = args.meta + inst;
    const int n_res = args.prog.n_res;
    const int node = (tile - args.tile_begin[inst]) * EZ_TILE + threadIdx.x;
    const int n_nodes = P.n_dir * P.n_u;

    double res[EZ_RES_MAX];
#pragma unroll
    for (int r = 0; r < EZ_RES_MAX; ++r) res[r] = 0.0;

    if (M->status == 0 && node < n_nodes) {
        const int dir = node / P.n_u;
        const int iu = node - dir * P.n_u;
        double B[D * D];
#pragma unroll
        for (int i = 0; i < D * D; ++i) B[i] = M->B[i];
        double w[3] = {0.0, 0.0, 0.0}, wh[3] = {0.0, 0.0, 0.0}, wv;
        ez_direction<D>(P, args.rules, B, dir, w, &wv, wh);
        const double u = args.rules[P.urule + iu];
        const double wu = args.rules[P.urule + P.n_u + iu];
        double k[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < D; ++i) k[i] = u * w[i];
        double W = 2.0 * wv * wu;
#pragma unroll
        for (int i = 0; i < D - 1; ++i) W *= u;

        double accr[NNU], acck[NNU];
#pragma unroll
        for (int i = 0; i < NNU; ++i) { accr[i] = 0.0; acck[i] = 0.0; }

        // real space: sum over pairs of 2 W_nu(z) Re e^{2 pi i k.z}, k.z = theta.n with
        // theta = A^T k = u w_hat.  Row by row (n2, n3 fixed, consecutive n1) the phase
        // advances by c1 = e^{2 pi i theta_1}; from row to row within a plane by
        // c2^{dn2} c1^{dn1}; each plane starts from one sincos.
        {
            const int rs = args.tab.rstride;
            const double *rt = args.tab.real + (size_t)inst * args.tab.real_cap * rs;
            const int *rows = args.tab.rows + (size_t)inst * args.tab.row_cap * 8;
            const int n_rows = M->n_rows;
            double th[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < D; ++i) th[i] = u * wh[i];
            double c1r, c1i, c2r = 1.0, c2i = 0.0;
            ez_sincos2pi(th[0], &c1i, &c1r);
            if (D > 1) ez_sincos2pi(th[1], &c2i, &c2r);
            double br = 1.0, bi = 0.0;
            for (int r = 0; r < n_rows; ++r) {
                const int *R = rows + (size_t)r * 8;
                const int first = R[0], cnt = R[1];
                if (R[5]) {
                    double ph = th[0] * (double)R[2];
                    if (D > 1) ph = fma(th[1], (double)R[3], ph);
                    if (D > 2) ph = fma(th[2], (double)R[4], ph);
                    const double2 sc = ez_sincos2pi_ool(ph);
                    bi = sc.x;
                    br = sc.y;
                } else {
                    for (int j = 0; j < R[7]; ++j) cmul(br, bi, c2r, c2i);
                    const int dl = R[6];
                    if (dl > 0) for (int j = 0; j < dl; ++j) cmul(br, bi, c1r, c1i);
                    else for (int j = 0; j < -dl; ++j) cmul(br, bi, c1r, -c1i);
                }
                double pr = br, pi = bi;
                const double *e = rt + (size_t)first * rs;
                for (int j = 0; j < cnt; ++j, e += rs) {
#pragma unroll
                    for (int i = 0; i < NNU; ++i) accr[i] = fma(e[3 + i], pr, accr[i]);
                    cmul(pr, pi, c1r, c1i);
                }
            }
        }

        // reciprocal space: sum over m* of E_{p_nu}(pi lam^2 |m* + k|^2).  Entry 0 is
        // m* = 0, where a = alpha |k|^2 can be small (series of E1); every other entry
        // has a >= alpha / (4 |A|_F^2) >= 1/4 (the setup raises lam to ensure it), so the
        // main loop is one branch-free formula with E1 from the wide rational.
        const double *kt = args.tab.rec + (size_t)inst * args.tab.rec_cap * 4;
        const int n_rec = M->n_rec;
        const double alpha = M->alpha, acut = M->a_cut;
        const bool need_e1 = pset_need_e1<SET, NNU>(args.prog), need_half = pset_need_half<SET, NNU>(args.prog);
        {
            double rho = k[0] * k[0];
            if (D > 1) rho = fma(k[1], k[1], rho);
            if (D > 2) rho = fma(k[2], k[2], rho);
            const double a = alpha * rho;
            if (a <= acut) {
                const double ex = ez_expm(a);
                const double inv = ez_rcp(a);
                double E1 = 0.0;
                if (need_e1) E1 = (a < 0.25) ? ez_e1_series(a) : ex * ez_e1w_scaled(inv);
                const double Eh = need_half ? ez_ehalf(a) : 0.0;
#pragma unroll
                for (int i = 0; i < NNU; ++i)
                    acck[i] += ez_ep_from(pset_p2<SET>(args.prog, i), a, ex, inv, E1, Eh);
            }
        }
        for (int q = 1; q < n_rec; ++q) {
            const double *e = kt + (size_t)q * 4;
            double qx = e[0] + k[0];
            double rho = qx * qx;
            if (D > 1) { double qy = e[1] + k[1]; rho = fma(qy, qy, rho); }
            if (D > 2) { double qz = e[2] + k[2]; rho = fma(qz, qz, rho); }
            const double a = alpha * rho;
            if (a <= acut) {
                const double ex = ez_expm(a);
                const double inv = ez_rcp(a);
                const double E1 = need_e1 ? ex * ez_e1w_scaled(inv) : 0.0;
                const double Eh = need_half ? ez_ehalf(a) : 0.0;
#pragma unroll
                for (int i = 0; i < NNU; ++i)
                    acck[i] += ez_ep_from(pset_p2<SET>(args.prog, i), a, ex, inv, E1, Eh);
            }
        }

        double Z[NNU];
#pragma unroll
        for (int i = 0; i < NNU; ++i) Z[i] = accr[i] + M->K[i] * acck[i] - M->self_[i];

        for (int t = 0; t < args.prog.n_terms; ++t) {
            double prod = args.prog.term_coef[t];
            for (int f = 0; f < args.prog.term_nfac[t]; ++f) {
                const int fi = args.prog.term_fac[t][f];
                double z = Z[0];
#pragma unroll
                for (int i = 1; i < NNU; ++i) z = (fi == i) ? Z[i] : z;
                for (int m = 0; m < args.prog.term_mult[t][f]; ++m) prod *= z;
            }
            const int rr = args.prog.term_res[t];
#pragma unroll
            for (int r = 0; r < EZ_RES_MAX; ++r)
                if (rr == r) res[r] += prod;
        }
#pragma unroll
        for (int r = 0; r < EZ_RES_MAX; ++r) res[r] *= W;
    }

    // tile reduction: wave butterflies, then the four waves in fixed order
    __shared__ double red[EZ_RES_MAX][EZ_TILE / 64][2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < EZ_RES_MAX; ++r) {
        if (r < n_res) {
            ez_dd v = ez_dd_wave_sum(ez_dd{res[r], 0.0});
            if (lane == 0) { red[r][wave][0] = v.hi; red[r][wave][1] = v.lo; }
        }
    }
    __syncthreads();
    if (threadIdx.x < n_res) {
        const int r = threadIdx.x;
        ez_dd s{red[r][0][0], red[r][0][1]};
        for (int wv = 1; wv < EZ_TILE / 64; ++wv) s = ez_dd_add(s, ez_dd{red[r][wv][0], red[r][wv][1]});
        args.tile_part[((size_t)tile * n_res + r) * 2 + 0] = s.hi;
        args.tile_part[((size_t)tile * n_res + r) * 2 + 1] = s.lo;
    }
}

// ---------------------------------------------------------------------------
// Hadamard part on (0, eps)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double binom(int n, int k) {
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

__device__ __forceinline__ double fact(int n) {
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= (double)i;
    return r;
}

// fp int_0^eps u^{mu-1} L(u)^q du, L(u) = log(pi u^2 |w|^2); Leps = L(eps)
__device__ double had_I(double mu, int q, double eps, double Leps, bool *bad) {
    if (mu == 0.0) { *bad = true; return 0.0; }
    const double em = pow(eps, mu);
    const double rmu = 1.0 / mu;
    double I = em * rmu;
    double Lp = 1.0;
    for (int j = 1; j <= q; ++j) {
        Lp *= Leps;
        I = (em * Lp - 2.0 * (double)j * I) * rmu;
    }
    return I;
}

constexpr int EZ_HCH = 32;                      // m* per LDS chunk in the Hadamard kernel
constexpr int EZ_NF = 2 * EZ_ELL_MAX + 1;       // derivative orders 0..2 ell

// binomial coefficient as a compile-time constant after unrolling
__host__ __device__ constexpr double cbinom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return (k < 0 || k > n) ? 0.0 : r;
}

// ---------------------------------------------------------------------------
// Taylor coefficients C_k(w) of Z^reg_nu(u w) in u are homogeneous polynomials of
// degree 2k in the fractional direction w_hat (w = B w_hat).  They are evaluated
// directly at a fixed set of probe directions per lattice (ez_probe_kernel),
// the polynomial coefficients are recovered by a precomputed least-squares
// inverse, and every quadrature direction contracts them with its monomials
// (ez_hadamard_kernel): the paper's precomputed derivatives + multinomial
// directional derivatives, organised for the GPU.
// ---------------------------------------------------------------------------
constexpr int EZ_HW = 4;                        // waves per probe workgroup

// Partial C[i][k] at direction w over one slice of the tables: real-space pairs,
// reciprocal m* != 0, and (slice 0 only) the self term and the m* = 0 series.
// Lane = direction, the slice's entries split over EZ_HW waves, summed in LDS in
// fixed order; on return wave 0 holds the slice's coefficients.
template <int D, int NNU>
__device__ void taylor_coeffs(const EzQuadArgs &args, int inst, const EzLatMeta *M, int ell, const double *w,
                              double (&C)[NNU][EZ_ELL_MAX + 1], double *lds, int slice, int n_slice) {
    double (*fsh)[NNU][EZ_NF] = reinterpret_cast<double (*)[NNU][EZ_NF]>(lds);
    const EzProgram &prog = args.prog;
    const int lane = (int)threadIdx.x & 63, part = (int)threadIdx.x >> 6;
    double w2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) w2 = fma(w[i], w[i], w2);
    const double alpha = M->alpha;
    double pw2[EZ_ELL_MAX + 1];
    pw2[0] = 1.0;
#pragma unroll
    for (int j = 1; j <= EZ_ELL_MAX; ++j) pw2[j] = pw2[j - 1] * w2;
#pragma unroll
    for (int i = 0; i < NNU; ++i) {
#pragma unroll
        for (int k = 0; k <= EZ_ELL_MAX; ++k) C[i][k] = 0.0;
        if (part == 0 && slice == 0) C[i][0] = -M->self_[i];
    }
    // real space: 2 W cos(2 pi u w.z) = 2 W sum_k (-1)^k (2 pi w.z)^{2k} u^{2k} / (2k)!
    {
        const int rs = args.tab.rstride;
        const double *rt = args.tab.real + (size_t)inst * args.tab.real_cap * rs;
        const int n_real = M->n_real;
        for (int p = slice * EZ_HW + part; p < n_real; p += EZ_HW * n_slice) {
            const double *e = rt + (size_t)p * rs;
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) t = fma(w[i], e[i], t);
            const double x = (2.0 * EZ_PI * t) * (2.0 * EZ_PI * t);
            double term = 1.0;
#pragma unroll
            for (int k = 0; k <= EZ_ELL_MAX; ++k) {
                if (k <= ell) {
#pragma unroll
                    for (int i = 0; i < NNU; ++i) C[i][k] = fma(e[3 + i], term, C[i][k]);
                    term *= -x * (1.0 / ((2.0 * k + 1.0) * (2.0 * k + 2.0)));
                }
            }
        }
    }
    // reciprocal space, m* != 0: F(rho) = K E_p(alpha rho), rho(u) = |m*|^2 + 2 u b + u^2 w2, b = w.m*.
    // With F_n = F^(n)(|m*|^2)/n! = K (-alpha)^n E_{p-n}(alpha |m*|^2)/n!, the u^{2k} coefficient is
    //   sum_{n=k}^{2k} F_n C(n, 2k-n) (4 b^2)^{n-k} w2^{2k-n}.
    {
        const double *kt = args.tab.rec + (size_t)inst * args.tab.rec_cap * 4;
        const int n_rec = M->n_rec;
        for (int base = 1 + slice * EZ_HCH; base < n_rec; base += EZ_HCH * n_slice) {
            __syncthreads();
            // F_n for (entry, nu) pairs, one per thread
            for (int task = (int)threadIdx.x; task < EZ_HCH * NNU; task += 64 * EZ_HW) {
                const int te = task / NNU, i = task - te * NNU;
                const int q = base + te;
                if (q < n_rec) {
                    const double a0 = alpha * kt[(size_t)q * 4 + 3];
                    const double ex = exp(-a0), inv = ez_rcp(a0);
                    const int p2 = prog.p2[i];
                    const double E1 = ((p2 & 1) == 0) ? ez_e1(a0, ex, inv) : 0.0;
                    const double Eh = (p2 & 1) ? ez_ehalf(a0) : 0.0;
                    double E = ez_ep_from(p2, a0, ex, inv, E1, Eh);
                    double sc = M->K[i];
#pragma unroll
                    for (int n = 0; n < EZ_NF; ++n) {
                        if (n <= 2 * ell) {
                            fsh[te][i][n] = sc * E;
                            const double pnm1 = 0.5 * (double)p2 - (double)n - 1.0;
                            E = (ex - pnm1 * E) * inv;          // E_{p-n-1}
                            sc *= -alpha * (1.0 / (double)(n + 1));
                        }
                    }
                }
            }
            __syncthreads();
            const int cnt = min(EZ_HCH, n_rec - base);
            for (int t = part; t < cnt; t += EZ_HW) {
                const double *e = kt + (size_t)(base + t) * 4;
                double b = 0.0;
#pragma unroll
                for (int i = 0; i < D; ++i) b = fma(w[i], e[i], b);
                const double b4 = 4.0 * b * b;
                double pb[EZ_ELL_MAX + 1];
                pb[0] = 1.0;
#pragma unroll
                for (int j = 1; j <= EZ_ELL_MAX; ++j) pb[j] = pb[j - 1] * b4;
#pragma unroll
                for (int k = 0; k <= EZ_ELL_MAX; ++k) {
                    if (k <= ell) {
#pragma unroll
                        for (int n = k; n <= 2 * k; ++n) {
                            const double H = cbinom(n, 2 * k - n) * pb[n - k] * pw2[2 * k - n];
#pragma unroll
                            for (int i = 0; i < NNU; ++i) C[i][k] = fma(fsh[t][i][n], H, C[i][k]);
                        }
                    }
                }
            }
        }
    }
    // fixed-order sum of the waves' coefficients into wave 0 (LDS reused)
    for (int src = 1; src < EZ_HW; ++src) {
        __syncthreads();
        if (part == src) {
#pragma unroll
            for (int i = 0; i < NNU; ++i)
#pragma unroll
                for (int k = 0; k <= EZ_ELL_MAX; ++k)
                    if (k <= ell) lds[(i * (EZ_ELL_MAX + 1) + k) * 64 + lane] = C[i][k];
        }
        __syncthreads();
        if (part == 0) {
#pragma unroll
            for (int i = 0; i < NNU; ++i)
#pragma unroll
                for (int k = 0; k <= EZ_ELL_MAX; ++k)
                    if (k <= ell) C[i][k] += lds[(i * (EZ_ELL_MAX + 1) + k) * 64 + lane];
        }
    }
    // m* = 0: regular part of K E_p(alpha |k|^2) as a series in a = alpha w2 u^2
    if (part != 0 || slice != 0) return;
    const double aw = alpha * w2;
#pragma unroll
    for (int i = 0; i < NNU; ++i) {
        const double s = 0.5 * ((double)D - prog.nu[i]);
        const int m = prog.logm[i];
        const double K = M->K[i];
        if (m < 0) {
            double awj = 1.0, jf = 1.0;
#pragma unroll
            for (int j = 0; j <= EZ_ELL_MAX; ++j) {
                if (j <= ell) {
                    if (j > 0) { awj *= aw; jf *= (double)j; }
                    C[i][j] += -K * (((j & 1) ? -awj : awj) / (jf * (s + (double)j)));
                }
            }
        } else {
            // K [ (-1)^{m+1}/m! a^m ln lam^2 + (-1)^m/m! ( a^m (-gamma - sum_{j>=1} (-a)^j/(j j!))
            //     - e^{-a} sum_{i<m} (-1)^i i! a^{m-i-1} ) ]  as a power series in a
            const double sm = (m & 1) ? -1.0 : 1.0;
            double mf = 1.0;
            for (int j = 2; j <= m; ++j) mf *= (double)j;
            const double lnl2 = log(M->lam * M->lam);
            double awj = 1.0;
#pragma unroll
            for (int J = 0; J <= EZ_ELL_MAX; ++J) {
                if (J > ell) continue;
                double c = 0.0;
                if (J == m) c += -sm / mf * lnl2 + sm / mf * (-EZ_EULER);
                if (J > m) {
                    const int j = J - m;
                    double jf = 1.0;
                    for (int q = 2; q <= j; ++q) jf *= (double)q;
                    c += -sm / mf * (((j & 1) ? -1.0 : 1.0) / ((double)j * jf));
                }
                double iif = 1.0;
                for (int ii = 0; ii < m; ++ii) {
                    if (ii > 0) iif *= (double)ii;
                    const int r = J - (m - ii - 1);
                    if (r >= 0) {
                        double rf = 1.0;
                        for (int q = 2; q <= r; ++q) rf *= (double)q;
                        c += -sm / mf * (((ii & 1) ? -iif : iif)) * (((r & 1) ? -1.0 : 1.0) / rf);
                    }
                }
                C[i][J] += K * c * awj;
                awj *= aw;
            }
        }
    }
}

// Probe kernel: partial C_k(B w_hat_p) over one table slice for 64 probe directions.
// Grid: batch x probe blocks x slices.
template <int D, int NNU>
__global__ __launch_bounds__(64 * EZ_HW) void ez_probe_kernel(EzQuadArgs args) {
    constexpr int FSZ = EZ_HCH * NNU * EZ_NF;
    constexpr int CSZ = 64 * NNU * (EZ_ELL_MAX + 1);
    __shared__ double lds[FSZ > CSZ ? FSZ : CSZ];
    const int nblk = (args.n_probe + 63) / 64;
    const int S = args.n_slice;
    const int inst = (int)blockIdx.x / (nblk * S);
    const int rem = (int)blockIdx.x - inst * nblk * S;
    const int pb = rem / S, slice = rem - pb * S;
    const EzLatMeta *M = args.meta + inst;
    const int lane = (int)threadIdx.x & 63, part = (int)threadIdx.x >> 6;
    const int p = pb * 64 + lane;
    const bool valid = p < args.n_probe;
    const int ell = args.ell_probe;
    double *out = args.probe_val +
                  (((size_t)inst * S + slice) * args.n_probe + (valid ? p : 0)) * NNU * (EZ_ELL_MAX + 1);
    if (M->status != 0) return;               // uniform; the direction kernel skips the lattice
    double wh[3] = {0.0, 0.0, 0.0}, w[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < D; ++i) wh[i] = args.rules[args.probe_off + (valid ? p : 0) * D + i];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) s = fma(M->B[i * D + c], wh[c], s);
        w[i] = s;
    }
    double C[NNU][EZ_ELL_MAX + 1];
    taylor_coeffs<D, NNU>(args, inst, M, ell, w, C, lds, slice, S);
    if (part != 0 || !valid) return;
#pragma unroll
    for (int i = 0; i < NNU; ++i)
#pragma unroll
        for (int k = 0; k <= EZ_ELL_MAX; ++k)
            if (k <= ell) out[i * (EZ_ELL_MAX + 1) + k] = C[i][k];
}

// number of monomials of degree g in D variables
__host__ __device__ constexpr int nmono(int D, int g) { return D == 1 ? 1 : (D == 2 ? g + 1 : (g + 1) * (g + 2) / 2); }

constexpr int EZ_TOUT = 16;                     // tensor coefficients per workgroup

// Tensor kernel: T[i][off_k + a] = sum_p pinv_k[a][p] C_k(probe p), the probe values
// first summed over the table slices in fixed order.  Grid: batch x n_nu x groups of
// EZ_TOUT coefficients; thread = (coefficient, probe residue mod 16).
template <int D, int NNU>
__global__ __launch_bounds__(256) void ez_tensor_kernel(EzQuadArgs args) {
    __shared__ double part[EZ_TOUT][17];
    const int lp = args.ell_probe, S = args.n_slice, np = args.n_probe;
    int tdim = 0;
    for (int k = 0; k <= lp; ++k) tdim += nmono(D, 2 * k);
    const int ngrp = (tdim + EZ_TOUT - 1) / EZ_TOUT;
    const int inst = (int)blockIdx.x / (NNU * ngrp);
    const int rem = (int)blockIdx.x - inst * NNU * ngrp;
    const int i = rem / ngrp, grp = rem - i * ngrp;
    if (args.meta[inst].status != 0) return;  // uniform over the workgroup
    const int o = (int)threadIdx.x >> 4, pp = (int)threadIdx.x & 15;
    const int aa = grp * EZ_TOUT + o;
    double s = 0.0;
    if (aa < tdim) {
        int a = aa, k = 0;
        while (a >= nmono(D, 2 * k)) { a -= nmono(D, 2 * k); ++k; }
        const double *pinv = args.rules + args.pinv_off[k] + (size_t)a * np;
        const double *pv = args.probe_val + (size_t)inst * S * np * NNU * (EZ_ELL_MAX + 1) +
                           (size_t)i * (EZ_ELL_MAX + 1) + k;
        for (int p = pp; p < np; p += 16) {
            double v = 0.0;
            for (int sl = 0; sl < S; ++sl) v += pv[((size_t)sl * np + p) * NNU * (EZ_ELL_MAX + 1)];
            s = fma(pinv[p], v, s);
        }
    }
    part[o][pp] = s;
    __syncthreads();
    if (pp == 0 && aa < tdim) {
        double t = 0.0;
        for (int q = 0; q < 16; ++q) t += part[o][q];
        args.tensor[((size_t)inst * NNU + i) * EZ_TDIM + aa] = t;
    }
}

// Direction kernel: a workgroup takes ndb = min(EZ_HDIR, 256 / n_combo) directions
// of one lattice.  Phase 0: direction geometry and the tensors into LDS; phase 1:
// one thread per (direction, order k) contracts the tensor with the monomials of
// w_hat of degree 2k (C_k); phase 2: one thread per (direction, combination) builds
// the product polynomial (PD coefficients, in registers) and its Hadamard
// integrals; phase 3: per direction, the combinations are summed in fixed order.
template <int D, int NNU, int PD>
__global__ __launch_bounds__(256) void ez_hadamard_kernel(EzQuadArgs args) {
    __shared__ double Tsh[NNU * EZ_TDIM];
    __shared__ double Csh[EZ_HDIR][NNU][EZ_ELL_MAX + 1];
    __shared__ double ssh[EZ_HDIR][NNU];   // sigma_i |w|^{nu_i - d}
    __shared__ double dsh[EZ_HDIR][6];     // 2 w_v, log(pi eps^2 |w|^2), validity, w_hat
    __shared__ double vsh[256];            // value of each (direction, combination)
    __shared__ uint32_t fsh_bad[EZ_HDIR];  // a Hadamard exponent mu = 0 was met
    const int blk = blockIdx.x;
    const int inst = find_segment(args.htile_begin, args.batch, blk);
    const EzInstPlan P = args.plans[inst];
    const EzLatMeta *M = args.meta + inst;
    const EzProgram &prog = args.prog;
    const int n_res = prog.n_res, nc = args.n_combo;
    const int ndb = args.n_dir_blk;
    const int d0 = (blk - args.htile_begin[inst]) * ndb;
    const int ell = P.ell;
    const int tid = (int)threadIdx.x;
    if (M->status != 0) {                           // uniform over the workgroup
        const int dl = d0 + tid;
        if (tid < ndb && dl < P.n_dir) {
            for (int r = 0; r < n_res; ++r) args.dir_part[(size_t)(P.dir_begin + dl) * n_res + r] = 0.0;
            args.dir_flag[P.dir_begin + dl] = 0;
        }
        return;
    }
    int tdim = 0;
    for (int k = 0; k <= ell; ++k) tdim += nmono(D, 2 * k);
    {
        const double *T = args.tensor + (size_t)inst * NNU * EZ_TDIM;
        for (int idx = tid; idx < NNU * tdim; idx += 256) {
            const int i = idx / tdim;
            Tsh[idx] = T[(size_t)i * EZ_TDIM + (idx - i * tdim)];
        }
    }
    if (tid < ndb) {
        const int dl = d0 + tid;
        const bool valid = dl < P.n_dir;
        double B[D * D];
#pragma unroll
        for (int i = 0; i < D * D; ++i) B[i] = M->B[i];
        double w[3] = {0.0, 0.0, 0.0}, wh[3] = {0.0, 0.0, 0.0}, wv = 0.0;
        ez_direction<D>(P, args.rules, B, valid ? dl : 0, w, &wv, wh);
        double w2 = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) w2 = fma(w[i], w[i], w2);
#pragma unroll
        for (int i = 0; i < NNU; ++i) ssh[tid][i] = M->sig[i] * pow(w2, 0.5 * prog.e[i]);
        dsh[tid][0] = 2.0 * wv;
        dsh[tid][1] = log(EZ_PI * P.eps * P.eps * w2);
        dsh[tid][2] = valid ? 1.0 : 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) dsh[tid][3 + i] = wh[i];
        fsh_bad[tid] = 0u;
    }
    __syncthreads();

    // phase 1: C_k(w) = sum over monomials of degree 2k of w_hat (order: a0 desc, a1 desc)
    for (int idx = tid; idx < ndb * (ell + 1); idx += 256) {
        const int dd = idx / (ell + 1), k = idx - dd * (ell + 1);
        const int g = 2 * k;
        int off = 0;
        for (int kk = 0; kk < k; ++kk) off += nmono(D, 2 * kk);
        const double x0 = dsh[dd][3], x1 = dsh[dd][4], x2 = dsh[dd][5];
        double acc[NNU];
#pragma unroll
        for (int i = 0; i < NNU; ++i) acc[i] = 0.0;
        if (D == 1) {
            double mono = 1.0;
            for (int q = 0; q < g; ++q) mono *= x0;
#pragma unroll
            for (int i = 0; i < NNU; ++i) acc[i] = Tsh[i * tdim + off] * mono;
        } else if (D == 2) {
            int a_idx = 0;
            for (int a = g; a >= 0; --a, ++a_idx) {
                double mono = 1.0;
                for (int q = 0; q < a; ++q) mono *= x0;
                for (int q = 0; q < g - a; ++q) mono *= x1;
#pragma unroll
                for (int i = 0; i < NNU; ++i) acc[i] = fma(Tsh[i * tdim + off + a_idx], mono, acc[i]);
            }
        } else {
            int a_idx = 0;
            for (int a = g; a >= 0; --a) {
                double p0 = 1.0;
                for (int q = 0; q < a; ++q) p0 *= x0;
                for (int b = g - a; b >= 0; --b, ++a_idx) {
                    double mono = p0;
                    for (int q = 0; q < b; ++q) mono *= x1;
                    for (int q = 0; q < g - a - b; ++q) mono *= x2;
#pragma unroll
                    for (int i = 0; i < NNU; ++i) acc[i] = fma(Tsh[i * tdim + off + a_idx], mono, acc[i]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < NNU; ++i) Csh[dd][i][k] = acc[i];
    }
    __syncthreads();

    // phase 2: one (direction, combination) per thread
    const int myd = tid / nc, myc = tid - myd * nc;
    bool bad = false;
    if (myd < ndb) {
        const EzCombo &cb = args.combo[myc];
        const int t = cb.t;
        const int nf = prog.term_nfac[t];
        double c = cb.coef;
        double poly[PD];
        poly[0] = 1.0;
#pragma unroll
        for (int J = 1; J < PD; ++J) poly[J] = 0.0;
        int deg = 0;
        for (int f = 0; f < nf; ++f) {
            const int i = prog.term_fac[t][f];
            for (int q = 0; q < cb.j[f]; ++q) c *= ssh[myd][i];
            double Ck[EZ_ELL_MAX + 1];
#pragma unroll
            for (int kk = 0; kk <= EZ_ELL_MAX; ++kk) Ck[kk] = (kk <= ell) ? Csh[myd][i][kk] : 0.0;
            for (int rep = 0; rep < prog.term_mult[t][f] - cb.j[f]; ++rep) {
                // poly <- poly * sum_k C_k u^{2k}, truncated to PD coefficients
#pragma unroll
                for (int J = PD - 1; J >= 0; --J) {
                    double sacc = 0.0;
#pragma unroll
                    for (int kk = 0; kk <= EZ_ELL_MAX; ++kk)
                        if (kk <= J) sacc = fma(poly[J - kk], Ck[kk], sacc);
                    poly[J] = sacc;
                }
                deg = min(deg + ell, PD - 1);
            }
        }
        // fp int_0^eps u^{mu-1} L^Q du, mu = d + E + 2J:
        //   I_0 = eps^mu/mu,  I_q = (eps^mu L(eps)^q - 2q I_{q-1})/mu
        const double eps = P.eps, eps2 = eps * eps;
        const double Leps = dsh[myd][1];
        double mu = (double)(D + cb.E);
        double em = pow(eps, mu);
        double acc = 0.0;
#pragma unroll
        for (int J = 0; J < PD; ++J) {
            if (J <= deg) {
                if (mu == 0.0) {
                    bad = true;
                } else {
                    const double rmu = ez_rcp(mu);
                    double I = em * rmu, Lp = 1.0;
                    for (int j = 1; j <= cb.Q; ++j) {
                        Lp *= Leps;
                        I = (em * Lp - 2.0 * (double)j * I) * rmu;
                    }
                    acc = fma(poly[J], I, acc);
                }
            }
            mu += 2.0;
            em *= eps2;
        }
        vsh[tid] = c * acc;
        if (bad) atomicOr(&fsh_bad[myd], 1u);
    }
    __syncthreads();
    // phase 3: per direction, fixed-order sum over the combinations
    if (tid < ndb) {
        const int dl = d0 + tid;
        if (dl < P.n_dir) {
            const int gd = P.dir_begin + dl;
            for (int r = 0; r < n_res; ++r) {
                double h = 0.0;
                for (int c = 0; c < nc; ++c)
                    if (args.combo[c].res == r) h += vsh[tid * nc + c];
                args.dir_part[(size_t)gd * n_res + r] = dsh[tid][0] * h;
            }
            // device-side guard for a Hadamard exponent mu = 0 (the host rejects such programs)
            args.dir_flag[gd] = fsh_bad[tid];
        }
    }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void ez_finalize_kernel(EzQuadArgs args) {
    const int inst = blockIdx.x;
    const int n_res = args.prog.n_res;
    const int tb = args.tile_begin[inst], te = args.tile_begin[inst + 1];
    const int db = args.dir_begin[inst], de = args.dir_begin[inst + 1];
    __shared__ double red[256 / 64][2];
    __shared__ uint32_t flag_sh;
    if (threadIdx.x == 0) flag_sh = 0;
    __syncthreads();
    uint32_t fl = 0;
    for (int g = db + (int)threadIdx.x; g < de; g += 256) fl |= args.dir_flag[g];
    if (fl) atomicOr(&flag_sh, 1u);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int r = 0; r < n_res; ++r) {
        ez_dd s{0.0, 0.0};
        for (int t = tb + (int)threadIdx.x; t < te; t += 256)
            s = ez_dd_add(s, ez_dd{args.tile_part[((size_t)t * n_res + r) * 2], args.tile_part[((size_t)t * n_res + r) * 2 + 1]});
        for (int g = db + (int)threadIdx.x; g < de; g += 256)
            s = ez_dd_add_d(s, args.dir_part[(size_t)g * n_res + r]);
        s = ez_dd_wave_sum(s);
        __syncthreads();
        if (lane == 0) { red[wave][0] = s.hi; red[wave][1] = s.lo; }
        __syncthreads();
        if (threadIdx.x == 0) {
            ez_dd tot{red[0][0], red[0][1]};
            for (int w = 1; w < 256 / 64; ++w) tot = ez_dd_add(tot, ez_dd{red[w][0], red[w][1]});
            double v = tot.hi + tot.lo;
            uint32_t st = args.meta[inst].status;
            if (flag_sh) st |= 0x8u;
            if (st) v = __longlong_as_double(0x7ff8000000000000ll);
            else if (!isfinite(v)) st |= 0x4u;
            args.out[(size_t)inst * n_res + r] = v;
            if (args.status && r == 0) args.status[inst] = st;
        }
    }
}

template <int D, int NNU, int SET = 0>
hipError_t launch_nodes_t(const EzQuadArgs &args, int n_tiles, hipStream_t stream) {
    hipLaunchKernelGGL((ez_node_kernel<D, NNU, SET>), dim3(n_tiles), dim3(EZ_TILE), 0, stream, args);
    return hipGetLastError();
}

template <int D>
hipError_t launch_nodes_d(const EzQuadArgs &args, int n_tiles, hipStream_t stream) {
    if (D == 3 && args.prog.pset == 1) return launch_nodes_t<D, 4, 1>(args, n_tiles, stream);
    if (D == 2 && args.prog.pset == 2) return launch_nodes_t<D, 4, 2>(args, n_tiles, stream);
    if (D == 1 && args.prog.pset == 3) return launch_nodes_t<D, 4, 3>(args, n_tiles, stream);
    if (D == 3 && args.prog.pset == 4) return launch_nodes_t<D, 7, 4>(args, n_tiles, stream);
    switch (args.prog.n_nu) {
        case 1: return launch_nodes_t<D, 1>(args, n_tiles, stream);
        case 2: return launch_nodes_t<D, 2>(args, n_tiles, stream);
        case 3: return launch_nodes_t<D, 3>(args, n_tiles, stream);
        case 4: return launch_nodes_t<D, 4>(args, n_tiles, stream);
        case 5: return launch_nodes_t<D, 5>(args, n_tiles, stream);
        case 6: return launch_nodes_t<D, 6>(args, n_tiles, stream);
        case 7: return launch_nodes_t<D, 7>(args, n_tiles, stream);
        case 8: return launch_nodes_t<D, 8>(args, n_tiles, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t ez_launch_nodes_impl(const EzQuadArgs &args, int n_tiles, hipStream_t stream) {
    switch (args.prog.d) {
        case 1: return launch_nodes_d<1>(args, n_tiles, stream);
        case 2: return launch_nodes_d<2>(args, n_tiles, stream);
        case 3: return launch_nodes_d<3>(args, n_tiles, stream);
        default: return hipErrorInvalidValue;
    }
}

template <int D, int NNU, int PD>
hipError_t launch_had_t(const EzQuadArgs &args, int n_htiles, hipStream_t stream) {
    const int nblk = (args.n_probe + 63) / 64;
    hipLaunchKernelGGL((ez_probe_kernel<D, NNU>), dim3(args.batch * nblk * args.n_slice), dim3(64 * EZ_HW), 0,
                       stream, args);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int tdim = 0;
    for (int k = 0; k <= args.ell_probe; ++k) tdim += nmono(D, 2 * k);
    const int ngrp = (tdim + EZ_TOUT - 1) / EZ_TOUT;
    hipLaunchKernelGGL((ez_tensor_kernel<D, NNU>), dim3(args.batch * NNU * ngrp), dim3(256), 0, stream, args);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((ez_hadamard_kernel<D, NNU, PD>), dim3(n_htiles), dim3(256), 0, stream, args);
    return hipGetLastError();
}

template <int D, int NNU>
hipError_t launch_had_p(const EzQuadArgs &args, int n_htiles, hipStream_t stream) {
    if (args.poly_deg == 13) return launch_had_t<D, NNU, 13>(args, n_htiles, stream);
    if (args.poly_deg == 33) return launch_had_t<D, NNU, 33>(args, n_htiles, stream);
    return hipErrorInvalidValue;
}

template <int D>
hipError_t launch_had_d(const EzQuadArgs &args, int n_htiles, hipStream_t stream) {
    switch (args.prog.n_nu) {
        case 1: return launch_had_p<D, 1>(args, n_htiles, stream);
        case 2: return launch_had_p<D, 2>(args, n_htiles, stream);
        case 3: return launch_had_p<D, 3>(args, n_htiles, stream);
        case 4: return launch_had_p<D, 4>(args, n_htiles, stream);
        case 5: return launch_had_p<D, 5>(args, n_htiles, stream);
        case 6: return launch_had_p<D, 6>(args, n_htiles, stream);
        case 7: return launch_had_p<D, 7>(args, n_htiles, stream);
        case 8: return launch_had_p<D, 8>(args, n_htiles, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t ez_launch_nodes(const EzQuadArgs &args, int n_tiles, hipStream_t stream) {
    return ez_launch_nodes_impl(args, n_tiles, stream);
}

hipError_t ez_launch_hadamard(const EzQuadArgs &args, int n_htiles, hipStream_t stream) {
    switch (args.prog.d) {
        case 1: return launch_had_d<1>(args, n_htiles, stream);
        case 2: return launch_had_d<2>(args, n_htiles, stream);
        case 3: return launch_had_d<3>(args, n_htiles, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t ez_launch_finalize(const EzQuadArgs &args, hipStream_t stream) {
    hipLaunchKernelGGL(ez_finalize_kernel, dim3(args.batch), dim3(256), 0, stream, args);
    return hipGetLastError();
}
