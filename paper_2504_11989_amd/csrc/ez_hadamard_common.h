// ez_hadamard_common.h -- Taylor coefficients of Z^reg on (0, eps) through probe
// directions and a least-squares tensor (probe and tensor kernels), shared by the
// Hadamard kernels (ez_hadamard.hip, ez_hadamard_adj.hip).
#pragma once
#include "ez_quad_common.h"

namespace {
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

// strain component s of a symmetric d x d tensor: the diagonal first, then (0,1), (0,2), (1,2)
__host__ __device__ constexpr int ez_sa(int D, int s) { return s < D ? s : (s - D < 2 ? 0 : 1); }
__host__ __device__ constexpr int ez_sb(int D, int s) { return s < D ? s : (s - D == 0 ? 1 : 2); }

// Partial C[i][k] at direction w over one slice of the tables: real-space pairs,
// reciprocal m* != 0, and (slice 0 only) the self term and the m* = 0 series.
// Channel ch = 0 gives the coefficients; ch = 1 + s (GR only) their derivative
// with respect to the strain component s = (a, b) at fixed fractional direction,
// using d|z|^2 = 2 z z^T, d|m*|^2 = -2 m* m*^T, d(w.m*) = -(w m*^T + m* w^T),
// d|w|^2 = -2 w w^T and dK = -K I.
// Lane = direction, the slice's entries split over EZ_HW waves, summed in LDS in
// fixed order; on return wave 0 holds the slice's coefficients.
template <int D, int NNU, bool GR, int LM = EZ_ELL_MAX>
__device__ void taylor_coeffs(const EzQuadArgs &args, int inst, const EzLatMeta *M, int ell, const double *w,
                              double (&C)[NNU][LM + 1], double *lds, int slice, int n_slice, int ch) {
    constexpr int NF = GR ? 2 * LM + 2 : 2 * LM + 1;
    double (*fsh)[NNU][NF] = reinterpret_cast<double (*)[NNU][NF]>(lds);
    const EzProgram &prog = args.prog;
    const int lane = (int)threadIdx.x & 63, part = (int)threadIdx.x >> 6;
    const bool dch = GR && ch > 0;
    const int sa = dch ? ez_sa(D, ch - 1) : 0, sb = dch ? ez_sb(D, ch - 1) : 0;
    const double delta = (dch && sa == sb) ? 1.0 : 0.0;
    double w2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) w2 = fma(w[i], w[i], w2);
    const double ww = w[sa] * w[sb];
    const double alpha = M->alpha;
    double pw2[LM + 1];
    pw2[0] = 1.0;
#pragma unroll
    for (int j = 1; j <= LM; ++j) pw2[j] = pw2[j - 1] * w2;
#pragma unroll
    for (int i = 0; i < NNU; ++i) {
#pragma unroll
        for (int k = 0; k <= LM; ++k) C[i][k] = 0.0;
        if (part == 0 && slice == 0 && !dch) C[i][0] = -M->self_[i];
    }
    // real space: 2 W cos(2 pi u w.z) = 2 W sum_k (-1)^k (2 pi w.z)^{2k} u^{2k} / (2k)!
    // (w.z is the fractional w_hat.n, so only the weight moves under strain)
    {
        const int rs = args.tab.rstride;
        const double *rt = args.tab.real + (size_t)inst * args.tab.real_cap * rs;
        const int n_real = M->n_real;
        const int woff = dch ? 3 + NNU : 3;
        // two entries per pass (their loads issued together), added in table order
        const int step = EZ_HW * n_slice;
        for (int p = slice * EZ_HW + part; p < n_real; p += 2 * step) {
            const bool two = p + step < n_real;
            const double *e0 = rt + (size_t)p * rs;
            const double *e1 = rt + (size_t)(two ? p + step : p) * rs;
            double ew0[NNU], ew1[NNU], t0 = 0.0, t1 = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) { t0 = fma(w[i], e0[i], t0); t1 = fma(w[i], e1[i], t1); }
#pragma unroll
            for (int i = 0; i < NNU; ++i) { ew0[i] = e0[woff + i]; ew1[i] = two ? e1[woff + i] : 0.0; }
            const double x0 = (2.0 * EZ_PI * t0) * (2.0 * EZ_PI * t0);
            const double x1 = (2.0 * EZ_PI * t1) * (2.0 * EZ_PI * t1);
            double term0 = dch ? e0[sa] * e0[sb] : 1.0;
            double term1 = dch ? e1[sa] * e1[sb] : 1.0;
#pragma unroll
            for (int k = 0; k <= LM; ++k) {
                if (k <= ell) {
#pragma unroll
                    for (int i = 0; i < NNU; ++i) C[i][k] = fma(ew1[i], term1, fma(ew0[i], term0, C[i][k]));
                    const double f = 1.0 / ((2.0 * k + 1.0) * (2.0 * k + 2.0));
                    term0 *= -x0 * f;
                    term1 *= -x1 * f;
                }
            }
        }
    }
    // reciprocal space, m* != 0: F(rho) = K E_p(alpha rho), rho(u) = |m*|^2 + 2 u b + u^2 w2, b = w.m*.
    // With F_n = F^(n)(|m*|^2)/n! = K (-alpha)^n E_{p-n}(alpha |m*|^2)/n!, the u^{2k} coefficient is
    //   sum_{n=k}^{2k} F_n H_{n,k},  H_{n,k} = C(n, 2k-n) (4 b^2)^{n-k} w2^{2k-n};
    // its strain derivative is sum_n [(-F_n I - 2 (n+1) F_{n+1} m* m*^T) H + F_n dH].
    {
        const double *kt = args.tab.rec + (size_t)inst * args.tab.rec_cap * 4;
        const int n_rec = M->n_rec;
        const int nfmax = dch ? 2 * ell + 1 : 2 * ell;
        // entries 1 .. n_rec - 1 in equal contiguous shares per slice, in chunks of EZ_HCH
        const int per = (n_rec - 1 + n_slice - 1) / n_slice;
        const int lo = 1 + slice * per, hi = min(n_rec, lo + per);
        for (int base = lo; base < hi; base += EZ_HCH) {
            __syncthreads();
            // F_n for (entry, nu) pairs, one per thread
            for (int task = (int)threadIdx.x; task < EZ_HCH * NNU; task += 64 * EZ_HW) {
                const int te = task / NNU, i = task - te * NNU;
                const int q = base + te;
                if (q < hi) {
                    const double a0 = alpha * kt[(size_t)q * 4 + 3];
                    const double ex = exp(-a0), inv = ez_rcp(a0);
                    double E, pi_;
                    if (prog.real_nu) {
                        pi_ = prog.preal[i];
                        E = ez_ep_real(pi_, a0);
                    } else {
                        const int p2 = prog.p2[i];
                        pi_ = 0.5 * (double)p2;
                        const double E1 = ((p2 & 1) == 0) ? ez_e1(a0, ex, inv) : 0.0;
                        const double Eh = (p2 & 1) ? ez_ehalf(a0) : 0.0;
                        E = ez_ep_from(p2, a0, ex, inv, E1, Eh);
                    }
                    double sc = M->K[i];
#pragma unroll
                    for (int n = 0; n < NF; ++n) {
                        if (n <= nfmax) {
                            fsh[te][i][n] = sc * E;
                            const double pnm1 = pi_ - (double)n - 1.0;
                            E = (ex - pnm1 * E) * inv;          // E_{p-n-1}
                            sc *= -alpha * (1.0 / (double)(n + 1));
                        }
                    }
                }
            }
            __syncthreads();
            const int cnt = min(EZ_HCH, hi - base);
            for (int t = part; t < cnt; t += EZ_HW) {
                const double *e = kt + (size_t)(base + t) * 4;
                double b = 0.0;
#pragma unroll
                for (int i = 0; i < D; ++i) b = fma(w[i], e[i], b);
                const double b4 = 4.0 * b * b;
                double pb[LM + 1];
                pb[0] = 1.0;
#pragma unroll
                for (int j = 1; j <= LM; ++j) pb[j] = pb[j - 1] * b4;
                if (!dch) {
#pragma unroll
                    for (int k = 0; k <= LM; ++k) {
                        if (k <= ell) {
#pragma unroll
                            for (int n = k; n <= 2 * k; ++n) {
                                const double H = cbinom(n, 2 * k - n) * pb[n - k] * pw2[2 * k - n];
#pragma unroll
                                for (int i = 0; i < NNU; ++i) C[i][k] = fma(fsh[t][i][n], H, C[i][k]);
                            }
                        }
                    }
                } else {
                    const double qq = e[sa] * e[sb];
                    const double wq = w[sa] * e[sb] + e[sa] * w[sb];
#pragma unroll
                    for (int k = 0; k <= LM; ++k) {
                        if (k <= ell) {
#pragma unroll
                            for (int n = k; n <= 2 * k; ++n) {
                                const double cb = cbinom(n, 2 * k - n);
                                const double H = cb * pb[n - k] * pw2[2 * k - n];
                                const double Hb = (n > k) ? cb * (double)(n - k) * 8.0 * b * pb[n - k - 1] * pw2[2 * k - n] : 0.0;
                                const double Hw = (n < 2 * k) ? cb * (double)(2 * k - n) * pb[n - k] * pw2[2 * k - n - 1] : 0.0;
                                const double X = -delta * H - Hb * wq - 2.0 * Hw * ww;
                                const double Y = -2.0 * (double)(n + 1) * qq * H;
#pragma unroll
                                for (int i = 0; i < NNU; ++i)
                                    C[i][k] = fma(fsh[t][i][n], X, fma(fsh[t][i][n + 1], Y, C[i][k]));
                            }
                        }
                    }
                }
            }
        }
    }
    // m* = 0 (slice 0; exponent i on wave i mod EZ_HW): regular part of K E_p(alpha |k|^2)
    // as a series in a = alpha w2 u^2; a term K c_J (alpha w2)^J has strain derivative
    // -(I + 2 J w w^T / w2) times itself
    if (slice == 0) {
        const double aw = alpha * w2;
        const double rw2 = dch ? ww / w2 : 0.0;
#pragma unroll
        for (int i = 0; i < NNU; ++i) {
            if (i % EZ_HW != part) continue;
            const double s = 0.5 * ((double)D - prog.nu[i]);
            const int m = prog.logm[i];
            const double K = M->K[i];
            if (m < 0) {
                double awj = 1.0, jf = 1.0;
#pragma unroll
                for (int j = 0; j <= LM; ++j) {
                    if (j <= ell) {
                        if (j > 0) { awj *= aw; jf *= (double)j; }
                        double v = -K * (((j & 1) ? -awj : awj) / (jf * (s + (double)j)));
                        if (dch) v *= -delta - 2.0 * (double)j * rw2;
                        C[i][j] += v;
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
                for (int J = 0; J <= LM; ++J) {
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
                    double v = K * c * awj;
                    if (dch) v *= -delta - 2.0 * (double)J * rw2;
                    C[i][J] += v;
                    awj *= aw;
                }
            }
        }
    }
    // fixed-order sum of the waves' coefficients into wave 0: waves 1 .. EZ_HW - 1 write
    // their orders k <= ell to regions of their own (the F_n table is no longer read),
    // and wave 0 adds the regions in wave order
    const int KL = ell + 1;
    __syncthreads();
    if (part != 0) {
        double *R = lds + (size_t)(part - 1) * NNU * KL * 64;
#pragma unroll
        for (int i = 0; i < NNU; ++i)
#pragma unroll
            for (int k = 0; k <= LM; ++k)
                if (k <= ell) R[(i * KL + k) * 64 + lane] = C[i][k];
    }
    __syncthreads();
    if (part == 0) {
        for (int src = 1; src < EZ_HW; ++src) {
            const double *R = lds + (size_t)(src - 1) * NNU * KL * 64;
#pragma unroll
            for (int i = 0; i < NNU; ++i)
#pragma unroll
                for (int k = 0; k <= LM; ++k)
                    if (k <= ell) C[i][k] += R[(i * KL + k) * 64 + lane];
        }
    }
}

// dynamic LDS of the probe kernel: the F_n table of one chunk, or the partial
// coefficients of waves 1 .. EZ_HW - 1 (orders k <= ell)
template <int NNU, bool GR>
inline size_t probe_lds_bytes(int ell) {
    const size_t fsz = (size_t)EZ_HCH * NNU * (GR ? EZ_NF + 1 : EZ_NF);
    const size_t csz = (size_t)(EZ_HW - 1) * NNU * (ell + 1) * 64;
    return sizeof(double) * (fsz > csz ? fsz : csz);
}

// Probe kernel: partial C_k(B w_hat_p) over one table slice for 64 probe directions,
// one channel (value or strain component).  Grid: batch x probe blocks x slices x channels.
template <int D, int NNU, bool GR, int LM = EZ_ELL_MAX>
__global__ __launch_bounds__(64 * EZ_HW) void ez_probe_kernel(EzQuadArgs args) {
    extern __shared__ double lds[];                 // probe_lds_bytes<NNU, GR>(args.ell_probe)
    const int nblk = (args.n_probe + 63) / 64;
    const int S = args.n_slice, NCH = GR ? args.n_ch : 1;
    const int per_inst = nblk * S * NCH;
    const int inst = (int)blockIdx.x / per_inst;
    int rem = (int)blockIdx.x - inst * per_inst;
    const int ch = rem / (nblk * S);
    rem -= ch * nblk * S;
    const int pb = rem / S, slice = rem - pb * S;
    const EzLatMeta *M = args.meta + inst;
    const int lane = (int)threadIdx.x & 63, part = (int)threadIdx.x >> 6;
    const int p = pb * 64 + lane;
    const bool valid = p < args.n_probe;
    const int ell = args.ell_probe;
    double *out = args.probe_val +
                  ((((size_t)inst * S + slice) * args.n_probe + (valid ? p : 0)) * NCH + ch) * NNU * (EZ_ELL_MAX + 1);
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
    double C[NNU][LM + 1];
    taylor_coeffs<D, NNU, GR, LM>(args, inst, M, ell, w, C, lds, slice, S, ch);
    if (part != 0 || !valid) return;
#pragma unroll
    for (int i = 0; i < NNU; ++i)
#pragma unroll
        for (int k = 0; k <= LM; ++k)
            if (k <= ell) out[i * (EZ_ELL_MAX + 1) + k] = C[i][k];
}

// number of monomials of degree g in D variables
__host__ __device__ constexpr int nmono(int D, int g) { return D == 1 ? 1 : (D == 2 ? g + 1 : (g + 1) * (g + 2) / 2); }

constexpr int EZ_TOUT = 4;                      // tensor coefficients per workgroup (one per wave)

// Tensor kernel: T[c][off_k + a] = sum_p pinv_k[a][p] C_k(probe p) for each channel
// c = ch * n_nu + i, the probe values first summed over the table slices in fixed
// order.  Grid: batch x channels x groups of EZ_TOUT coefficients; wave = coefficient,
// lane = probe residue mod 64 (the slice loads of a probe issued eight at a time);
// the lanes' sums are added by a fixed butterfly.
template <int D, int NNU>
__global__ __launch_bounds__(64 * EZ_TOUT) void ez_tensor_kernel(EzQuadArgs args) {
    const int lp = args.ell_probe, S = args.n_slice, np = args.n_probe;
    const int NC = NNU * args.n_ch;
    int tdim = 0;
    for (int k = 0; k <= lp; ++k) tdim += nmono(D, 2 * k);
    const int ngrp = (tdim + EZ_TOUT - 1) / EZ_TOUT;
    const int inst = (int)blockIdx.x / (NC * ngrp);
    const int rem = (int)blockIdx.x - inst * NC * ngrp;
    const int c = rem / ngrp, grp = rem - c * ngrp;
    if (args.meta[inst].status != 0) return;  // uniform over the workgroup
    const int lane = (int)threadIdx.x & 63;
    const int aa = grp * EZ_TOUT + ((int)threadIdx.x >> 6);
    if (aa >= tdim) return;                   // uniform over the wave
    int a = aa, k = 0;
    while (a >= nmono(D, 2 * k)) { a -= nmono(D, 2 * k); ++k; }
    const double *pinv = args.rules + args.pinv_off[k] + (size_t)a * np;
    const double *pv = args.probe_val + (size_t)inst * S * np * NC * (EZ_ELL_MAX + 1) + (size_t)c * (EZ_ELL_MAX + 1) + k;
    double s = 0.0;
    for (int p = lane; p < np; p += 64) {
        // the slices in fixed order, their loads issued eight at a time
        double v = 0.0;
        for (int sl0 = 0; sl0 < S; sl0 += 8) {
            double t[8];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                t[q] = (sl0 + q < S) ? pv[((size_t)(sl0 + q) * np + p) * NC * (EZ_ELL_MAX + 1)] : 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) v += t[q];
        }
        s = fma(pinv[p], v, s);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
    if (lane == 0) args.tensor[((size_t)inst * NC + c) * EZ_TDIM + aa] = s;
}

// C_k(w_hat), k = 0 .. ell, of one channel from its tensor row T (monomials of degree
// 2k in the order a0 desc, a1 desc, orders one after the other): homogeneous Horner
// in (x0, x1, x2); T is uniform over the wave
template <int D, int LM>
__device__ __forceinline__ void horner_orders(const double *T, int ell, double x0, double x1, double x2,
                                              double (&C)[LM + 1]) {
    int off = 0;
#pragma unroll
    for (int k = 0; k <= LM; ++k) {
        C[k] = 0.0;
        if (k > ell) continue;
        const int g = 2 * k;
        if (D == 1) {
            double m = 1.0;
            for (int q = 0; q < g; ++q) m *= x0;
            C[k] = T[off] * m;
            off += 1;
        } else if (D == 2) {
            // sum_a T[g - a] x0^a x1^(g - a), a descending
            double acc = T[off], p1 = 1.0;
            for (int a = g - 1; a >= 0; --a) {
                p1 *= x1;
                acc = fma(acc, x0, T[off + g - a] * p1);
            }
            C[k] = acc;
            off += g + 1;
        } else {
            // sum_a x0^a S_a(x1, x2), S_a homogeneous of degree g - a in (x1, x2) with
            // its coefficients in b = g - a .. 0 order
            double acc = 0.0;
            for (int a = g; a >= 0; --a) {
                const int m = g - a;
                double S = T[off], p2 = 1.0;
                for (int b = m - 1; b >= 0; --b) {
                    p2 *= x2;
                    S = fma(S, x1, T[off + m - b] * p2);
                }
                off += m + 1;
                acc = fma(acc, x0, S);
            }
            C[k] = acc;
        }
    }
}


// Direction kernel (value calls): a workgroup takes EZ_HDIR = 64 directions of one
// lattice, one per lane, and its waves (16, or 4 for a large batch) share out the
// channels (phase 1: the tensor contracted with the monomials of w_hat, C_k) and the
// combinations (phase 2: the product polynomial, PD coefficients in registers, and
// its Hadamard integrals), so that a wave's control flow is uniform; phase 3 adds the
// waves' per-result sums in wave order.  The adjoint kernel has the same layout, one
// workgroup per (direction block, strain component).
}  // namespace
