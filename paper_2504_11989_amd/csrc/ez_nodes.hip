// ez_nodes.hip -- quadrature nodes on (eps, 1/2] and the final reduction.
//
// ez_node_kernel      : one thread per node k = u w: Z_nu(k) for the exponent set by
//                       the split (real-space table + reciprocal table), the products
//                       of the terms, weight, then a double-double reduction to one
//                       partial per 256-node tile (paper, Sec. 2, Theorem (Epstein
//                       representation); Sec. 3, Corollary (Duffy transformation)).
// ez_node_split_kernel: the last few tiles of a call, each node's terms shared by
//                       many waves (see below).
// ez_finalize_kernel  : fixed-order double-double sum of tiles and directions; the
//                       derivatives with respect to A when requested.
#include <algorithm>

#include "ez_quad_common.h"

namespace {

// E_1(a) and E_{1/2}(a) for any a > 0 (series below 1/4, rationals above), out
// of line for the rarely used near-list loop
__device__ __attribute__((noinline, const)) double ez_e1_ool(double a) {
    if (a < 0.25) return ez_e1_series(a);
    return ez_expm(a) * ez_e1w_scaled(ez_rcp(a));
}
__device__ __attribute__((noinline, const)) double ez_ehalf_ool(double a) {
    if (a < 0.25) return ez_ehalf(a);
    const double inv = ez_rcp(a);
    return ez_expm(a) * inv * ez_ehw_scaled(inv);
}

// Geometry of node (dir, iu): k = u w, theta = u w_hat (so that k.z = theta.n for
// z = A n) and the quadrature weight W (Duffy Jacobian u^{d-1}, Gauss weights, factor 2).
template <int D>
__device__ __forceinline__ void node_geometry(const EzInstPlan &P, const double *rules, const EzLatMeta *M, int dir,
                                              int iu, double *k, double *th, double *W) {
    double B[D * D];
#pragma unroll
    for (int i = 0; i < D * D; ++i) B[i] = M->B[i];
    double w[3] = {0.0, 0.0, 0.0}, wh[3] = {0.0, 0.0, 0.0}, wv;
    ez_direction<D>(P, rules, B, dir, w, &wv, wh);
    const double u = rules[P.urule + iu];
    const double wu = rules[P.urule + P.n_u + iu];
#pragma unroll
    for (int i = 0; i < 3; ++i) { k[i] = 0.0; th[i] = 0.0; }
#pragma unroll
    for (int i = 0; i < D; ++i) { k[i] = u * w[i]; th[i] = u * wh[i]; }
    double Wt = 2.0 * wv * wu;
#pragma unroll
    for (int i = 0; i < D - 1; ++i) Wt *= u;
    *W = Wt;
}

// Real space: sum over pairs of 2 W_nu(z) Re e^{2 pi i k.z}, k.z = theta.n, over the
// rows [r0, r1) of the table.  Row by row (n2, n3 fixed, consecutive n1) the phase
// advances by c1 = e^{2 pi i theta_1}; from row to row within a plane by
// c2^{dn2} c1^{dn1}; each plane, and the first row of the range, starts from one sincos.
template <int D, int NNU>
__device__ __forceinline__ void real_rows(const EzQuadArgs &args, int inst, const double *th, int r0, int r1,
                                          double *accr) {
    const int rs = args.tab.rstride;
    const double *rt = args.tab.real + (size_t)inst * args.tab.real_cap * rs;
    const int *rows = args.tab.rows + (size_t)inst * args.tab.row_cap * 8;
    double c1r, c1i, c2r = 1.0, c2i = 0.0;
    ez_sincos2pi(th[0], &c1i, &c1r);
    if (D > 1) ez_sincos2pi(th[1], &c2i, &c2r);
    double br = 1.0, bi = 0.0;
    for (int r = r0; r < r1; ++r) {
        const int *R = rows + (size_t)r * 8;
        const int first = R[0], cnt = R[1];
        if (R[5] || r == r0) {
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

// Reciprocal space: sum over m* of E_{p_nu}(pi lam^2 |m* + k|^2).  Entry 0 is m* = 0,
// where a = alpha |k|^2 can be small (series of E1); so can the entries of the
// culling's near list.  rec_origin adds m* = 0 (inline), then the near list in
// table order; that list is usually empty, so its special functions are called
// out of line and take no registers from the main loop.  Every entry of the main
// list has a >= 1/4 at every node of the tile, so rec_list is one branch-free
// formula with E1 and E_{1/2} from the wide rationals.
template <int D, int NNU, int SET>
__device__ __forceinline__ void rec_origin(const EzQuadArgs &args, const double *kt, const unsigned short *klist,
                                           int n_near, const double *k, double alpha, double acut, double *acck) {
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
            const double Eh = need_half ? ((a < 0.25) ? ez_ehalf(a) : ex * inv * ez_ehw_scaled(inv)) : 0.0;
#pragma unroll
            for (int i = 0; i < NNU; ++i)
                acck[i] += pset_ep<SET>(args.prog, i, a, ex, inv, E1, Eh);
        }
    }
    for (int j = 1; j <= n_near; ++j) {
        const double *e = kt + (size_t)__builtin_amdgcn_readfirstlane((int)klist[EZ_KCULL - j]) * 4;
        double rho = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) { const double t = e[i] + k[i]; rho = fma(t, t, rho); }
        const double a = alpha * rho;
        if (a <= acut) {
            const double ex = ez_expm(a);
            const double inv = ez_rcp(a);
            const double E1 = need_e1 ? ez_e1_ool(a) : 0.0;
            const double Eh = need_half ? ez_ehalf_ool(a) : 0.0;
#pragma unroll
            for (int i = 0; i < NNU; ++i)
                acck[i] += pset_ep<SET>(args.prog, i, a, ex, inv, E1, Eh);
        }
    }
}

template <int D, int NNU, int SET>
__device__ __forceinline__ void rec_list(const EzQuadArgs &args, const double *kt, const unsigned short *klist,
                                         int j0, int j1, const double *k, double alpha, double acut, double *acck) {
    const bool need_e1 = pset_need_e1<SET, NNU>(args.prog), need_half = pset_need_half<SET, NNU>(args.prog);
    if (j0 >= j1) return;
    // software pipeline: the list index two entries ahead and the table entry one
    // entry ahead are loaded while the current term is evaluated
    auto entry = [&](int j) { return kt + (size_t)__builtin_amdgcn_readfirstlane((int)klist[j]) * 4; };
    int qn = (int)klist[j0 + 1 < j1 ? j0 + 1 : j0];
    const double *en = entry(j0);
    double m0 = en[0], m1 = D > 1 ? en[1] : 0.0, m2 = D > 2 ? en[2] : 0.0;
    for (int j = j0; j < j1; ++j) {
        const double c0 = m0, c1 = m1, c2 = m2;
        {
            const double *e2 = kt + (size_t)__builtin_amdgcn_readfirstlane(qn) * 4;
            m0 = e2[0];
            if (D > 1) m1 = e2[1];
            if (D > 2) m2 = e2[2];
            qn = (int)klist[j + 2 < j1 ? j + 2 : j1 - 1];
        }
        double qx = c0 + k[0];
        double rho = qx * qx;
        if (D > 1) { double qy = c1 + k[1]; rho = fma(qy, qy, rho); }
        if (D > 2) { double qz = c2 + k[2]; rho = fma(qz, qz, rho); }
        const double a = alpha * rho;
        if (a <= acut) {
            const double ex = ez_expm(a);
            const double inv = ez_rcp(a);
            const double E1 = need_e1 ? ex * ez_e1w_scaled(inv) : 0.0;
            const double Eh = need_half ? ex * inv * ez_ehw_scaled(inv) : 0.0;
#pragma unroll
            for (int i = 0; i < NNU; ++i)
                acck[i] += pset_ep<SET>(args.prog, i, a, ex, inv, E1, Eh);
        }
    }
}

// Reciprocal sum of one wave of the tile kernel over the table entries [q0, q1) (and
// m* = 0 if `origin`), culled per wave.  The table is read in chunks of 64 entries (one per lane); with c and r_w
// the centre and half-diagonal of the bounding box of the wave's k, an entry is
//   beyond the cutoff for every node   if |m* + c| > sqrt(a_cut/alpha) + r_w,
//   near  (a may be < 1/4 at a node)   if |m* + c| <= 1/(2 sqrt alpha) + r_w,
//   mid   (a may be < 4, never < 1/4)  if |m* + c| <= 2/sqrt(alpha) + r_w,
//   far   (a >= 4 at every node)       otherwise.
// Far entries (most of them) are summed as the chunk is read, taken one by one
// from the chunk's ballot mask and loaded through the scalar cache, with e^{-a}
// from a 256-entry table of 2^{-j/256} in LDS and E_1, E_{1/2} and 1/a from the
// (7,7) rationals for a >= 4 with one reciprocal.  Mid and near entries go to the
// wave's lists in LDS and are summed afterwards, mid ones with the (12,12)
// rationals for a >= 1/4, near ones with the series forms below 1/4 (out of
// line); a list longer than its capacity makes the sums NaN.
// Order of the terms: m* = 0, far entries, mid list, near list (table order in each).
#define EZ_NEAR_MAX 128
#define EZ_MID_MAX 256

// a value equal on all lanes of the wave, moved to scalar registers
__device__ __forceinline__ double wave_uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// appends the lanes with `sel` to a wave's index list at position *n (in lane order)
__device__ __forceinline__ void wave_append(bool sel, int q, unsigned short *list, int cap, int *n) {
    const unsigned long long bal = __ballot(sel);
    if (bal) {
        const int lane = (int)threadIdx.x & 63;
        const int slot = *n + __popcll(bal & ((1ull << lane) - 1ull));
        if (sel && slot < cap) list[slot] = (unsigned short)q;
        *n += __popcll(bal);
    }
}

// Largest 2p of the integer chain (which = 0; 0 when its largest p is <= 0, -1 when
// no exponent has an integer p) and of the half-integer chain (which = 1; 1 when its
// largest p is <= 1/2, -1 when there is none)
template <int SET, int NNU>
__device__ __forceinline__ int mix_top2(const EzQuadArgs &args, int which) {
    if constexpr (SET == 0) {
        return args.mix_top2[which];
    } else {
        bool any = false;
        int t = 0;
#pragma unroll
        for (int i = 0; i < NNU; ++i) {
            const int p2 = ez_pset(SET).p2[i];
            if ((p2 & 1) == which) {
                t = (any && t > p2) ? t : p2;
                any = true;
            }
        }
        return any ? (t < which ? which : t) : -1;
    }
}

// One far-field reciprocal term in FP32 (a >= a_mix >= EZ_EPF_XMIN): e^{-a}, 1/a, the
// chain tops E_p = e^{-a} t g_p(t) from the fits, every exponent's E_p by the downward
// recurrence E_{p-1} = (e^{-a} - (p-1) E_p) / a from its chain's top (stable for
// a > p), added to accf
template <int SET, int NNU>
__device__ __forceinline__ void far32_term(const EzQuadArgs &args, double a, float *accf) {
    const float ex = ez_expm_f32(a);
    const float t = __builtin_amdgcn_rcpf((float)a);
    const float ext = ex * t;
    const int ti = mix_top2<SET, NNU>(args, 0), th = mix_top2<SET, NNU>(args, 1);
    float Ei = ext, Eh = 0.0f;
    if (ti >= 2) Ei = ext * ez_epf(ti - 1, t);
    if (th >= 1) Eh = ext * ez_epf(th - 1, t);
#pragma unroll
    for (int i = 0; i < NNU; ++i) {
        const int p2 = pset_p2<SET>(args.prog, i);
        const bool odd = (p2 & 1) != 0;
        float E = odd ? Eh : Ei;
        for (int q2 = odd ? th : ti; q2 > p2; q2 -= 2) E = fmaf(-0.5f * (float)(q2 - 2), E, ex) * t;
        accf[i] += E;
    }
}

template <int D, int NNU, int SET, bool MIX>
__device__ __forceinline__ void rec_wave(const EzQuadArgs &args, const double *kt, int q0, int q1, bool origin,
                                         const double *k, bool valid, double alpha, double acut,
                                         unsigned short *nearl, unsigned short *midl, const double *exptab,
                                         double *acck, double *far32) {
    const bool need_e1 = pset_need_e1<SET, NNU>(args.prog), need_half = pset_need_half<SET, NNU>(args.prog);
    const int lane = (int)threadIdx.x & 63;
    double c[3] = {0.0, 0.0, 0.0}, rt2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double lo = k[i], hi = k[i];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, m, 64));
            hi = fmax(hi, __shfl_xor(hi, m, 64));
        }
        c[i] = wave_uniform(0.5 * (lo + hi));
        rt2 += 0.25 * (hi - lo) * (hi - lo);
    }
    const double rt = sqrt(rt2), ra = 1.0 / sqrt(alpha);
    const double rmax = (sqrt(acut / alpha) + rt) * (1.0 + 1e-9) + 1e-12;
    const double rnear = (0.5 * ra + rt) * (1.0 + 1e-9) + 1e-12;
    const double rmid = (2.0 * ra + rt) * (1.0 + 1e-9) + 1e-12;
    const double rmax2 = wave_uniform(rmax * rmax), rnear2 = wave_uniform(rnear * rnear);
    const double rmid2 = wave_uniform(rmid * rmid);
    // mixed precision: entries with |m* + c| >= sqrt(a_mix / alpha) + r_w have a >= a_mix
    // at every node of the wave and are summed in FP32
    double r32sq = 1e300;
    if constexpr (MIX) {
        const double r32 = (sqrt(args.a_mix / alpha) + rt) * (1.0 + 1e-9) + 1e-12;
        r32sq = wave_uniform(r32 * r32);
#pragma unroll
        for (int i = 0; i < NNU; ++i) far32[i] = 0.0;
    }
    // m* = 0
    if (valid && origin) {
        double rho = k[0] * k[0];
        if (D > 1) rho = fma(k[1], k[1], rho);
        if (D > 2) rho = fma(k[2], k[2], rho);
        const double a = alpha * rho;
        if (a <= acut) {
            const double ex = ez_expm(a);
            const double inv = ez_rcp(a);
            double E1 = 0.0;
            if (need_e1) E1 = (a < 0.25) ? ez_e1_series(a) : ex * ez_e1w_scaled(inv);
            const double Eh = need_half ? ((a < 0.25) ? ez_ehalf(a) : ex * inv * ez_ehw_scaled(inv)) : 0.0;
#pragma unroll
            for (int i = 0; i < NNU; ++i)
                acck[i] += pset_ep<SET>(args.prog, i, a, ex, inv, E1, Eh);
        }
    }
    int n_near = 0, n_mid = 0;
    for (int base = q0; base < q1; base += 64) {
        // the chunk's entries, one per lane (a prefetch of the next chunk held 14 more
        // registers)
        const int q = base + lane;
        const bool in = q < q1;
        double d2 = 0.0;
        {
            const double *e = kt + (size_t)(in ? q : base) * 4;
            const double t0 = e[0] + c[0];
            d2 = t0 * t0;
            if (D > 1) { const double t1 = e[1] + c[1]; d2 = fma(t1, t1, d2); }
            if (D > 2) { const double t2 = e[2] + c[2]; d2 = fma(t2, t2, d2); }
        }
        const bool near = in && d2 <= rnear2;
        const bool mid = in && !near && d2 <= rmid2;
        const bool keep = in && !near && !mid && d2 <= rmax2;
        const bool lo32 = MIX && keep && d2 >= r32sq;
        wave_append(near, q, nearl, EZ_NEAR_MAX, &n_near);
        wave_append(mid, q, midl, EZ_MID_MAX, &n_mid);
        unsigned long long bal = __ballot(keep && !lo32);
        while (bal) {
            const int j = __builtin_ctzll(bal);
            bal &= bal - 1ull;
            const double *e = kt + (size_t)(base + j) * 4;
            double qx = e[0] + k[0];
            double rho = qx * qx;
            if (D > 1) { const double qy = e[1] + k[1]; rho = fma(qy, qy, rho); }
            if (D > 2) { const double qz = e[2] + k[2]; rho = fma(qz, qz, rho); }
            const double a = alpha * rho;
            if (a <= acut) {
                const double ex = ez_expm_tab(a, exptab);
                double E1, Eh, inv;
                ez_far_bases(a, ex, need_e1, need_half, &E1, &Eh, &inv);
#pragma unroll
                for (int i = 0; i < NNU; ++i)
                    acck[i] += pset_ep<SET>(args.prog, i, a, ex, inv, E1, Eh);
            }
        }
        if constexpr (MIX) {
            // the chunk's FP32 far field: at most 64 terms summed in FP32 per exponent,
            // then added to the FP64 sums (and to far32, for the error bound)
            unsigned long long b32 = __ballot(lo32);
            if (b32) {
                float accf[NNU];
#pragma unroll
                for (int i = 0; i < NNU; ++i) accf[i] = 0.0f;
                while (b32) {
                    const int j = __builtin_ctzll(b32);
                    b32 &= b32 - 1ull;
                    const double *e = kt + (size_t)(base + j) * 4;
                    double qx = e[0] + k[0];
                    double rho = qx * qx;
                    if (D > 1) { const double qy = e[1] + k[1]; rho = fma(qy, qy, rho); }
                    if (D > 2) { const double qz = e[2] + k[2]; rho = fma(qz, qz, rho); }
                    const double a = alpha * rho;
                    if (a <= acut) far32_term<SET, NNU>(args, a, accf);
                }
#pragma unroll
                for (int i = 0; i < NNU; ++i) {
                    acck[i] += (double)accf[i];
                    far32[i] += (double)accf[i];
                }
            }
        }
    }
    if (n_near > EZ_NEAR_MAX || n_mid > EZ_MID_MAX) {
#pragma unroll
        for (int i = 0; i < NNU; ++i) acck[i] = __longlong_as_double(0x7ff8000000000000ll);
        return;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int j = 0; j < n_mid; ++j) {
        const double *e = kt + (size_t)__builtin_amdgcn_readfirstlane((int)midl[j]) * 4;
        double rho = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) { const double t = e[i] + k[i]; rho = fma(t, t, rho); }
        const double a = alpha * rho;
        if (a <= acut) {
            const double ex = ez_expm(a);
            const double inv = ez_rcp(a);
            const double E1 = need_e1 ? ex * ez_e1w_scaled(inv) : 0.0;
            const double Eh = need_half ? ex * inv * ez_ehw_scaled(inv) : 0.0;
#pragma unroll
            for (int i = 0; i < NNU; ++i)
                acck[i] += pset_ep<SET>(args.prog, i, a, ex, inv, E1, Eh);
        }
    }
    for (int j = 0; j < n_near; ++j) {
        const double *e = kt + (size_t)__builtin_amdgcn_readfirstlane((int)nearl[j]) * 4;
        double rho = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) { const double t = e[i] + k[i]; rho = fma(t, t, rho); }
        const double a = alpha * rho;
        if (a <= acut) {
            const double ex = ez_expm(a);
            const double inv = ez_rcp(a);
            const double E1 = need_e1 ? ez_e1_ool(a) : 0.0;
            const double Eh = need_half ? ez_ehalf_ool(a) : 0.0;
#pragma unroll
            for (int i = 0; i < NNU; ++i)
                acck[i] += pset_ep<SET>(args.prog, i, a, ex, inv, E1, Eh);
        }
    }
}

// First-order bound of the change of the node's weighted products when each Z_i
// moves by at most dZ_i: sum over terms of |coef| W sum_f m_f dZ_f |Z_f|^{m_f - 1}
// prod_{g != f} |Z_g|^{m_g}, added to rb (the second-order part is smaller by a
// factor dZ/|Z| <= 1e-9 and is covered by the margin of the per-term bounds)
template <int NNU>
__device__ __forceinline__ void node_product_bounds(const EzQuadArgs &args, const double *Z, const double *dZ,
                                                    double W, double *rb) {
    for (int t = 0; t < args.prog.n_terms; ++t) {
        const int nf = args.prog.term_nfac[t];
        double b = 0.0;
        for (int f = 0; f < nf; ++f) {
            const int fi = args.prog.term_fac[t][f];
            double dz = dZ[0];
#pragma unroll
            for (int i = 1; i < NNU; ++i) dz = (fi == i) ? dZ[i] : dz;
            double part = (double)args.prog.term_mult[t][f] * dz;
            for (int g = 0; g < nf; ++g) {
                const int gi = args.prog.term_fac[t][g];
                double z = Z[0];
#pragma unroll
                for (int i = 1; i < NNU; ++i) z = (gi == i) ? Z[i] : z;
                const int mg = args.prog.term_mult[t][g] - (g == f ? 1 : 0);
                for (int m = 0; m < mg; ++m) part *= fabs(z);
            }
            b += part;
        }
        const int rr = args.prog.term_res[t];
#pragma unroll
        for (int r = 0; r < EZ_RES_MAX; ++r)
            if (rr == r) rb[r] += fabs(args.prog.term_coef[t]) * b * W;
    }
}

// Z_nu = real part + K_nu (reciprocal part) - self term, then the weighted
// products of the program's terms added to res; with far32 (mixed precision) the
// bound of the products' change from the FP32 far-field sums is added to rb
template <int NNU>
__device__ __forceinline__ void node_products(const EzQuadArgs &args, const EzLatMeta *M, const double *accr,
                                              const double *acck, double W, double *res,
                                              const double *far32 = nullptr, double *rb = nullptr) {
    double Z[NNU];
#pragma unroll
    for (int i = 0; i < NNU; ++i) Z[i] = accr[i] + M->K[i] * acck[i] - M->self_[i];
    if (far32) {
        double dZ[NNU];
#pragma unroll
        for (int i = 0; i < NNU; ++i) dZ[i] = args.mix_eps[i] * fabs(M->K[i]) * far32[i];
        node_product_bounds<NNU>(args, Z, dZ, fabs(W), rb);
    }
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

// LDS of the split kernel.  kpool holds the culled reciprocal list (unsigned
// short) and, once the list is done, the partial sums.
template <int NW>
struct NodeLds {
    double kpool[EZ_KCULL / 4];
    double kbox[NW][6];
    double red[EZ_RES_MAX][EZ_TILE / 64][2];
    int kwave[NW];
    int kcount;
};
using TailLds = NodeLds<EZ_TAIL_WAVES>;

// LDS of the tile kernel: each wave's near and mid lists, the tile reduction.  A
// half-tile workgroup passes its odd waves' sums to the even waves through `xch`,
// which takes the place of the table and the lists once every wave has summed.
struct TileTables {
    double exptab[EZ_EXP2_TAB_N];
    unsigned short nearl[EZ_TILE / 64][EZ_NEAR_MAX];
    unsigned short midl[EZ_TILE / 64][EZ_MID_MAX];
};
struct TileLds {
    union {
        TileTables t;
        double xch[EZ_TILE / 128][4][64];
    } u;
    double red[EZ_RES_MAX][EZ_TILE / 64][2];
    double rbnd[EZ_RES_MAX][EZ_TILE / 64];
};

// One node tile: four wave blocks of the lattice, each wave culls and sums on its own.
//
// half = 0 or 1: a tile of the tail of a call whose tiles pass a multiple of a round
// of workgroups by a large part of a round.  Its last round would run at about half
// the occupancy of the others, and waves alone on a SIMD are latency-bound, so each
// tail tile goes to two workgroups: workgroup `half` takes wave blocks 2 half and
// 2 half + 1, wave 2j + p of it takes block 2 half + j with part p of the terms:
// real-space rows [p n_rows/2, (p+1) n_rows/2), reciprocal entries [1, q_m) with
// m* = 0 (p = 0) or [q_m, n_rec) (p = 1), q_m on a 64-entry chunk boundary.  The
// even wave adds the odd wave's sums to its own (part 0 + part 1, in that order),
// forms the products, and the workgroup's partial goes to sub_part.
template <int D, int NNU, int SET, bool MIX = false>
__device__ __forceinline__ void node_tile(const EzQuadArgs &args, const int tile, TileLds &L, const int half = -1) {
    const int inst = find_segment(args.tile_begin, args.batch, tile);
    const EzInstPlan P = args.plans[inst];
    const EzLatMeta *M = args.meta + inst;
    const int n_res = args.prog.n_res;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool split = half >= 0;                   // uniform over the workgroup
    // uniform over the wave: kept in scalar registers, so that the entry loops below
    // keep their table reads on the scalar path
    const int part = __builtin_amdgcn_readfirstlane(split ? (wave & 1) : 0);
    const int wb = (tile - args.tile_begin[inst]) * (EZ_TILE / 64) + (split ? 2 * half + (wave >> 1) : wave);

    double res[EZ_RES_MAX], rbound[EZ_RES_MAX];
#pragma unroll
    for (int r = 0; r < EZ_RES_MAX; ++r) { res[r] = 0.0; rbound[r] = 0.0; }
    for (int j = (int)threadIdx.x; j < EZ_EXP2_TAB_N; j += EZ_TILE) L.u.t.exptab[j] = ez_exp2_tab[j];
    __syncthreads();

    const bool ok = M->status == 0 && wb < P.n_wblk;   // uniform over the wave
    bool valid = false;
    double W = 0.0;
    double accr[NNU], acck[NNU], far32[NNU];
#pragma unroll
    for (int i = 0; i < NNU; ++i) { accr[i] = 0.0; acck[i] = 0.0; far32[i] = 0.0; }
    if (ok) {
        int dir, iu;
        valid = block_node(P, wb, lane, &dir, &iu);
        double k[3], th[3];
        node_geometry<D>(P, args.rules, M, dir, iu, k, th, &W);

        const double *kt = args.tab.rec + (size_t)inst * args.tab.rec_cap * 4;
        const int n_rec = M->n_rec, n_rows = M->n_rows;
        int q0 = 1, q1 = n_rec, r0 = 0, r1 = n_rows;
        if (split) {
            const int qm = min(n_rec, 1 + 64 * (((n_rec - 1) / 2 + 63) / 64));
            q0 = __builtin_amdgcn_readfirstlane(part ? qm : 1);
            q1 = __builtin_amdgcn_readfirstlane(part ? n_rec : qm);
            r0 = __builtin_amdgcn_readfirstlane(part ? n_rows / 2 : 0);
            r1 = __builtin_amdgcn_readfirstlane(part ? n_rows : n_rows / 2);
        }
        if (valid) real_rows<D, NNU>(args, inst, th, r0, r1, accr);
        rec_wave<D, NNU, SET, MIX>(args, kt, q0, q1, part == 0, k, valid, M->alpha, M->a_cut, L.u.t.nearl[wave],
                                   L.u.t.midl[wave], L.u.t.exptab, acck, far32);
    }
    if (split) {
        // the odd waves' sums (and FP32 far-field sums of mixed calls) to the even
        // waves, four values per pass
        constexpr int NV = (MIX ? 3 : 2) * NNU;
#pragma unroll
        for (int c0 = 0; c0 < NV; c0 += 4) {
            __syncthreads();                        // the table, lists or last pass are read
            if (part == 1) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int c = c0 + u;
                    if (c < NV)
                        L.u.xch[wave >> 1][u][lane] = c < NNU ? accr[c] : (c < 2 * NNU ? acck[c - NNU] : far32[c - 2 * NNU]);
                }
            }
            __syncthreads();
            if (part == 0) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int c = c0 + u;
                    if (c < NNU) accr[c] += L.u.xch[wave >> 1][u][lane];
                    else if (c < 2 * NNU) acck[c - NNU] += L.u.xch[wave >> 1][u][lane];
                    else if (c < NV) far32[c - 2 * NNU] += L.u.xch[wave >> 1][u][lane];
                }
            }
        }
    }
    if (ok && valid && part == 0) {
        if constexpr (MIX) node_products<NNU>(args, M, accr, acck, W, res, far32, rbound);
        else node_products<NNU>(args, M, accr, acck, W, res);
    }

    // tile reduction: wave butterflies, then the four waves in fixed order
#pragma unroll
    for (int r = 0; r < EZ_RES_MAX; ++r) {
        if (r < n_res) {
            ez_dd v = ez_dd_wave_sum(ez_dd{res[r], 0.0});
            if (lane == 0) { L.red[r][wave][0] = v.hi; L.red[r][wave][1] = v.lo; }
        }
    }
    if constexpr (MIX) {                          // the bound: plain sums in fixed order
#pragma unroll
        for (int r = 0; r < EZ_RES_MAX; ++r) {
            if (r < n_res) {
                double v = rbound[r];
#pragma unroll
                for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
                if (lane == 0) L.rbnd[r][wave] = v;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < n_res) {
        const int r = threadIdx.x;
        ez_dd s{L.red[r][0][0], L.red[r][0][1]};
        for (int wv = 1; wv < EZ_TILE / 64; ++wv) s = ez_dd_add(s, ez_dd{L.red[r][wv][0], L.red[r][wv][1]});
        if (split) {
            const size_t g = (size_t)(tile - args.n_main) * (EZ_TILE / 64) + half;
            args.sub_part[(g * n_res + r) * 2 + 0] = s.hi;
            args.sub_part[(g * n_res + r) * 2 + 1] = s.lo;
            args.sub_part[((g + 2) * n_res + r) * 2 + 0] = 0.0;
            args.sub_part[((g + 2) * n_res + r) * 2 + 1] = 0.0;
        } else {
            args.tile_part[((size_t)tile * n_res + r) * 2 + 0] = s.hi;
            args.tile_part[((size_t)tile * n_res + r) * 2 + 1] = s.lo;
        }
        if constexpr (MIX) {
            // half 1 of a tail tile: the slot n_tiles + (tile - n_main)
            double b = L.rbnd[r][0];
            for (int wv = 1; wv < EZ_TILE / 64; ++wv) b += L.rbnd[r][wv];
            const size_t slot = half == 1 ? (size_t)args.n_tiles + (tile - args.n_main) : (size_t)tile;
            args.tile_bound[slot * n_res + r] = b;
        }
    }
}

// The last tiles of a call.  The tile kernel's workgroups run in rounds of (CUs x
// workgroups per CU); when the tile count is just above a multiple of a round, the
// last round holds a few tiles whose waves then run alone on their SIMDs for about
// the time of a full round.  The host hands those tiles [n_main, n_tiles) to the
// split kernel instead, launched after the tile kernel with one workgroup per CU:
// each 64-node group of a tail tile is shared by EZ_TAIL_PARTS workgroups of
// EZ_TAIL_WAVES waves, and wave s of part p takes the (EZ_TAIL_WAVES p + s)-th of
// EZ_TAIL_WAVES EZ_TAIL_PARTS contiguous shares of the real-space rows and of the
// culled reciprocal list (share 0 also m* = 0) for all 64 nodes.  A workgroup adds
// its waves' partial sums in LDS in wave order.  With several parts, each stores
// its sums and the last of the group's workgroups to finish (a counter, reset by
// that workgroup) adds the stored parts in part order; wave 0 of the workgroup
// holding the total forms the products and writes the 64-node partial to
// sub_part.  The finalize kernel adds the four partials of a tile in the order the
// tile path adds its four waves.
template <int D, int NNU, int SET>
__device__ __forceinline__ void node_group_split(const EzQuadArgs &args, const int g, const int p, TailLds &L) {
    constexpr int NS = EZ_TAIL_WAVES;             // waves per workgroup
    constexpr int NSH = NS * EZ_TAIL_PARTS;       // shares of a group's terms
    constexpr int GPT = EZ_TILE / 64;             // 64-node groups per tile
    const int tile = args.n_main + g / GPT;
    const int quarter = g % GPT;
    const int lane = (int)threadIdx.x & 63, s = (int)threadIdx.x >> 6;
    const int j = p * NS + s;                     // this wave's share
    const int inst = find_segment(args.tile_begin, args.batch, tile);
    const EzInstPlan P = args.plans[inst];
    const EzLatMeta *M = args.meta + inst;
    const int n_res = args.prog.n_res;
    const int wb = (tile - args.tile_begin[inst]) * GPT + quarter;   // the group is this wave block
    unsigned short *klist = reinterpret_cast<unsigned short *>(L.kpool);

    // uniform over the workgroup: lattice flags, a block past the lattice's last
    const bool ok = M->status == 0 && wb < P.n_wblk;
    int dir, iu;
    const bool valid = block_node(P, wb, lane, &dir, &iu);
    double accr[NNU], acck[NNU], W = 0.0;
#pragma unroll
    for (int i = 0; i < NNU; ++i) { accr[i] = 0.0; acck[i] = 0.0; }
    if (ok) {
        double k[3], th[3];
        node_geometry<D>(P, args.rules, M, dir, iu, k, th, &W);
        const double *kt = args.tab.rec + (size_t)inst * args.tab.rec_cap * 4;
        const double alpha = M->alpha, acut = M->a_cut;
        int n_near = 0;
        const int nk = cull_reciprocal<D, 64 * NS>(kt, M->n_rec, k, alpha, acut, klist, L.kbox, L.kwave, &L.kcount,
                                                   &n_near);
        if (valid) {
            const int n_rows = M->n_rows;
            real_rows<D, NNU>(args, inst, th, j * n_rows / NSH, (j + 1) * n_rows / NSH, accr);
            if (j == 0) rec_origin<D, NNU, SET>(args, kt, klist, n_near, k, alpha, acut, acck);
            rec_list<D, NNU, SET>(args, kt, klist, j * nk / NSH, (j + 1) * nk / NSH, k, alpha, acut, acck);
        }
    }
    __syncthreads();                              // the list is done: kpool takes the partial sums
    double *acc = L.kpool;                        // [2 NNU][64]
    for (int w = 0; w < NS; ++w) {
        if (s == w) {
#pragma unroll
            for (int i = 0; i < NNU; ++i) {
                acc[i * 64 + lane] = (w == 0) ? accr[i] : acc[i * 64 + lane] + accr[i];
                acc[(NNU + i) * 64 + lane] = (w == 0) ? acck[i] : acc[(NNU + i) * 64 + lane] + acck[i];
            }
        }
        __syncthreads();
    }
    if (s != 0) return;

    double res[EZ_RES_MAX];
#pragma unroll
    for (int r = 0; r < EZ_RES_MAX; ++r) res[r] = 0.0;
    if constexpr (EZ_TAIL_PARTS > 1) {
        // wave 0: store this part; the group's last part adds them all
        constexpr int PART = 2 * NNU * 64;
        double *mine = args.tail_acc + ((size_t)g * EZ_TAIL_PARTS + p) * PART;
#pragma unroll
        for (int i = 0; i < 2 * NNU; ++i) mine[i * 64 + lane] = acc[i * 64 + lane];
        __threadfence();
        int old = 0;
        if (lane == 0) old = atomicAdd(args.tail_cnt + g, 1);
        old = __shfl(old, 0, 64);
        if (old != EZ_TAIL_PARTS - 1) return;
        __threadfence();
        if (lane == 0) args.tail_cnt[g] = 0;      // ready for the next call
        if (ok && valid) {
            const double *parts = args.tail_acc + (size_t)g * EZ_TAIL_PARTS * PART;
#pragma unroll
            for (int i = 0; i < NNU; ++i) {
                double a = parts[i * 64 + lane], b = parts[(NNU + i) * 64 + lane];
                for (int q = 1; q < EZ_TAIL_PARTS; ++q) {
                    a += parts[(size_t)q * PART + i * 64 + lane];
                    b += parts[(size_t)q * PART + (NNU + i) * 64 + lane];
                }
                accr[i] = a;
                acck[i] = b;
            }
            node_products<NNU>(args, M, accr, acck, W, res);
        }
    } else if (ok && valid) {
#pragma unroll
        for (int i = 0; i < NNU; ++i) { accr[i] = acc[i * 64 + lane]; acck[i] = acc[(NNU + i) * 64 + lane]; }
        node_products<NNU>(args, M, accr, acck, W, res);
    }
#pragma unroll
    for (int r = 0; r < EZ_RES_MAX; ++r) {
        if (r < n_res) {
            ez_dd v = ez_dd_wave_sum(ez_dd{res[r], 0.0});
            if (lane == 0) {
                args.sub_part[((size_t)g * n_res + r) * 2 + 0] = v.hi;
                args.sub_part[((size_t)g * n_res + r) * 2 + 1] = v.lo;
            }
        }
    }
}

// one workgroup per tile (tiles [0, n_main)); MIX: the mixed-precision far field
// waves per SIMD the compiler is held to: one more than the registers alone allow for
// the ATM (4 exponents, 8) and scan (7 exponents, 6) sets, at the cost of a few
// bytes of spill
template <int NNU, int SET>
constexpr int node_waves() { return (SET == 1) ? 8 : (SET == 4 ? 6 : 1); }

template <int D, int NNU, int SET, bool MIX = false>
__global__ __launch_bounds__(EZ_TILE) __attribute__((amdgpu_waves_per_eu(node_waves<NNU, SET>())))
void ez_node_kernel(EzQuadArgs args) {
    __shared__ TileLds L;
    // workgroups [0, n_main) take whole tiles; with tail_halves, workgroup n_main + 2 t + h
    // takes half h of tail tile n_main + t
    const int b = (int)blockIdx.x;
    int tile = b, half = -1;
    if (args.tail_halves && b >= args.n_main) {
        tile = args.n_main + ((b - args.n_main) >> 1);
        half = (b - args.n_main) & 1;
    }
    node_tile<D, NNU, SET, MIX>(args, tile, L, half);
}

// mixed precision held to 8 waves per SIMD (64 registers, a few bytes of spill)
template <int D, int NNU, int SET>
__global__ __launch_bounds__(EZ_TILE) __attribute__((amdgpu_waves_per_eu(8))) void ez_node_mix_kernel(EzQuadArgs args) {
    __shared__ TileLds L;
    const int b = (int)blockIdx.x;
    int tile = b, half = -1;
    if (args.tail_halves && b >= args.n_main) {
        tile = args.n_main + ((b - args.n_main) >> 1);
        half = (b - args.n_main) & 1;
    }
    node_tile<D, NNU, SET, true>(args, tile, L, half);
}

// persistent: a fixed grid of workgroups takes tiles from a queue, costliest first;
// every workgroup leaves once the queue position passes the last tile.  Tiles from
// n_main on are left to the split kernel.
template <int D, int NNU, int SET>
__global__ __launch_bounds__(EZ_TILE) void ez_node_persist_kernel(EzQuadArgs args) {
    __shared__ TileLds L;
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(args.queue, 1);
        __syncthreads();
        // the tile index is uniform over the workgroup: keep it in scalar registers
        const int t = __builtin_amdgcn_readfirstlane(next);
        __syncthreads();
        if (t >= args.n_tiles) break;
        const int tile = __builtin_amdgcn_readfirstlane(args.tile_order[t]);
        if (tile < args.n_main) node_tile<D, NNU, SET>(args, tile, L);
    }
}

// the tail: workgroup b takes part b % EZ_TAIL_PARTS of 64-node group b / EZ_TAIL_PARTS
template <int D, int NNU, int SET>
__global__ __launch_bounds__(64 * EZ_TAIL_WAVES) void ez_node_split_kernel(EzQuadArgs args) {
    __shared__ TailLds L;
    const int b = (int)blockIdx.x;
    node_group_split<D, NNU, SET>(args, b / EZ_TAIL_PARTS, b % EZ_TAIL_PARTS, L);
}

__global__ void ez_fill_int_kernel(int *p, int n, int value) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}


// ---------------------------------------------------------------------------
// partial of tile t: from the tile kernels, or the split kernel's four 64-node
// partials added in the order of the tile kernel's four waves
__device__ __forceinline__ ez_dd tile_value(const EzQuadArgs &args, int t, int r, int n_res) {
    if (t < args.n_main)
        return ez_dd{args.tile_part[((size_t)t * n_res + r) * 2], args.tile_part[((size_t)t * n_res + r) * 2 + 1]};
    const size_t g0 = (size_t)(t - args.n_main) * (EZ_TILE / 64);
    ez_dd s{args.sub_part[(g0 * n_res + r) * 2], args.sub_part[(g0 * n_res + r) * 2 + 1]};
    for (int q = 1; q < EZ_TILE / 64; ++q)
        s = ez_dd_add(s, ez_dd{args.sub_part[((g0 + q) * n_res + r) * 2], args.sub_part[((g0 + q) * n_res + r) * 2 + 1]});
    return s;
}

// one workgroup of FT threads per lattice (the sums are short: latency-bound)
constexpr int FT = 1024;

__global__ __launch_bounds__(FT) void ez_finalize_kernel(EzQuadArgs args) {
    const int inst = blockIdx.x;
    const int n_res = args.prog.n_res;
    const int tb = args.tile_begin[inst], te = args.tile_begin[inst + 1];
    const int db = args.dir_begin[inst], de = args.dir_begin[inst + 1];
    __shared__ double red[FT / 64][2];
    __shared__ uint32_t flag_sh;
    if (threadIdx.x == 0) flag_sh = 0;
    __syncthreads();
    uint32_t fl = 0;
    for (int g = db + (int)threadIdx.x; g < de; g += FT) fl |= args.dir_flag[g];
    if (fl) atomicOr(&flag_sh, 1u);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int r = 0; r < n_res; ++r) {
        ez_dd s{0.0, 0.0};
        for (int t = tb + (int)threadIdx.x; t < te; t += FT)
            s = ez_dd_add(s, tile_value(args, t, r, n_res));
        for (int g = db + (int)threadIdx.x; g < de; g += FT)
            s = ez_dd_add_d(s, args.dir_part[(size_t)g * n_res + r]);
        s = ez_dd_wave_sum(s);
        __syncthreads();
        if (lane == 0) { red[wave][0] = s.hi; red[wave][1] = s.lo; }
        __syncthreads();
        if (threadIdx.x == 0) {
            ez_dd tot{red[0][0], red[0][1]};
            for (int w = 1; w < FT / 64; ++w) tot = ez_dd_add(tot, ez_dd{red[w][0], red[w][1]});
            double v = tot.hi + tot.lo;
            uint32_t st = args.meta[inst].status;
            if (flag_sh) st |= 0x8u;
            if (st) v = __longlong_as_double(0x7ff8000000000000ll);
            else if (!isfinite(v)) st |= 0x4u;
            args.out[(size_t)inst * n_res + r] = v;
            if (args.status && r == 0) args.status[inst] = st;
        }
    }
    if (args.bound_out) {
        // a-priori bound of the FP32 far field's effect on each result: the tile bounds
        // (mixed calls keep every tile in the tile kernel) added by a fixed tree, each
        // thread a strided share, then the waves in order; 0 in FP64 calls
        for (int r = 0; r < n_res; ++r) {
            double b = 0.0;
            if (args.mixed) {
                for (int t = tb + (int)threadIdx.x; t < te; t += FT) b += args.tile_bound[(size_t)t * n_res + r];
                // second halves of the lattice's tail tiles
                if (args.tail_halves)
                    for (int t = max(tb, args.n_main) + (int)threadIdx.x; t < te; t += FT)
                        b += args.tile_bound[((size_t)args.n_tiles + (t - args.n_main)) * n_res + r];
            }
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) b += __shfl_xor(b, m, 64);
            __syncthreads();
            if (lane == 0) red[wave][0] = b;
            __syncthreads();
            if (threadIdx.x == 0) {
                double tot = red[0][0];
                for (int w = 1; w < FT / 64; ++w) tot += red[w][0];
                args.bound_out[(size_t)inst * n_res + r] =
                    args.meta[inst].status ? __longlong_as_double(0x7ff8000000000000ll) : tot;
            }
        }
    }
    if (!args.grad_out) return;
    // d result / d A = S A^{-T}, S the symmetric strain derivative (d(d+1)/2 components),
    // all components summed in one sweep: each in the same fixed order as the value
    const int d = args.prog.d, ns = d * (d + 1) / 2;
    __shared__ double Ssh[6];
    __shared__ double red6[FT / 64][6][2];
    for (int r = 0; r < n_res; ++r) {
        ez_dd s[6];
#pragma unroll
        for (int sc = 0; sc < 6; ++sc) s[sc] = ez_dd{0.0, 0.0};
        for (int t = tb + (int)threadIdx.x; t < te; t += FT) {
            const double *tg = args.tile_grad + ((size_t)t * n_res + r) * 12;
#pragma unroll
            for (int sc = 0; sc < 6; ++sc)
                if (sc < ns) s[sc] = ez_dd_add(s[sc], ez_dd{tg[2 * sc], tg[2 * sc + 1]});
        }
        for (int g = db + (int)threadIdx.x; g < de; g += FT) {
            const double *dg = args.dir_grad + ((size_t)g * n_res + r) * 6;
#pragma unroll
            for (int sc = 0; sc < 6; ++sc)
                if (sc < ns) s[sc] = ez_dd_add_d(s[sc], dg[sc]);
        }
#pragma unroll
        for (int sc = 0; sc < 6; ++sc) s[sc] = ez_dd_wave_sum(s[sc]);
        __syncthreads();
        if (lane == 0) {
#pragma unroll
            for (int sc = 0; sc < 6; ++sc) { red6[wave][sc][0] = s[sc].hi; red6[wave][sc][1] = s[sc].lo; }
        }
        __syncthreads();
        if ((int)threadIdx.x < ns) {
            const int sc = (int)threadIdx.x;
            ez_dd tot{red6[0][sc][0], red6[0][sc][1]};
            for (int w = 1; w < FT / 64; ++w) tot = ez_dd_add(tot, ez_dd{red6[w][sc][0], red6[w][sc][1]});
            Ssh[sc] = tot.hi + tot.lo;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const EzLatMeta *M = args.meta + inst;
            double Sf[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int a = 0; a < d; ++a) Sf[a][a] = Ssh[a];
            if (d > 1) { Sf[0][1] = Sf[1][0] = Ssh[d]; }
            if (d > 2) { Sf[0][2] = Sf[2][0] = Ssh[d + 1]; Sf[1][2] = Sf[2][1] = Ssh[d + 2]; }
            const bool bad = M->status != 0 || flag_sh;
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) {
                    double g = 0.0;
                    for (int c = 0; c < d; ++c) g = fma(Sf[a][c], M->B[c * d + b], g);
                    args.grad_out[(((size_t)inst * n_res + r) * d + a) * d + b] =
                        bad ? __longlong_as_double(0x7ff8000000000000ll) : g;
                }
        }
        __syncthreads();
    }
}

// mode 0: one workgroup per tile (n = tiles); mode 1: persistent (n = workgroups);
// mode 2: report the persistent kernel's resident workgroups per CU in *bpc;
// mode 3: split kernel (n = workgroups); mode 4: the tile kernel's workgroups per CU
template <int D, int NNU, int SET = 0>
hipError_t launch_nodes_t(const EzQuadArgs &args, int n_tiles, hipStream_t stream, int mode = 0, int *bpc = nullptr) {
    if (mode == 2) {
        static int cached = 0;
        if (!cached) {
            int nb = 0;
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ez_node_persist_kernel<D, NNU, SET>,
                                                                        EZ_TILE, 0);
            if (e != hipSuccess) return e;
            cached = nb > 0 ? nb : 1;
        }
        *bpc = cached;
        return hipSuccess;
    }
    if (mode == 4) {
        static int cached_t = 0;
        if (!cached_t) {
            int nb = 0;
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ez_node_kernel<D, NNU, SET>, EZ_TILE, 0);
            if (e != hipSuccess) return e;
            cached_t = nb > 0 ? nb : 1;
        }
        *bpc = cached_t;
        return hipSuccess;
    }
    if (mode == 3) {
        // unused dynamic LDS (more than half a CU's LDS with the static part, within the
        // per-workgroup limit) keeps the split kernel at one workgroup per CU, so that
        // its few workgroups spread over the device instead of filling a few CUs
        static int pad = -1;
        if (pad < 0) {
            hipFuncAttributes fa;
            int dev = 0, per_cu = 0, per_blk = 0;
            hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&ez_node_split_kernel<D, NNU, SET>));
            if (e == hipSuccess) e = hipGetDevice(&dev);
            if (e == hipSuccess) e = hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
            if (e == hipSuccess) e = hipDeviceGetAttribute(&per_blk, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
            if (e != hipSuccess) return e;
            const long want = (long)per_cu / 2 + 1024 - (long)fa.sharedSizeBytes;
            const long cap = (long)per_blk - (long)fa.sharedSizeBytes;
            pad = (int)std::max(0L, std::min(want, cap));
        }
        hipLaunchKernelGGL((ez_node_split_kernel<D, NNU, SET>), dim3(n_tiles), dim3(64 * EZ_TAIL_WAVES), pad, stream, args);
    } else if (mode == 1) {
        hipLaunchKernelGGL((ez_node_persist_kernel<D, NNU, SET>), dim3(n_tiles), dim3(EZ_TILE), 0, stream, args);
    } else if (args.mixed) {
        hipLaunchKernelGGL((ez_node_mix_kernel<D, NNU, SET>), dim3(n_tiles), dim3(EZ_TILE), 0, stream, args);
    } else {
        hipLaunchKernelGGL((ez_node_kernel<D, NNU, SET>), dim3(n_tiles), dim3(EZ_TILE), 0, stream, args);
    }
    return hipGetLastError();
}

// real (non-integer) exponents: the tile kernel only (mode 0) and its occupancy (mode 4);
// such calls take no tail split, no persistent schedule and no mixed precision
template <int D, int NNU>
hipError_t launch_nodes_real(const EzQuadArgs &args, int n_tiles, hipStream_t stream, int mode, int *bpc) {
    if (mode == 4) {
        static int cached_r = 0;
        if (!cached_r) {
            int nb = 0;
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ez_node_kernel<D, NNU, EZ_PSET_REAL>,
                                                                        EZ_TILE, 0);
            if (e != hipSuccess) return e;
            cached_r = nb > 0 ? nb : 1;
        }
        *bpc = cached_r;
        return hipSuccess;
    }
    if (mode != 0 || args.mixed) return hipErrorInvalidValue;
    hipLaunchKernelGGL((ez_node_kernel<D, NNU, EZ_PSET_REAL>), dim3(n_tiles), dim3(EZ_TILE), 0, stream, args);
    return hipGetLastError();
}

template <int D>
hipError_t launch_nodes_d(const EzQuadArgs &args, int n_tiles, hipStream_t stream, int mode, int *bpc) {
    if (args.prog.real_nu) {
        switch (args.prog.n_nu) {
            case 1: return launch_nodes_real<D, 1>(args, n_tiles, stream, mode, bpc);
            case 2: return launch_nodes_real<D, 2>(args, n_tiles, stream, mode, bpc);
            case 3: return launch_nodes_real<D, 3>(args, n_tiles, stream, mode, bpc);
            case 4: return launch_nodes_real<D, 4>(args, n_tiles, stream, mode, bpc);
            case 5: return launch_nodes_real<D, 5>(args, n_tiles, stream, mode, bpc);
            case 6: return launch_nodes_real<D, 6>(args, n_tiles, stream, mode, bpc);
            case 7: return launch_nodes_real<D, 7>(args, n_tiles, stream, mode, bpc);
            case 8: return launch_nodes_real<D, 8>(args, n_tiles, stream, mode, bpc);
            default: return hipErrorInvalidValue;
        }
    }
    if (D == 3 && args.prog.pset == 1) return launch_nodes_t<D, 4, 1>(args, n_tiles, stream, mode, bpc);
    if (D == 2 && args.prog.pset == 2) return launch_nodes_t<D, 4, 2>(args, n_tiles, stream, mode, bpc);
    if (D == 1 && args.prog.pset == 3) return launch_nodes_t<D, 4, 3>(args, n_tiles, stream, mode, bpc);
    if (D == 3 && args.prog.pset == 4) return launch_nodes_t<D, 7, 4>(args, n_tiles, stream, mode, bpc);
    switch (args.prog.n_nu) {
        case 1: return launch_nodes_t<D, 1>(args, n_tiles, stream, mode, bpc);
        case 2: return launch_nodes_t<D, 2>(args, n_tiles, stream, mode, bpc);
        case 3: return launch_nodes_t<D, 3>(args, n_tiles, stream, mode, bpc);
        case 4: return launch_nodes_t<D, 4>(args, n_tiles, stream, mode, bpc);
        case 5: return launch_nodes_t<D, 5>(args, n_tiles, stream, mode, bpc);
        case 6: return launch_nodes_t<D, 6>(args, n_tiles, stream, mode, bpc);
        case 7: return launch_nodes_t<D, 7>(args, n_tiles, stream, mode, bpc);
        case 8: return launch_nodes_t<D, 8>(args, n_tiles, stream, mode, bpc);
        default: return hipErrorInvalidValue;
    }
}

hipError_t ez_launch_nodes_impl(const EzQuadArgs &args, int n_tiles, hipStream_t stream, int mode = 0,
                                int *bpc = nullptr) {
    switch (args.prog.d) {
        case 1: return launch_nodes_d<1>(args, n_tiles, stream, mode, bpc);
        case 2: return launch_nodes_d<2>(args, n_tiles, stream, mode, bpc);
        case 3: return launch_nodes_d<3>(args, n_tiles, stream, mode, bpc);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t ez_launch_nodes(const EzQuadArgs &args, int n_tiles, hipStream_t stream) {
    return ez_launch_nodes_impl(args, n_tiles, stream);
}

hipError_t ez_launch_nodes_split(const EzQuadArgs &args, hipStream_t stream) {
    const int groups = (args.n_tiles - args.n_main) * (EZ_TILE / 64);
    if (groups <= 0) return hipSuccess;
    return ez_launch_nodes_impl(args, groups * EZ_TAIL_PARTS, stream, 3);
}

int ez_nodes_tile_blocks_per_cu(const EzQuadArgs &args) {
    int bpc = 1;
    if (ez_launch_nodes_impl(args, 0, nullptr, 4, &bpc) != hipSuccess) return 1;
    return bpc;
}

hipError_t ez_launch_nodes_persistent(const EzQuadArgs &args, int n_blocks, hipStream_t stream) {
    return ez_launch_nodes_impl(args, n_blocks, stream, 1);
}

int ez_nodes_blocks_per_cu(const EzQuadArgs &args) {
    int bpc = 1;
    if (ez_launch_nodes_impl(args, 0, nullptr, 2, &bpc) != hipSuccess) return 1;
    return bpc;
}

hipError_t ez_launch_fill_int(int *p, int n, int value, hipStream_t stream) {
    hipLaunchKernelGGL(ez_fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, p, n, value);
    return hipGetLastError();
}

hipError_t ez_launch_finalize(const EzQuadArgs &args, hipStream_t stream) {
    hipLaunchKernelGGL(ez_finalize_kernel, dim3(args.batch), dim3(FT), 0, stream, args);
    return hipGetLastError();
}
