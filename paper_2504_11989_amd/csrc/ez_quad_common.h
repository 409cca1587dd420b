// ez_quad_common.h -- device helpers shared by the quadrature kernels
// (ez_nodes.hip, ez_nodes_adj.hip, ez_hadamard.hip, ez_hadamard_adj.hip).
//
// The quadrature of products of Epstein zeta functions over the Brillouin zone
// (paper, Sec. 2, Theorem (Epstein representation); Sec. 3, Corollary (Duffy
// transformation) and the meromorphic continuation):
//
//   zeta = 2 sum_{p,j} int_0^{1/2} u^{d-1} int_{[0,1]^{d-1}} f(u w(v)) dv du,
//   w(v) = A^{-T} sigma^j (p1 v1, ..., p_{d-1} v_{d-1}, 1),
//
// with u in (eps, 1/2] on quadrature nodes and u in (0, eps) through the Taylor
// expansion of Z^reg and closed-form Hadamard integrals.
//
// Direction numbering: dir = block * n_q^{d-1} + iv, block = j 2^{d-1} + ip,
// bit b of ip set <=> p_{b+1} = -1, iv = sum_b iv_b n_q^b; node = dir * n_u + iu.
#pragma once
#include "ez_internal.h"
#include "ez_math.h"
#include "ez_kernels.h"

namespace {

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

// Node of lane `lane` in wave block wb of a lattice (see EzInstPlan): the block's
// db directions x ub consecutive u-nodes.  Returns false for lanes past the last
// direction or u-node, and for blocks past the lattice's last one; invalid lanes
// of a valid block take the block's first node (geometry only).
__device__ __forceinline__ bool block_node(const EzInstPlan &P, int wb, int lane, int *dir, int *iu) {
    if (wb >= P.n_wblk) { *dir = 0; *iu = 0; return false; }
    const int dg = wb / P.n_ublk, uc = wb - dg * P.n_ublk;
    const int dd = lane >> P.ub_log2, uu = lane & ((1 << P.ub_log2) - 1);
    const int d0 = dg * P.db, u0 = uc << P.ub_log2;
    const bool ok = d0 + dd < P.n_dir && u0 + uu < P.n_u;
    *dir = ok ? d0 + dd : d0;
    *iu = ok ? u0 + uu : u0;
    return ok;
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
    if constexpr (SET == EZ_PSET_REAL) return false;
    if constexpr (SET == 0) return prog.need_e1 != 0;
    bool r = false;
    for (int i = 0; i < NNU; ++i) r = r || ((ez_pset(SET).p2[i] & 1) == 0 && ez_pset(SET).p2[i] >= 2);
    return r;
}
template <int SET, int NNU>
__device__ __forceinline__ bool pset_need_half(const EzProgram &prog) {
    if constexpr (SET == EZ_PSET_REAL) return false;
    if constexpr (SET == 0) return prog.need_half != 0;
    bool r = false;
    for (int i = 0; i < NNU; ++i) r = r || (ez_pset(SET).p2[i] & 1);
    return r;
}

// E_{p_i}(a) of exponent i: from the bases E_1, E_{1/2} and the recurrences, or, for
// real exponents, by the incomplete gamma of its own order
template <int SET>
__device__ __forceinline__ double pset_ep(const EzProgram &prog, int i, double a, double e, double inv, double E1,
                                          double Eh) {
    if constexpr (SET == EZ_PSET_REAL) return ez_ep_real(prog.preal[i], a);
    else return ez_ep_from(pset_p2<SET>(prog, i), a, e, inv, E1, Eh);
}

// The reciprocal table covers every node of the cell; a workgroup needs only the
// entries within the cutoff radius of some of its nodes.  With c and r_t the
// centre and half-diagonal of the bounding box of the workgroup's k, an entry with
// |m* + c| > sqrt(a_cut / alpha) + r_t is beyond the cutoff for every node of it.
// The others are listed in table order (so each node adds the same nonzero terms
// in the same order as over the whole table); the host keeps the table capacity
// within the list (EZ_KCULL entries).  NT threads; returns the list length.
// With knear (the value node kernels), entries that may reach an argument
// alpha |m* + k|^2 below 1/4 at a node of the workgroup (|m* + c| <= r_t +
// 1/(2 sqrt alpha): small lam, or a skewed lattice near the corners of the cell)
// go to a second list instead, in table order from klist[EZ_KCULL - 1] downward,
// and *knear receives its length: the main list then needs no series forms of
// E_1 and E_{1/2}.  Per-wave counts are packed as (main | near << 16).
template <int D, int NT>
__device__ __forceinline__ int cull_reciprocal(const double *kt, int n_rec, const double *k, double alpha, double acut,
                                               unsigned short *klist, double (*kbox)[6], int *kwave, int *kcount,
                                               int *knear = nullptr) {
    constexpr int NWV = NT / 64;
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    double bl[3] = {k[0], k[1], k[2]}, bh[3] = {k[0], k[1], k[2]};
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            bl[i] = fmin(bl[i], __shfl_xor(bl[i], m, 64));
            bh[i] = fmax(bh[i], __shfl_xor(bh[i], m, 64));
        }
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < 3; ++i) { kbox[wave][i] = bl[i]; kbox[wave][3 + i] = bh[i]; }
    if (threadIdx.x == 0) *kcount = 0;
    __syncthreads();
    double c[3] = {0.0, 0.0, 0.0}, rt2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double lo = kbox[0][i], hi = kbox[0][3 + i];
        for (int w2 = 1; w2 < NWV; ++w2) { lo = fmin(lo, kbox[w2][i]); hi = fmax(hi, kbox[w2][3 + i]); }
        c[i] = 0.5 * (lo + hi);
        rt2 += 0.25 * (hi - lo) * (hi - lo);
    }
    const double rmax = (sqrt(acut / alpha) + sqrt(rt2)) * (1.0 + 1e-9) + 1e-12;
    const bool split_near = knear != nullptr;
    const double rnear = (0.5 / sqrt(alpha) + sqrt(rt2)) * (1.0 + 1e-9) + 1e-12;
    for (int base = 1; base < n_rec; base += NT) {
        const int q = base + (int)threadIdx.x;
        bool keep = false, near = false;
        if (q < n_rec) {
            const double *e = kt + (size_t)q * 4;
            double d2 = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) { const double t = e[i] + c[i]; d2 = fma(t, t, d2); }
            near = split_near && d2 <= rnear * rnear;
            keep = !near && d2 <= rmax * rmax;
        }
        const unsigned long long bal = __ballot(keep), baln = __ballot(near);
        const unsigned long long below = (1ull << lane) - 1ull;
        if (lane == 0) kwave[wave] = __popcll(bal) | (__popcll(baln) << 16);
        __syncthreads();
        int off = *kcount;
        for (int w2 = 0; w2 < wave; ++w2) off += kwave[w2];
        // q < n_rec <= rec_cap <= EZ_KCULL, and the two lists together hold at most n_rec - 1 entries
        if (keep) klist[(off & 0xFFFF) + __popcll(bal & below)] = (unsigned short)q;
        if (near) klist[EZ_KCULL - 1 - ((off >> 16) + __popcll(baln & below))] = (unsigned short)q;
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int w2 = 0; w2 < NWV; ++w2) tot += kwave[w2];
            *kcount += tot;
        }
        __syncthreads();
    }
    const int packed = *kcount;
    if (knear) *knear = packed >> 16;
    return packed & 0xFFFF;
}

}  // namespace
