// ez_grid.hip -- Z_{Lambda,nu}(x_j, y_m) on a grid of shifts x_j and reciprocal-cell
// points y_m (paper, Sec. 2, Definition (Epstein zeta function)), with the two
// lattice sums of the incomplete-gamma split written as matrix products:
//
//   real space : R_nu[j][m] = sum_z W_nu(|z - x_j|) e^{-2 pi i y_m.z}
//                = (W_nu [cos | sin](2 pi y.z))  over the union table of z;
//   reciprocal : Q_nu[j][m] = sum_m* e^{-2 pi i m*.x_j} G_nu(|m* + y_m|^2)
//                = ([cos ; sin](2 pi m*.x) G_nu),  G_nu = K_nu E_p(pi lam^2 |m*+y|^2),
//   Z_nu = R_nu + e^{-2 pi i y.x} Q_nu - [x in Lambda] (pi/lam^2)^{nu/2}/Gamma(nu/2+1).
//
// x_j is reduced to the cell A[-1/2,1/2)^d (quasi-periodicity, phase e^{-2 pi i y.z0})
// and y_m to B[-1/2,1/2)^d (periodicity); every phase is taken in fractional
// coordinates (y.z = s.n, m*.x = h.t).  The K index (table entries) is split into
// "near" columns, entries that can be large for some x (|z| <= r_near + r_cell) or
// some y (|m*| <= r_near' + r_BZ), and "far" columns, whose weights are below
// e^{-a_near}.  FP64 precision: every column in FP64 MFMA products
// (v_mfma_f64_16x16x4).  Mixed precision: near columns in FP64 MFMA; far columns as
// split-BF16 products (a = a_hi + a_lo, three v_mfma_f32_16x16x32_bf16 per tile:
// hi*hi + hi*lo + lo*hi) accumulated in FP32 per 32-wide K chunk and in FP64 across
// chunks.  The FP64 special functions (weights, E_p) and the combination stay FP64.
#include "ez_internal.h"
#include "ez_math.h"
#include "ez_grid.h"

#include <type_traits>

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ double half_diag_g(int d, const double *M) {
    double best = 0.0;
    for (int s = 0; s < (1 << d); ++s) {
        double n2 = 0.0;
        for (int i = 0; i < d; ++i) {
            double v = 0.0;
            for (int j = 0; j < d; ++j) v += M[i * d + j] * (((s >> j) & 1) ? -1.0 : 1.0);
            n2 += v * v;
        }
        best = fmax(best, n2);
    }
    return 0.5 * sqrt(best);
}

__global__ __launch_bounds__(256) void grid_zero_kernel(double *p, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// workgroup sum of one value per thread (256 threads), result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double *sh) {
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    return sh[0] + sh[1] + sh[2] + sh[3];
}


// ---------------------------------------------------------------------------
// points: t_j = A^{-1} x_j reduced to [-1/2,1/2) (n0_j the integer part, on-lattice
// flag), s_m = A^T y_m reduced likewise.  pts_x: [n_x][8] = t(3), n0(3), xin, 0;
// pts_y: [n_y][4] = s(3), yin.
__global__ __launch_bounds__(256) void grid_points_kernel(EzGridArgs g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const EzLatMeta *M = g.meta;
    const int d = g.d;
    if (i < g.n_x) {
        double f[3] = {0, 0, 0};
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c) f[r] += M->B[c * d + r] * g.x[(size_t)i * d + c];
        double *o = g.pts_x + (size_t)i * 8;
        bool xin = true;
        for (int r = 0; r < 3; ++r) {
            const double n0 = (r < d) ? rint(f[r]) : 0.0;
            double t = (r < d) ? f[r] - n0 : 0.0;
            if (fabs(t) < 1e-12) t = 0.0; else xin = false;
            o[r] = t;
            o[3 + r] = n0;
        }
        o[6] = xin ? 1.0 : 0.0;
        o[7] = 0.0;
    }
    if (i < g.n_y) {
        double f[3] = {0, 0, 0};
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c) f[r] += M->A[c * d + r] * g.y[(size_t)i * d + c];
        double *o = g.pts_y + (size_t)i * 4;
        bool yin = true;
        for (int r = 0; r < 3; ++r) {
            double s = (r < d) ? f[r] - rint(f[r]) : 0.0;
            if (fabs(s) < 1e-12) s = 0.0; else yin = false;
            o[r] = s;
        }
        o[3] = yin ? 1.0 : 0.0;
    }
}

// stable compaction step of a 256-thread workgroup: slot of this thread's item
// (or -1) among the kept items, after *count kept earlier; advances *count
__device__ int grid_compact(bool keep, int *wave_tot, int *count) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long m = __ballot(keep);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wave_tot[wave] = __popcll(m);
    __syncthreads();
    int off = *count;
    for (int w = 0; w < wave; ++w) off += wave_tot[w];
    const int slot = keep ? off + before : -1;
    __syncthreads();
    if (threadIdx.x == 0) *count += wave_tot[0] + wave_tot[1] + wave_tot[2] + wave_tot[3];
    __syncthreads();
    return slot;
}

// near/far split of the table columns, near first, table order kept within each
// part (deterministic), and the reciprocal prefactors
//   K_nu = pi^{nu - d/2} / (Gamma(nu/2) V) (pi lam^2)^{(d - nu)/2}
// counts: [0] near real, [1] far real, [2] near reciprocal, [3] far reciprocal
__global__ __launch_bounds__(256) void grid_classify_kernel(EzGridArgs g) {
    __shared__ int wave_tot[4];
    __shared__ int count;
    const EzLatMeta *M = g.meta;
    const int d = g.d;
    const double rcell = half_diag_g(d, M->A), rbz = half_diag_g(d, M->B);
    const double rn = M->lam * sqrt(g.a_near / EZ_PI) + rcell;
    const double rk = sqrt(g.a_near / EZ_PI) / M->lam + rbz;
    const int nr = M->status ? 0 : M->n_real, nk = M->status ? 0 : M->n_rec;
    if (threadIdx.x < g.n_nu) {
        const double nu = g.nu[threadIdx.x];
        g.kpref[threadIdx.x] = pow(EZ_PI, nu - 0.5 * d) * ez_rgamma(0.5 * nu) / M->V * pow(M->alpha, 0.5 * (d - nu));
    }
    for (int part = 0; part < 4; ++part) {        // real near, real far, rec near, rec far
        const bool rec = part >= 2, wantnear = (part & 1) == 0;
        const int total = rec ? nk : nr;
        int *perm = rec ? g.perm_rec : g.perm_real;
        if (threadIdx.x == 0) count = (part & 1) ? g.counts[part - 1] : 0;
        __syncthreads();
        for (int base = 0; base < total; base += 256) {
            const int n = base + (int)threadIdx.x;
            bool keep = false;
            if (n < total) {
                const double r = rec ? sqrt(g.tab.rec[(size_t)n * 4 + 3])
                                     : sqrt(g.tab.real[(size_t)n * g.tab.rstride] * g.tab.real[(size_t)n * g.tab.rstride] +
                                            g.tab.real[(size_t)n * g.tab.rstride + 1] * g.tab.real[(size_t)n * g.tab.rstride + 1] +
                                            g.tab.real[(size_t)n * g.tab.rstride + 2] * g.tab.real[(size_t)n * g.tab.rstride + 2]);
                const bool near = g.mixed == 0 || r <= (rec ? rk : rn);
                keep = near == wantnear;
            }
            const int slot = grid_compact(keep, wave_tot, &count);
            if (keep) perm[slot] = n;
        }
        if (threadIdx.x == 0) g.counts[part] = (part & 1) ? count - g.counts[part - 1] : count;
        __syncthreads();
    }
}

// integer coordinates of a table vector: A^{-1} z (real) or A^T m* (reciprocal)
__device__ __forceinline__ void frac_coords(const EzLatMeta *M, int d, const double *v, bool recip, double *n) {
    for (int r = 0; r < 3; ++r) {
        double s = 0.0;
        for (int c = 0; c < d; ++c) s += (recip ? M->A[c * d + r] : M->B[c * d + r]) * v[c];
        n[r] = (r < d) ? rint(s) : 0.0;
    }
}

__device__ __forceinline__ void split_bf16(double v, __bf16 *hi, __bf16 *lo) {
    const float vf = (float)v;
    const __bf16 h = (__bf16)vf;
    *hi = h;
    *lo = (__bf16)(float)(v - (double)(float)h);
}

// A operands: real-space weights W_nu(|z - x_j|), rows (nu, j), columns = table
// entries in near/far order; reciprocal phases [cos; sin](2 pi h.t_j).  Column c < n_near
// goes to the FP64 matrix, column n_near + c' to column c' of the BF16 pair.  Both have
// leading dimension K_pad >= n_near + n_far + 32, and the grid covers every column
// c < K_pad, so the zero padding up to the next multiple of 16 (FP64) or 32 (BF16)
// past each count is always written.
__global__ __launch_bounds__(256) void grid_build_a_kernel(EzGridArgs g) {
    __shared__ double red[4];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;    // padded column
    const int row = blockIdx.y;                              // padded row of W (n_nu * Mp) or of P (2 Mp)
    const EzLatMeta *M = g.meta;
    const int d = g.d;
    const bool isP = row >= g.n_nu * g.Mp;
    if (!isP) {
        const int nu_i = row / g.Mp, j = row - nu_i * g.Mp;
        const int nnear = g.counts[0], nfar = g.counts[1];
        double w = 0.0;
        int n = -1;
        if (c < nnear + nfar && j < g.n_x) n = g.perm_real[c];
        if (n >= 0 && M->status == 0) {
            const double *e = g.tab.real + (size_t)n * g.tab.rstride;
            const double *px = g.pts_x + (size_t)j * 8;
            double xr[3] = {0, 0, 0};
            for (int r = 0; r < d; ++r)
                for (int k = 0; k < d; ++k) xr[r] += M->A[r * d + k] * px[k];
            double r2 = 0.0;
            for (int t = 0; t < d; ++t) { const double dt = e[t] - xr[t]; r2 += dt * dt; }
            const double a = EZ_PI * r2 / (M->lam * M->lam);
            const double nu = g.nu[nu_i];
            if (r2 > 0.0 && a <= M->a_cut)
                w = ez_gamma_upper(0.5 * nu, a) * ez_rgamma(0.5 * nu) * pow(r2, -0.5 * nu);
        }
        if (c < g.Kr_pad) {
            // near (or every) column in FP64; positions past the near count hold zeros
            g.A64r[(size_t)row * g.Krn_pad + c] = (c < nnear) ? w : 0.0;
            const int cf = c - nnear;
            if (g.mixed && cf >= 0 && cf < g.Krf_pad) {
                __bf16 h, l;
                split_bf16(cf < nfar ? w : 0.0, &h, &l);
                g.Ahr[(size_t)row * g.Krf_pad + cf] = h;
                g.Alr[(size_t)row * g.Krf_pad + cf] = l;
            }
        }
        if (g.mixed) {            // sums of |weights| for the error bound, one atomic per workgroup
            const double far = block_sum((c >= nnear && c < nnear + nfar) ? fabs(w) : 0.0, red);
            const double all = block_sum(fabs(w), red);
            if (threadIdx.x == 0) {
                if (far != 0.0) atomicAdd(&g.wsum[row], far);
                if (all != 0.0) atomicAdd(&g.wall[row], all);
            }
        }
    } else {
        if (c >= g.Kk_pad) return;                           // uniform over the workgroup row
        const int prow = row - g.n_nu * g.Mp;                // 0..2Mp-1
        const int j = prow < g.Mp ? prow : prow - g.Mp;
        const bool sinpart = prow >= g.Mp;
        const int nnear = g.counts[2], nfar = g.counts[3];
        double v = 0.0;
        int n = -1;
        if (c < nnear + nfar && j < g.n_x) n = g.perm_rec[c];
        if (n >= 0 && M->status == 0) {
            double h[3];
            frac_coords(M, d, g.tab.rec + (size_t)n * 4, true, h);
            const double *px = g.pts_x + (size_t)j * 8;
            double ht = 0.0;
            for (int t = 0; t < d; ++t) ht += h[t] * px[t];
            double sn, cs;
            ez_sincos2pi(ht, &sn, &cs);
            v = sinpart ? sn : cs;
        }
        if (c < g.Kkn_pad) g.A64k[(size_t)prow * g.Kkn_pad + c] = (c < nnear) ? v : 0.0;
        const int cf = c - nnear;
        if (g.mixed && cf >= 0 && cf < g.Kkf_pad) {
            __bf16 hh, ll;
            split_bf16(cf < nfar ? v : 0.0, &hh, &ll);
            g.Ahk[(size_t)prow * g.Kkf_pad + cf] = hh;
            g.Alk[(size_t)prow * g.Kkf_pad + cf] = ll;
        }
    }
}

// real-space B operand [cos | sin](2 pi s_m.n_z), K x 2Np: FP64 rows for near
// entries; BF16 pairs for far entries, stored transposed (K contiguous per column)
// for the MFMA operand loads.  Grid: (2Np / 256, Kr_pad).
__global__ __launch_bounds__(256) void grid_build_b_kernel(EzGridArgs g) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int krow = blockIdx.y;
    const EzLatMeta *M = g.meta;
    const int d = g.d;
    {
        if (col >= 2 * g.Np) return;
        const int m = col < g.Np ? col : col - g.Np;
        const bool sinpart = col >= g.Np;
        const int nnear = g.counts[0], nfar = g.counts[1];
        double v = 0.0;
        if (krow < nnear + nfar && m < g.n_y && M->status == 0) {
            double n[3];
            frac_coords(M, d, g.tab.real + (size_t)g.perm_real[krow] * g.tab.rstride, false, n);
            const double *ps = g.pts_y + (size_t)m * 4;
            double sn_ = 0.0;
            for (int t = 0; t < d; ++t) sn_ += ps[t] * n[t];
            double sn, cs;
            ez_sincos2pi(sn_, &sn, &cs);
            v = sinpart ? sn : cs;
        }
        if (krow < g.Krn_pad) g.B64r[(size_t)krow * (2 * g.Np) + col] = (krow < nnear) ? v : 0.0;
        const int kf = krow - nnear;
        if (g.mixed && kf >= 0 && kf < g.Krf_pad) {
            __bf16 h, l;
            split_bf16(kf < nfar ? v : 0.0, &h, &l);
            g.Bhr[(size_t)col * g.Krf_pad + kf] = h;
            g.Blr[(size_t)col * g.Krf_pad + kf] = l;
        }
        return;
    }
}

// reciprocal B operand G_nu(h, m) = K_nu E_{p_nu}(pi lam^2 |m*_h + y_m|^2) of column
// kr (near columns first) at the reduced point yr, every exponent: one base per
// entry (e^{-a} with E_1 or E_{1/2}) and the recurrences p E_{p+1} = e^{-a} - a E_p
// when every 2p is an integer, else the incomplete gamma per exponent; zero past the
// table, for a failed lattice and beyond a_cut.
__device__ __forceinline__ void grid_g_values(const EzGridArgs &g, int kr, bool pt, const double *yr,
                                              double (&vals)[EZ_NU_MAX]) {
    const EzLatMeta *M = g.meta;
    const int d = g.d;
    for (int i = 0; i < EZ_NU_MAX; ++i) vals[i] = 0.0;
    if (!pt || kr >= g.counts[2] + g.counts[3] || M->status != 0) return;
    const double *e = g.tab.rec + (size_t)g.perm_rec[kr] * 4;
    double r2 = 0.0;
    for (int t = 0; t < d; ++t) { const double q = e[t] + yr[t]; r2 += q * q; }
    const double a = M->alpha * r2;
    if (r2 == 0.0) {                     // m* + y = 0: continuation in nu, -K_nu / s
        for (int i = 0; i < g.n_nu; ++i) {
            const double s = 0.5 * ((double)d - g.nu[i]);
            if (s == 0.0) {
                atomicOr(g.status_acc, 0x10u);
                vals[i] = __longlong_as_double(0x7ff8000000000000ll);
            } else {
                vals[i] = -g.kpref[i] / s;
            }
        }
    } else if (a <= M->a_cut) {
        if (g.ladder) {
            const double ex = ez_expm(a), inv = ez_rcp(a);
            bool ne1 = false, nh = false;
            for (int i = 0; i < g.n_nu; ++i) {
                ne1 = ne1 || ((g.p2[i] & 1) == 0 && g.p2[i] >= 2);
                nh = nh || (g.p2[i] & 1);
            }
            double E1 = 0.0;
            if (ne1) E1 = (a < 0.25) ? ez_e1_small(a) : ex * ez_e1w_scaled(inv);
            const double Eh = nh ? ez_ehalf(a) : 0.0;
            for (int i = 0; i < g.n_nu; ++i) vals[i] = g.kpref[i] * ez_ep_from(g.p2[i], a, ex, inv, E1, Eh);
        } else {
            for (int i = 0; i < g.n_nu; ++i) {
                const double s = 0.5 * ((double)d - g.nu[i]);
                vals[i] = g.kpref[i] * pow(a, -s) * ez_gamma_upper(s, a);
            }
        }
    }
}

// B operands of the reciprocal product, near columns (every column in FP64
// precision): G_nu(|m* + y_m|^2) as FP64 rows of B64k, one thread per (column,
// point), stores coalesced over the points.  Grid: (Np / 256, Kkn_pad).
__global__ __launch_bounds__(256) void grid_build_g_kernel(EzGridArgs g) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const int kr = blockIdx.y;
    const EzLatMeta *M = g.meta;
    const int d = g.d;
    const bool pt = m < g.n_y;
    double yr[3] = {0, 0, 0};
    if (pt) {
        const double *ps = g.pts_y + (size_t)m * 4;
        for (int r = 0; r < d; ++r)
            for (int k = 0; k < d; ++k) yr[r] += M->B[r * d + k] * ps[k];
    }
    double vals[EZ_NU_MAX];
    grid_g_values(g, kr < g.counts[2] ? kr : 1 << 30, pt, yr, vals);
    if (m < g.Np)
        for (int i = 0; i < g.n_nu; ++i) g.B64k[(size_t)kr * (g.n_nu * g.Np) + (size_t)i * g.Np + m] = vals[i];
}

// mixed precision, for the error bound: sum of |G| over the near columns per
// (exponent, point) column of B64k, added to the far columns' sum (the kernels run
// one after the other on one stream)
__global__ __launch_bounds__(256) void grid_gsum_kernel(EzGridArgs g) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= g.n_nu * g.Np || col % g.Np >= g.n_y) return;
    const size_t ld = (size_t)g.n_nu * g.Np;
    double s = 0.0;
    for (int kr = 0; kr < g.counts[2]; ++kr) {
        const double v = g.B64k[(size_t)kr * ld + col];
        if (v == v) s += fabs(v);
    }
    g.gall[col] += s;
}

// Far columns (mixed precision): the split-BF16 pairs of G, K-contiguous per
// (exponent, point) column.  A workgroup takes one point and 256 consecutive far
// columns, one per thread, so the two-byte stores of a wave are contiguous; the
// workgroup adds up |G| per exponent for the bound (one atomic per exponent).
__global__ __launch_bounds__(256) void grid_build_gfar_kernel(EzGridArgs g) {
    __shared__ double red[4];
    const int kf = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    const EzLatMeta *M = g.meta;
    const int d = g.d;
    const bool pt = m < g.n_y;
    double yr[3] = {0, 0, 0};
    if (pt) {
        const double *ps = g.pts_y + (size_t)m * 4;
        for (int r = 0; r < d; ++r)
            for (int k = 0; k < d; ++k) yr[r] += M->B[r * d + k] * ps[k];
    }
    double vals[EZ_NU_MAX];
    grid_g_values(g, kf < g.counts[3] ? g.counts[2] + kf : 1 << 30, pt, yr, vals);
    for (int i = 0; i < g.n_nu; ++i) {
        const double v = vals[i];
        if (kf < g.Kkf_pad) {
            __bf16 h, l;
            split_bf16(v, &h, &l);
            const size_t col = (size_t)i * g.Np + m;
            g.Bhk[col * g.Kkf_pad + kf] = h;
            g.Blk[col * g.Kkf_pad + kf] = l;
        }
        const double s = block_sum((kf < g.Kkf_pad && v == v) ? fabs(v) : 0.0, red);
        if (threadIdx.x == 0 && pt && s != 0.0) {
            atomicAdd(&g.gfar[(size_t)i * g.Np + m], s);
            atomicAdd(&g.gall[(size_t)i * g.Np + m], s);
        }
    }
}

// ---------------------------------------------------------------------------
// C[r][c] = sum_{k < Kn} A[r][k] B[k][c]                      (FP64, v_mfma_f64_16x16x4)
//         + sum_{k < Kf} (Ah + Al)[r][k] (Bh + Bl)[k][c]        (split BF16, far entries)
// The FP64 part runs over the near table entries (zero-padded to multiples of 16),
// the BF16 part over the far ones (padded to 32): per 32-wide step Ah Bh + Ah Bl +
// Al Bh by v_mfma_f32_16x16x32_bf16 into a zeroed FP32 tile, which is then added to
// the FP64 accumulators (the FP32 rounding covers 96 products at a time), and C is
// written once.  A, A64 row-major; B64 row-major
// (K x ldb); Bh, Bl stored transposed (columns x ldbh, K contiguous).  64 x 64 tile
// per workgroup, each wave a 32 x 32 quarter.
struct GemmF64Tiles {                // two buffers: the next K step is stored while this one is read
    double As[2][64][17];
    double Bs[2][16][65];
};
struct alignas(16) GemmBf16Tiles {
    __bf16 Ash[64][40];
    __bf16 Asl[64][40];
    __bf16 Bsh[64][40];
    __bf16 Bsl[64][40];
};
// mixed: the BF16 tiles reuse the FP64 tiles once the FP64 loop is done
struct alignas(16) GemmLdsMixed {
    union {
        GemmF64Tiles f;
        GemmBf16Tiles b;
    } u;
};
__device__ __forceinline__ GemmF64Tiles &f64_tiles(GemmF64Tiles &L) { return L; }
__device__ __forceinline__ GemmF64Tiles &f64_tiles(GemmLdsMixed &L) { return L.u.f; }

template <bool MIXED>
__global__ __launch_bounds__(256) void gemm_mixed_kernel(const double *A, int lda, const double *B, int ldb,
                                                         const int *Kn_dev, const __bf16 *Ah, const __bf16 *Al,
                                                         int ldah, const __bf16 *Bh, const __bf16 *Bl, int ldbh,
                                                         const int *Kf_dev, double *C, int ldc) {
    __shared__ typename std::conditional<MIXED, GemmLdsMixed, GemmF64Tiles>::type L;
    GemmF64Tiles &F = f64_tiles(L);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    // workgroups go to the XCDs in turn (g mod 8): XCD x takes the x-th eighth of the
    // tiles, column block by column block with the row blocks innermost, so that the
    // workgroups an XCD runs one after another share their B columns in its L2 (the
    // tile count is a multiple of 8: rows and columns are padded to multiples of 128)
    const int T = (int)(gridDim.x * gridDim.y), Mt = (int)gridDim.y;
    const int g = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    const int t = (g & 7) * (T >> 3) + (g >> 3);
    const int row0 = (t % Mt) * 64, col0 = (t / Mt) * 64;
    f64x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    const int nkt = (*Kn_dev + 15) / 16;
    // K steps of 16: the next step's A and B are loaded into registers while this
    // step's MFMAs run, and stored to the other LDS buffer at the top of the next
    // iteration (that buffer's last readers passed this iteration's barrier)
    double ra[4], rb[4];
    auto gload = [&](int kt) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + 256 * q;
            ra[q] = A[(size_t)(row0 + (idx >> 4)) * lda + kt * 16 + (idx & 15)];
            rb[q] = B[(size_t)(kt * 16 + (idx >> 6)) * ldb + col0 + (idx & 63)];
        }
    };
    if (nkt > 0) gload(0);
    for (int kt = 0; kt < nkt; ++kt) {
        const int buf = kt & 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + 256 * q;
            F.As[buf][idx >> 4][idx & 15] = ra[q];
            F.Bs[buf][idx >> 6][idx & 63] = rb[q];
        }
        __syncthreads();
        if (kt + 1 < nkt) gload(kt + 1);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            double a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = F.As[buf][32 * wr + 16 * i + (lane & 15)][4 * kk + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = F.Bs[buf][4 * kk + (lane >> 4)][32 * wc + 16 * j + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    if constexpr (MIXED) {
        const int nft = (*Kf_dev + 31) / 32;
        __syncthreads();                                 // the BF16 tiles reuse the FP64 ones
        __bf16 (*Ash)[40] = L.u.b.Ash, (*Asl)[40] = L.u.b.Asl, (*Bsh)[40] = L.u.b.Bsh, (*Bsl)[40] = L.u.b.Bsl;
        {
            // the next 32-wide step's operands are loaded into registers while this
            // step's MFMAs run
            const int lr = tid >> 2, k8 = (tid & 3) * 8;
            bf16x8 pah, pal, pbh, pbl;
            auto bload = [&](int kt) {
                pah = *reinterpret_cast<const bf16x8 *>(Ah + (size_t)(row0 + lr) * ldah + kt * 32 + k8);
                pal = *reinterpret_cast<const bf16x8 *>(Al + (size_t)(row0 + lr) * ldah + kt * 32 + k8);
                pbh = *reinterpret_cast<const bf16x8 *>(Bh + (size_t)(col0 + lr) * ldbh + kt * 32 + k8);
                pbl = *reinterpret_cast<const bf16x8 *>(Bl + (size_t)(col0 + lr) * ldbh + kt * 32 + k8);
            };
            if (nft > 0) bload(0);
            for (int kt = 0; kt < nft; ++kt) {
                *reinterpret_cast<bf16x8 *>(&Ash[lr][k8]) = pah;
                *reinterpret_cast<bf16x8 *>(&Asl[lr][k8]) = pal;
                *reinterpret_cast<bf16x8 *>(&Bsh[lr][k8]) = pbh;
                *reinterpret_cast<bf16x8 *>(&Bsl[lr][k8]) = pbl;
                __syncthreads();
                if (kt + 1 < nft) bload(kt + 1);
                bf16x8 bh[2], bl[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    bh[j] = *reinterpret_cast<const bf16x8 *>(&Bsh[32 * wc + 16 * j + (lane & 15)][8 * (lane >> 4)]);
                    bl[j] = *reinterpret_cast<const bf16x8 *>(&Bsl[32 * wc + 16 * j + (lane & 15)][8 * (lane >> 4)]);
                }
                // v_mfma_f32_16x16x32_bf16 leaves D[4 (l/16) + r][l % 16] in lane l, register
                // r, and v_mfma_f64_16x16x4 D[l/16 + 4 r][l % 16]: the A rows are fed in the
                // order pi(rho) = rho/4 + 4 (rho % 4), so that each lane's FP32 results are
                // the rows of its FP64 accumulators
                const int pr = ((lane & 15) >> 2) + 4 * (lane & 3);
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const bf16x8 ah = *reinterpret_cast<const bf16x8 *>(&Ash[32 * wr + 16 * i + pr][8 * (lane >> 4)]);
                    const bf16x8 al = *reinterpret_cast<const bf16x8 *>(&Asl[32 * wr + 16 * i + pr][8 * (lane >> 4)]);
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        f32x4 t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], f32x4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
                        t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], t, 0, 0, 0);
                        t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], t, 0, 0, 0);
                        // FP32 over the chunk's 3 x 32 products, FP64 across chunks
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)t[r];
                    }
                }
                __syncthreads();
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // v_mfma_f64_16x16x4: lane l, register r holds D[l/16 + 4 r][l % 16]
                const int rl = 32 * wr + 16 * i + (lane >> 4) + 4 * r, cl = 32 * wc + 16 * j + (lane & 15);
                C[(size_t)(row0 + rl) * ldc + col0 + cl] = acc[i][j][r];
            }
}

// ---------------------------------------------------------------------------
// Z_nu(x_j, y_m) = R + e^{-2 pi i s.t} Q - self, times e^{-2 pi i s.n0} (quasi-periodicity)
__global__ __launch_bounds__(256) void grid_combine_kernel(EzGridArgs g) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)g.n_nu * g.n_x * g.n_y;
    if (gid >= total) return;
    const int m = (int)(gid % g.n_y);
    const long long rest = gid / g.n_y;
    const int j = (int)(rest % g.n_x), nu_i = (int)(rest / g.n_x);
    const EzLatMeta *M = g.meta;
    double *o = g.out + 2 * gid;
    if (M->status != 0) {
        o[0] = o[1] = __longlong_as_double(0x7ff8000000000000ll);
        return;
    }
    const double *px = g.pts_x + (size_t)j * 8, *ps = g.pts_y + (size_t)m * 4;
    const size_t rrow = (size_t)(nu_i * g.Mp + j) * (2 * g.Np);
    const double rre = g.R[rrow + m], rim = -g.R[rrow + g.Np + m];
    const size_t qcol = (size_t)nu_i * g.Np + m, ldq = (size_t)g.n_nu * g.Np;
    const double qre = g.Q[(size_t)j * ldq + qcol], qim = -g.Q[(size_t)(g.Mp + j) * ldq + qcol];
    double st = 0.0, sn0 = 0.0;
    for (int t = 0; t < g.d; ++t) { st += ps[t] * px[t]; sn0 += ps[t] * px[3 + t]; }
    double sn, cs;
    ez_sincos2pi(-st, &sn, &cs);                       // e^{-2 pi i s.t}
    double zre = rre + qre * cs - qim * sn;
    double zim = rim + qre * sn + qim * cs;
    if (px[6] != 0.0) {
        const double nu = g.nu[nu_i];
        zre -= pow(EZ_PI / (M->lam * M->lam), 0.5 * nu) * ez_rgamma(0.5 * nu + 1.0);
    }
    ez_sincos2pi(-sn0, &sn, &cs);
    o[0] = zre * cs - zim * sn;
    o[1] = zre * sn + zim * cs;
}

// a-priori bound of |Z_mixed - Z_fp64| per (nu, x_j), all phases having modulus <= 1:
// at (x_j, y_m) the real-space sum over z has the weights of row j and the reciprocal
// sum over m* those of point m, so the bound is a term per shift plus a term per point:
//  split-BF16 far products: with a = a_hi + a_lo + da (a_hi = bf16(fp32(a)), a_lo =
//    bf16(fp32(a - a_hi)), |da| <= (2^-8 + 2^-24)^2 |a|, |a_lo| <= 2^-8 (1 + 2^-7) |a|),
//    ab - (a_hi b_hi + a_hi b_lo + a_lo b_hi) = a_lo b_lo + a_hi db + da b_hi + da db,
//    at most 3.05 2^-16 |ab|; the products are exact in FP32 and each chunk adds 96 of
//    them from zero in FP32, at most gamma_97 (1.01 sum |ab|), gamma_n = n 2^-24 /
//    (1 - n 2^-24); so (3.05 2^-16 + 1.01 gamma_97) times (the sum of |far weights|
//    of row j + the sum of |far G| of point m);
//  FP64 products and sums (both forms, their summation orders differ): 2 gamma_K with
//    gamma_K = K 2^-53 / (1 - K 2^-53), K the table size, times the same sums over
//    every column;
// each for the real and the imaginary part (factor 2)
__global__ __launch_bounds__(256) void grid_bound_kernel(EzGridArgs g) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int nxy = g.n_x + g.n_y;
    if (idx >= g.n_nu * nxy) return;
    const int nu_i = idx / nxy, q = idx - nu_i * nxy;
    const double g97 = 97.0 * 0x1p-24 / (1.0 - 97.0 * 0x1p-24);
    const double ubf = 3.05 * 0x1p-16 + 1.01 * g97;
    const double K = (double)(g.counts[0] + g.counts[1] + g.counts[2] + g.counts[3]) + 4.0;
    const double g64 = 2.0 * K * 0x1p-53 / (1.0 - K * 0x1p-53);
    double far, all;
    if (q < g.n_x) {                   // shift term: the real-space row sums
        far = g.wsum[nu_i * g.Mp + q];
        all = g.wall[nu_i * g.Mp + q];
    } else {                           // point term: the reciprocal column sums
        far = g.gfar[(size_t)nu_i * g.Np + (q - g.n_x)];
        all = g.gall[(size_t)nu_i * g.Np + (q - g.n_x)];
    }
    g.bound[idx] = 2.0 * (ubf * far + g64 * all);
}

}  // namespace

hipError_t ez_grid_launch(const EzGridArgs &g, hipStream_t s, int part) {
    hipError_t e = hipSuccess;
    if (part & EZ_GRID_PRE) {
        const int mx = std::max(g.n_x, g.n_y);
        if (g.mixed) {
            const long long nz = 2 * ((long long)g.n_nu * g.Mp + (long long)g.n_nu * g.Np);   // wsum, gfar, wall, gall
            hipLaunchKernelGGL(grid_zero_kernel, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, s, g.wsum, nz);
        }
        hipLaunchKernelGGL(grid_points_kernel, dim3((mx + 255) / 256), dim3(256), 0, s, g);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(grid_classify_kernel, dim3(1), dim3(256), 0, s, g);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int kmax = std::max(g.Kr_pad, g.Kk_pad);
        hipLaunchKernelGGL(grid_build_a_kernel, dim3((kmax + 255) / 256, g.n_nu * g.Mp + 2 * g.Mp), dim3(256), 0, s, g);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(grid_build_b_kernel, dim3((2 * g.Np + 255) / 256, g.Kr_pad), dim3(256), 0, s, g);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(grid_build_g_kernel, dim3((g.Np + 255) / 256, g.Kkn_pad), dim3(256), 0, s, g);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (g.mixed) {
            hipLaunchKernelGGL(grid_build_gfar_kernel, dim3((g.Kkf_pad + 255) / 256, g.Np), dim3(256), 0, s, g);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(grid_gsum_kernel, dim3((g.n_nu * g.Np + 255) / 256), dim3(256), 0, s, g);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (part & EZ_GRID_GEMM) {
        // the products' tile remap takes the tile count to be a multiple of 8
        if ((((2 * g.Np / 64) * (g.n_nu * g.Mp / 64)) & 7) || (((g.n_nu * g.Np / 64) * (2 * g.Mp / 64)) & 7))
            return hipErrorInvalidValue;
        // real space: (n_nu Mp) x (2 Np);  reciprocal: (2 Mp) x (n_nu Np)
        auto gemm = g.mixed ? gemm_mixed_kernel<true> : gemm_mixed_kernel<false>;
        hipLaunchKernelGGL(gemm, dim3(2 * g.Np / 64, g.n_nu * g.Mp / 64), dim3(256), 0, s, g.A64r, g.Krn_pad, g.B64r,
                           2 * g.Np, g.counts + 0, g.Ahr, g.Alr, g.Krf_pad, g.Bhr, g.Blr, g.Krf_pad, g.counts + 1, g.R,
                           2 * g.Np);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(gemm, dim3(g.n_nu * g.Np / 64, 2 * g.Mp / 64), dim3(256), 0, s, g.A64k, g.Kkn_pad, g.B64k,
                           g.n_nu * g.Np, g.counts + 2, g.Ahk, g.Alk, g.Kkf_pad, g.Bhk, g.Blk, g.Kkf_pad, g.counts + 3, g.Q,
                           g.n_nu * g.Np);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!(part & EZ_GRID_POST)) return hipSuccess;
    const long long total = (long long)g.n_nu * g.n_x * g.n_y;
    hipLaunchKernelGGL(grid_combine_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (g.bound) {
        if (g.mixed)   // FP64 products: no bound beyond rounding, zeros
            hipLaunchKernelGGL(grid_bound_kernel, dim3((g.n_nu * (g.n_x + g.n_y) + 255) / 256), dim3(256), 0, s, g);
        else
            hipLaunchKernelGGL(grid_zero_kernel, dim3((g.n_nu * (g.n_x + g.n_y) + 255) / 256), dim3(256), 0, s,
                               g.bound, (long long)g.n_nu * (g.n_x + g.n_y));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}
