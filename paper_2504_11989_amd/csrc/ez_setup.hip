// ez_setup.hip -- per-lattice precompute on the device: B = A^{-T}, V, lam, the
// real-space point table with its incomplete-gamma weights and the reciprocal
// point table (paper, Sec. 2, Definition (Lattices); the split itself follows
// from the Mellin integral of |r|^{-nu} and Poisson summation).
//
// Real space (x = 0, pairs mode): one representative of each pair +-z,
// 0 < |z| <= lam sqrt(a_cut/pi), with 2 W_nu(z),
//   W_nu(z) = Gamma(nu/2, pi |z|^2 / lam^2) / (Gamma(nu/2) |z|^nu).
// Real space (general-x mode): every z with |z| <= lam sqrt(a_cut/pi) + r_cell.
// Reciprocal space: every m* with |m*| <= sqrt(a_cut/pi)/lam + r_BZ, m* = 0 first,
// where r_BZ bounds |k| over the reduced cell B[-1/2,1/2]^d of the nodes.
//
// One workgroup per lattice; point order is the enumeration order of the
// integer box, made deterministic by a ballot/prefix compaction.
#include "ez_internal.h"
#include "ez_math.h"
#include "ez_kernels.h"

namespace {

constexpr int SB = 256;   // threads per setup workgroup

struct SetupShared {
    double A[9], Ai[9], B[9];
    double V, lam, alpha, Rr, Rk;
    int lo[3], hi[3];        // enumeration box
    long long nbox;
    int count;
    uint32_t status;
    int wave_tot[SB / 64];
};

__device__ void mat_inverse(int d, const double *M, double *Mi, double *det) {
    if (d == 1) { *det = M[0]; Mi[0] = 1.0 / M[0]; return; }
    if (d == 2) {
        double dt = M[0] * M[3] - M[1] * M[2];
        *det = dt;
        Mi[0] = M[3] / dt; Mi[1] = -M[1] / dt; Mi[2] = -M[2] / dt; Mi[3] = M[0] / dt;
        return;
    }
    double c00 = M[4] * M[8] - M[5] * M[7];
    double c01 = M[5] * M[6] - M[3] * M[8];
    double c02 = M[3] * M[7] - M[4] * M[6];
    double dt = M[0] * c00 + M[1] * c01 + M[2] * c02;
    *det = dt;
    double r = 1.0 / dt;
    Mi[0] = c00 * r; Mi[1] = (M[2] * M[7] - M[1] * M[8]) * r; Mi[2] = (M[1] * M[5] - M[2] * M[4]) * r;
    Mi[3] = c01 * r; Mi[4] = (M[0] * M[8] - M[2] * M[6]) * r; Mi[5] = (M[2] * M[3] - M[0] * M[5]) * r;
    Mi[6] = c02 * r; Mi[7] = (M[1] * M[6] - M[0] * M[7]) * r; Mi[8] = (M[0] * M[4] - M[1] * M[3]) * r;
}

// half of the largest |M s|, s in {+-1}^d: bounds |M t| over t in [-1/2,1/2]^d
__device__ double half_diag(int d, const double *M) {
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

// Block-wide deterministic compaction: returns this thread's slot (or -1) and
// advances sh->count by the number of kept items, in thread order.
__device__ int compact_slot(bool keep, SetupShared *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long m = __ballot(keep);
    int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) sh->wave_tot[wave] = __popcll(m);
    __syncthreads();
    int off = sh->count;
    for (int w = 0; w < wave; ++w) off += sh->wave_tot[w];
    int slot = keep ? off + before : -1;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < SB / 64; ++w) tot += sh->wave_tot[w];
        sh->count += tot;
    }
    __syncthreads();
    return slot;
}

__device__ void box_index(long long idx, const int *lo, const int *hi, int d, int *n) {
    for (int i = 0; i < 3; ++i) n[i] = 0;
    for (int i = 0; i < d; ++i) {
        long long w = hi[i] - lo[i] + 1;
        n[i] = lo[i] + (int)(idx % w);
        idx /= w;
    }
}

__global__ __launch_bounds__(SB) void ez_setup_kernel(EzSetupArgs args) {
    __shared__ SetupShared sh;
    const int inst = blockIdx.x;
    const int d = args.prog.d;
    const EzInstPlan plan = args.plans[inst];
    EzLatMeta *meta = args.meta + inst;
    const double lam_rel = plan.lam_rel;
    const double a_cut = args.a_cut;

    if (threadIdx.x == 0) {
        uint32_t st = 0;
        for (int i = 0; i < 9; ++i) sh.A[i] = 0.0;
        for (int i = 0; i < d * d; ++i) {
            sh.A[i] = args.A[(size_t)inst * d * d + i];
            if (!isfinite(sh.A[i])) st |= 0x1u;
        }
        double det = 0.0;
        if (!st) {
            mat_inverse(d, sh.A, sh.Ai, &det);
            if (!(fabs(det) > 1e-300) || !isfinite(det)) st |= 0x1u;
        }
        if (!st) {
            for (int i = 0; i < d; ++i)
                for (int j = 0; j < d; ++j) sh.B[i * d + j] = sh.Ai[j * d + i];
            sh.V = fabs(det);
            sh.lam = lam_rel * pow(sh.V, 1.0 / d);
            // every m* != 0 then has pi lam^2 |m* + k|^2 >= 1/4 for the quadrature nodes
            // k in B[-1/2,1/2]^d (|m* + k| >= sigma_min(B)/2 >= 1/(2 |A|_F)); the node
            // kernel's rational E1 is fitted for arguments >= 1/4
            if (!args.general_x) {
                double fro2 = 0.0;
                for (int i = 0; i < d * d; ++i) fro2 += sh.A[i] * sh.A[i];
                sh.lam = fmax(sh.lam, sqrt(fro2 / EZ_PI) * (1.0 + 1e-12));
            }
            sh.alpha = EZ_PI * sh.lam * sh.lam;
            sh.Rr = sh.lam * sqrt(a_cut / EZ_PI);
            sh.Rk = sqrt(a_cut / EZ_PI) / sh.lam;
            if (args.general_x) sh.Rr += half_diag(d, sh.A);
            // box for |A n| <= Rr: |n_i| <= Rr |row_i(A^{-1})|
            long long nb = 1;
            for (int i = 0; i < 3; ++i) { sh.lo[i] = 0; sh.hi[i] = 0; }
            for (int i = 0; i < d; ++i) {
                double r = 0.0;
                for (int j = 0; j < d; ++j) r += sh.Ai[i * d + j] * sh.Ai[i * d + j];
                int h = (int)floor(sh.Rr * sqrt(r));
                sh.lo[i] = -h; sh.hi[i] = h;
                nb *= (long long)(2 * h + 1);
            }
            sh.nbox = nb;
            if (nb > (1ll << 26)) st |= 0x2u;
        }
        sh.status = st;
        sh.count = 0;
    }
    __syncthreads();
    if (sh.status) {
        if (threadIdx.x == 0) {
            meta->status = sh.status; meta->n_real = 0; meta->n_rec = 0;
            if (args.status_out) args.status_out[0] = sh.status;
        }
        return;
    }

    // ---------------- real-space table ----------------
    const int rs = args.tab.rstride;
    double *rtab = args.tab.real + (size_t)inst * args.tab.real_cap * rs;
    const double Rr2 = sh.Rr * sh.Rr;
    for (long long base = 0; base < sh.nbox; base += SB) {
        long long idx = base + threadIdx.x;
        bool keep = false;
        double z[3] = {0.0, 0.0, 0.0};
        int n[3] = {0, 0, 0};
        if (idx < sh.nbox) {
            box_index(idx, sh.lo, sh.hi, d, n);
            bool nonzero = (n[0] | n[1] | n[2]) != 0;
            // pairs mode: keep the representative whose last nonzero coordinate is > 0
            bool half = true;
            if (!args.general_x) {
                int last = 0;
                for (int i = 0; i < d; ++i) if (n[i] != 0) last = n[i];
                half = last > 0;
            }
            for (int i = 0; i < d; ++i) {
                double s = 0.0;
                for (int j = 0; j < d; ++j) s += sh.A[i * d + j] * (double)n[j];
                z[i] = s;
            }
            double r2 = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
            keep = (args.general_x ? true : nonzero) && half && r2 <= Rr2;
        }
        int slot = compact_slot(keep, &sh);
        if (keep) {
            if (slot < args.tab.real_cap) {
                double *e = rtab + (size_t)slot * rs;
                e[0] = z[0]; e[1] = z[1]; e[2] = z[2];
                if (!args.general_x) {
                    int *ni = args.tab.rn + ((size_t)inst * args.tab.real_cap + slot) * 4;
                    ni[0] = n[0]; ni[1] = n[1]; ni[2] = n[2]; ni[3] = 0;
                }
            } else {
                atomicOr(&sh.status, 0x2u);
            }
        }
    }
    __syncthreads();
    const int n_real = min(sh.count, args.tab.real_cap);
    // weights (pairs mode only; general-x weights depend on x)
    if (!args.general_x) {
        for (int t = threadIdx.x; t < n_real; t += SB) {
            double *e = rtab + (size_t)t * rs;
            double r2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
            double a = EZ_PI * r2 / (sh.lam * sh.lam);
            for (int i = 0; i < args.prog.n_nu; ++i) {
                double nu = args.prog.nu[i];
                double w = ez_gamma_upper(0.5 * nu, a) * ez_rgamma(0.5 * nu) * pow(r2, -0.5 * nu);
                e[3 + i] = 2.0 * w;
            }
            int used = 3 + args.prog.n_nu;
            if (args.grad) {
                // strain weights: d(2 W_nu)/d|z|^2 times 2 (from d|z|^2 = 2 z^T G z), with
                // dW_nu/d|z|^2 = -Gamma(nu/2 + 1, a) / (Gamma(nu/2) |z|^{nu+2})
                for (int i = 0; i < args.prog.n_nu; ++i) {
                    double nu = args.prog.nu[i];
                    e[used + i] = -4.0 * ez_gamma_upper(0.5 * nu + 1.0, a) * ez_rgamma(0.5 * nu) *
                                  pow(r2, -0.5 * nu - 1.0);
                }
                used += args.prog.n_nu;
            }
            for (int i = used; i < rs; ++i) e[i] = 0.0;
        }
    }
    __syncthreads();
    // rows of the real-space table (pairs mode)
    if (!args.general_x) {
        const int *rn = args.tab.rn + (size_t)inst * args.tab.real_cap * 4;
        int *rows = args.tab.rows + (size_t)inst * args.tab.row_cap * 8;
        if (threadIdx.x == 0) sh.count = 0;
        __syncthreads();
        for (int base = 0; base < n_real; base += SB) {
            const int t = base + (int)threadIdx.x;
            bool start = false;
            if (t < n_real) {
                start = (t == 0) || rn[4 * t + 1] != rn[4 * (t - 1) + 1] || rn[4 * t + 2] != rn[4 * (t - 1) + 2];
            }
            int slot = compact_slot(start, &sh);
            if (start && slot < args.tab.row_cap) {
                int cnt = 1;
                while (t + cnt < n_real && rn[4 * (t + cnt) + 1] == rn[4 * t + 1] && rn[4 * (t + cnt) + 2] == rn[4 * t + 2]) ++cnt;
                int *R = rows + (size_t)slot * 8;
                R[0] = t; R[1] = cnt; R[2] = rn[4 * t]; R[3] = rn[4 * t + 1]; R[4] = rn[4 * t + 2];
            } else if (start) {
                atomicOr(&sh.status, 0x2u);
            }
        }
        __syncthreads();
        const int n_rows = min(sh.count, args.tab.row_cap);
        for (int r = threadIdx.x; r < n_rows; r += SB) {
            int *R = rows + (size_t)r * 8;
            const int *Rp = rows + (size_t)(r > 0 ? r - 1 : 0) * 8;
            const bool np = (r == 0) || R[4] != Rp[4];
            R[5] = np ? 1 : 0;
            R[6] = np ? 0 : R[2] - Rp[2];
            R[7] = np ? 0 : R[3] - Rp[3];
        }
        __syncthreads();
        if (threadIdx.x == 0) meta->n_rows = n_rows;
    } else if (threadIdx.x == 0) {
        meta->n_rows = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        sh.count = 0;
        // reciprocal box: |B m| <= Rk + r_BZ  ->  |m_i| <= R |row_i(B^{-1})| = R |col_i(A)|
        double R = sh.Rk + half_diag(d, sh.B);
        long long nb = 1;
        for (int i = 0; i < 3; ++i) { sh.lo[i] = 0; sh.hi[i] = 0; }
        for (int i = 0; i < d; ++i) {
            double r = 0.0;
            for (int j = 0; j < d; ++j) r += sh.A[j * d + i] * sh.A[j * d + i];
            int h = (int)floor(R * sqrt(r));
            sh.lo[i] = -h; sh.hi[i] = h;
            nb *= (long long)(2 * h + 1);
        }
        sh.nbox = nb;
        if (nb > (1ll << 26)) sh.status |= 0x2u;
        sh.Rk = R;
        // m* = 0 first
        double *e = args.tab.rec + (size_t)inst * args.tab.rec_cap * 4;
        e[0] = e[1] = e[2] = e[3] = 0.0;
        sh.count = 1;
    }
    __syncthreads();
    double *ktab = args.tab.rec + (size_t)inst * args.tab.rec_cap * 4;
    const double Rk2 = sh.Rk * sh.Rk;
    // inner: entries that can reach a = alpha |m* + k|^2 < 1 for a node k in B[-1/2,1/2]^d.
    // |m* + k| >= sigma_min(B) (|m|_inf - 1/2) and sigma_min(B) >= 1/|A|_F give the test.
    double fro2 = 0.0;
    for (int i = 0; i < d * d; ++i) fro2 += sh.A[i] * sh.A[i];
    int n_inner = 1;
    for (int pass = 0; pass < 2; ++pass) {
        if (sh.status & 0x2u) break;
        for (long long base = 0; base < sh.nbox; base += SB) {
            long long idx = base + threadIdx.x;
            bool keep = false;
            double m[3] = {0.0, 0.0, 0.0};
            if (idx < sh.nbox) {
                int n[3];
                box_index(idx, sh.lo, sh.hi, d, n);
                for (int i = 0; i < d; ++i) {
                    double s = 0.0;
                    for (int j = 0; j < d; ++j) s += sh.B[i * d + j] * (double)n[j];
                    m[i] = s;
                }
                double r2 = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
                int ninf = max(abs(n[0]), max(abs(n[1]), abs(n[2])));
                double g = (double)ninf - 0.5;
                bool inner = sh.alpha * g * g < fro2;
                keep = ((n[0] | n[1] | n[2]) != 0) && r2 <= Rk2 && (pass == 0 ? inner : !inner);
            }
            int slot = compact_slot(keep, &sh);
            if (keep) {
                if (slot < args.tab.rec_cap) {
                    double *e = ktab + (size_t)slot * 4;
                    e[0] = m[0]; e[1] = m[1]; e[2] = m[2];
                    e[3] = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
                } else {
                    atomicOr(&sh.status, 0x2u);
                }
            }
        }
        if (pass == 0) n_inner = sh.count;
        __syncthreads();
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < 9; ++i) { meta->A[i] = sh.A[i]; meta->B[i] = sh.B[i]; }
        meta->V = sh.V;
        meta->lam = sh.lam;
        meta->alpha = sh.alpha;
        meta->a_cut = a_cut;
        for (int i = 0; i < EZ_NU_MAX; ++i) { meta->K[i] = 0.0; meta->self_[i] = 0.0; meta->sig[i] = 0.0; }
        for (int i = 0; i < args.prog.n_nu; ++i) {
            double nu = args.prog.nu[i];
            double s = 0.5 * (d - nu);
            double rg = ez_rgamma(0.5 * nu);
            double cp = pow(EZ_PI, nu - 0.5 * d) * rg / sh.V;
            meta->K[i] = cp * pow(sh.alpha, s);
            meta->self_[i] = pow(EZ_PI / (sh.lam * sh.lam), 0.5 * nu) * ez_rgamma(0.5 * nu + 1.0);
            int m = args.prog.logm[i];
            if (m >= 0) {
                double mf = 1.0;
                for (int j = 2; j <= m; ++j) mf *= (double)j;
                meta->sig[i] = pow(EZ_PI, 2.0 * m + 0.5 * d) * ez_rgamma(m + 0.5 * d) *
                               (((m + 1) & 1) ? -1.0 : 1.0) / mf / sh.V;
            } else {
                meta->sig[i] = cp * tgamma(s);
            }
        }
        meta->n_real = n_real;
        meta->n_rec = min(sh.count, args.tab.rec_cap);
        meta->n_inner = min(n_inner, meta->n_rec);
        uint32_t st = sh.status;
        if (sh.count > args.tab.rec_cap) st |= 0x2u;
        meta->status = st;
        if (args.status_out) args.status_out[0] = st;
    }
}

}  // namespace

hipError_t ez_launch_setup(const EzSetupArgs &args, int batch, hipStream_t stream) {
    hipLaunchKernelGGL(ez_setup_kernel, dim3(batch), dim3(SB), 0, stream, args);
    return hipGetLastError();
}
