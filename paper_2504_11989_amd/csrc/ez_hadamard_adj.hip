// ez_hadamard_adj.hip -- the Hadamard part on (0, eps) with its strain derivatives.
#include <hip/hip_ext.h>

#include "ez_hadamard_common.h"

namespace {

template <int PD>
__device__ __forceinline__ void poly_mul_trunc(double (&p)[PD], const double (&c)[EZ_ELL_MAX + 1]) {
#pragma unroll
    for (int J = PD - 1; J >= 0; --J) {
        double s = 0.0;
#pragma unroll
        for (int kk = 0; kk <= EZ_ELL_MAX; ++kk)
            if (kk <= J) s = fma(p[J - kk], c[kk], s);
        p[J] = s;
    }
}

// (p, dp) <- (p c, dp c + p dc): a product and its derivative, truncated to PD coefficients
template <int PD>
__device__ __forceinline__ void poly_mul_trunc_d(double (&p)[PD], double (&dp)[PD], const double (&c)[EZ_ELL_MAX + 1],
                                                 const double (&dc)[EZ_ELL_MAX + 1]) {
#pragma unroll
    for (int J = PD - 1; J >= 0; --J) {
        double s = 0.0, sd = 0.0;
#pragma unroll
        for (int kk = 0; kk <= EZ_ELL_MAX; ++kk) {
            if (kk <= J) {
                sd = fma(dp[J - kk], c[kk], fma(p[J - kk], dc[kk], sd));
                s = fma(p[J - kk], c[kk], s);
            }
        }
        p[J] = s;
        dp[J] = sd;
    }
}

// sum_{J <= deg} p_J fp int_0^eps u^{mu_J - 1} L^Q du with mu_J = d + E + 2J (returned),
// and the same with L^{Q-1} (in *s_qm1; 0 when Q = 0)
template <int D, int PD>
__device__ __forceinline__ double had_sum(const double (&p)[PD], int deg, double E, int Q, double eps, double Leps,
                                          double *s_qm1, bool *bad) {
    const double eps2 = eps * eps;
    double mu = (double)D + E;
    double em = pow(eps, mu);
    double acc = 0.0, accm = 0.0;
#pragma unroll
    for (int J = 0; J < PD; ++J) {
        if (J <= deg) {
            if (mu == 0.0) {
                *bad = true;
            } else {
                const double rmu = ez_rcp(mu);
                double I = em * rmu, Ip = 0.0, Lp = 1.0;
                for (int j = 1; j <= Q; ++j) {
                    Lp *= Leps;
                    Ip = I;
                    I = (em * Lp - 2.0 * (double)j * I) * rmu;
                }
                acc = fma(p[J], I, acc);
                accm = fma(p[J], Ip, accm);
            }
        }
        mu += 2.0;
        em *= eps2;
    }
    *s_qm1 = accm;
    return acc;
}

// Adjoint of the direction kernel: the (0, eps) part and its strain derivative.
// Under the strain G at fixed fractional direction, sigma |w|^e moves by
// -(I + e w w^T/|w|^2) times itself, L(u) = log(pi u^2 |w|^2) by -2 w w^T/|w|^2,
// and C_k by the strain channels of the tensors.  A workgroup takes ndb <=
// EZ_HDIR_GRAD directions (ndb n_combo <= 256).  Phase 1 contracts the tensors of
// every channel, one thread per (channel, direction, order k); in phase 2 one thread
// per (direction, combination) builds the product polynomial with its derivative
// along each of the d(d+1)/2 strain components; phase 3 sums the combinations in
// fixed order.
// LDS (dynamic, laid out by had_adj_lds): staged tensors, C_k per (direction,
// channel), direction data, and the value and derivatives per (direction, combination).
struct HadAdjLds {
    int tsh, csh, ssh, dsh, whsh, psh, vsh, bad, bytes;   // offsets in doubles; bytes in total
};

// tensor coefficients per channel: monomials of even degree <= 2 ell in D variables
__host__ __device__ inline int had_adj_tdim(int D, int ell) {
    int tdim = 0;
    for (int k = 0; k <= ell; ++k) tdim += nmono(D, 2 * k);
    return tdim;
}

// tdim: tensor coefficients per channel (of the largest Taylor order of the batch)
__host__ __device__ inline HadAdjLds had_adj_lds(int NNU, int NCH, int ndb, int nc, int tdim) {
    HadAdjLds L;
    const int ts = NCH * NNU * tdim < EZ_HADJ_TSTAGE ? NCH * NNU * tdim : EZ_HADJ_TSTAGE;
    L.tsh = 0;
    L.csh = ts;
    L.ssh = L.csh + ndb * NCH * NNU * (EZ_ELL_MAX + 1);
    L.dsh = L.ssh + ndb * NNU;
    L.whsh = L.dsh + ndb * 3;
    L.psh = L.whsh + ndb * 3;
    L.vsh = L.psh + ndb * 6;
    L.bad = L.vsh + ndb * nc * NCH;
    L.bytes = 8 * L.bad + 4 * ndb;
    return L;
}

template <int D, int NNU, int PD>
__global__ __launch_bounds__(256) void ez_hadamard_adj_kernel(EzQuadArgs args) {
    constexpr int NS = D * (D + 1) / 2;
    constexpr int NCH = 1 + NS;
    constexpr int KS = EZ_ELL_MAX + 1;
    extern __shared__ double lds_dyn[];
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
            const size_t gd = (size_t)(P.dir_begin + dl);
            for (int r = 0; r < n_res; ++r) {
                args.dir_part[gd * n_res + r] = 0.0;
                for (int s = 0; s < 6; ++s) args.dir_grad[(gd * n_res + r) * 6 + s] = 0.0;
            }
            args.dir_flag[gd] = 0;
        }
        return;
    }
    const HadAdjLds L = had_adj_lds(NNU, NCH, ndb, nc, had_adj_tdim(D, args.ell_probe));
    double *Tsh = lds_dyn + L.tsh;
    double *Csh = lds_dyn + L.csh;                              // [ndb][NCH][NNU][KS]
    double (*ssh)[NNU] = reinterpret_cast<double (*)[NNU]>(lds_dyn + L.ssh);   // sigma_i |w|^{nu_i - d}
    double (*dsh)[3] = reinterpret_cast<double (*)[3]>(lds_dyn + L.dsh);       // 2 w_v, log(pi eps^2 |w|^2), validity
    double (*whsh)[3] = reinterpret_cast<double (*)[3]>(lds_dyn + L.whsh);     // w_hat
    double (*psh)[6] = reinterpret_cast<double (*)[6]>(lds_dyn + L.psh);       // w_a w_b / |w|^2 per strain component
    double (*vsh)[NCH] = reinterpret_cast<double (*)[NCH]>(lds_dyn + L.vsh);   // per (direction, combination)
    uint32_t *fsh_bad = reinterpret_cast<uint32_t *>(lds_dyn + L.bad);
    const int tdim = had_adj_tdim(D, ell);
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
        for (int i = 0; i < 3; ++i) whsh[tid][i] = wh[i];
#pragma unroll
        for (int s = 0; s < NS; ++s) psh[tid][s] = w[ez_sa(D, s)] * w[ez_sb(D, s)] / w2;
        fsh_bad[tid] = 0u;
    }
    // phase 1: C_k(w) of every channel from the tensors, as many channels staged at a
    // time as the LDS holds (at least one: NNU tdim <= EZ_HADJ_TSTAGE)
    {
        const int NC = NNU * NCH;
        const int cb = min(NCH, EZ_HADJ_TSTAGE / (NNU * tdim));
        const double *T = args.tensor + (size_t)inst * NC * EZ_TDIM;
        for (int c0 = 0; c0 < NCH; c0 += cb) {
            const int cn = min(cb, NCH - c0);
            __syncthreads();
            for (int idx = tid; idx < cn * NNU * tdim; idx += 256) {
                const int row = idx / tdim;
                Tsh[idx] = T[(size_t)(c0 * NNU + row) * EZ_TDIM + (idx - row * tdim)];
            }
            __syncthreads();
            for (int idx = tid; idx < cn * ndb * (ell + 1); idx += 256) {
                const int cc = idx / (ndb * (ell + 1));
                const int r = idx - cc * ndb * (ell + 1);
                const int dd = r / (ell + 1), k = r - dd * (ell + 1);
                double acc[NNU];
                contract_order<D, NNU>(Tsh + cc * NNU * tdim, tdim, k, whsh[dd][0], whsh[dd][1], whsh[dd][2], acc);
                double *Co = Csh + ((size_t)(dd * NCH + c0 + cc) * NNU) * KS + k;
#pragma unroll
                for (int i = 0; i < NNU; ++i) Co[i * KS] = acc[i];
            }
        }
    }
    __syncthreads();

    // phase 2: one (direction, combination) per thread
    const int myd = tid / nc, myc = tid - myd * nc;
    bool bad = false;
    if (myd < ndb) {
        const EzCombo &cb = args.combo[myc];
        const int t = cb.t;
        const int nf = prog.term_nfac[t];
        double c = cb.coef, jsum = 0.0, jse = 0.0;
        int deg = 0, rest = 0;
        for (int f = 0; f < nf; ++f) {
            const int i = prog.term_fac[t][f];
            for (int q = 0; q < cb.j[f]; ++q) c *= ssh[myd][i];
            jsum += (double)cb.j[f];
            jse += (double)cb.j[f] * prog.e[i];
            for (int rep = 0; rep < prog.term_mult[t][f] - cb.j[f]; ++rep) deg = min(deg + ell, PD - 1);
            rest += prog.term_mult[t][f] - cb.j[f];
        }
        const double Leps = dsh[myd][1];
        const double *Cd = Csh + (size_t)myd * NCH * NNU * KS;
#pragma unroll 1
        for (int s = 0; s < NS; ++s) {
            // (p, dp): the product polynomial and its derivative along strain component s
            double p[PD], dp[PD];
            p[0] = 1.0;
            dp[0] = 0.0;
#pragma unroll
            for (int J = 1; J < PD; ++J) { p[J] = 0.0; dp[J] = 0.0; }
            // the Taylor factors of the product in one loop of `rest` multiplications
            // (factor f taken mult_f - j_f times in turn), so that the lanes of a wave,
            // which hold different combinations, differ only in its trip count
            int f = 0, left = nf > 0 ? prog.term_mult[t][0] - cb.j[0] : 0;
            for (int m = 0; m < rest; ++m) {
                while (left == 0) { ++f; left = prog.term_mult[t][f] - cb.j[f]; }
                --left;
                const int i = prog.term_fac[t][f];
                double Ck[EZ_ELL_MAX + 1], dCk[EZ_ELL_MAX + 1];
#pragma unroll
                for (int kk = 0; kk <= EZ_ELL_MAX; ++kk) {
                    Ck[kk] = (kk <= ell) ? Cd[i * KS + kk] : 0.0;
                    dCk[kk] = (kk <= ell) ? Cd[((1 + s) * NNU + i) * KS + kk] : 0.0;
                }
                poly_mul_trunc_d<PD>(p, dp, Ck, dCk);
            }
            double base_m1 = 0.0, dummy = 0.0;
            const double base = had_sum<D, PD>(p, deg, cb.E, cb.Q, P.eps, Leps, &base_m1, &bad);
            const double dsum = had_sum<D, PD>(dp, deg, cb.E, cb.Q, P.eps, Leps, &dummy, &bad);
            if (s == 0) vsh[tid][0] = c * base;
            const double Ps = psh[myd][s];
            const double delta = (s < D) ? 1.0 : 0.0;
            vsh[tid][1 + s] = c * (dsum + (-jsum * delta - jse * Ps) * base - 2.0 * (double)cb.Q * Ps * base_m1);
        }
        if (bad) atomicOr(&fsh_bad[myd], 1u);
    }
    __syncthreads();
    // phase 3: per direction, fixed-order sums over the combinations
    if (tid < ndb) {
        const int dl = d0 + tid;
        if (dl < P.n_dir) {
            const size_t gd = (size_t)(P.dir_begin + dl);
            for (int r = 0; r < n_res; ++r) {
                double h[NCH];
#pragma unroll
                for (int q = 0; q < NCH; ++q) h[q] = 0.0;
                for (int c = 0; c < nc; ++c)
                    if (args.combo[c].res == r) {
#pragma unroll
                        for (int q = 0; q < NCH; ++q) h[q] += vsh[tid * nc + c][q];
                    }
                args.dir_part[gd * n_res + r] = dsh[tid][0] * h[0];
                for (int s = 0; s < 6; ++s)
                    args.dir_grad[(gd * n_res + r) * 6 + s] = (s < NS) ? dsh[tid][0] * h[1 + s] : 0.0;
            }
            args.dir_flag[gd] = fsh_bad[tid];
        }
    }
}


template <int D, int NNU, int PD>
hipError_t launch_had_t(const EzQuadArgs &args, int n_htiles, hipStream_t stream, int part, hipEvent_t pre_done) {
    hipError_t e = hipSuccess;
    if (part & EZ_HAD_PRE) {            // probe values and Taylor tensors
        const int nblk = (args.n_probe + 63) / 64;
        const int nch = true ? args.n_ch : 1;
        // Taylor orders up to 4 (the usual plans) keep 5 coefficients per exponent in
        // registers, higher ones 9
        if (args.ell_probe <= 4)
            hipLaunchKernelGGL((ez_probe_kernel<D, NNU, true, 4>), dim3(args.batch * nblk * args.n_slice * nch),
                               dim3(64 * EZ_HW), (probe_lds_bytes<NNU, true>(args.ell_probe)), stream, args);
        else
            hipLaunchKernelGGL((ez_probe_kernel<D, NNU, true>), dim3(args.batch * nblk * args.n_slice * nch),
                               dim3(64 * EZ_HW), (probe_lds_bytes<NNU, true>(args.ell_probe)), stream, args);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        int tdim = 0;
        for (int k = 0; k <= args.ell_probe; ++k) tdim += nmono(D, 2 * k);
        const int ngrp = (tdim + EZ_TOUT - 1) / EZ_TOUT;
        // pre_done (if given) is recorded by the tensor launch itself: no marker packet
        // on `stream` between the tensors and the node kernel
        if (pre_done)
            hipExtLaunchKernelGGL((ez_tensor_kernel<D, NNU>), dim3(args.batch * NNU * nch * ngrp), dim3(256), 0, stream,
                                  nullptr, pre_done, 0, args);
        else
            hipLaunchKernelGGL((ez_tensor_kernel<D, NNU>), dim3(args.batch * NNU * nch * ngrp), dim3(256), 0, stream, args);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!(part & EZ_HAD_DIR)) return hipSuccess;   // direction kernel
    const HadAdjLds L = had_adj_lds(NNU, 1 + D * (D + 1) / 2, args.n_dir_blk, args.n_combo, had_adj_tdim(D, args.ell_probe));
    if (L.bytes > 160 * 1024) return hipErrorInvalidConfiguration;   // a CU's LDS on gfx950
    hipLaunchKernelGGL((ez_hadamard_adj_kernel<D, NNU, PD>), dim3(n_htiles), dim3(256), L.bytes, stream, args);
    return hipGetLastError();
}

template <int D, int NNU>
hipError_t launch_had_p(const EzQuadArgs &args, int n_htiles, hipStream_t stream, int part, hipEvent_t pre_done) {
    if (args.poly_deg == 13) return launch_had_t<D, NNU, 13>(args, n_htiles, stream, part, pre_done);
    if (args.poly_deg == 33) return launch_had_t<D, NNU, 33>(args, n_htiles, stream, part, pre_done);
    return hipErrorInvalidValue;
}

template <int D>
hipError_t launch_had_d(const EzQuadArgs &args, int n_htiles, hipStream_t stream, int part, hipEvent_t pre_done) {
    switch (args.prog.n_nu) {
        case 1: return launch_had_p<D, 1>(args, n_htiles, stream, part, pre_done);
        case 2: return launch_had_p<D, 2>(args, n_htiles, stream, part, pre_done);
        case 3: return launch_had_p<D, 3>(args, n_htiles, stream, part, pre_done);
        case 4: return launch_had_p<D, 4>(args, n_htiles, stream, part, pre_done);
        case 5: return launch_had_p<D, 5>(args, n_htiles, stream, part, pre_done);
        case 6: return launch_had_p<D, 6>(args, n_htiles, stream, part, pre_done);
        case 7: return launch_had_p<D, 7>(args, n_htiles, stream, part, pre_done);
        case 8: return launch_had_p<D, 8>(args, n_htiles, stream, part, pre_done);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t ez_launch_hadamard_adj(const EzQuadArgs &args, int n_htiles, hipStream_t stream, int part, hipEvent_t pre_done) {
    switch (args.prog.d) {
        case 1: return launch_had_d<1>(args, n_htiles, stream, part, pre_done);
        case 2: return launch_had_d<2>(args, n_htiles, stream, part, pre_done);
        case 3: return launch_had_d<3>(args, n_htiles, stream, part, pre_done);
        default: return hipErrorInvalidValue;
    }
}
