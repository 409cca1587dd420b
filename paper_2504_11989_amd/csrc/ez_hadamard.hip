// ez_hadamard.hip -- the Hadamard part on (0, eps) (paper, Sec. 3, Taylor
// expansion of Z^reg and closed-form Hadamard integrals): probe, tensor and
// direction kernels.
#include <hip/hip_ext.h>

#include "ez_hadamard_common.h"

namespace {

template <int D, int NNU, int PD>
__global__ __launch_bounds__(256) void ez_hadamard_kernel(EzQuadArgs args) {
    __shared__ double Tsh[NNU * EZ_TDIM];
    __shared__ double Csh[EZ_HDIR][NNU][EZ_ELL_MAX + 1];
    __shared__ double ssh[EZ_HDIR][NNU];   // sigma_i |w|^{nu_i - d}
    __shared__ double dsh[EZ_HDIR][3];     // 2 w_v, log(pi eps^2 |w|^2), validity
    __shared__ double whsh[EZ_HDIR][3];    // w_hat
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
        fsh_bad[tid] = 0u;
    }
    // phase 1: C_k(w) from the tensors
    contract_tensor<D, NNU>(args, inst, 0, NNU, ndb, ell, tdim, Tsh, whsh, &Csh[0][0][0], NNU * (EZ_ELL_MAX + 1),
                            EZ_ELL_MAX + 1);
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
        int deg = 0, rest = 0;
        for (int f = 0; f < nf; ++f) {
            const int i = prog.term_fac[t][f];
            for (int q = 0; q < cb.j[f]; ++q) c *= ssh[myd][i];
            for (int rep = 0; rep < prog.term_mult[t][f] - cb.j[f]; ++rep) deg = min(deg + ell, PD - 1);
            rest += prog.term_mult[t][f] - cb.j[f];
        }
        // the Taylor factors in one loop of `rest` multiplications (factor f taken
        // mult_f - j_f times in turn): the lanes of a wave hold different combinations
        // and differ only in its trip count
        int f = 0, left = nf > 0 ? prog.term_mult[t][0] - cb.j[0] : 0;
        for (int m = 0; m < rest; ++m) {
            while (left == 0) { ++f; left = prog.term_mult[t][f] - cb.j[f]; }
            --left;
            const int i = prog.term_fac[t][f];
            double Ck[EZ_ELL_MAX + 1];
#pragma unroll
            for (int kk = 0; kk <= EZ_ELL_MAX; ++kk) Ck[kk] = (kk <= ell) ? Csh[myd][i][kk] : 0.0;
            // poly <- poly * sum_k C_k u^{2k}, truncated to PD coefficients
#pragma unroll
            for (int J = PD - 1; J >= 0; --J) {
                double sacc = 0.0;
#pragma unroll
                for (int kk = 0; kk <= EZ_ELL_MAX; ++kk)
                    if (kk <= J) sacc = fma(poly[J - kk], Ck[kk], sacc);
                poly[J] = sacc;
            }
        }
        // fp int_0^eps u^{mu-1} L^Q du, mu = d + E + 2J:
        //   I_0 = eps^mu/mu,  I_q = (eps^mu L(eps)^q - 2q I_{q-1})/mu
        const double eps = P.eps, eps2 = eps * eps;
        const double Leps = dsh[myd][1];
        double mu = (double)D + cb.E;
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

// poly <- poly * sum_k c_k u^{2k}, truncated to PD coefficients

template <int D, int NNU, int PD>
hipError_t launch_had_t(const EzQuadArgs &args, int n_htiles, hipStream_t stream, int part, hipEvent_t pre_done) {
    hipError_t e = hipSuccess;
    if (part & EZ_HAD_PRE) {            // probe values and Taylor tensors
        const int nblk = (args.n_probe + 63) / 64;
        const int nch = false ? args.n_ch : 1;
        hipLaunchKernelGGL((ez_probe_kernel<D, NNU, false>), dim3(args.batch * nblk * args.n_slice * nch), dim3(64 * EZ_HW),
                           (probe_lds_bytes<NNU, false>(args.ell_probe)), stream, args);
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
    hipLaunchKernelGGL((ez_hadamard_kernel<D, NNU, PD>), dim3(n_htiles), dim3(256), 0, stream, args);
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

hipError_t ez_launch_hadamard(const EzQuadArgs &args, int n_htiles, hipStream_t stream, int part, hipEvent_t pre_done) {
    switch (args.prog.d) {
        case 1: return launch_had_d<1>(args, n_htiles, stream, part, pre_done);
        case 2: return launch_had_d<2>(args, n_htiles, stream, part, pre_done);
        case 3: return launch_had_d<3>(args, n_htiles, stream, part, pre_done);
        default: return hipErrorInvalidValue;
    }
}
