// ez_nodes_adj.hip -- the node kernel with its adjoint pass: values and strain
// derivatives of the results at the quadrature nodes on (eps, 1/2].
#include "ez_quad_common.h"

namespace {

// ---------------------------------------------------------------------------
// Adjoint of the node part.  Under the strain A -> (I + G) A at fixed fractional
// node coordinates, k.z is unchanged, |z|^2 moves by 2 z^T G z, |m* + k|^2 by
// -2 (m* + k)^T G (m* + k) and 1/V by -tr(G)/V; so with
//   dW/d|z|^2 = -Gamma(nu/2+1, .)/(Gamma(nu/2) |z|^{nu+2})  and  dE_p(a)/da = -E_{p-1}(a)
// the strain derivative of Z_nu(k) is
//   sum_pairs (4 W') cos(2 pi k.z) z z^T + sum_m* K [2 alpha E_{p-1} (m*+k)(m*+k)^T - E_p I].
// Pass 1 evaluates Z_nu and fbar_{r,nu} = W d f_r / d Z_nu; pass 2 walks the tables
// again and accumulates S_r = sum_nu fbar_{r,nu} dZ_nu/dG (symmetric, d(d+1)/2
// components: the diagonal, then (0,1), (0,2), (1,2)).  d result / d A = S A^{-T}.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void sym_acc(double *S, double t, const double *v) {
    // S += t v v^T
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double tv = t * v[a];
        S[a] = fma(tv, v[a], S[a]);
        if (D > 1 && a == 0) S[D] = fma(tv, v[1], S[D]);
        if (D > 2 && a == 0) S[D + 1] = fma(tv, v[2], S[D + 1]);
        if (D > 2 && a == 1) S[D + 2] = fma(tv, v[2], S[D + 2]);
    }
}

// The d = 3 ATM exponent set (set 1) takes 147 VGPRs unconstrained (three waves per
// SIMD, rounds of 768 tiles); held to four waves it spills 64 bytes per lane and
// runs the three-lattice ATM derivative 5% faster (709 against 746 us).
template <int D, int NNU, int SET, int NR>
__global__ __launch_bounds__(EZ_TILE) __attribute__((amdgpu_waves_per_eu(SET == 1 ? 5 : 1)))
void ez_node_adj_kernel(EzQuadArgs args) {
    constexpr int NS = D * (D + 1) / 2;
    const int tile = blockIdx.x;
    const int inst = find_segment(args.tile_begin, args.batch, tile);
    const EzInstPlan P = args.plans[inst];
    const EzLatMeta *M = args.meta + inst;
    const int n_res = args.prog.n_res;
    const int node = (tile - args.tile_begin[inst]) * EZ_TILE + threadIdx.x;
    const int n_nodes = P.n_dir * P.n_u;

    double res[NR], S[NR][NS];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        res[r] = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) S[r][s] = 0.0;
    }

    // reciprocal entries this tile needs, in table order (cull_reciprocal)
    __shared__ unsigned short klist[EZ_KCULL];
    __shared__ double kbox[EZ_TILE / 64][6];
    __shared__ int kwave[EZ_TILE / 64];
    __shared__ int kcount;

    if (M->status == 0) {                         // uniform over the workgroup
        const bool valid = node < n_nodes;
        // threads past the last node take the tile's first node (geometry only)
        const int nd = valid ? node : (tile - args.tile_begin[inst]) * EZ_TILE;
        const int dir = nd / P.n_u;
        const int iu = nd - dir * P.n_u;
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
        const double *kt = args.tab.rec + (size_t)inst * args.tab.rec_cap * 4;
        const int n_rec = M->n_rec;
        const double alpha = M->alpha, acut = M->a_cut;
        const bool need_e1 = pset_need_e1<SET, NNU>(args.prog), need_half = pset_need_half<SET, NNU>(args.prog);
        // m* = 0, then the culled list: the entries left out are beyond the cutoff for
        // every node of the tile, so both passes add the same terms in the same order
        const int nk = cull_reciprocal<D, EZ_TILE>(kt, n_rec, k, alpha, acut, klist, kbox, kwave, &kcount);
        auto entry = [&](int j) { return j == 0 ? 0 : __builtin_amdgcn_readfirstlane((int)klist[j - 1]); };
        if (valid) {

        // ---- pass 1: Z_nu(k) ----
        double accr[NNU], acck[NNU];
#pragma unroll
        for (int i = 0; i < NNU; ++i) { accr[i] = 0.0; acck[i] = 0.0; }
        {
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
        for (int j = 0; j <= nk; ++j) {
            const double *e = kt + (size_t)entry(j) * 4;
            double qv[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < D; ++i) qv[i] = e[i] + k[i];
            double rho = qv[0] * qv[0];
            if (D > 1) rho = fma(qv[1], qv[1], rho);
            if (D > 2) rho = fma(qv[2], qv[2], rho);
            const double a = alpha * rho;
            if (a <= acut) {
                const double ex = ez_expm(a);
                const double inv = ez_rcp(a);
                double E1 = 0.0;
                if (need_e1) E1 = (a < 0.25) ? ez_e1_small(a) : ex * ez_e1w_scaled(inv);
                const double Eh = need_half ? ((a < 0.25) ? ez_ehalf(a) : ex * inv * ez_ehw_scaled(inv)) : 0.0;
#pragma unroll
                for (int i = 0; i < NNU; ++i)
                    acck[i] += ez_ep_from(pset_p2<SET>(args.prog, i), a, ex, inv, E1, Eh);
            }
        }
        double Z[NNU];
#pragma unroll
        for (int i = 0; i < NNU; ++i) Z[i] = accr[i] + M->K[i] * acck[i] - M->self_[i];

        // ---- results and fbar = W d f_r / d Z_nu ----
        double fb[NR][NNU];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int i = 0; i < NNU; ++i) fb[r][i] = 0.0;
        for (int t = 0; t < args.prog.n_terms; ++t) {
            const int nf = args.prog.term_nfac[t];
            const int rr = args.prog.term_res[t];
            double zf[EZ_FAC_MAX], pf[EZ_FAC_MAX];
            double prod = args.prog.term_coef[t];
            for (int f = 0; f < EZ_FAC_MAX; ++f) {
                zf[f] = 1.0;
                pf[f] = 1.0;
                if (f < nf) {
                    const int fi = args.prog.term_fac[t][f];
                    double z = Z[0];
#pragma unroll
                    for (int i = 1; i < NNU; ++i) z = (fi == i) ? Z[i] : z;
                    zf[f] = z;
                    const int m = args.prog.term_mult[t][f];
                    double pm1 = 1.0;
                    for (int q = 1; q < m; ++q) pm1 *= z;
                    pf[f] = pm1;                      // z^{m-1}
                    prod *= pm1 * z;
                }
            }
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (rr == r) res[r] += prod;
            for (int f = 0; f < nf; ++f) {
                // d/dz_f of coef prod_g z_g^{m_g} = coef m_f z_f^{m_f - 1} prod_{g != f} z_g^{m_g}
                double part = args.prog.term_coef[t] * (double)args.prog.term_mult[t][f] * pf[f];
                for (int g = 0; g < nf; ++g)
                    if (g != f) part *= pf[g] * zf[g];
                const int fi = args.prog.term_fac[t][f];
#pragma unroll
                for (int r = 0; r < NR; ++r)
#pragma unroll
                    for (int i = 0; i < NNU; ++i)
                        if (rr == r && fi == i) fb[r][i] += part;
            }
        }
        // fbar K_nu, and the -E_p I part of the reciprocal derivative (sum over m* known from pass 1)
        double fbK[NR][NNU];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            res[r] *= W;
            double diag = 0.0;
#pragma unroll
            for (int i = 0; i < NNU; ++i) {
                fb[r][i] *= W;
                fbK[r][i] = fb[r][i] * M->K[i];
                diag = fma(fbK[r][i], acck[i], diag);
            }
#pragma unroll
            for (int a = 0; a < D; ++a) S[r][a] = -diag;
        }

        // ---- pass 2, real space: S_r += cos(2 pi k.z) (sum_nu fbar 4W') z z^T ----
        {
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
                    double z[3] = {e[0], e[1], e[2]};
#pragma unroll
                    for (int r2 = 0; r2 < NR; ++r2) {
                        double g = 0.0;
#pragma unroll
                        for (int i = 0; i < NNU; ++i) g = fma(fb[r2][i], e[3 + NNU + i], g);
                        sym_acc<D>(S[r2], g * pr, z);
                    }
                    cmul(pr, pi, c1r, c1i);
                }
            }
        }
        // ---- pass 2, reciprocal space: S_r += 2 alpha (sum_nu fbar K E_{p-1}) (m*+k)(m*+k)^T ----
        for (int j = 0; j <= nk; ++j) {
            const double *e = kt + (size_t)entry(j) * 4;
            double qv[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < D; ++i) qv[i] = e[i] + k[i];
            double rho = qv[0] * qv[0];
            if (D > 1) rho = fma(qv[1], qv[1], rho);
            if (D > 2) rho = fma(qv[2], qv[2], rho);
            const double a = alpha * rho;
            if (a <= acut) {
                const double ex = ez_expm(a);
                const double inv = ez_rcp(a);
                double E1 = 0.0;
                if (need_e1) E1 = (a < 0.25) ? ez_e1_small(a) : ex * ez_e1w_scaled(inv);
                const double Eh = need_half ? ((a < 0.25) ? ez_ehalf(a) : ex * inv * ez_ehw_scaled(inv)) : 0.0;
                double Em[NNU];
#pragma unroll
                for (int i = 0; i < NNU; ++i) Em[i] = ez_ep_from(pset_p2<SET>(args.prog, i) - 2, a, ex, inv, E1, Eh);
#pragma unroll
                for (int r2 = 0; r2 < NR; ++r2) {
                    double h = 0.0;
#pragma unroll
                    for (int i = 0; i < NNU; ++i) h = fma(fbK[r2][i], Em[i], h);
                    sym_acc<D>(S[r2], 2.0 * alpha * h, qv);
                }
            }
        }
        }   // valid
    }

    // tile reduction of the values and the strain tensors
    __shared__ double red[NR * (1 + NS)][EZ_TILE / 64][2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (r < n_res) {
            ez_dd v = ez_dd_wave_sum(ez_dd{res[r], 0.0});
            if (lane == 0) { red[r * (1 + NS)][wave][0] = v.hi; red[r * (1 + NS)][wave][1] = v.lo; }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                ez_dd g = ez_dd_wave_sum(ez_dd{S[r][s], 0.0});
                if (lane == 0) { red[r * (1 + NS) + 1 + s][wave][0] = g.hi; red[r * (1 + NS) + 1 + s][wave][1] = g.lo; }
            }
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < n_res * (1 + NS)) {
        const int c = threadIdx.x;
        const int r = c / (1 + NS), s = c - r * (1 + NS) - 1;
        ez_dd t{red[c][0][0], red[c][0][1]};
        for (int wv = 1; wv < EZ_TILE / 64; ++wv) t = ez_dd_add(t, ez_dd{red[c][wv][0], red[c][wv][1]});
        if (s < 0) {
            args.tile_part[((size_t)tile * n_res + r) * 2 + 0] = t.hi;
            args.tile_part[((size_t)tile * n_res + r) * 2 + 1] = t.lo;
        } else {
            args.tile_grad[(((size_t)tile * n_res + r) * 6 + s) * 2 + 0] = t.hi;
            args.tile_grad[(((size_t)tile * n_res + r) * 6 + s) * 2 + 1] = t.lo;
        }
    }
}


template <int D, int NNU, int SET>
hipError_t launch_nodes_adj_t(const EzQuadArgs &args, int n_tiles, hipStream_t stream) {
    if (args.prog.n_res == 1)
        hipLaunchKernelGGL((ez_node_adj_kernel<D, NNU, SET, 1>), dim3(n_tiles), dim3(EZ_TILE), 0, stream, args);
    else
        hipLaunchKernelGGL((ez_node_adj_kernel<D, NNU, SET, 2>), dim3(n_tiles), dim3(EZ_TILE), 0, stream, args);
    return hipGetLastError();
}

template <int D>
hipError_t launch_nodes_adj_d(const EzQuadArgs &args, int n_tiles, hipStream_t stream) {
    if (D == 3 && args.prog.pset == 1) return launch_nodes_adj_t<D, 4, 1>(args, n_tiles, stream);
    switch (args.prog.n_nu) {
        case 1: return launch_nodes_adj_t<D, 1, 0>(args, n_tiles, stream);
        case 2: return launch_nodes_adj_t<D, 2, 0>(args, n_tiles, stream);
        case 3: return launch_nodes_adj_t<D, 3, 0>(args, n_tiles, stream);
        case 4: return launch_nodes_adj_t<D, 4, 0>(args, n_tiles, stream);
        case 5: return launch_nodes_adj_t<D, 5, 0>(args, n_tiles, stream);
        case 6: return launch_nodes_adj_t<D, 6, 0>(args, n_tiles, stream);
        case 7: return launch_nodes_adj_t<D, 7, 0>(args, n_tiles, stream);
        case 8: return launch_nodes_adj_t<D, 8, 0>(args, n_tiles, stream);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t ez_launch_nodes_adj(const EzQuadArgs &args, int n_tiles, hipStream_t stream) {
    switch (args.prog.d) {
        case 1: return launch_nodes_adj_d<1>(args, n_tiles, stream);
        case 2: return launch_nodes_adj_d<2>(args, n_tiles, stream);
        case 3: return launch_nodes_adj_d<3>(args, n_tiles, stream);
        default: return hipErrorInvalidValue;
    }
}
