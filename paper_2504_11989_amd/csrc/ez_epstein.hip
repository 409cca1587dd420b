// ez_epstein.hip -- Z_{Lambda,nu}(x, y) at arbitrary x, y (paper, Sec. 2,
// Definition (Epstein zeta function)) by the incomplete-gamma split:
//
//  Z(x,y) = sum_{z != x} e^{-2 pi i y.z} Gamma(nu/2, pi|z-x|^2/lam^2) / (Gamma(nu/2) |z-x|^nu)
//         + pi^{nu-d/2}/(Gamma(nu/2) V) sum_{m*} e^{-2 pi i (m*+y).x} |m*+y|^{nu-d} Gamma((d-nu)/2, pi lam^2 |m*+y|^2)
//         - [x in Lambda] (pi/lam^2)^{nu/2} / Gamma(nu/2 + 1)
//
// x is first reduced to the cell A[-1/2,1/2)^d (quasi-periodicity
// Z(x + z0, y) = e^{-2 pi i y.z0} Z(x, y)) and y to B[-1/2,1/2)^d (periodicity in
// Lambda*), so that one real-space table (|z| <= lam sqrt(a_cut/pi) + r_cell)
// and one reciprocal table serve every point.  A coordinate within 1e-12 of an
// integer is snapped onto the lattice; at y in Lambda* the m* + y = 0 term takes
// its continuation in nu, -(pi lam^2)^s / s with s = (d - nu)/2.
// One thread per (nu, point).
#include "ez_internal.h"
#include "ez_math.h"
#include "ez_kernels.h"

namespace {

__global__ __launch_bounds__(256) void ez_epstein_kernel(EzEpsteinArgs args) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)args.n_nu * args.n_pts;
    if (gid >= total) return;
    const int j = (int)(gid / args.n_pts);
    const long long i = gid - (long long)j * args.n_pts;
    const int d = args.d;
    const EzLatMeta *M = args.meta;
    double *o = args.out + 2 * gid;
    if (M->status != 0) {
        o[0] = o[1] = __longlong_as_double(0x7ff8000000000000ll);
        return;
    }
    const double nu = args.nu[j];
    double A[9], B[9];
    for (int t = 0; t < 9; ++t) { A[t] = M->A[t]; B[t] = M->B[t]; }
    double x[3] = {0, 0, 0}, y[3] = {0, 0, 0};
    for (int t = 0; t < d; ++t) { x[t] = args.x[i * d + t]; y[t] = args.y[i * d + t]; }

    // fractional coordinates: A^{-1} x = B^T x,  A^T y
    double f[3] = {0, 0, 0}, g[3] = {0, 0, 0};
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            f[r] += B[c * d + r] * x[c];
            g[r] += A[c * d + r] * y[c];
        }
    double n0[3] = {0, 0, 0}, m0[3] = {0, 0, 0};
    bool xin = true, yin = true;
    for (int r = 0; r < d; ++r) {
        n0[r] = rint(f[r]);
        m0[r] = rint(g[r]);
        if (fabs(f[r] - n0[r]) >= 1e-12) xin = false;
        if (fabs(g[r] - m0[r]) >= 1e-12) yin = false;
    }
    double xr[3] = {0, 0, 0}, yr[3] = {0, 0, 0};
    if (!xin)
        for (int r = 0; r < d; ++r) {
            double s = x[r];
            for (int c = 0; c < d; ++c) s -= A[r * d + c] * n0[c];
            xr[r] = s;
        }
    if (!yin)
        for (int r = 0; r < d; ++r) {
            double s = y[r];
            for (int c = 0; c < d; ++c) s -= B[r * d + c] * m0[c];
            yr[r] = s;
        }
    // phase of the quasi-periodicity: y.z0 = (A^T y).n0, reduced mod 1 in fractional form
    double ph0 = 0.0;
    for (int r = 0; r < d; ++r) {
        double gi = g[r] - rint(g[r]);
        ph0 += gi * n0[r];
    }

    const double lam = M->lam, lam2 = lam * lam, alpha = M->alpha, acut = M->a_cut;
    const double rg = ez_rgamma(0.5 * nu);
    double sre = 0.0, sim = 0.0;
    const int rs = args.tab.rstride;
    for (int p = 0; p < M->n_real; ++p) {
        const double *e = args.tab.real + (size_t)p * rs;
        double r2 = 0.0, yz = 0.0;
        for (int t = 0; t < d; ++t) {
            double rt = e[t] - xr[t];
            r2 += rt * rt;
            yz += yr[t] * e[t];
        }
        if (r2 == 0.0) continue;                 // z = x (x on the lattice)
        const double a = EZ_PI * r2 / lam2;
        if (a > acut) continue;
        const double wgt = ez_gamma_upper(0.5 * nu, a) * rg * pow(r2, -0.5 * nu);
        double sn, cs;
        ez_sincos2pi(-yz, &sn, &cs);
        sre += wgt * cs;
        sim += wgt * sn;
    }
    const double s = 0.5 * ((double)d - nu);
    double kre = 0.0, kim = 0.0;
    for (int q = 0; q < M->n_rec; ++q) {
        const double *e = args.tab.rec + (size_t)q * 4;
        double qv[3] = {0, 0, 0}, r2 = 0.0, qx = 0.0;
        for (int t = 0; t < d; ++t) {
            qv[t] = e[t] + yr[t];
            r2 += qv[t] * qv[t];
            qx += qv[t] * xr[t];
        }
        double val;
        if (r2 == 0.0) {                         // m* + y = 0: continuation in nu
            if (s == 0.0) {
                if (args.status) atomicOr(args.status, 0x10u);
                val = __longlong_as_double(0x7ff8000000000000ll);
            } else {
                val = -pow(alpha, s) / s;
            }
        } else {
            const double a = alpha * r2;
            if (a > acut) continue;
            val = pow(r2, -s) * ez_gamma_upper(s, a);
        }
        double sn, cs;
        ez_sincos2pi(-qx, &sn, &cs);
        kre += val * cs;
        kim += val * sn;
    }
    const double pref = pow(EZ_PI, nu - 0.5 * d) * rg / M->V;
    double zre = sre + pref * kre, zim = sim + pref * kim;
    if (xin) zre -= pow(EZ_PI / lam2, 0.5 * nu) * ez_rgamma(0.5 * nu + 1.0);
    double sn, cs;
    ez_sincos2pi(-ph0, &sn, &cs);
    o[0] = zre * cs - zim * sn;
    o[1] = zre * sn + zim * cs;
}

}  // namespace

hipError_t ez_launch_epstein(const EzEpsteinArgs &args, hipStream_t stream) {
    const long long total = (long long)args.n_nu * args.n_pts;
    if (total == 0) return hipSuccess;
    const long long blocks = (total + 255) / 256;
    hipLaunchKernelGGL(ez_epstein_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, args);
    return hipGetLastError();
}
