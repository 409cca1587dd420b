// ez_direct.hip -- direct summation of the Axilrod-Teller-Muto lattice sum over a
// box of the lattice, an independent check of the Epstein zeta method (paper,
// Sec. 4.3: the two-dimensional square lattice compared with direct sums).
//
//   E_L = (1/6) sum_{x, y in A{-L..L}^d, x != 0, y != 0, x != y} U(x, y),
//   U(x, y) = 1/r^3 - 3 (x.y)(y.z)(z.x)/r^5,  z = y - x,  r = |x| |y| |z|
//
// (the ATM potential of the triangle 0, x, y: (1 + 3 cos g1 cos g2 cos g3) /
// (|x| |y| |z|)^3).  The outer points x come from a host list with weights: every
// nonzero box point with weight 1, or, when the lattice metric is a multiple of the
// identity (square and cubic lattices, whose box is invariant under the signed
// permutations of the coordinates), one point per orbit of that group with the
// orbit size as weight.  Workgroups take 256 outer points and one contiguous chunk
// of the inner points; each thread adds its terms in a double-double sum, the
// workgroup adds its threads in fixed order, and a last kernel adds the partials in
// fixed order, so the result is deterministic.
#include "ez_internal.h"
#include "ez_math.h"
#include "ez_kernels.h"

namespace {

constexpr int DT = 256;

template <int D>
__global__ __launch_bounds__(DT) void direct_atm_kernel(EzDirectArgs g) {
    __shared__ double red[DT / 64][2];
    const int xi = (int)blockIdx.x * DT + (int)threadIdx.x;
    const int chunk = (int)blockIdx.y;
    const long long M = 2ll * g.L + 1;
    const long long y0 = (long long)chunk * g.per_chunk;
    const long long y1 = min(g.n_box, y0 + g.per_chunk);
    double x[3] = {0.0, 0.0, 0.0}, w = 0.0;
    if (xi < g.n_x) {
        const int *nx = g.xlist + (size_t)xi * 4;
        w = (double)nx[3];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) s = fma(g.A[i * 3 + j], (double)nx[j], s);
            x[i] = s;
        }
    }
    double xx = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) xx = fma(x[i], x[i], xx);
    ez_dd acc{0.0, 0.0};
    // inner point of index k: n = (k mod M, k / M mod M, k / M^2) - L, uniform over the
    // wave; decomposed once, then advanced as an odometer
    int c[3] = {0, 0, 0};
    {
        long long q = y0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            c[j] = (int)(q % M) - g.L;
            q /= M;
        }
    }
    for (long long k = y0; k < y1; ++k) {
        double ny[3] = {0.0, 0.0, 0.0};
        bool zero = true;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            ny[j] = (double)c[j];
            zero = zero && c[j] == 0;
        }
        // next index
        ++c[0];
#pragma unroll
        for (int j = 0; j + 1 < D; ++j)
            if (c[j] > g.L) { c[j] = -g.L; ++c[j + 1]; }
        if (zero) continue;
        double y[3] = {0.0, 0.0, 0.0}, yy = 0.0, zz = 0.0, xy = 0.0, yz = 0.0, zx = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) s = fma(g.A[i * 3 + j], ny[j], s);
            y[i] = s;
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double zi = y[i] - x[i];
            yy = fma(y[i], y[i], yy);
            zz = fma(zi, zi, zz);
            xy = fma(x[i], y[i], xy);
            yz = fma(y[i], zi, yz);
            zx = fma(zi, x[i], zx);
        }
        const double r2 = xx * yy * zz;
        if (r2 > 0.0) {                        // z = 0 (y = x) and padding lanes add nothing
            const double ir = 1.0 / sqrt(r2);
            const double ir3 = ir * ir * ir;
            const double U = ir3 - 3.0 * xy * yz * zx * (ir3 * ir * ir);
            acc = ez_dd_add_d(acc, w * U);
        }
    }
    acc = ez_dd_wave_sum(acc);
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    if (lane == 0) { red[wave][0] = acc.hi; red[wave][1] = acc.lo; }
    __syncthreads();
    if (threadIdx.x == 0) {
        ez_dd s{red[0][0], red[0][1]};
        for (int v = 1; v < DT / 64; ++v) s = ez_dd_add(s, ez_dd{red[v][0], red[v][1]});
        const size_t o = ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 2;
        g.part[o] = s.hi;
        g.part[o + 1] = s.lo;
    }
}

// fixed-order double-double sum of the n partials (one workgroup), / 6
__global__ __launch_bounds__(DT) void direct_finish_kernel(const double *part, long long n, double *out) {
    __shared__ double red[DT / 64][2];
    ez_dd s{0.0, 0.0};
    for (long long i = threadIdx.x; i < n; i += DT) s = ez_dd_add(s, ez_dd{part[2 * i], part[2 * i + 1]});
    s = ez_dd_wave_sum(s);
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    if (lane == 0) { red[wave][0] = s.hi; red[wave][1] = s.lo; }
    __syncthreads();
    if (threadIdx.x == 0) {
        ez_dd t{red[0][0], red[0][1]};
        for (int v = 1; v < DT / 64; ++v) t = ez_dd_add(t, ez_dd{red[v][0], red[v][1]});
        out[0] = (t.hi + t.lo) / 6.0;
    }
}

}  // namespace

// number of partial sums the kernels write for a launch of n_x outer points
long long ez_direct_parts(long long n_x, int n_chunks) { return ((n_x + DT - 1) / DT) * (long long)n_chunks; }

hipError_t ez_launch_direct_atm(const EzDirectArgs &g, int n_chunks, double *out, hipStream_t stream) {
    const dim3 grid((unsigned)((g.n_x + DT - 1) / DT), (unsigned)n_chunks);
    switch (g.d) {
        case 1: hipLaunchKernelGGL(direct_atm_kernel<1>, grid, dim3(DT), 0, stream, g); break;
        case 2: hipLaunchKernelGGL(direct_atm_kernel<2>, grid, dim3(DT), 0, stream, g); break;
        case 3: hipLaunchKernelGGL(direct_atm_kernel<3>, grid, dim3(DT), 0, stream, g); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(direct_finish_kernel, dim3(1), dim3(DT), 0, stream, (const double *)g.part,
                       ez_direct_parts(g.n_x, n_chunks), out);
    return hipGetLastError();
}
