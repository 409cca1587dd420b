// ez_internal.h -- structures shared by the host and the kernels of libezeta.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define EZ_NU_MAX 8      // distinct exponents per call
#define EZ_TERM_MAX 8    // product terms per call
#define EZ_FAC_MAX 4     // distinct factors per term
#define EZ_RES_MAX 8     // results per lattice
#define EZ_ELL_MAX 8     // Taylor cutoff
#define EZ_MULT_MAX 64   // total degree of a product term
#define EZ_TILE 256      // quadrature nodes per workgroup of the node kernel
#define EZ_TDIM 525      // monomials of even degree <= 2 EZ_ELL_MAX in 3 variables
#define EZ_HDIR 64       // quadrature directions per workgroup of the Hadamard direction kernel
#define EZ_KCULL 8192    // reciprocal table capacity per lattice in the quadrature (node tiles list it in LDS)
#define EZ_SLICE_MAX 8   // table slices of the probe kernel
#define EZ_GRAD_RES_MAX 2  // results per call when strain derivatives are requested
#define EZ_TAIL_WAVES 4  // waves per workgroup of the tail node kernel
#define EZ_TAIL_PARTS 4  // workgroups sharing one 64-node group of the tail node tiles

// Which lattice sums one call computes (host-built, passed by value).
// Exponent nu_i enters the reciprocal sum through E_{p_i}(a), p_i = (nu_i - d + 2)/2
// (E_p the generalised exponential integral), so 2 p_i = nu_i - d + 2 is an integer.
struct EzProgram {
    int d, n_nu, n_res, n_terms;
    double nu[EZ_NU_MAX];
    int p2[EZ_NU_MAX];      // 2 p_i
    int logm[EZ_NU_MAX];    // m if nu_i = d + 2m (logarithmic singular part), else -1
    double e[EZ_NU_MAX];    // nu_i - d, exponent of the singular part
    int term_res[EZ_TERM_MAX];
    double term_coef[EZ_TERM_MAX];
    int term_nfac[EZ_TERM_MAX];
    int term_fac[EZ_TERM_MAX][EZ_FAC_MAX];
    int term_mult[EZ_TERM_MAX][EZ_FAC_MAX];
    int need_e1;            // some p_i is an integer >= 1
    int need_half;          // some p_i is a half-integer
    int pset;               // id of a compile-time exponent set matching p2, or 0
    int real_nu;            // some nu_i is not an integer: p2 unused, E_p from preal
    double preal[EZ_NU_MAX];// p_i = (nu_i - d + 2)/2
};

// Exponent sets with kernels specialised at compile time (2 p_i = nu_i - d + 2);
// set 0 reads the exponents at run time.
struct EzPSet { int n; int p2[EZ_NU_MAX]; };
#define EZ_NPSETS 5
#define EZ_PSET_REAL 15     // kernels for real (non-integer) exponents: E_p per exponent
__host__ __device__ constexpr EzPSet ez_pset(int id) {
    return id == 1 ? EzPSet{4, {-2, 0, 2, 4}}                 // d = 3, nu = -1, 1, 3, 5 (ATM)
         : id == 2 ? EzPSet{4, {-1, 1, 3, 5}}                 // d = 2, ATM
         : id == 3 ? EzPSet{4, {0, 2, 4, 6}}                  // d = 1, ATM
         : id == 4 ? EzPSet{7, {-2, 0, 2, 4, 5, 8, 11}}       // d = 3, ATM and nu = 6, 9, 12
                   : EzPSet{0, {0}};
}

// Per-lattice constants written by the setup kernel.
struct EzLatMeta {
    double A[9], B[9];      // row-major; B = A^{-T}
    double V, lam, alpha;   // |det A|, Ewald parameter, pi lam^2
    double a_cut;
    double K[EZ_NU_MAX];    // pi^{nu-d/2} / (Gamma(nu/2) V) * alpha^{(d-nu)/2}
    double self_[EZ_NU_MAX];// (pi/lam^2)^{nu/2} / Gamma(nu/2 + 1)
    double sig[EZ_NU_MAX];  // s_hat(k)/V = sig |k|^{nu-d} [ * log(pi |k|^2) ]
    int n_real;             // real-space entries (pairs +-z stored once)
    int n_rec;              // reciprocal entries (all m*, m* = 0 first)
    uint32_t status;
    int n_rows;             // rows of the real-space table (pairs mode)
    int pad_[2];
};

// Per-lattice quadrature plan (host-built).
// The nodes (direction, u-node) of a lattice are grouped into wave blocks of 64:
// db directions x ub consecutive u-nodes (ub = 2^ub_log2, db ub = 64), blocks
// numbered direction group first, u-chunk fastest; a node tile (one workgroup
// of the node kernel) is four consecutive blocks.
struct EzInstPlan {
    int n_q, n_u, n_dir, ell;
    int tile_begin;         // first node tile of this lattice
    int dir_begin;          // first direction of this lattice (Hadamard output)
    int vrule;              // offset of the n_q-point Gauss rule on [0,1] (nodes, then weights)
    int urule;              // offset of the n_u u-nodes on (eps,1/2] (nodes, then weights)
    int ub_log2, db;        // wave block: 2^ub_log2 u-nodes x db directions
    int n_ublk, n_wblk;     // u-chunks per direction group, wave blocks of the lattice
    double eps;
    double lam_rel;         // Ewald parameter in units of V^{1/d}
};

// Real-space table (pairs mode): points ordered by (n3, n2, n1), so that each
// row (n2, n3 fixed) is a run of consecutive n1.  A row record holds
// {first point, count, n1 of the first point, n2, n3, starts a new plane,
//  n1 shift from the previous row's first point, n2 step from the previous row}.
struct EzTables {
    int real_cap, rec_cap, rstride, row_cap;  // capacities per lattice, doubles per real entry
    double *real;                     // [batch][real_cap][rstride]: z (3), 2 W_nu(z) (n_nu)
    int *rn;                          // [batch][real_cap][4]: integer coordinates of each point
    int *rows;                        // [batch][row_cap][8]: row records
    double *rec;                      // [batch][rec_cap][4]: m* (3), |m*|^2
};

#define EZ_PI 3.141592653589793238462643383279502884
#define EZ_EULER 0.577215664901532860606512090082402431
