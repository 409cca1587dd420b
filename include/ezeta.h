/*
 * ezeta.h -- C ABI of libezeta, the MI355X (gfx950) implementation of the
 * Epstein zeta method for many-body lattice sums (Buchheit & Busse,
 * arXiv 2504.11989).
 *
 * Conventions shared by every entry point
 *  - d in {1, 2, 3}.  A lattice is given by its generator matrix A, d x d,
 *    row-major, whose COLUMNS are the basis vectors: Lambda = A Z^d,
 *    Lambda* = A^{-T} Z^d, V = |det A| (paper, Sec. 2, Definition (Lattices)).
 *  - Pointers named *_dev are device pointers (HBM of the current HIP device);
 *    pointers named *_host are host pointers.  The caller owns every buffer it
 *    passes.  The library owns its cached workspace, rule tables and plans,
 *    keyed by device, and frees them in ez_finalize().
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every entry point
 *    only enqueues work on `stream` and returns; results are valid once the
 *    stream has been synchronised.  Host arguments are consumed before return.
 *  - Argument errors are detected on the host before any launch and returned
 *    as ez_status; per-lattice problems found on the device (singular or
 *    too-skewed lattice, non-finite result) set bits in status_dev[i] and
 *    write NaN to that lattice's results without failing the batch.  Every
 *    status_dev entry is written by the call (no zeroing needed beforehand).
 *  - Calls that overlap on one device are serialised by the caller's stream
 *    order; the library workspace is shared per device, so concurrent calls
 *    from different host threads on one device must use one stream.
 */
#ifndef EZETA_H
#define EZETA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EZ_OK = 0,
    EZ_ERR_INVALID_ARG = 1,      /* bad d, sizes, null pointer, bad spec          */
    EZ_ERR_SINGULAR_LATTICE = 2, /* reserved for host-side lattice checks         */
    EZ_ERR_POLE = 3,             /* exponent on a pole of the requested function  */
    EZ_ERR_UNSUPPORTED = 4,      /* Hadamard exponent mu + 2k = 0 (paper, Sec. 3)  */
    EZ_ERR_NOMEM = 5,            /* device allocation failed                      */
    EZ_ERR_HIP = 6               /* a HIP runtime call failed                     */
} ez_status;

/* bits of status_dev[i] */
#define EZ_FLAG_SINGULAR 0x1u   /* A not finite or |det A| <= 1e-300               */
#define EZ_FLAG_CAPACITY 0x2u   /* lattice too skewed for the point-table capacity */
#define EZ_FLAG_NONFINITE 0x4u  /* a result came out NaN or Inf                    */
#define EZ_FLAG_HADAMARD 0x8u   /* a Hadamard exponent mu + 2k hit 0 on the device  */
#define EZ_FLAG_POLE 0x10u      /* ez_epstein_zeta: nu = d at y in Lambda*          */

#define EZ_PREC_FP64 0
#define EZ_PREC_MIXED 1

/* Quadrature plan of the Epstein representation (paper, Sec. 3):
 * v in [0,1]^{d-1}: n_q-point Gauss-Legendre per dimension (paper: n_q = 14);
 * u in (0, eps): Taylor expansion of Z^reg to order 2*ell and Hadamard
 *   integrals (paper: eps = 1e-2, ell = 4; 0 <= ell <= 6);
 * u in (eps, 1/2]: n_panels geometric panels eps*r^i (r = (1/(2 eps))^{1/n_panels}),
 *   n_g Gauss-Legendre points each.
 * lam: Ewald split parameter in units of V^{1/d} (0 selects 1.0), used as given;
 * a_cut: terms whose incomplete-gamma argument exceeds a_cut are dropped
 *   (0 selects 36, a truncation below 1e-15 relative for nu <= 12 at lam = 1).
 * precision: EZ_PREC_MIXED (ez_lattice_sums, ez_lattice_sums_bound, ez_atm_energy
 *   and ez_nbody_lattice_sum without derivatives) sums the reciprocal-space terms
 *   whose incomplete-gamma argument is at least a_mix at every node of a 64-node
 *   wave block in FP32: e^{-a} by the hardware exponential, E_p from FP32 rational
 *   fits at the largest p and the stable downward recurrence; a_mix = 16 unless
 *   EZ_SPEC_MIX_A(n) sets n >= 8.  Everything else (real-space sum, small and
 *   middle arguments, the origin split, products, Hadamard part, reductions) stays
 *   FP64.  ez_lattice_sums_bound returns an a-priori bound of the result's change.
 *   When an exponent has 2p > 12 (p = (nu - d + 2)/2) or a_cut > 80 the call
 *   computes in FP64 throughout (bound 0).  Derivatives and the no-allocation
 *   entry point refuse it (EZ_ERR_UNSUPPORTED). */
typedef struct ez_quad_spec {
    int32_t n_q;
    int32_t n_panels;
    int32_t n_g;
    int32_t ell;
    double eps;
    double lam;
    double a_cut;
    int32_t precision; /* EZ_PREC_FP64, or EZ_PREC_MIXED for value calls (below) */
    int32_t flags;     /* execution options below (0: defaults); equal for all specs of a call */
} ez_quad_spec;

/* spec.flags: how the work is scheduled (results do not depend on them beyond
 * the order of floating-point sums in the node reduction, which stays fixed)
 *  EZ_SPEC_PERSISTENT : the node kernel runs as a persistent grid that takes node
 *                       tiles from a work queue, costliest tiles first
 *  EZ_SPEC_SERIAL     : the kernels of the Hadamard part (probe, tensor,
 *                       direction) run on the caller's stream before the nodes
 *                       instead of concurrently on a second stream
 *  EZ_SPEC_BPC(n)     : persistent workgroups per CU (0: as many as fit)
 *  EZ_SPEC_NO_SPLIT   : value calls hand the last node tiles, when they pass a
 *                       multiple of a round of workgroups over the device by a
 *                       few tiles (at most one per 16 CUs), to a kernel that
 *                       shares each node's terms among 16 waves on four CUs;
 *                       this flag keeps every tile in the tile kernel (the split
 *                       changes the order in which a node's terms are added, so
 *                       the two agree to rounding, not bit for bit) */
#define EZ_SPEC_PERSISTENT 0x1
#define EZ_SPEC_SERIAL 0x2
#define EZ_SPEC_NO_SPLIT 0x4
#define EZ_SPEC_BPC(n) (((n) & 0xFF) << 8)
/*  EZ_SPEC_MIX_A(n)   : mixed precision: FP32 far field from argument a_mix = n
 *                       (n >= 8; 0 selects 16) */
#define EZ_SPEC_MIX_A(n) (((n) & 0xFF) << 16)
/*  EZ_SPEC_WAVE_U(k)  : shape of the 64-node wave blocks of the node kernel in
 *                       d >= 2: 2^(k+2) consecutive u-nodes x 2^(4-k) directions
 *                       (k = 1..4); 0 picks the shape with the fewest empty lanes
 *                       (results do not depend on it beyond rounding) */
#define EZ_SPEC_WAVE_U(k) (((k) & 0x7) << 24)

/* Epstein zeta Z_{Lambda,nu}(x, y) = sum'_{z in Lambda} e^{-2 pi i y.z} |z - x|^{-nu},
 * meromorphically continued in nu (paper, Sec. 2, Definition (Epstein zeta
 * function)), evaluated by the incomplete-gamma split into a real-space and a
 * reciprocal-space sum.  The primed sum omits z = x.
 *   A_dev   : d*d doubles (one lattice)
 *   nu_host : n_nu exponents
 *   x_dev, y_dev : n_pts points each, row-major (n_pts x d)
 *   lam, a_cut   : as in ez_quad_spec (0 selects the defaults)
 *   out_dev : n_nu x n_pts x 2 doubles, (re, im) of Z(nu_j; x_i, y_i) at
 *             out_dev[2*(j*n_pts + i) + {0,1}]
 *   status_dev : 1 uint32 (lattice flags), may be NULL
 * y on Lambda* (within 1e-12 in fractional coordinates) takes the value of the
 * continuation in nu at that y; x within 1e-12 of a lattice point is taken on it.
 * Errors: EZ_ERR_INVALID_ARG (d, n_nu < 1, n_pts < 0, null pointers, non-finite nu),
 *         EZ_ERR_POLE (nu == d: pole at y in Lambda*). */
ez_status ez_epstein_zeta(int d, const double *A_dev, int n_nu, const double *nu_host,
                          int64_t n_pts, const double *x_dev, const double *y_dev,
                          double lam, double a_cut, double *out_dev, uint32_t *status_dev,
                          void *stream);

/* Epstein zeta on a grid: Z_{Lambda,nu_k}(x_j, y_m) for every exponent, shift x_j
 * and point y_m (paper, Sec. 2, Definition (Epstein zeta function)), with the
 * real-space sum sum_z W_nu(|z - x_j|) e^{-2 pi i y_m.z} and the reciprocal sum
 * sum_m* e^{-2 pi i m*.x_j} G_nu(|m* + y_m|) each computed as one matrix product
 * over the lattice-point tables (MFMA).
 *   A_dev   : d*d doubles (one lattice)
 *   x_dev   : n_x x d shifts, y_dev : n_y x d points (Cartesian, row-major)
 *   precision : EZ_PREC_FP64 (FP64 products throughout) or EZ_PREC_MIXED (table
 *             entries whose weight exceeds e^{-21} for some x or y in FP64, the rest
 *             as split-BF16 products with FP32 accumulation per 32 entries and FP64
 *             accumulation across them)
 *   out_dev : n_nu x n_x x n_y x 2 doubles, (re, im) of Z(nu_k; x_j, y_m) at
 *             out_dev[2*((k*n_x + j)*n_y + m) + {0,1}]
 *   bound_dev : NULL or n_nu x (n_x + n_y) doubles, a shift term b[k][j] and a point
 *             term b[k][n_x + m] per exponent: |Z_mixed - Z_fp64| at (nu_k, x_j, y_m) is
 *             at most b[k][j] + b[k][n_x + m], a priori (zeros for FP64)
 *   status_dev : 1 uint32 (lattice flags, EZ_FLAG_POLE at nu = d, y in Lambda*), may be NULL
 * The call reads the lattice table sizes back once (it synchronises `stream`
 * after the setup kernel), so it cannot be captured into a graph.
 * Errors: EZ_ERR_INVALID_ARG (d, sizes, null pointers, non-finite nu, precision). */
ez_status ez_epstein_grid(int d, const double *A_dev, int n_nu, const double *nu_host, int n_x,
                          const double *x_dev, int n_y, const double *y_dev, double lam, double a_cut,
                          int precision, double *out_dev, double *bound_dev, uint32_t *status_dev,
                          void *stream);

/* n-body zeta zeta^(n)_Lambda(nu) (paper, Sec. 2, Definition (Many-body zeta
 * function)) by the Epstein representation V int_BZ prod_i Z_{Lambda,nu_i}(k) dk
 * (Sec. 2, Theorem) with the Duffy transform and the Hadamard continuation
 * (Sec. 3), for a batch of lattices.
 *   A_dev   : batch*d*d doubles
 *   n, nu_host : number of bodies and their n exponents (integers, |nu| <= 64)
 *   spec    : host pointer to one plan used for every lattice
 *   out_dev : batch doubles
 *   status_dev : batch uint32 (may be NULL)
 * Errors: EZ_ERR_INVALID_ARG, EZ_ERR_UNSUPPORTED (a Hadamard exponent mu+2k = 0). */
ez_status ez_nbody_lattice_sum(int batch, int d, const double *A_dev, int n, const double *nu_host,
                               const ez_quad_spec *spec, double *out_dev, uint32_t *status_dev,
                               void *stream);

/* Axilrod-Teller-Muto cohesive energy per particle (paper, Sec. 2, Definition
 * (ATM potential)) via E = 1/24 zeta(3,3,3) - 3/16 zeta(-1,5,5) + 3/8 zeta(1,3,5)
 * (Sec. 2, Proposition), the three integrands fused at one node set.
 *   A_dev   : batch*d*d doubles;  E_dev : batch doubles
 *   dEdA_dev: batch*d*d doubles of dE/dA (row-major like A), or NULL.  The
 *             derivative is that of the quadrature value on the given plan (the
 *             nodes are fixed in fractional coordinates, lam is held fixed); it
 *             comes from the adjoint kernels, at about twice the cost of E alone.
 *   status_dev : batch uint32 (may be NULL) */
ez_status ez_atm_energy(int batch, int d, const double *A_dev, const ez_quad_spec *spec,
                        double *E_dev, double *dEdA_dev, uint32_t *status_dev, void *stream);

/* General form behind the two entry points above: several results per lattice,
 * each a linear combination of products of Epstein zeta functions integrated
 * over the Brillouin zone,
 *   result_r = sum_{t : term_result[t] = r} term_coef[t] * V int_BZ prod_f Z_{nu[fac]}^{mult} dk.
 *   nu_host  : n_nu distinct integer exponents (n_nu <= 8)
 *   term_*   : n_terms terms (n_terms <= 8); term t has term_nfac[t] (<= 4) distinct
 *              factors; its factors are term_fac[4*t + f] (index into nu_host) with
 *              multiplicity term_mult[4*t + f] (>= 1, total degree <= 64)
 *   specs    : n_specs == 1 (shared plan) or n_specs == batch (one plan per lattice)
 *   out_dev  : batch x n_results doubles (n_results <= 8) */
ez_status ez_lattice_sums(int batch, int d, const double *A_dev, int n_nu, const double *nu_host,
                          int n_terms, const int *term_result, const double *term_coef,
                          const int *term_nfac, const int *term_fac, const int *term_mult,
                          int n_results, const ez_quad_spec *specs, int n_specs, double *out_dev,
                          uint32_t *status_dev, void *stream);

/* Direct summation of the Axilrod-Teller-Muto cohesive energy over the box
 * A{-L..L}^d (paper, Sec. 2, Definition (ATM potential); Sec. 4.3 compares the
 * Epstein zeta method with such sums on the square lattice):
 *   E_L = (1/6) sum_{x, y in box, x, y, x - y != 0} U(x, y),
 *   U = (1 + 3 cos g1 cos g2 cos g3) / (|x| |y| |x - y|)^3  (g_i the triangle's angles).
 * An independent check of ez_atm_energy: the box sum converges to the lattice sum
 * like L^{-d-2}.
 *   A_host       : d*d doubles (host), row-major, columns the basis vectors
 *   use_symmetry : 1 sums over one point per orbit of the signed coordinate
 *                  permutations, with the orbit size as weight (needs A^T A = c I:
 *                  square and cubic lattices; about 2^d d! times less work); 0 sums
 *                  over every box point
 *   out_dev      : 1 double (device), written on `stream`
 * Deterministic (fixed-order double-double sums).  The outer-point list is copied
 * from pageable host memory (the copy completes before the call returns).
 * Errors: EZ_ERR_INVALID_ARG (d, L beyond 2^28 / 8192 / 512 for d = 1 / 2 / 3, null
 * pointers, non-finite or singular A, use_symmetry without A^T A = c I). */
ez_status ez_direct_atm(int d, const double *A_host, int L, int use_symmetry, double *out_dev, void *stream);

/* ez_lattice_sums with an a-priori error bound per result, for EZ_PREC_MIXED specs:
 *   bound_dev : batch x n_results doubles (device), |result_mixed - result_FP64| <=
 *               bound_dev[b * n_results + r], where result_FP64 is the FP64 value on
 *               the same plan up to FP64 rounding (about 1e-16 relative, not part of
 *               the bound).  The bound propagates, to first order, the FP32 error of
 *               each far-field chunk sum (a fixed multiple of u = 2^-24 per exponent,
 *               from the error of e^{-a}, 1/a, the fits, the recurrence steps and 63
 *               FP32 additions) through K_nu, the products and the quadrature
 *               weights, with 1% for the second-order terms.  It is 0 for FP64 specs
 *               and NaN for a lattice with a nonzero status.
 * (The mixed-precision path: the spec's precision field.)
 * Errors: as ez_lattice_sums; EZ_ERR_INVALID_ARG for a NULL bound_dev. */
ez_status ez_lattice_sums_bound(int batch, int d, const double *A_dev, int n_nu, const double *nu_host,
                                int n_terms, const int *term_result, const double *term_coef,
                                const int *term_nfac, const int *term_fac, const int *term_mult,
                                int n_results, const ez_quad_spec *specs, int n_specs, double *out_dev,
                                double *bound_dev, uint32_t *status_dev, void *stream);

/* ez_lattice_sums for callers that cannot allocate device memory (code under HIP
 * graph capture elsewhere in their stream, tight serving loops, harnesses that
 * forbid hipMalloc): the same arguments, results and kernels as ez_lattice_sums
 * (values only), with every intermediate buffer -- lattice tables, quadrature
 * plan, partial sums, counters -- carved from a static device array of 64 MiB
 * per GPU that the library holds from its first use until the process ends.
 * The call allocates and frees nothing.  It runs the whole sequence on `stream`
 * (no second stream, no events; results are bit-identical to ez_lattice_sums
 * with EZ_SPEC_SERIAL and, like every schedule, to ez_lattice_sums itself).
 * The plan is uploaded from host memory with hipMemcpyAsync when it differs
 * from the one resident in the scratch (pageable source: the copy completes
 * before the call returns), so a first call with a new plan cannot be captured.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (different streams or host threads) race and give undefined results.
 * Errors: as ez_lattice_sums; EZ_ERR_INVALID_ARG when the plan and workspace of
 * the call exceed the 64 MiB (the message gives the size needed). */
ez_status ez_lattice_sums_noalloc(int batch, int d, const double *A_dev, int n_nu, const double *nu_host,
                                  int n_terms, const int *term_result, const double *term_coef,
                                  const int *term_nfac, const int *term_fac, const int *term_mult,
                                  int n_results, const ez_quad_spec *specs, int n_specs, double *out_dev,
                                  uint32_t *status_dev, void *stream);

/* ez_lattice_sums with the derivatives of the results with respect to the
 * generator matrix (reverse mode through every step of the quadrature; the
 * derivative of the quadrature value on the given plan, lam held fixed).
 *   n_results <= 2
 *   grad_dev : batch x n_results x d x d doubles, grad_dev[((b*n_results + r)*d + i)*d + j]
 *              = d result_r / d A_ij of lattice b (NULL: values only)
 * Errors: as ez_lattice_sums; EZ_ERR_INVALID_ARG for n_results > 2 with grad_dev. */
ez_status ez_lattice_sums_grad(int batch, int d, const double *A_dev, int n_nu, const double *nu_host,
                               int n_terms, const int *term_result, const double *term_coef,
                               const int *term_nfac, const int *term_fac, const int *term_mult,
                               int n_results, const ez_quad_spec *specs, int n_specs, double *out_dev,
                               double *grad_dev, uint32_t *status_dev, void *stream);

/* Kernel timing (tracing aid).  When enabled, every kernel the library launches
 * is bracketed by a pair of HIP events recorded on the launch stream; reading
 * synchronises the recorded events and returns the accumulated elapsed time and
 * launch count of one kernel kind.  Costs two event records per launch. */
#define EZ_KERNEL_SETUP 0      /* per-lattice tables                    */
#define EZ_KERNEL_NODES 1      /* quadrature nodes on (eps, 1/2]         */
#define EZ_KERNEL_HADAMARD 2   /* Hadamard part on (0, eps), directions  */
#define EZ_KERNEL_FINALIZE 3   /* fixed-order reduction                  */
#define EZ_KERNEL_EPSTEIN 4    /* Z(x, y) at arbitrary points            */
#define EZ_KERNEL_NODES_ADJ 5  /* quadrature nodes with the adjoint pass  */
#define EZ_KERNEL_GRID 6       /* Z on a (shift x point) grid            */
#define EZ_KERNEL_NODES_TAIL 7 /* last node tiles, terms split over waves */
#define EZ_KERNEL_TAYLOR 8     /* probe values and Taylor tensors          */
#define EZ_KERNEL_GRID_GEMM 9  /* the two matrix products of the grid (EZ_KERNEL_GRID: the rest) */
#define EZ_KERNEL_COUNT 10
ez_status ez_timing_enable(int enable);
ez_status ez_timing_reset(void);
ez_status ez_timing_read(int kernel, double *total_ms, int64_t *launches);

/* Table sizes of the last ez_epstein_grid call on the current device (a tracing
 * aid): n_real real-space and n_rec reciprocal entries, the inner dimensions of the
 * real-space product ((n_nu n_x) x n_real times n_real x (2 n_y)) and of the
 * reciprocal product ((2 n_x) x n_rec times n_rec x (n_nu n_y)); 0, 0 before the
 * first call.  Errors: EZ_ERR_INVALID_ARG (null pointer). */
ez_status ez_grid_last_tables(int64_t *n_real, int64_t *n_rec);

/* Node tiles of the last lattice-sum call (ez_atm_energy, ez_nbody_lattice_sum,
 * ez_lattice_sums and their variants) on the current device (a tracing aid): n_tiles
 * tiles of 256 nodes, n_main of them taken whole by the tile kernel, and the tail
 * [n_main, n_tiles): tail_mode 0 none, 1 the split kernel (a few tiles past a full
 * round of workgroups), 2 two half-term workgroups per tile in the tile kernel (up to
 * about half a round).  All 0 before the first call.  Errors: EZ_ERR_INVALID_ARG
 * (null pointer). */
ez_status ez_last_sum_tiles(int64_t *n_tiles, int64_t *n_main, int *tail_mode);

/* Text of the last error on the calling host thread (never NULL). */
const char *ez_last_error(void);

/* Frees the library's cached device workspace and plans on every device. */
ez_status ez_finalize(void);

/* A counter that changes whenever the library frees or moves device memory it
 * owns: a workspace buffer grown for a larger call, a cached plan evicted (the
 * cache keeps the 128 most recently used plans per device), ez_finalize.  Work captured
 * into a HIP graph from calls of the library records the library's device
 * pointers; such a graph may be replayed only while this value is the one read
 * after the capture (the Python GraphedLatticeSums checks it). */
uint64_t ez_workspace_generation(void);

/* Library version string. */
const char *ez_version(void);

#ifdef __cplusplus
}
#endif
#endif /* EZETA_H */
