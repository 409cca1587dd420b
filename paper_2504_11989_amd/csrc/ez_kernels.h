// ez_kernels.h -- launch arguments and launchers of the libezeta kernels.
#pragma once
#include "ez_internal.h"

struct EzSetupArgs {
    EzProgram prog;
    const double *A;           // batch x d x d
    const EzInstPlan *plans;
    EzLatMeta *meta;
    EzTables tab;
    double a_cut;
    int general_x;             // 0: pairs table for x = 0; 1: full table for general x
    int grad;                  // pairs mode: also store the strain weights -4 Gamma(nu/2+1, a)/(Gamma(nu/2) r^{nu+2})
    uint32_t *status_out;      // general-x mode: receives the lattice flags (may be NULL)
    // per exponent, lattice-independent factors (host-computed from nu and d):
    // [0] pi^{nu-d/2}/Gamma(nu/2), [1] 1/Gamma(nu/2+1), [2] V times the singular
    // coefficient sig, [3] 1/Gamma(nu/2); 1/Gamma is 0 at the poles
    double nuc[EZ_NU_MAX][4];
};

// One term of the (0, eps) expansion: term t with factor slot f taking its singular
// part j[f] times and its Taylor part mult - j[f] times; coef holds the term
// coefficient times the binomials; the integrand is u^{d-1+E} L^Q times a
// polynomial in u^2.
#define EZ_COMBO_MAX 64
struct EzCombo {
    double coef;
    double E;                  // sum_f j_f (nu_f - d): the u-exponent of the singular factors
    int Q;                     // number of logarithmic singular factors
    signed char t, res, j[EZ_FAC_MAX];
    short pad_;
};

struct EzQuadArgs {
    EzProgram prog;
    int batch;
    const EzInstPlan *plans;
    const int *tile_begin;     // batch + 1 prefix of node tiles
    int n_tiles;               // node tiles of the whole batch
    int n_main;                // tiles [0, n_main) whole, [n_main, n_tiles) the tail (below)
    int tail_halves;           // 0: the tail goes to the split kernel (64-node groups); 1: the
                               // tile kernel takes each tail tile as two workgroups of half its terms
    const int *tile_order;     // persistent node kernel: tiles in the order they are taken (costliest first)
    int *queue;                // persistent node kernel: next position in tile_order (reset before launch)
    const int *dir_begin;      // batch + 1 prefix of directions
    const int *htile_begin;    // batch + 1 prefix of Hadamard direction tiles
    int n_dir_blk;             // directions per Hadamard direction workgroup (<= EZ_HDIR)
    int poly_deg;              // 13 or 33: coefficients kept in the (0, eps) product polynomials
    int n_probe, ell_probe;    // probe directions per lattice, Taylor order they carry
    int n_slice;               // table slices per probe set (workgroups that split the sums)
    int n_ch;                  // 1 (values) or 1 + d(d+1)/2 (values and strain derivatives)
    int probe_off;             // offset of the probe directions (n_probe x d) in rules
    int pinv_off[EZ_ELL_MAX + 1];  // offsets of the least-squares inverses (nmono x n_probe) in rules
    double *probe_val;         // [batch][n_slice][n_probe][n_ch * n_nu][EZ_ELL_MAX + 1] partial sums
    double *tensor;            // [batch][n_ch * n_nu][EZ_TDIM] coefficients of C_k in w_hat monomials
    int n_combo;
    EzCombo combo[EZ_COMBO_MAX];
    const EzLatMeta *meta;
    EzTables tab;
    const double *rules;       // Gauss rules (v on [0,1], u on (eps,1/2])
    double *tile_part;         // [n_tiles][n_res][2] double-double partials
    // mixed precision (EZ_PREC_MIXED): reciprocal entries with alpha |m* + k|^2 >= a_mix at
    // every node of a wave are summed in FP32 (E_p from the fit at the largest p of each
    // chain, smaller p by the downward recurrence); an a-priori bound per result
    int mixed;                 // 0: FP64 throughout
    double a_mix;              // FP32 threshold on the incomplete-gamma argument (>= EZ_EPF_XMIN)
    int mix_top2[2];           // largest 2p of the integer (>= 0) and half-integer (>= 1) chains
    double mix_eps[EZ_NU_MAX]; // relative error bound of one FP32 chunk sum of exponent i
    double *tile_bound;        // [n_tiles (+ n_tiles - n_main with tail_halves)][n_res] bound
                               // partials (mixed calls; half 1 of tail tile t at n_tiles + t - n_main)
    double *bound_out;         // [batch][n_res] per-result bound, or NULL
    double *sub_part;          // [4 (n_tiles - n_main)][n_res][2] partials of the 64-node groups
                               // (tail_halves: slot 4t + h of workgroup h of tail tile t, 4t + 2 + h zero)
    double *tail_acc;          // [4 (n_tiles - n_main)][EZ_TAIL_PARTS][2 n_nu][64] partial sums of the split kernel
    int *tail_cnt;             // [4 (n_tiles - n_main)] parts finished per group (zero between calls)
    double *dir_part;          // [n_dirs][n_res] Hadamard part per direction (times 2 w_v)
    uint32_t *dir_flag;        // [n_dirs] flags (Hadamard mu = 0)
    double *tile_grad;         // [n_tiles][n_res][6][2] strain-derivative partials (gradient calls)
    double *dir_grad;          // [n_dirs][n_res][6] (gradient calls)
    double *out;               // [batch][n_res]
    double *grad_out;          // [batch][n_res][d][d] d result / d A, or NULL
    uint32_t *status;          // [batch] or NULL
};

struct EzEpsteinArgs {
    int d, n_nu;
    double nu[EZ_NU_MAX];
    long long n_pts;
    const double *x, *y;       // n_pts x d
    const EzLatMeta *meta;
    EzTables tab;
    double *out;               // [n_nu][n_pts][2]
    uint32_t *status;
};

hipError_t ez_launch_setup(const EzSetupArgs &args, int batch, hipStream_t stream, hipEvent_t done = nullptr);
hipError_t ez_launch_nodes(const EzQuadArgs &args, int n_tiles, hipStream_t stream);
// tiles [n_main, n_tiles): EZ_TAIL_PARTS workgroups per 64-node group
hipError_t ez_launch_nodes_split(const EzQuadArgs &args, hipStream_t stream);
// workgroups of the tile node kernel that fit on one CU at once
int ez_nodes_tile_blocks_per_cu(const EzQuadArgs &args);
// persistent form: n_blocks workgroups take tiles from args.queue until all are done
hipError_t ez_launch_nodes_persistent(const EzQuadArgs &args, int n_blocks, hipStream_t stream);
// blocks of the persistent node kernel that fit on one CU at once
int ez_nodes_blocks_per_cu(const EzQuadArgs &args);
hipError_t ez_launch_fill_int(int *p, int n, int value, hipStream_t stream);
// Taylor/Hadamard branch: part EZ_HAD_PRE = probe and tensor kernels, EZ_HAD_DIR = the
// direction kernel (it reads the tensors), or both; pre_done (may be NULL) is recorded
// when the tensors are complete
#define EZ_HAD_PRE 1
#define EZ_HAD_DIR 2
hipError_t ez_launch_hadamard(const EzQuadArgs &args, int n_htiles, hipStream_t stream, int part,
                              hipEvent_t pre_done = nullptr);
hipError_t ez_launch_finalize(const EzQuadArgs &args, hipStream_t stream);
hipError_t ez_launch_nodes_adj(const EzQuadArgs &args, int n_tiles, hipStream_t stream);
hipError_t ez_launch_hadamard_adj(const EzQuadArgs &args, int n_htiles, hipStream_t stream, int part,
                                  hipEvent_t pre_done = nullptr);
hipError_t ez_launch_epstein(const EzEpsteinArgs &args, hipStream_t stream);

// direct ATM sum over the box A{-L..L}^d (ez_direct.hip)
struct EzDirectArgs {
    int d, L;
    double A[9];               // row-major, padded to 3 x 3
    const int *xlist;          // [n_x][4]: outer point n (3 ints) and its weight
    long long n_x;
    long long n_box;           // (2L + 1)^d inner points
    long long per_chunk;       // inner points per workgroup column
    double *part;              // [ez_direct_parts][2] double-double partials
};
long long ez_direct_parts(long long n_x, int n_chunks);
hipError_t ez_launch_direct_atm(const EzDirectArgs &g, int n_chunks, double *out, hipStream_t stream);
