// ez_grid.h -- launch arguments of the Epstein-zeta grid kernels (ez_grid.hip).
#pragma once
#include "ez_internal.h"

struct EzGridArgs {
    int d, n_nu;
    double nu[EZ_NU_MAX];
    int n_x, n_y;              // shifts x_j, reciprocal-cell points y_m
    int Mp, Np;                // n_x, n_y padded to multiples of 128
    int Kr_pad, Kk_pad;        // real / reciprocal table capacity + 32, multiple of 32
    int Krn_pad, Krf_pad;      // leading dimensions of the near (FP64) / far (BF16) real operands
    int Kkn_pad, Kkf_pad;      // same, reciprocal
    int mixed;                 // 0: every column FP64; 1: far columns split-BF16
    double a_near;             // far columns: incomplete-gamma argument >= a_near for every point
    const EzLatMeta *meta;
    EzTables tab;              // general-x tables of the lattice
    const double *x, *y;       // n_x x d, n_y x d (Cartesian)
    double *pts_x;             // [n_x][8]
    double *pts_y;             // [n_y][4]
    int *perm_real, *perm_rec; // table entries, near first
    int *counts;               // near real, far real, near reciprocal, far reciprocal
    double *kpref;             // [n_nu] reciprocal prefactors K_nu
    int p2[EZ_NU_MAX];         // 2 p = nu - d + 2 of E_p, when every nu is a half-integer multiple
    int ladder;                // 1: every 2 p is an integer in [-64, 64] (one E_p base per entry, recurrences)
    double *A64r, *B64r;       // (n_nu Mp) x Krn_pad ; Kr_pad x (2 Np)
    double *A64k, *B64k;       // (2 Mp) x Kkn_pad ; Kk_pad x (n_nu Np)
    __bf16 *Ahr, *Alr, *Bhr, *Blr;   // (n_nu Mp) x Krf_pad ; (2 Np) x Krf_pad (transposed)
    __bf16 *Ahk, *Alk, *Bhk, *Blk;   // (2 Mp) x Kkf_pad ; (n_nu Np) x Kkf_pad (transposed)
    double *R;                 // (n_nu Mp) x (2 Np)
    double *Q;                 // (2 Mp) x (n_nu Np)
    double *wsum;              // [n_nu Mp] sum of |far real weights| per shift x_j (mixed)
    double *gfar;              // [n_nu Np] sum of |far G| per point y_m (mixed), follows wsum
    double *wall;              // [n_nu Mp] sum of |weights| over every real column (mixed), follows gfar
    double *gall;              // [n_nu Np] sum of |G| over every reciprocal column (mixed), follows wall
    double *out;               // [n_nu][n_x][n_y][2]
    double *bound;             // [n_nu][n_x + n_y] (shift terms, then point terms) or NULL
    uint32_t *status_acc;      // lattice status word (POLE bit)
};

// the launch sequence in three parts: operands (points, classification, builds), the
// two matrix products, and the combination with the bound
#define EZ_GRID_PRE 1
#define EZ_GRID_GEMM 2
#define EZ_GRID_POST 4
hipError_t ez_grid_launch(const EzGridArgs &g, hipStream_t s, int part);
