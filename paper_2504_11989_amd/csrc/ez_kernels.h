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
    uint32_t *status_out;      // general-x mode: receives the lattice flags (may be NULL)
};

struct EzQuadArgs {
    EzProgram prog;
    int batch;
    const EzInstPlan *plans;
    const int *tile_begin;     // batch + 1 prefix of node tiles
    const int *dir_begin;      // batch + 1 prefix of directions
    const int *htile_begin;    // batch + 1 prefix of 64-direction Hadamard tiles
    const EzLatMeta *meta;
    EzTables tab;
    const double *rules;       // Gauss rules (v on [0,1], u on (eps,1/2])
    double *tile_part;         // [n_tiles][n_res][2] double-double partials
    double *dir_part;          // [n_dirs][n_res] Hadamard part per direction (times 2 w_v)
    uint32_t *dir_flag;        // [n_dirs] flags (Hadamard mu = 0)
    double *out;               // [batch][n_res]
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

hipError_t ez_launch_setup(const EzSetupArgs &args, int batch, hipStream_t stream);
hipError_t ez_launch_nodes(const EzQuadArgs &args, int n_tiles, hipStream_t stream);
hipError_t ez_launch_hadamard(const EzQuadArgs &args, int n_htiles, hipStream_t stream);
hipError_t ez_launch_finalize(const EzQuadArgs &args, hipStream_t stream);
hipError_t ez_launch_epstein(const EzEpsteinArgs &args, hipStream_t stream);
