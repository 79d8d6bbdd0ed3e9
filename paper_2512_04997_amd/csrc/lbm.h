// lbm.h -- fused in-place (AA pattern) D3Q19 BGK/TRT-PSM collide-and-stream.
#pragma once
#include "common.h"

struct LbmArgs {
    GeoArgs g;
    void* f;                   // populations [19][N], storage type S, shifted f - w_i
    double omega;              // dt / tau (tau+ of TRT)
    double omega_m;            // dt / tau- of TRT; equal to omega for BGK
    int forcing;               // Guo forcing on
    double F[3];               // constant force density
    int kolm_axis, kolm_dir;
    const double* kolm_prof;   // [n_axis] sine profile of the Kolmogorov forcing or NULL
    const double* wall_corr;   // [6 * 19] 6 w_i rho0 (c_i . u_w) per walled face (0 for no-slip)
    TileArgs t;
    const double* kin;         // [9 np] position, v^p, w^p
    int np;
    int ms;
    double L[3];
    unsigned long long* flags;  // device flags word (PSM_FLAG_UNSTABLE raised on a non-positive density)
};

// storage: 0 double, 1 float, 2 bf16, 3 fp16 (psmdem_precision)
hipError_t lbm_step(const LbmArgs& A, int precision, int odd, hipStream_t s);
hipError_t lbm_init(void* f, int precision, long long N, double rho0, hipStream_t s);
hipError_t lbm_to_double(const void* f, int precision, long long n, double* out, hipStream_t s);
hipError_t lbm_from_double(void* f, int precision, long long n, const double* in, hipStream_t s);
