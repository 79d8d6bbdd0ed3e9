// dem.h -- DEM kernel arguments and launchers (FP64 on the device).
#pragma once
#include "common.h"

struct DemArgs {
    GeoArgs g;
    PartArgs p;
    double L[3];
    int nc[3];
    double h[3];
    long long ncell;
    int* cell_count;       // [ncell]
    int* cell_start;       // [ncell + 1]
    int* cell_fill;        // [ncell]
    int* cell_pid;         // [reg_cap] particle ids per cell, ascending
    long long reg_cap;
    int* pcount;           // [np] pairs per row
    int* prow;             // [np + 1] row offsets; prow[np] = number of pairs
    unsigned long long* pairs;  // [pair_cap] (i << 32 | j), ascending
    double *hist, *cF, *cMi, *cMj;  // [3 pair_cap]
    unsigned char* incontact;       // [pair_cap]
    long long pair_cap;
    const unsigned long long* prev_pairs;  // previous substep's list
    const double* prev_hist;
    const int* prev_n;     // device count of the previous list (NULL: empty)
    double kn, beta_e, mu, kt_ratio, gt_ratio;
    double wall_u[6][3];
    double gravity[3];
    DevCounters* ctr;
};

hipError_t dem_predict(const DemArgs& A, double dt, int write_kin, hipStream_t s);
hipError_t dem_lists(const DemArgs& A, int* scan_tmp, hipStream_t s);
hipError_t dem_contacts(const DemArgs& A, const double* vv, const double* ww, double dth, hipStream_t s);
hipError_t dem_correct(const DemArgs& A, double dt, hipStream_t s);
hipError_t dem_initial_accel(const DemArgs& A, hipStream_t s);
hipError_t dem_zero(double* p, long long n, hipStream_t s);
