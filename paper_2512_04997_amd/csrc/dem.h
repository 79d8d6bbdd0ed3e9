// dem.h -- DEM kernel arguments and launchers (FP64 on the device).
#pragma once
#include "common.h"

// particles up to this count take the fused single-workgroup substep kernel
#define DEM_FUSED_MAX 2048
#define DEM_ROWS_PER_WG 64  // particles per workgroup of the multi-launch row kernel

struct DemArgs {
    GeoArgs g;
    PartArgs p;
    double L[3];
    int nc[3];
    double h[3];
    long long ncell;
    int* pc;               // [8 np] per-axis registration cells of each particle
    int* cell_count;       // [ncell]
    int* cell_start;       // [ncell + 1]
    int* cell_fill;        // [ncell]
    int* cell_pid;         // [reg_cap] particle ids per cell, ascending
    long long reg_cap;
    unsigned long long* row_lb;  // [np / DEM_ROWS_PER_WG + 2] the row kernel's ticket counter and
                                 // per-chunk status words (cleared by the cell histogram)
    double *cF, *cMi, *cMj;         // [3 pair_cap] force on i, torque on i, torque on j
    unsigned char* incontact;       // [pair_cap] bit 0: in contact now; bit 1: at the evaluation before (or unknown)
    int *col_count, *col_fill;      // [np]
    int* col_start;                 // [np + 1]
    int* col_list;                  // [pair_cap] pair indices by second member, ascending
    long long pair_cap;
    double kn, beta_e, mu, kt_ratio, gt_ratio;
    int hertz;             // Hertz law from the material, else the linear law
    double ystar, gstar;   // Hertz: Y*, G*
    double wall_u[6][3];
    double gravity[3];
    int ellipsoids;        // any particle is an ellipsoid (else the sphere-only kernels run)
    int* fused_age;        // [2] substeps the pair list has been kept (pc holds the cells it was built
                           // from, the wall candidates in pc's last word); -1: rebuild.  The fused
                           // kernel uses word 0, the multi-launch path one word per substep parity
    unsigned char* fz;     // [dem_fused_save_bytes()] the fused kernel's skip state of its kept list,
                           // saved at the end of a launch for the next one (null: not kept)
    int* list_flag;        // [2] multi-launch path: the list changed in this substep (by substep parity)
    const int* list_run;   // multi-launch path: list_flag of this substep, or null (always build)
    int* ell_list;         // [DEM_ELL_SEGS * ell_seg_cap] multi-launch path: pairs whose ellipsoid
                           // iteration is deferred to a dense second launch, in DEM_ELL_SEGS segments
                           // (a wave appends to segment wave % DEM_ELL_SEGS), or null (no ellipsoids)
    unsigned* ell_cnt;     // [DEM_ELL_SEGS] pairs queued per segment this substep
    long long ell_seg_cap;
    DevCounters* ctr;
};

#define DEM_ELL_SEGS 64
#define DEM_CONTACT_GRID_MAX 2048u
// capacity of one deferral segment for pair_cap pairs: the contact launch has
// at most DEM_CONTACT_GRID_MAX workgroups of 128 lanes striding over the list,
// and the waves of one segment cover at most a DEM_ELL_SEGS-th of its lanes
inline long long dem_ell_seg_cap(long long pair_cap) {
    const long long blocks = (pair_cap + 127) / 128 < DEM_CONTACT_GRID_MAX ? (pair_cap + 127) / 128 : DEM_CONTACT_GRID_MAX;
    const long long lanes = 128 * (blocks > 0 ? blocks : 1);
    const long long iters = (pair_cap + lanes - 1) / lanes;
    return (pair_cap + lanes) / DEM_ELL_SEGS + 64 * iters + 64;
}

// the current and the previous substep's pair lists
struct PairBufs {
    unsigned long long* pairs;   // [pair_cap] (i << 32 | j), ascending
    int* prow;                   // [np + 1] row offsets; prow[np] = number of pairs
    double* hist;                // [3 pair_cap] tangential history
    const unsigned long long* prev_pairs;
    const double* prev_hist;
    const int* prev_n;           // device count of the previous list (NULL: empty)
};

// both pair buffers for the fused kernel (substeps alternate between them)
struct PairSet {
    unsigned long long* pairs[2];
    int* prow[2];
    double* hist[2];
};

hipError_t dem_predict(const DemArgs& A, double dt, int write_kin, hipStream_t s);
// cells, rows and column lists of the current positions (one launch per phase)
hipError_t dem_lists(const DemArgs& A, const PairBufs& B, int* scan_tmp, hipStream_t s);
// the column lists of the rows in B (the per-particle sums read them) from the
// column counts: the row emission forms them; rows placed otherwise (copied)
// take dem_count_columns first
hipError_t dem_columns(const DemArgs& A, const PairBufs& B, int* scan_tmp, hipStream_t s);
// each cell's list of the last build in ascending particle order (the step
// itself leaves them in arrival order; a read-back of the lists sorts them)
hipError_t dem_sort_cells(const DemArgs& A, hipStream_t s);
hipError_t dem_count_columns(const DemArgs& A, const PairBufs& B, hipStream_t s);
// multi-launch substeps that keep an unchanged list (A.list_run = A.list_flag + par)
hipError_t dem_predict_keep(const DemArgs& A, double dt, int write_kin, int par, hipStream_t s);
// the list of a multi-launch substep: cells and rows rebuilt when
// list_flag[par] is set, else kept (the list kernels return at once); the
// column lists follow with dem_columns (gated the same way)
hipError_t dem_lists_kept(const DemArgs& A, const PairBufs& B, int par, int* scan_tmp, hipStream_t s);
// contacts of the pairs in B, then (sums) the per-particle sums
hipError_t dem_contacts(const DemArgs& A, const PairBufs& B, const double* vv, const double* ww, double dth,
                        int* scan_tmp, hipStream_t s, bool sums = true);
// the per-particle sums of a substep whose contacts ran without them
hipError_t dem_sums(const DemArgs& A, const PairBufs& B, hipStream_t s);
// the per-particle sums of a substep whose contacts ran without them, its
// corrector and the next substep's predictor (its parity par)
hipError_t dem_sum_correct_predict(const DemArgs& A, const PairBufs& B, double dt, int write_kin, int par,
                                   hipStream_t s);
hipError_t dem_correct(const DemArgs& A, double dt, hipStream_t s);
// hydrodynamic sums of the tile partials (T) and the corrector, one launch
hipError_t dem_hydro_correct(const DemArgs& A, const TileArgs& T, double dt, hipStream_t s);
hipError_t dem_initial_accel(const DemArgs& A, hipStream_t s);
hipError_t dem_zero(double* p, long long n, hipStream_t s);
// nsub substeps in one workgroup starting from buffer `cur` (the first substep
// writes buffer cur ^ 1); with stop_before_correct the last substep ends after
// the DEM sums (the corrector then runs after the fluid coupling)
// bytes of DemArgs::fz; its first int is -1 while it holds no state
size_t dem_fused_save_bytes();
hipError_t dem_fused(const DemArgs& A, const PairSet& P, int cur, int nsub, double dt, int stop_before_correct,
                     hipStream_t s);
