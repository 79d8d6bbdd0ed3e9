// serve.h -- batched launches of many independent domains (ensemble serving).
//
// A serving step runs one coupled step of every active domain with six
// launches in total, whatever the number of domains: fused DEM substeps (one
// workgroup per domain), tile registration (one workgroup per domain),
// voxelisation and the two LBM passes over a (domain, tile) map of every
// domain's tiles, and the hydrodynamic sums with the corrector (one workgroup
// per domain).  Each domain's arithmetic is the one of its single-domain step:
// the same device bodies on the same data (the voxelisation in a one-workgroup
// form that counts the same samples), so a result does not depend on the other
// domains of the batch.
#pragma once
#include "common.h"
#include "dem.h"
#include "lbm.h"
#include "voxel.h"

#define SRV_MAX_JOBS 128

// per-step state of every slot, passed by value at each launch as bit sets
// (read with selects: a kernel argument indexed by a lane-uniform value would
// otherwise be copied to private memory)
struct SrvDyn {
    unsigned long long cur[2];   // bit i: DEM pair buffer of slot i holding the previous list
    unsigned long long odd[2];   // bit i: AA parity of slot i's LBM step
};

__host__ __device__ inline int srv_bit(const unsigned long long (&w)[2], int i) {
    const unsigned long long v = i < 64 ? w[0] : w[1];
    return (int)((v >> (i & 63)) & 1ull);
}

__host__ inline void srv_set(unsigned long long (&w)[2], int i, int b) {
    if (b) w[i >> 6] |= 1ull << (i & 63);
}

// the DEM and particle side of one domain
struct DemJob {
    DemArgs A;
    PairSet P;
    TileArgs t;
    double dt;
    int nsub;
    int dem;      // DEM substeps run (dem_on and particles present)
    int fluid;    // fluid coupled (fluid_on)
};

hipError_t dem_fused_batch(const DemJob* jobs, int njobs, const SrvDyn& dyn, int ellipsoids, hipStream_t s);
hipError_t dem_finish_batch(const DemJob* jobs, int njobs, hipStream_t s);
hipError_t vox_register_batch(const VoxArgs* jobs, int njobs, hipStream_t s);
hipError_t vox_voxelize_batch(const VoxArgs* jobs, const int2* map, long long nmap, int ctype_double,
                              hipStream_t s);
hipError_t lbm_step_batch(const LbmArgs* jobs, const SrvDyn& dyn, const int2* map, long long nmap, int ms,
                          int precision, hipStream_t s);
