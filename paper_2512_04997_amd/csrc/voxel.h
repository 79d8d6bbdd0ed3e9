// voxel.h -- solid-fraction (voxelisation) arguments and launchers.
#pragma once
#include "common.h"

#define VOX_AXIS_MAX 12  // distinct tiles one particle box may touch per axis (radius up to about 15 cells)

struct VoxArgs {
    GeoArgs g;
    PartArgs p;
    TileArgs t;
    int* tile_count;     // [ntiles]
    int* tile_fill;      // [ntiles]
    int sf_method;       // 0 subdivision, 1 distance
    int ns;              // samples per direction
    double Rc;           // (3 / (4 pi))^(1/3)
    double tau;
    int ms;              // solids kept per cell
    // subdivision method: each particle's count box, the inside samples of every
    // cell of its lattice box (x fastest), 16 bits per cell, box_stride cells apart
    unsigned short* vbox;
    long long box_stride;
    void* vpart;                 // [np] per-step particle records of the tile kernels (vox_part_bytes
                                 // each), formed by vox_register; null: each tile forms its own
    const void* btab;            // [ns^3 + 1] subdivision method: B of each inside-sample count, in the
                                 // compute type, and beta (betatab); null: formed per slot
    const double* betatab;
    int stream;                  // store the slots with streaming stores (lattices that take the
                                 // LBM pass's streaming accesses: beyond the last-level cache)
    DevCounters* ctr;
};

// registration: the tile lists (on lattices of up to 8192 tiles left in
// arbitrary order within a tile, which vox_voxelize's select kernel then
// sets, clearing the registration counters: it follows every vox_register)
hipError_t vox_register(const VoxArgs& A, int* scan_tmp, hipStream_t s);
// voxelisation of registered tiles (with A.t.slot_beta null, beta itself is
// not stored: only the slots' local indices and B)
hipError_t vox_voxelize(const VoxArgs& A, int ctype_double, hipStream_t s);
// the selection alone, again, from the particle records and count boxes of the
// last vox_voxelize (they are kept until the next one): the same slots, and
// beta when A.t.slot_beta is set
hipError_t vox_select(const VoxArgs& A, int ctype_double, hipStream_t s);
hipError_t vox_reduce_hydro(const VoxArgs& A, hipStream_t s);
// the subdivision method's tables of B and beta per inside-sample count (ns^3 + 1
// entries each; btab in double when ctype_double, else float), from the same
// expressions the selection would evaluate per slot
hipError_t vox_fill_tables(void* btab, double* betatab, int ns, double tau, int ctype_double, hipStream_t s);
// bytes of one particle record (VoxArgs::vpart)
size_t vox_part_bytes();
// cells of a count box's x-y plane the row-counting kernel holds (per z-slab)
size_t vox_box_cells_max();
