// common.h -- internal definitions of the gfx950 coupled LBM-PSM-DEM library.
//
// Device data layout (lattice units):
//   populations  f[i * N + cell], shifted g_i = f_i - w_i, storage type S
//                (double / float / bf16 bits / half), updated in place with the
//                AA pattern (even steps read and write the own cell, odd steps
//                read from and write to the neighbours);
//   lattice tiles of TX x TY x TZ = 64 x 4 x 4 cells; a workgroup of 256 lanes
//                owns one tile, one wave per x-row (64 cells, coalesced), four
//                z-planes per lane;
//   per-cell solid slots in tile-major order (tile * 1024 + local cell);
//   particles    interleaved xyz double arrays [3 n], quaternions [4 n].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "psmdem.h"

#define PSM_TX 64
#define PSM_TY 4
#define PSM_TZ 4
#define PSM_TILE (PSM_TX * PSM_TY * PSM_TZ)
#define PSM_PMAX 128          // particles registered in one tile (LBM-PSM / voxelisation)
#define PSM_MAXNB 96          // unique neighbours j > i of one particle
#define PSM_SLOTS_MAX 4

// device-side flag bits (psmdem_counters_t.flags)
#define PSM_FLAG_PAIRS 1
#define PSM_FLAG_TILE 2
#define PSM_FLAG_NEIGH 4
#define PSM_FLAG_VREG 8
#define PSM_FLAG_CAPACITY_MASK 15ull
// a cell density that is not a positive finite number (LBM), or a particle
// centre that is not finite or lies more than one box length outside the
// domain (DEM predictor, voxelisation): the state has blown up
#define PSM_FLAG_UNSTABLE 16

// ---------------------------------------------------------------------------
// D3Q19 (Sec. 2.3): velocities, weights, opposite directions
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int d3q19_cx(int i) {
    constexpr int v[19] = {0, 1, 0, 0, 1, 1, 1, 1, 0, 0, -1, 0, 0, -1, -1, -1, -1, 0, 0};
    return v[i];
}
__host__ __device__ constexpr int d3q19_cy(int i) {
    constexpr int v[19] = {0, 0, 1, 0, 1, -1, 0, 0, 1, 1, 0, -1, 0, -1, 1, 0, 0, -1, -1};
    return v[i];
}
__host__ __device__ constexpr int d3q19_cz(int i) {
    constexpr int v[19] = {0, 0, 0, 1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 0, 0, -1, 1, -1, 1};
    return v[i];
}
__host__ __device__ constexpr int d3q19_opp(int i) { return i == 0 ? 0 : (i <= 9 ? i + 9 : i - 9); }
__host__ __device__ constexpr double d3q19_w(int i) {
    return i == 0 ? 1.0 / 3.0 : (((i - 1) % 9) < 3 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// ---------------------------------------------------------------------------
// kernel argument blocks
// ---------------------------------------------------------------------------
struct GeoArgs {
    int nx, ny, nz;
    long long N;
    int ntx, nty, ntz;
    long long ntiles;
    int periodic[3];
    int bc[6];
};

struct PartArgs {          // particle state, all double
    int np;
    const int* shape;
    const unsigned char* fixed;
    double *semi, *mass, *inertia, *rb, *dens;
    double *pos, *q, *qold, *v, *w, *vp, *wp, *a, *al;
    double *fh, *mh, *fd, *md;
    double *kin;           // [9 np]: position, v^p, w^p (read by the LBM-PSM kernel)
};

// tile registrations of particles (solid fractions and hydrodynamic partial sums)
struct TileArgs {
    int* tile_start;       // [ntiles + 1] exclusive offsets into tile_list
    unsigned long long* tile_list;  // (pid << 32 | emission index), sorted by pid per tile
    int* vcount;           // [np] tiles per particle
    int* voff;             // [np + 1] emission offsets
    int* vinv;             // [cap] emission index -> position in tile_list
    long long cap;         // capacity of tile_list / vinv / partial
    unsigned int* slot_lp; // [ntiles * 1024] byte k = local particle index of slot k (0xff none)
    void* slot_B;          // [ms][ntiles * 1024] B_k in the compute type
    double* partial;       // [cap][6] per (tile, particle): force then torque
    double* slot_beta;     // [ms][ntiles * 1024] beta of kept slots (double, for read-back)
    unsigned* tile_ed;     // [2 ntiles] entries (beta > 0) and dropped entries of each tile's last
                           // selection, summed when read; null: the step counters take atomics
};

// device error flags and counters (one 64-bit word each)
struct DevCounters {
    unsigned long long flags;
    unsigned long long entries;
    unsigned long long dropped;
    unsigned long long contacts;
    unsigned long long items;     // boundary cells queued for sampling this step
};

// ---------------------------------------------------------------------------
// device helpers shared by several kernels
// ---------------------------------------------------------------------------
// Exclusive scan of in[0..n) into out[0..n], out[n] = total, by one workgroup
// of NT threads (every thread of the workgroup calls it).
template <int NT>
__device__ inline void psm_block_scan(const int* in, int* out, long long n) {
    __shared__ int wsum[NT / 64];
    __shared__ int carry;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (long long base = 0; base < n; base += NT) {
        const long long i = base + tid;
        const int v = i < n ? in[i] : 0;
        int x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wid] = x;
        __syncthreads();
        int off = 0, tot = 0;
        for (int w = 0; w < NT / 64; ++w) {
            off += w < wid ? wsum[w] : 0;
            tot += wsum[w];
        }
        const int c = carry;
        if (i < n) out[i] = c + off + x - v;
        __syncthreads();
        if (tid == 0) carry = c + tot;
        __syncthreads();
    }
    if (tid == 0) out[n] = carry;
    __syncthreads();
}

// hydrodynamic force and torque of particle k (Sec. 2.4, momentum exchange):
// minus the sum of its per-tile partials, in emission order
__device__ inline void psm_reduce_hydro(const TileArgs& t, const PartArgs& p, int k) {
    double F[3] = {0.0, 0.0, 0.0}, M[3] = {0.0, 0.0, 0.0};
    const int e0 = t.voff[k], e1 = t.voff[k + 1];
    for (int e = e0; e < e1 && e < t.cap; ++e) {
        const long long s = t.vinv[e];
        if (s < 0 || s >= t.cap) continue;
        const double* P = t.partial + 6 * s;
        for (int c = 0; c < 3; ++c) {
            F[c] -= P[c];
            M[c] -= P[3 + c];
        }
    }
    for (int c = 0; c < 3; ++c) {
        p.fh[3 * k + c] = F[c];
        p.mh[3 * k + c] = M[c];
    }
}

// The same sums by one wave (every lane calls it): lanes fetch the
// particle's partials into the wave's LDS buffer buf[64 * 6], lane 0 adds
// them in emission order and stores fh, mh.
__device__ inline void psm_reduce_hydro_wave(const TileArgs& t, const PartArgs& p, int k, int lane, double* buf) {
    const int e0 = t.voff[k], e1 = t.voff[k + 1];
    double F[3] = {0.0, 0.0, 0.0}, M[3] = {0.0, 0.0, 0.0};
    for (int b = e0; b < e1 && b < t.cap; b += 64) {
        const int e = b + lane;
        bool ok = false;
        if (e < e1 && e < t.cap) {
            const long long s = t.vinv[e];
            ok = s >= 0 && s < t.cap;
            if (ok)
#pragma unroll
                for (int c = 0; c < 6; ++c) buf[6 * lane + c] = t.partial[6 * s + c];
        }
        const unsigned long long okm = __ballot(ok);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane == 0) {
            const int m = (e1 - b < 64 ? e1 - b : 64);
            for (int j = 0; j < m; ++j)
                if ((okm >> j) & 1ull)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        F[c] -= buf[6 * j + c];
                        M[c] -= buf[6 * j + 3 + c];
                    }
        }
        // the buffer is refilled only after lane 0 has read it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (lane == 0)
        for (int c = 0; c < 3; ++c) {
            p.fh[3 * k + c] = F[c];
            p.mh[3 * k + c] = M[c];
        }
}

// host helpers
#define PSM_CHECK(call)                                                      \
    do {                                                                     \
        hipError_t e__ = (call);                                             \
        if (e__ != hipSuccess) return psm_hip_fail(e__, #call, __FILE__, __LINE__); \
    } while (0)

// error value usable as an int stage code or as a psmdem_status
struct PsmErr {
    int v;
    operator int() const { return v; }
    operator psmdem_status() const { return (psmdem_status)v; }
};
PsmErr psm_hip_fail(hipError_t e, const char* what, const char* file, int line);
void psm_set_error(const char* fmt, ...);

// exclusive scan of n ints into out[0..n], out[n] = total (device); tmp >= scan_tmp_size(n)
size_t psm_scan_tmp_ints(long long n);
// exclusive scan of in[0..n) into out[0..n], out[n] = total; with run, only if *run != 0
hipError_t psm_scan(const int* in, int* out, long long n, int* tmp, hipStream_t s, const int* run = nullptr);
// two independent scans; one launch when both are short
hipError_t psm_scan2(const int* in0, int* out0, long long n0, const int* in1, int* out1, long long n1, int* tmp,
                     hipStream_t s);
hipError_t psm_fill_int(int* p, int v, long long n, hipStream_t s);
