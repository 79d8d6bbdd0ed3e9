// voxel.hip -- solid fractions of spheres and ellipsoids on lattice tiles
// (Sec. 2.4: subdivision and distance-based methods; Sec. 3.2.3: at most k
// solids per fluid cell) and the per-particle hydrodynamic reduction.
// Compiled with -ffp-contract=off: the subdivision sample test decides an
// integer count and is evaluated with separately rounded operations.  The row
// counting's root arithmetic (whose results only need to lie within the
// margins it tests against) is contracted locally.
//
// Pipeline per coupled step:
//   k_vox_parts    each particle's record (centre, rotation, extents, lattice box)
//   k_vox_count    tiles touched by each particle's lattice box (count + tile histogram)
//   (scans)        emission offsets per particle, list offsets per tile
//   k_vox_scatter  counting-sort scatter of (pid, emission index) into tiles
//   (k_tile_sort)  order each tile's list by pid; inverse map emission -> position
//                  (lattices of up to VOX_SORT_IN_TILE_MAX tiles do this in the
//                  select kernel instead)
//   k_vox_rows     subdivision method: one workgroup per particle counts the
//                  inside samples of every cell of its lattice box, a row of
//                  samples at a time, into the particle's count box
//   k_vox_select   per tile: beta of every (cell, particle) (a count-box entry, or
//                  the distance formula), keep the max_solids largest (ties to
//                  the smaller pid), B_k, slots
//   k_reduce_hydro per particle: minus the sum of its tile partials (F, M)
// Serving batches classify, sample and select a tile in one workgroup
// (k_voxelize_batch); both forms count the same samples.
#include <math.h>

#include "common.h"
#include "serve.h"
#include "voxel.h"

namespace {

__device__ inline void quat_rbw(const double* q, double R[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

__device__ inline void half_extents(const VoxArgs& A, int k, double e[3]) {
    const double* s = A.p.semi + 3 * k;
    if (A.p.shape[k] == 0) {
        e[0] = e[1] = e[2] = s[0];
        return;
    }
    double R[9];
    quat_rbw(A.p.q + 4 * k, R);
    for (int r = 0; r < 3; ++r) {
        double t0 = s[0] * R[3 * r + 0], t1 = s[1] * R[3 * r + 1], t2 = s[2] * R[3 * r + 2];
        e[r] = sqrt((t0 * t0 + t1 * t1) + t2 * t2);
    }
}

// lattice box of particle k: unwrapped lo..hi per axis, clamped on walled
// axes.  A centre that is not finite or lies more than one box length outside
// the domain (a blown-up state) gets an empty box (hi < lo on every axis) and
// returns true; every other box lies within [-1.5 n - 1, 2.5 n + 1) per axis
// (the half extent stays below n / 2, checked at creation).
__device__ inline bool lattice_box(const VoxArgs& A, int k, int lo[3], int hi[3]) {
    double e[3];
    half_extents(A, k, e);
    const int n[3] = {A.g.nx, A.g.ny, A.g.nz};
    bool far = false;
    for (int a = 0; a < 3; ++a) {
        const double c = A.p.pos[3 * k + a];
        far = far || !(c >= -(double)n[a] && c < 2.0 * (double)n[a]);
    }
    if (far) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = 0;
            hi[a] = -1;
        }
        return true;
    }
    for (int a = 0; a < 3; ++a) {
        double E = e[a] + 1e-6;
        if (A.sf_method == 1) E += A.Rc;
        double c = A.p.pos[3 * k + a];
        lo[a] = (int)floor(c - E);
        hi[a] = (int)floor(c + E);
        if (!A.g.periodic[a]) {
            lo[a] = lo[a] < 0 ? 0 : lo[a];
            hi[a] = hi[a] > n[a] - 1 ? n[a] - 1 : hi[a];
        }
    }
    return false;
}

// distinct tile indices along one axis for the cell range lo..hi (unwrapped
// on a periodic axis: walked tile by tile in wrapped coordinates)
__device__ inline int axis_tiles(int lo, int hi, int n, int T, int periodic, int* out) {
    int cnt = 0;
    if (hi < lo) return 0;
    if (!periodic) {
        for (int t = lo / T; t <= hi / T && cnt < VOX_AXIS_MAX; ++t) out[cnt++] = t;
        return cnt;
    }
    for (int c = lo; c <= hi && cnt < VOX_AXIS_MAX;) {
        int w = c % n;
        w = w < 0 ? w + n : w;
        const int t = w / T;
        bool dup = false;
        for (int u = 0; u < cnt; ++u) dup |= out[u] == t;
        if (!dup) out[cnt++] = t;
        int step = T - w % T;          // to the start of the next tile
        step = w + step > n ? n - w : step;  // or to the wrap
        c += step;
    }
    for (int u = 1; u < cnt; ++u)
        for (int v = u; v > 0 && out[v] < out[v - 1]; --v) {
            int t = out[v]; out[v] = out[v - 1]; out[v - 1] = t;
        }
    return cnt;
}

// per-particle data staged in LDS for a tile (8-byte words, copied as such)
struct VoxPart {
    double c[3];
    double ax[3];
    double R[9];
    double inv[3];
    double e[3];
    double r[3];   // ellipsoids: body-frame half-widths of a cell's sample box, h sum_r |R_rk|
    int lo[3], hi[3];
    int shape;
    int pid;
};
static_assert(sizeof(VoxPart) % 8 == 0, "VoxPart is copied in 8-byte words");

struct TileSet {
    int tx[VOX_AXIS_MAX], ty[VOX_AXIS_MAX], tz[VOX_AXIS_MAX];
    int nx, ny, nz;
};

// returns true for a blown-up particle (no tiles); the lattice box comes from
// the step's particle record when there is one (formed at the start of the
// registration), else it is formed here
__device__ inline bool particle_tiles(const VoxArgs& A, int k, TileSet& S) {
    int lo[3], hi[3];
    bool far;
    if (A.vpart) {
        const VoxPart& V = ((const VoxPart*)A.vpart)[k];
        const int n[3] = {A.g.nx, A.g.ny, A.g.nz};
        far = false;
        for (int a = 0; a < 3; ++a) {
            lo[a] = V.lo[a];
            hi[a] = V.hi[a];
            far = far || !(V.c[a] >= -(double)n[a] && V.c[a] < 2.0 * (double)n[a]);
        }
    } else {
        far = lattice_box(A, k, lo, hi);
    }
    S.nx = axis_tiles(lo[0], hi[0], A.g.nx, PSM_TX, A.g.periodic[0], S.tx);
    S.ny = axis_tiles(lo[1], hi[1], A.g.ny, PSM_TY, A.g.periodic[1], S.ty);
    S.nz = axis_tiles(lo[2], hi[2], A.g.nz, PSM_TZ, A.g.periodic[2], S.tz);
    return far;
}

// Registration of particle k by a group of lanes: lane l of the group takes
// the l-th tile of the particle's box (x fastest, then y, then z), then the
// (l + group size)-th, ...; the tile's place in that order is also its
// emission index.
__device__ inline long long tile_of(const VoxArgs& A, const TileSet& S, int l) {
    const int a = l % S.nx, b = (l / S.nx) % S.ny, c = l / (S.nx * S.ny);
    return S.tx[a] + (long long)A.g.ntx * (S.ty[b] + (long long)A.g.nty * S.tz[c]);
}

// tile count of particle k and one tile-histogram increment per tile (through
// `hist`), by lane `lane` of a group of `gs` lanes
__device__ inline void reg_count_wave(const VoxArgs& A, int k, int lane, int* hist, int gs = 64) {
    TileSet S;
    const bool far = particle_tiles(A, k, S);
    const int n = S.nx * S.ny * S.nz;
    if (lane == 0) A.t.vcount[k] = n;
    if (lane == 0 && far) atomicOr(&A.ctr->flags, (unsigned long long)PSM_FLAG_UNSTABLE);
    for (int l = lane; l < n; l += gs) atomicAdd(&hist[tile_of(A, S, l)], 1);
}

// counting-sort scatter of particle k's (pid, emission) entries; `fill` counts per tile
__device__ inline void reg_scatter_wave(const VoxArgs& A, int k, int lane, int* fill, int gs = 64) {
    TileSet S;
    particle_tiles(A, k, S);
    const int n = S.nx * S.ny * S.nz;
    const int e0 = A.t.voff[k];
    bool full = false;
    for (int l = lane; l < n; l += gs) {
        const long long t = tile_of(A, S, l);
        const int e = e0 + l;
        const int slot = atomicAdd(&fill[t], 1);
        const long long at = (long long)A.t.tile_start[t] + slot;
        if (at < A.t.cap && e < A.t.cap)
            A.t.tile_list[at] = ((unsigned long long)k << 32) | (unsigned)e;
        else
            full = true;
    }
    if (full) atomicOr(&A.ctr->flags, (unsigned long long)PSM_FLAG_VREG);
}

// order tile t's list by (pid, emission) and record where each emission landed
__device__ inline void reg_sort(const VoxArgs& A, long long t) {
    long long s0 = A.t.tile_start[t], s1 = A.t.tile_start[t + 1];
    if (s1 > A.t.cap) s1 = A.t.cap;
    if (s0 >= s1) return;
    if (s1 - s0 > PSM_PMAX) atomicOr(&A.ctr->flags, (unsigned long long)PSM_FLAG_TILE);
    unsigned long long* L = A.t.tile_list;
    for (long long u = s0 + 1; u < s1; ++u)
        for (long long v = u; v > s0 && L[v] < L[v - 1]; --v) {
            unsigned long long x = L[v]; L[v] = L[v - 1]; L[v - 1] = x;
        }
    for (long long u = s0; u < s1; ++u) {
        unsigned e = (unsigned)(L[u] & 0xffffffffu);
        if (e < A.t.cap) A.t.vinv[e] = (int)u;
    }
}

// VOX_REG_G lanes per particle (a particle's box touches a few tiles, most
// often fewer than eight); block 0 also clears the step's entry counters
#define VOX_REG_G 8
__global__ void k_vox_count(VoxArgs A) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        A.ctr->entries = 0;
        A.ctr->dropped = 0;
        A.ctr->items = 0;
    }
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = (int)(g / VOX_REG_G);
    if (k >= A.p.np) return;
    reg_count_wave(A, k, (int)(g % VOX_REG_G), A.tile_count, VOX_REG_G);
}

__global__ void k_vox_scatter(VoxArgs A) {
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = (int)(g / VOX_REG_G);
    if (k >= A.p.np) return;
    reg_scatter_wave(A, k, (int)(g % VOX_REG_G), A.tile_fill, VOX_REG_G);
}

#define VOX_T 256  // lanes of the per-tile voxelisation workgroups
// Up to this many tiles the lists are ordered inside the first per-tile
// voxelisation kernel (saving a launch); larger lattices order them in a
// kernel of their own, one thread per tile, which costs less than the added
// latency in every tile workgroup.
#define VOX_SORT_IN_TILE_MAX 8192

// Tile t's list ordered by (pid, emission) by the tile's workgroup, the
// emission -> position map, and the tile's counters cleared for the next step.
// Up to VOX_T entries rank-sort through LDS (keys are unique); longer lists
// (beyond the tile capacity, flagged) take the serial sort.  Every thread of
// the workgroup calls it; the list is ordered when it returns.  Returns ks,
// which then holds the ordered list, or null (the list is in global memory only).
__device__ inline const unsigned long long* sort_tile_list(const VoxArgs& A, long long t, unsigned long long* ks) {
    const int tid = threadIdx.x;
    long long s0 = A.t.tile_start[t], s1 = A.t.tile_start[t + 1];
    if (s1 > A.t.cap) s1 = A.t.cap;
    if (tid == 0) {
        A.tile_count[t] = 0;
        A.tile_fill[t] = 0;
    }
    const long long n = s1 - s0;
    if (n <= 0) return nullptr;
    unsigned long long* L = A.t.tile_list + s0;
    if (n <= VOX_T) {
        if (n > PSM_PMAX && tid == 0) atomicOr(&A.ctr->flags, (unsigned long long)PSM_FLAG_TILE);
        const unsigned long long key = tid < n ? L[tid] : 0ull;
        if (tid < n) ks[tid] = key;
        __syncthreads();
        int r = 0;
        if (tid < n)
            for (int v = 0; v < (int)n; ++v) r += ks[v] < key ? 1 : 0;
        __syncthreads();
        if (tid < n) {
            ks[r] = key;
            L[r] = key;
            const unsigned e = (unsigned)(key & 0xffffffffu);
            if (e < A.t.cap) A.t.vinv[e] = (int)(s0 + r);
        }
    } else if (tid == 0) {
        reg_sort(A, t);
    }
    __syncthreads();
    return n <= VOX_T ? ks : nullptr;
}

// Registration of one domain by one workgroup (serving batches): the tile
// histogram and fill counters live in LDS, the lists and offsets are the ones
// of the multi-launch path above.
#define VOX_RT 1024
#define VOX_REG_LDS_TILES 8192

__global__ __launch_bounds__(VOX_RT) void k_vox_register_batch(const VoxArgs* __restrict__ jobs) {
    __shared__ int hist_s[VOX_REG_LDS_TILES];
    const VoxArgs& A = jobs[blockIdx.x];
    const int tid = threadIdx.x;
    if (A.g.ntiles > VOX_REG_LDS_TILES) return;  // refused on the host
    const int nt = (int)A.g.ntiles, np = A.p.np;
    if (tid == 0) {
        A.ctr->entries = 0;
        A.ctr->dropped = 0;
    }
    for (int t = tid; t < nt; t += VOX_RT) hist_s[t] = 0;
    __syncthreads();
    for (int k = tid >> 6; k < np; k += VOX_RT / 64) reg_count_wave(A, k, tid & 63, hist_s);
    __syncthreads();
    for (int t = tid; t < nt; t += VOX_RT) A.tile_count[t] = hist_s[t];
    __syncthreads();
    psm_block_scan<VOX_RT>(A.t.vcount, A.t.voff, np);
    psm_block_scan<VOX_RT>(A.tile_count, A.t.tile_start, nt);
    for (int t = tid; t < nt; t += VOX_RT) hist_s[t] = 0;
    __syncthreads();
    for (int k = tid >> 6; k < np; k += VOX_RT / 64) reg_scatter_wave(A, k, tid & 63, hist_s);
    __syncthreads();
    for (int t = tid; t < nt; t += VOX_RT) {
        reg_sort(A, t);
        A.tile_count[t] = 0;  // left cleared, as the multi-launch path leaves it
    }
}


// what the selection needs of a candidate (a quarter of a full record)
struct SelPart {
    double c[3];
    double ax[1];   // radius (the distance method)
    int lo[3], hi[3];
    int shape, pid;
};
static_assert(sizeof(SelPart) % 8 == 0, "SelPart is copied in 8-byte words");

__device__ inline void sel_of(const VoxPart& V, SelPart& P) {
    for (int a = 0; a < 3; ++a) {
        P.c[a] = V.c[a];
        P.lo[a] = V.lo[a];
        P.hi[a] = V.hi[a];
    }
    P.ax[0] = V.ax[0];
    P.shape = V.shape;
    P.pid = V.pid;
}

// orders each tile's list, then clears the tile's counters for the next step
__global__ void k_tile_sort(VoxArgs A) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= A.g.ntiles) return;
    reg_sort(A, t);
    A.tile_count[t] = 0;
    A.tile_fill[t] = 0;
}


template <typename PT>
__device__ inline bool in_box(const PT& P, int x, int n, int axis, int periodic, int* X) {
    int lo = P.lo[axis], hi = P.hi[axis];
    int v;
    if (periodic) {
        // lo lies within one period below x: shift by whole periods without a division
        int d = x - lo;
        while (d < 0) d += n;
        while (d >= n) d -= n;
        v = lo + d;
    } else {
        v = x;
    }
    *X = v;
    return v >= lo && v <= hi;
}

__device__ inline double ell_q(const VoxPart& P, double dx, double dy, double dz) {
    double p0 = (P.R[0] * dx + P.R[3] * dy) + P.R[6] * dz;
    double p1 = (P.R[1] * dx + P.R[4] * dy) + P.R[7] * dz;
    double p2 = (P.R[2] * dx + P.R[5] * dy) + P.R[8] * dz;
    return ((p0 * p0) * P.inv[0] + (p1 * p1) * P.inv[1]) + (p2 * p2) * P.inv[2];
}

// Classification of lattice cell (X,Y,Z) against particle P for the subdivision
// method: 0 every sample outside, 1 every sample inside, 2 samples needed.
// The shortcuts are exact: they only fire with a margin far above the rounding
// of any sample's test value.  Spheres are bounded over the box the samples
// span, offsets slo..shi from the cell corner (the first and last sample
// offset), not over the whole cell.
__device__ int classify(const VoxPart& P, int X, int Y, int Z, double slo, double shi) {
    const int Xc[3] = {X, Y, Z};
    if (P.shape == 0) {
        const double R2 = P.ax[0] * P.ax[0];
        double maxr2 = 0.0, minr2 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double dl = ((double)Xc[a] + slo) - P.c[a];
            double dh = ((double)Xc[a] + shi) - P.c[a];
            double l2 = dl * dl, h2 = dh * dh;
            maxr2 += l2 > h2 ? l2 : h2;
            minr2 += dl > 0.0 ? l2 : (dh < 0.0 ? h2 : 0.0);
        }
        const double m = 1e-8 * (1.0 + R2);
        if (maxr2 < R2 - m) return 1;
        if (minr2 > R2 + m) return 0;
        return 2;
    }
    // Ellipsoids, over the cell's sample box (centre X + 1/2, half-width h =
    // (ns - 1) / (2 ns) per axis, widened by 1e-9 for the rounding of the
    // sample coordinates).  In the body frame the box's points p satisfy
    // |p_k - pc_k| <= r_k with r_k = h sum_r |R_rk|, so
    //   Q >= sum_k inv_k max(0, |pc_k| - r_k)^2   (every sample outside) and
    //   Q <= sum_k inv_k (|pc_k| + r_k)^2          (every sample inside);
    // between them, Q being convex its maximum over the box is at one of the
    // box's eight vertices: all eight inside means every sample is inside.
    // The margin 1e-9 lies far above the rounding of any sample's Q.
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double dl = (double)Xc[a] - P.c[a];
        double dh = ((double)Xc[a] + 1.0) - P.c[a];
        if (dh < -P.e[a] - 1e-6 || dl > P.e[a] + 1e-6) return 0;
    }
    const double h = 0.5 * (shi - slo) + 1e-9;
    const double d0 = ((double)X + 0.5) - P.c[0], d1 = ((double)Y + 0.5) - P.c[1], d2 = ((double)Z + 0.5) - P.c[2];
    double pc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) pc[k] = (P.R[0 + k] * d0 + P.R[3 + k] * d1) + P.R[6 + k] * d2;
    double qmin = 0.0, qmax = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double a = fabs(pc[k]);
        const double lo = a > P.r[k] ? a - P.r[k] : 0.0, hi = a + P.r[k];
        qmin += lo * lo * P.inv[k];
        qmax += hi * hi * P.inv[k];
    }
    if (qmin > 1.0 + 1e-9) return 0;
    if (qmax < 1.0 - 1e-9) return 1;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const double sx = (v & 1) ? h : -h, sy = (v & 2) ? h : -h, sz = (v & 4) ? h : -h;
        double q = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double pk = pc[k] + ((P.R[0 + k] * sx + P.R[3 + k] * sy) + P.R[6 + k] * sz);
            q += pk * pk * P.inv[k];
        }
        if (!(q < 1.0 - 1e-9)) return 2;
    }
    return 1;
}

// one sample m (a fastest): inside test in the evaluation order of the definition
__device__ inline bool sample_in(const VoxPart& P, int X, int Y, int Z, const double* off, int ns, int m) {
    const int a = m % ns, b = (m / ns) % ns, c = m / (ns * ns);
    const double dz = ((double)Z + off[c]) - P.c[2];
    const double dy = ((double)Y + off[b]) - P.c[1];
    const double dx = ((double)X + off[a]) - P.c[0];
    if (P.shape == 0) {
        const double R2 = P.ax[0] * P.ax[0];
        return ((dx * dx + dy * dy) + dz * dz) < R2;
    }
    return ell_q(P, dx, dy, dz) < 1.0;
}

template <typename PT>
__device__ inline double beta_distance(const PT& P, int X, int Y, int Z, double Rc) {
    const double R = P.ax[0];
    double dx = ((double)X + 0.5) - P.c[0], dy = ((double)Y + 0.5) - P.c[1], dz = ((double)Z + 0.5) - P.c[2];
    double dist = sqrt((dx * dx + dy * dy) + dz * dz);
    double delta = (R + Rc) - dist;
    if (delta < 0.0) return 0.0;
    if (delta > 2.0 * Rc) return 1.0;
    return delta / (2.0 * Rc);
}

#define VOX_QCAP 2048
#define VOX_NS_REG 12   // spheres with at most this many samples per direction keep the x terms in registers

// the ms largest beta of a cell (ties: the earlier, smaller pid wins), kept in
// four named registers in descending order
struct Top4 {
    double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
    int l0 = 0, l1 = 0, l2 = 0, l3 = 0;
    int n = 0;
};

__device__ inline void top_swap(double& a, double& b, int& i, int& j) {
    const double t = a;
    a = b;
    b = t;
    const int k = i;
    i = j;
    j = k;
}

__device__ inline void keep_top(Top4& T, int ms, double beta, int u, unsigned long long& dropped) {
    int pos;
    if (T.n < ms) {
        pos = T.n++;
    } else {
        ++dropped;
        const double last = ms == 1 ? T.b0 : (ms == 2 ? T.b1 : (ms == 3 ? T.b2 : T.b3));
        if (!(beta > last)) return;
        pos = ms - 1;
    }
    if (pos == 0) { T.b0 = beta; T.l0 = u; }
    else if (pos == 1) { T.b1 = beta; T.l1 = u; }
    else if (pos == 2) { T.b2 = beta; T.l2 = u; }
    else { T.b3 = beta; T.l3 = u; }
    if (pos >= 3 && T.b2 < T.b3) top_swap(T.b2, T.b3, T.l2, T.l3);
    if (pos >= 2 && T.b1 < T.b2) top_swap(T.b1, T.b2, T.l1, T.l2);
    if (pos >= 1 && T.b0 < T.b1) top_swap(T.b0, T.b1, T.l0, T.l1);
}

// the kept slots reordered by pid (local index order is pid order)
__device__ inline void top_by_pid(Top4& T) {
    for (int pass = 0; pass < 3; ++pass) {
        if (1 < T.n && T.l1 < T.l0) top_swap(T.b0, T.b1, T.l0, T.l1);
        if (2 < T.n && T.l2 < T.l1) top_swap(T.b1, T.b2, T.l1, T.l2);
        if (3 < T.n && T.l3 < T.l2) top_swap(T.b2, T.b3, T.l2, T.l3);
    }
}

// ---------------------------------------------------------------------------
// pieces of the per-tile voxelisation, shared by the one-kernel form (serving
// batches) and the three-kernel form (classify / sample / select)
// ---------------------------------------------------------------------------
// the voxelisation record of particle k (ns samples per direction)
__device__ inline void make_part(const VoxArgs& A, int k, VoxPart& P) {
    P.pid = k;
    P.shape = A.p.shape[k];
    for (int a = 0; a < 3; ++a) {
        P.c[a] = A.p.pos[3 * k + a];
        P.ax[a] = A.p.semi[3 * k + a];
        P.inv[a] = 1.0 / (P.ax[a] * P.ax[a]);
    }
    quat_rbw(A.p.q + 4 * k, P.R);
    half_extents(A, k, P.e);
    lattice_box(A, k, P.lo, P.hi);
    const double h = (double)(A.ns - 1) / (double)(2 * A.ns) + 1e-9;
    for (int a = 0; a < 3; ++a) P.r[a] = h * ((fabs(P.R[a]) + fabs(P.R[3 + a])) + fabs(P.R[6 + a]));
}

// the step's records, one per particle, for the per-tile kernels
__global__ void k_vox_parts(VoxArgs A) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.p.np) return;
    VoxPart P;
    make_part(A, k, P);
    ((VoxPart*)A.vpart)[k] = P;
}

// the tile's registered particles staged in LDS, and the sample offsets (the
// list from keys when given, else from global memory); the records come from
// the step's record array when there is one (copied in 8-byte words by the
// whole workgroup), else each is formed here
__device__ inline void stage_particles(const VoxArgs& A, VoxPart* sp, double* off, long long s0, int count,
                                       const unsigned long long* keys = nullptr) {
    const int tid = threadIdx.x;
    if (tid < A.ns) off[tid] = (double)(2 * tid + 1) / (double)(2 * A.ns);
    if (A.vpart) {
        constexpr int WORDS = (int)(sizeof(VoxPart) / 8);
        const unsigned long long* src = (const unsigned long long*)A.vpart;
        unsigned long long* dst = (unsigned long long*)sp;
        for (int w = tid; w < count * WORDS; w += VOX_T) {
            const int u = w / WORDS;
            int k = (int)((keys ? keys[u] : A.t.tile_list[s0 + u]) >> 32);
            if (k >= A.p.np) k = 0;
            dst[w] = src[(long long)k * WORDS + (w - u * WORDS)];
        }
        return;
    }
    for (int u = tid; u < count; u += VOX_T) {
        int k = (int)((keys ? keys[u] : A.t.tile_list[s0 + u]) >> 32);
        if (k >= A.p.np) k = 0;
        make_part(A, k, sp[u]);
    }
}

// candidates of a lane's (x, y) column: bit u set when particle u's lattice box
// holds x and y (ascending u = ascending pid)
template <typename PT>
__device__ inline void column_masks(const VoxArgs& A, const PT* sp, int count, int x, int y, bool xy_ok,
                                    unsigned long long& cm0, unsigned long long& cm1) {
    cm0 = cm1 = 0;
    if (!xy_ok) return;
    for (int u = 0; u < count; ++u) {
        int X, Y;
        if (in_box(sp[u], x, A.g.nx, 0, A.g.periodic[0], &X) && in_box(sp[u], y, A.g.ny, 1, A.g.periodic[1], &Y)) {
            if (u < 64) cm0 |= 1ull << u;
            else cm1 |= 1ull << (u - 64);
        }
    }
}

// Visits the lane's (plane, candidate) pairs whose cell lies in the particle's
// box, in the order planes ascending, then pid ascending:
// f(lz, u, P, X, Y, Z) returns false to stop.
template <typename F>
__device__ inline void for_each_pair(const VoxArgs& A, const VoxPart* sp, int tz, int x, int y, bool xy_ok,
                                     unsigned long long cm0, unsigned long long cm1, F f) {
    if (!xy_ok) return;
    for (int lz = 0; lz < PSM_TZ; ++lz) {
        const int z = tz * PSM_TZ + lz;
        if (z >= A.g.nz) break;
        for (int w = 0; w < 2; ++w)
            for (unsigned long long bits = w ? cm1 : cm0; bits; bits &= bits - 1) {
                const int u = 64 * w + __ffsll((long long)bits) - 1;
                const VoxPart& P = sp[u];
                int X, Y, Z;
                in_box(P, x, A.g.nx, 0, A.g.periodic[0], &X);
                in_box(P, y, A.g.ny, 1, A.g.periodic[1], &Y);
                if (!in_box(P, z, A.g.nz, 2, A.g.periodic[2], &Z)) continue;
                if (!f(lz, u, P, X, Y, Z)) return;
            }
    }
}

// exclusive prefix of the per-lane counts over the workgroup, and the total
__device__ inline void block_offsets(int mine, int* tcnt, int& my_off, int& total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int incl = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane == 63) tcnt[wid] = incl;
    __syncthreads();
    my_off = incl - mine;
    total = 0;
    for (int w = 0; w < VOX_T / 64; ++w) {
        const int c = tcnt[w];
        if (w < wid) my_off += c;
        total += c;
    }
    __syncthreads();
}

// Inside samples of cell (X, Y, Z) for particle P, counted by one wave.  The
// per-axis terms of the sample test are formed once in wave-private LDS (tab)
// with the same rounding as the definition: squared offsets for spheres,
// rotated components for ellipsoids; then each lane takes one row (b, c) of
// samples and walks its ns samples along x.  The count is the sum of exact
// per-row counts.  Every lane of the wave calls it; all get the count.
__device__ inline int sample_count(const VoxPart& P, int X, int Y, int Z, const double* off, int ns, double* tab) {
    const int lane = threadIdx.x & 63;
    const bool sph = P.shape == 0;
    if (lane < ns) {
        const double dx = ((double)X + off[lane]) - P.c[0];
        const double dy = ((double)Y + off[lane]) - P.c[1];
        const double dz = ((double)Z + off[lane]) - P.c[2];
        if (sph) {
            tab[lane] = dx * dx;
            tab[ns + lane] = dy * dy;
            tab[2 * ns + lane] = dz * dz;
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                tab[(3 * k + 0) * ns + lane] = P.R[0 + k] * dx;
                tab[(3 * k + 1) * ns + lane] = P.R[3 + k] * dy;
                tab[(3 * k + 2) * ns + lane] = P.R[6 + k] * dz;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int nrows = ns * ns;
    int cnt = 0;
    if (sph && ns <= VOX_NS_REG) {
        // x terms in registers (LDS broadcasts, once per item)
        const double R2 = P.ax[0] * P.ax[0];
        double x2[VOX_NS_REG];
#pragma unroll
        for (int a = 0; a < VOX_NS_REG; ++a) x2[a] = a < ns ? tab[a] : 0.0;
        for (int r0 = 0; r0 < nrows; r0 += 64) {
            const int r = r0 + lane;
            const bool act = r < nrows;
            const int b = act ? r % ns : 0, c = act ? r / ns : 0;
            const double y2 = tab[ns + b], z2 = tab[2 * ns + c];
            int rc = 0;
#pragma unroll
            for (int a = 0; a < VOX_NS_REG; ++a) rc += (a < ns && ((x2[a] + y2) + z2) < R2) ? 1 : 0;
            cnt += act ? rc : 0;
        }
    } else if (sph) {
        const double R2 = P.ax[0] * P.ax[0];
        for (int r0 = 0; r0 < nrows; r0 += 64) {
            const int r = r0 + lane;
            const bool act = r < nrows;
            const int b = act ? r % ns : 0, c = act ? r / ns : 0;
            const double y2 = tab[ns + b], z2 = tab[2 * ns + c];
            int rc = 0;
            for (int a = 0; a < ns; ++a) rc += ((tab[a] + y2) + z2) < R2 ? 1 : 0;
            cnt += act ? rc : 0;
        }
    } else {
        const double i0 = P.inv[0], i1 = P.inv[1], i2 = P.inv[2];
        for (int r0 = 0; r0 < nrows; r0 += 64) {
            const int r = r0 + lane;
            const bool act = r < nrows;
            const int b = act ? r % ns : 0, c = act ? r / ns : 0;
            const double y0 = tab[ns + b], z0 = tab[2 * ns + c];
            const double y1 = tab[4 * ns + b], z1 = tab[5 * ns + c];
            const double y2 = tab[7 * ns + b], z2 = tab[8 * ns + c];
            int rc = 0;
            for (int a = 0; a < ns; ++a) {
                const double p0 = (tab[a] + y0) + z0;
                const double p1 = (tab[3 * ns + a] + y1) + z1;
                const double p2 = (tab[6 * ns + a] + y2) + z2;
                rc += (((p0 * p0) * i0 + (p1 * p1) * i1) + (p2 * p2) * i2) < 1.0 ? 1 : 0;
            }
            cnt += act ? rc : 0;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return cnt;
}

// Phase C: beta per (cell, particle) in pid order, keep the largest ms, write
// the slots.  BOX: the subdivision count of every (cell, particle) is
// lookup(j, P, X, Y, Z) (the count box); else boundary cells take their count
// from lookup(j, P, X, Y, Z), j running from my_off in the order of
// for_each_pair, and the others are classified.
// the kept slots of one cell (T in descending beta, ties to the smaller pid),
// ordered by pid, into slot_lp, slot_B and slot_beta
template <typename C>
__device__ inline void write_slots(const VoxArgs& A, Top4& T, long long cell) {
    C* Bout = (C*)A.t.slot_B;
    const long long plane = A.g.ntiles * (long long)PSM_TILE;
    top_by_pid(T);
    unsigned int lp = 0xffffffffu;
    if (T.n > 0) lp = (lp & ~0xffu) | (unsigned)T.l0;
    if (T.n > 1) lp = (lp & ~0xff00u) | ((unsigned)T.l1 << 8);
    if (T.n > 2) lp = (lp & ~0xff0000u) | ((unsigned)T.l2 << 16);
    if (T.n > 3) lp = (lp & ~0xff000000u) | ((unsigned)T.l3 << 24);
    A.t.slot_lp[cell] = lp;
    const double bq[PSM_SLOTS_MAX] = {T.n > 0 ? T.b0 : 0.0, T.n > 1 ? T.b1 : 0.0, T.n > 2 ? T.b2 : 0.0,
                                      T.n > 3 ? T.b3 : 0.0};
    // only the kept slots are written: readers stop at the first empty index of slot_lp
#pragma unroll
    for (int q = 0; q < PSM_SLOTS_MAX; ++q)
        if (q < A.ms && q < T.n) {
            const double beta = bq[q];
            const double B = beta * (A.tau - 0.5) / ((1.0 - beta) + (A.tau - 0.5));
            Bout[q * plane + cell] = (C)B;
            if (A.t.slot_beta) A.t.slot_beta[q * plane + cell] = beta;
        }
}

// the workgroup's entry and drop counts: into the tile's own words when the
// domain keeps them (a global atomic per workgroup on one address would queue
// every tile of the lattice behind it), else into the step's counters
__device__ inline void add_entry_counts(const VoxArgs& A, long long t, unsigned long long my_e,
                                        unsigned long long my_d, unsigned long long* cnt_e,
                                        unsigned long long* cnt_d) {
    if (my_e) atomicAdd(cnt_e, my_e);
    if (my_d) atomicAdd(cnt_d, my_d);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (A.t.tile_ed) {
            A.t.tile_ed[2 * t] = (unsigned)*cnt_e;
            A.t.tile_ed[2 * t + 1] = (unsigned)*cnt_d;
        } else {
            if (*cnt_e) atomicAdd(&A.ctr->entries, *cnt_e);
            if (*cnt_d) atomicAdd(&A.ctr->dropped, *cnt_d);
        }
    }
}

// Phase C: beta per (cell, particle) in pid order, keep the largest ms, write
// the slots.  BOX: the subdivision count of every (cell, particle) is
// lookup(P, X, Y, Z) (the count box); the candidates are visited once for the
// lane's four planes together, so the four planes' count loads are in flight
// at once.  Else boundary cells take their count from lookup(j, P, X, Y, Z), j
// running from my_off in the order of for_each_pair, and the others are
// classified.  Every plane sees its candidates in ascending pid, as the
// selection's tie rule needs.
template <typename C, bool BOX, typename PT, typename L>
__device__ inline void select_slots(const VoxArgs& A, const PT* sp, long long t, int tz, int x, int y, bool xy_ok,
                                    unsigned long long cm0, unsigned long long cm1, double slo, double shi,
                                    int my_off, L lookup, unsigned long long* cnt_e, unsigned long long* cnt_d) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int ms = A.ms, n3 = A.ns * A.ns * A.ns;
    const bool subdiv = A.sf_method == 0;
    const long long base = t * (long long)PSM_TILE;
    unsigned long long my_e = 0, my_d = 0;
    if constexpr (BOX) {
        Top4 T[PSM_TZ];
        if (xy_ok)
            for (int w = 0; w < 2; ++w)
                for (unsigned long long bits = w ? cm1 : cm0; bits; bits &= bits - 1) {
                    const int u = 64 * w + __ffsll((long long)bits) - 1;
                    const PT& P = sp[u];
                    int X, Y;
                    in_box(P, x, A.g.nx, 0, A.g.periodic[0], &X);
                    in_box(P, y, A.g.ny, 1, A.g.periodic[1], &Y);
                    double beta[PSM_TZ];
#pragma unroll
                    for (int lz = 0; lz < PSM_TZ; ++lz) {
                        const int z = tz * PSM_TZ + lz;
                        int Z;
                        beta[lz] = 0.0;
                        if (z < A.g.nz && in_box(P, z, A.g.nz, 2, A.g.periodic[2], &Z))
                            beta[lz] = subdiv ? (double)lookup(P, X, Y, Z) / (double)n3 : beta_distance(P, X, Y, Z, A.Rc);
                    }
#pragma unroll
                    for (int lz = 0; lz < PSM_TZ; ++lz)
                        if (beta[lz] > 0.0) {
                            ++my_e;
                            keep_top(T[lz], ms, beta[lz], u, my_d);
                        }
                }
#pragma unroll
        for (int lz = 0; lz < PSM_TZ; ++lz)
            if (xy_ok && tz * PSM_TZ + lz < A.g.nz) write_slots<C>(A, T[lz], base + lane + PSM_TX * (wid + PSM_TY * lz));
        add_entry_counts(A, t, my_e, my_d, cnt_e, cnt_d);
        return;
    } else {
        int j = my_off;
        for (int lz = 0; lz < PSM_TZ; ++lz) {
            const int z = tz * PSM_TZ + lz;
            Top4 T;
            if (xy_ok && z < A.g.nz) {
                for (int w = 0; w < 2; ++w)
                    for (unsigned long long bits = w ? cm1 : cm0; bits; bits &= bits - 1) {
                        const int u = 64 * w + __ffsll((long long)bits) - 1;
                        const PT& P = sp[u];
                        int X, Y, Z;
                        in_box(P, x, A.g.nx, 0, A.g.periodic[0], &X);
                        in_box(P, y, A.g.ny, 1, A.g.periodic[1], &Y);
                        if (!in_box(P, z, A.g.nz, 2, A.g.periodic[2], &Z)) continue;
                        double beta;
                        if (!subdiv) {
                            beta = beta_distance(P, X, Y, Z, A.Rc);
                        } else {
                            const int cl = classify(P, X, Y, Z, slo, shi);
                            if (cl == 0) continue;
                            if (cl == 1) {
                                beta = 1.0;
                            } else {
                                const int cnt = lookup(j, P, X, Y, Z);
                                ++j;
                                beta = (double)cnt / (double)n3;
                            }
                        }
                        if (!(beta > 0.0)) continue;
                        ++my_e;
                        keep_top(T, ms, beta, u, my_d);
                    }
                write_slots<C>(A, T, base + lane + PSM_TX * (wid + PSM_TY * lz));
            }
        }
        add_entry_counts(A, t, my_e, my_d, cnt_e, cnt_d);
    }
}

struct TileRange {
    long long s0;
    int count;
    int tx, ty, tz;
};

__device__ inline TileRange tile_range(const VoxArgs& A, long long t) {
    TileRange r;
    long long s0 = A.t.tile_start[t], s1 = A.t.tile_start[t + 1];
    if (s1 > A.t.cap) s1 = A.t.cap;
    r.s0 = s0;
    r.count = (int)(s1 - s0) < PSM_PMAX ? (int)(s1 - s0) : PSM_PMAX;
    r.tx = (int)(t % A.g.ntx);
    r.ty = (int)((t / A.g.ntx) % A.g.nty);
    r.tz = (int)(t / ((long long)A.g.ntx * A.g.nty));
    return r;
}

// One tile in one workgroup (serving batches): classify, queue the boundary
// cells in LDS, count their samples (one wave per item), select.
template <typename C>
__device__ void voxelize_tile(const VoxArgs& A, const long long t) {
    __shared__ VoxPart sp[PSM_PMAX];
    __shared__ double off[32];
    __shared__ unsigned qitem[VOX_QCAP];
    __shared__ int qcnt[VOX_QCAP];
    __shared__ int tcnt[VOX_T / 64];
    __shared__ double tab_s[(VOX_T / 64) * 9 * 32];
    __shared__ unsigned long long cnt_e, cnt_d;
    const TileRange R = tile_range(A, t);
    if (R.count <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int ns = A.ns, n3 = ns * ns * ns;
    const bool subdiv = A.sf_method == 0;
    if (tid == 0) { cnt_e = 0; cnt_d = 0; }
    stage_particles(A, sp, off, R.s0, R.count);
    __syncthreads();
    const double slo = off[0], shi = off[A.ns - 1];  // first and last sample offset
    const int x = R.tx * PSM_TX + lane, y = R.ty * PSM_TY + wid;
    const bool xy_ok = x < A.g.nx && y < A.g.ny;
    unsigned long long cm0, cm1;
    column_masks(A, sp, R.count, x, y, xy_ok, cm0, cm1);
    int mine = 0;
    if (subdiv)
        for_each_pair(A, sp, R.tz, x, y, xy_ok, cm0, cm1, [&](int, int, const VoxPart& P, int X, int Y, int Z) {
            mine += classify(P, X, Y, Z, slo, shi) == 2;
            return true;
        });
    int my_off, total;
    block_offsets(mine, tcnt, my_off, total);
    if (mine) {
        int j = my_off;
        for_each_pair(A, sp, R.tz, x, y, xy_ok, cm0, cm1, [&](int lz, int u, const VoxPart& P, int X, int Y, int Z) {
            if (classify(P, X, Y, Z, slo, shi) == 2) {
                const unsigned l = lane + PSM_TX * (wid + PSM_TY * lz);
                qitem[j++] = (l << 8) | (unsigned)u;
            }
            return j < VOX_QCAP;
        });
    }
    __syncthreads();
    const int nq = total < VOX_QCAP ? total : VOX_QCAP;
    double* tab = tab_s + wid * (9 * 32);
    for (int it = wid; it < nq; it += VOX_T / 64) {
        const unsigned item = qitem[it];
        const int u = (int)(item & 0xffu), l = (int)(item >> 8);
        const int cx = R.tx * PSM_TX + (l % PSM_TX), cy = R.ty * PSM_TY + (l / PSM_TX) % PSM_TY;
        const int cz = R.tz * PSM_TZ + l / (PSM_TX * PSM_TY);
        const VoxPart& P = sp[u];
        int X, Y, Z;
        in_box(P, cx, A.g.nx, 0, A.g.periodic[0], &X);
        in_box(P, cy, A.g.ny, 1, A.g.periodic[1], &Y);
        in_box(P, cz, A.g.nz, 2, A.g.periodic[2], &Z);
        const int cnt = sample_count(P, X, Y, Z, off, ns, tab);
        if (lane == 0) qcnt[it] = cnt;
    }
    __syncthreads();
    select_slots<C, false, VoxPart>(A, sp, t, R.tz, x, y, xy_ok, cm0, cm1, slo, shi, my_off,
                    [&](int j, const VoxPart& P, int X, int Y, int Z) {
                        if (j < VOX_QCAP) return qcnt[j];
                        int cnt = 0;
                        for (int m = 0; m < n3; ++m) cnt += sample_in(P, X, Y, Z, off, ns, m);
                        return cnt;
                    },
                    &cnt_e, &cnt_d);
}

// ---------------------------------------------------------------------------
// single-domain form: count boxes per particle, then the per-tile selection
// ---------------------------------------------------------------------------
// Inside samples of every cell of particle P's lattice box, by one workgroup,
// a row of samples at a time.  Along a row (fixed y and z offsets dy, dz) the
// normalised test value is a quadratic in the x offset,
//   Q(x) = A x^2 + 2 B x + C,   inside when Q < 1,
// with A, B, C from the inverse shape matrix (an ellipsoid: p = R^T d and
// A = sum_k inv_k R_0k^2, B = sum_k inv_k R_0k w_k, C = sum_k inv_k w_k^2,
// w_k = R_1k dy + R_2k dz; a sphere: A = 1/r^2, B = 0, C = (dy^2 + dz^2)/r^2).
// The inside samples of a row lie between the roots r1 < r2 of Q = 1.  A
// sample farther than m = 1e-5 (1 + a_max) from both roots is decided by its
// side, since there |Q - 1| >= A m min(m, r2 - r1) lies far above the
// rounding of any evaluation of Q (the roots are formed only when the
// discriminant clears its own rounding bound by a factor 1e6); samples within
// m of a root, and every sample of a row whose discriminant is within that
// bound of zero (a row grazing the surface), are tested with the definition's
// own evaluation order.  Per z-sample plane only the rows whose discriminant
// can be positive are visited: as a function of dy it is the concave
// quadratic a2 dy^2 + a1 dy + a0, and outside its roots widened by 1e-3 it is
// below a2 1e-6 < 0, far beyond its rounding.  The counts therefore equal the
// per-sample definition's bit for bit; a row costs a root and a few
// comparisons instead of one test per sample.  The counts accumulate in LDS
// (z-slabs of the box that fit) and go to the particle's count box in global
// memory, one 16-bit count per cell, x fastest.
#define VOX_BOX_LDS 8192

__device__ inline int sample_exact(const VoxPart& P, double dx, double dy, double dz) {
    if (P.shape == 0) {
        const double R2 = P.ax[0] * P.ax[0];
        return ((dx * dx + dy * dy) + dz * dz) < R2 ? 1 : 0;
    }
    const double p0 = (P.R[0] * dx + P.R[3] * dy) + P.R[6] * dz;
    const double p1 = (P.R[1] * dx + P.R[4] * dy) + P.R[7] * dz;
    const double p2 = (P.R[2] * dx + P.R[5] * dy) + P.R[8] * dz;
    return (((p0 * p0) * P.inv[0] + (p1 * p1) * P.inv[1]) + (p2 * p2) * P.inv[2]) < 1.0 ? 1 : 0;
}

// sqrt(x) for x > 0 from the hardware reciprocal-square-root estimate refined
// by two Newton steps (a few units in the last place): the row roots only
// need to be within the margin of the exact test
__device__ inline double sqrt_est(double x) {
#pragma clang fp contract(fast)
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * (1.5 - h * y * y);
    y = y * (1.5 - h * y * y);
    return x * y;
}

// the row quadratic's coefficients of one particle (see k_vox_rows)
struct RowQ {
    double A, iA, by, bz, cyy, cyz, czz, a2, i2a2, mt, xl, gmax, fns;
};

// Row dy, dz of the cell row `row` (LDS counts of the box's x cells): the
// samples certainly inside are the global sample indices glo..ghi along the
// row (g = (X - lo_x) ns + a, at x = xl + (g + 1/2) / ns; empty: glo > ghi),
// returned for the caller to add; samples within the margin of a root, and
// every sample of a grazing row, are tested and added here.
__device__ inline void row_inside(const VoxPart& P, const RowQ& q, const double* off, int ns, double dy, double dz,
                                  double bzz, double cyzz, double czzz, int* row, int& glo, int& ghi) {
    glo = 1;
    ghi = 0;
    double B, disc, tol;
    {
#pragma clang fp contract(fast)
        B = q.by * dy + bzz;
        const double Cm1 = (q.cyy * dy * dy + cyzz * dy + czzz) - 1.0;
        disc = B * B - q.A * Cm1;
        tol = 1e-6 * (B * B + q.A * fabs(Cm1)) + 1e-10;
    }
    if (disc <= -tol) return;  // the row misses it
    if (disc < tol) {          // a row grazing the surface: every sample
        for (int X = P.lo[0]; X <= P.hi[0]; ++X) {
            int kx = 0;
            for (int a = 0; a < ns; ++a) kx += sample_exact(P, ((double)X + off[a]) - P.c[0], dy, dz);
            if (kx) atomicAdd(&row[X - P.lo[0]], kx);
        }
        return;
    }
    double G1, G2;
    {
#pragma clang fp contract(fast)
        const double sq = sqrt_est(disc);  // disc >= tol > 0 here
        G1 = ((-B - sq) * q.iA - q.xl) * q.fns - 0.5;
        G2 = ((-B + sq) * q.iA - q.xl) * q.fns - 0.5;
    }
    const double lo = fmax(floor(G1 + q.mt) + 1.0, 0.0), hi = fmin(ceil(G2 - q.mt) - 1.0, q.gmax);
    if (hi >= lo) {
        glo = (int)lo;
        ghi = (int)hi;
    }
    const double u0 = fmax(ceil(G1 - q.mt), 0.0), u1 = fmin(floor(G1 + q.mt), q.gmax);
    for (double g = u0; g <= u1; g += 1.0) {
        const int gi = (int)g;
        if (sample_exact(P, ((double)(P.lo[0] + gi / ns) + off[gi % ns]) - P.c[0], dy, dz))
            atomicAdd(&row[gi / ns], 1);
    }
    const double v0 = fmax(ceil(G2 - q.mt), 0.0), v1 = fmin(floor(G2 + q.mt), q.gmax);
    for (double g = v0; g <= v1; g += 1.0) {
        if (fabs(g - G1) <= q.mt) continue;
        const int gi = (int)g;
        if (sample_exact(P, ((double)(P.lo[0] + gi / ns) + off[gi % ns]) - P.c[0], dy, dz))
            atomicAdd(&row[gi / ns], 1);
    }
}

// samples of the index range glo..ghi per cell of the row
__device__ inline int range_in_cell(int glo, int ghi, int i, int ns) {
    const int a0 = i * ns, a1 = a0 + ns - 1;
    const int n = (ghi < a1 ? ghi : a1) - (glo > a0 ? glo : a0) + 1;
    return n > 0 ? n : 0;
}

// Inside samples of every cell of particle P's lattice box, by one workgroup,
// a row of samples at a time.  Along a row (fixed y and z offsets dy, dz) the
// normalised test value is a quadratic in the x offset,
//   Q(x) = A x^2 + 2 B x + C,   inside when Q < 1,
// with A, B, C from the inverse shape matrix (an ellipsoid: p = R^T d and
// A = sum_k inv_k R_0k^2, B = sum_k inv_k R_0k w_k, C = sum_k inv_k w_k^2,
// w_k = R_1k dy + R_2k dz; a sphere: A = 1/r^2, B = 0, C = (dy^2 + dz^2)/r^2).
// The inside samples of a row lie between the roots r1 < r2 of Q = 1.  A
// sample farther than m = 1e-5 (1 + a_max) from both roots is decided by its
// side, since there |Q - 1| >= A m min(m, r2 - r1) lies far above the
// rounding of any evaluation of Q (the roots are formed only when the
// discriminant clears its own rounding bound by a factor 1e6); samples within
// m of a root, and every sample of a row whose discriminant is within that
// bound of zero (a row grazing the surface), are tested with the definition's
// own evaluation order.  Per z-sample plane only the rows whose discriminant
// can be positive are visited: as a function of dy it is the concave
// quadratic a2 dy^2 + a1 dy + a0, and outside its roots widened by 1e-3 it is
// below a2 1e-6 < 0, far beyond its rounding.  The counts therefore equal the
// per-sample definition's bit for bit; a row costs a root and a few integer
// operations instead of one test per sample.  A work item is one z-sample
// plane of one cell row: with NS (compile-time samples per direction) its NS
// sample rows are summed per cell before one LDS add per cell, else each row
// adds its own.  The counts accumulate in LDS (z-slabs of the box that fit)
// and go to the particle's count box in global memory, one 16-bit count per
// cell, x fastest.
template <int NS>
__global__ __launch_bounds__(VOX_T) void k_vox_rows(VoxArgs A) {
    __shared__ VoxPart P;
    __shared__ double off[32];
    __shared__ int cnt_s[VOX_BOX_LDS];
    const int k = blockIdx.x;
    if (k >= A.p.np) return;
    const int tid = threadIdx.x;
    if (tid < A.ns) off[tid] = (double)(2 * tid + 1) / (double)(2 * A.ns);
    if (tid == 0) P = ((const VoxPart*)A.vpart)[k];
    __syncthreads();
    const int ns = NS > 0 ? NS : A.ns;
    const int bx = P.hi[0] - P.lo[0] + 1, by_ = P.hi[1] - P.lo[1] + 1, bz_ = P.hi[2] - P.lo[2] + 1;
    if (bx <= 0 || by_ <= 0 || bz_ <= 0) return;  // a blown-up particle: no box
    unsigned short* box = A.vbox + (long long)k * A.box_stride;
    RowQ q;
    double amax;
    if (P.shape == 0) {
        const double i2 = 1.0 / (P.ax[0] * P.ax[0]);
        q.A = i2; q.by = 0.0; q.bz = 0.0; q.cyy = i2; q.cyz = 0.0; q.czz = i2;
        amax = P.ax[0];
    } else {
        q.A = q.by = q.bz = q.cyy = q.cyz = q.czz = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double r0 = P.R[d], r1 = P.R[3 + d], r2 = P.R[6 + d], iv = P.inv[d];
            q.A += iv * r0 * r0;
            q.by += iv * r0 * r1;
            q.bz += iv * r0 * r2;
            q.cyy += iv * r1 * r1;
            q.cyz += iv * r1 * r2;
            q.czz += iv * r2 * r2;
        }
        amax = fmax(P.ax[0], fmax(P.ax[1], P.ax[2]));
    }
    q.iA = 1.0 / q.A;
    q.fns = (double)ns;
    q.mt = 1e-5 * (1.0 + amax) * q.fns;
    q.a2 = q.by * q.by - q.A * q.cyy;
    q.i2a2 = 1.0 / (2.0 * q.a2);  // a2 < 0: the shape matrix is positive definite
    q.xl = (double)P.lo[0] - P.c[0];
    q.gmax = (double)(bx * ns - 1);
    const double my = 1e-3;
    const int plane_cells = bx * by_;
    const int pz = VOX_BOX_LDS / plane_cells;  // z-planes per slab (the box's x-y plane fits: checked at creation)
    for (int z0 = 0; z0 < bz_; z0 += pz) {
        const int nzs = bz_ - z0 < pz ? bz_ - z0 : pz;
        for (int c = tid; c < nzs * plane_cells; c += VOX_T) cnt_s[c] = 0;
        __syncthreads();
        const int items = nzs * ns * by_;
        for (int it = tid; it < items; it += VOX_T) {
            const int Yr = it % by_, cz = (it / by_) % ns, Zr = it / (by_ * ns);
            const int Z = P.lo[2] + z0 + Zr, Y = P.lo[1] + Yr;
            const double dz = ((double)Z + off[cz]) - P.c[2];
            double bzz, czzz, cyzz, ylo, yhi;
            bool miss;
            {
#pragma clang fp contract(fast)
                bzz = q.bz * dz;
                czzz = q.czz * dz * dz;
                cyzz = 2.0 * q.cyz * dz;
                const double a1 = 2.0 * q.by * bzz - q.A * cyzz;
                const double a0 = bzz * bzz - q.A * (czzz - 1.0);
                const double D = a1 * a1 - 4.0 * q.a2 * a0;
                miss = D < -(1e-9 * (a1 * a1 + 4.0 * fabs(q.a2 * a0)) + 1e-12);
                const double sD = D > 0.0 ? sqrt_est(D) : 0.0;
                const double y1 = (-a1 + sD) * q.i2a2, y2 = (-a1 - sD) * q.i2a2;  // widened by my below
                ylo = fmin(y1, y2) - my;
                yhi = fmax(y1, y2) + my;
            }
            if (miss) continue;  // the plane misses it
            int* row = cnt_s + plane_cells * Zr + bx * Yr;
            if (NS > 0) {
                int glo[NS > 0 ? NS : 1], ghi[NS > 0 ? NS : 1];
                int i0 = 1 << 30, i1 = -1;
#pragma unroll
                for (int b = 0; b < NS; ++b) {
                    glo[b] = 1;
                    ghi[b] = 0;
                    const double dy = ((double)Y + off[b]) - P.c[1];
                    if (dy < ylo || dy > yhi) continue;
                    row_inside(P, q, off, NS, dy, dz, bzz, cyzz, czzz, row, glo[b], ghi[b]);
                    if (glo[b] <= ghi[b]) {
                        i0 = min(i0, glo[b] / NS);
                        i1 = max(i1, ghi[b] / NS);
                    }
                }
                // the per-cell sum over the rows on packed 16-bit lanes (two rows
                // per operation; sample indices stay below 2^15)
                typedef short s2_t __attribute__((ext_vector_type(2)));
                s2_t lo2[NS > 1 ? NS / 2 : 1], hi2[NS > 1 ? NS / 2 : 1];
#pragma unroll
                for (int b = 0; b < NS / 2; ++b) {
                    lo2[b] = s2_t{(short)glo[2 * b], (short)glo[2 * b + 1]};
                    hi2[b] = s2_t{(short)ghi[2 * b], (short)ghi[2 * b + 1]};
                }
                for (int i = i0; i <= i1; ++i) {
                    const short a0 = (short)(i * NS), a1 = (short)(i * NS + NS - 1);
                    const s2_t va0 = s2_t{a0, a0}, va1 = s2_t{a1, a1}, one = s2_t{1, 1}, zero = s2_t{0, 0};
                    s2_t acc = zero;
#pragma unroll
                    for (int b = 0; b < NS / 2; ++b) {
                        const s2_t m = __builtin_elementwise_min(hi2[b], va1) - __builtin_elementwise_max(lo2[b], va0) + one;
                        acc += __builtin_elementwise_max(m, zero);
                    }
                    int n = (int)acc.x + (int)acc.y;
#pragma unroll
                    for (int b = 2 * (NS / 2); b < NS; ++b) n += range_in_cell(glo[b], ghi[b], i, NS);
                    if (n) atomicAdd(&row[i], n);
                }
            } else {
                for (int b = 0; b < ns; ++b) {
                    const double dy = ((double)Y + off[b]) - P.c[1];
                    if (dy < ylo || dy > yhi) continue;
                    int glo, ghi;
                    row_inside(P, q, off, ns, dy, dz, bzz, cyzz, czzz, row, glo, ghi);
                    for (int i = glo / ns; glo <= ghi && i <= ghi / ns; ++i) atomicAdd(&row[i], range_in_cell(glo, ghi, i, ns));
                }
            }
        }
        __syncthreads();
        for (int c = tid; c < nzs * plane_cells; c += VOX_T)
            box[(long long)z0 * plane_cells + c] = (unsigned short)cnt_s[c];
        __syncthreads();
    }
}

// B of a solid fraction beta (Sec. 2.3): beta (tau - 1/2) / ((1 - beta) + (tau - 1/2)), tm = tau - 1/2
template <typename C>
__device__ inline C sel_B(double beta, double tm) {
    return (C)(beta * tm / ((1.0 - beta) + tm));
}

// the tables of B and beta per inside-sample count n = 0 .. n3
template <typename C>
__global__ void k_fill_tables(C* btab, double* betatab, int n3, double tau) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n > n3) return;
    const double beta = (double)n / (double)n3;
    btab[n] = sel_B<C>(beta, tau - 0.5);
    betatab[n] = beta;
}

// Phase C of the subdivision method from the count boxes, on integer keys:
// an entry of candidate u with count n > 0 is the key n * 256 + (255 - u), so
// that a larger key is a larger beta = n / ns^3 (the division is monotone and
// one-to-one on the counts) and, for equal counts, the smaller local index
// (the smaller pid).  Each of the lane's four planes keeps its four largest
// keys in a sorted list updated by max/min exchanges, which equals keeping
// the largest ms betas with ties to the smaller pid (the first ms of the list);
// every entry past the ms-th is counted as dropped.  beta and B are formed
// only for the kept slots.
template <typename C>
__device__ inline void select_counts(const VoxArgs& A, const SelPart* sp, long long t, int tz, int x, int y,
                                     bool xy_ok, unsigned long long cm0, unsigned long long cm1,
                                     const unsigned short* vbox, long long stride, unsigned long long* cnt_e,
                                     unsigned long long* cnt_d) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int ms = A.ms;
    unsigned key[PSM_TZ][4];
    int ne[PSM_TZ];
#pragma unroll
    for (int lz = 0; lz < PSM_TZ; ++lz) {
        ne[lz] = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) key[lz][q] = 0u;
    }
    if (xy_ok)
        for (int w = 0; w < 2; ++w)
            for (unsigned long long bits = w ? cm1 : cm0; bits; bits &= bits - 1) {
                const int u = 64 * w + __ffsll((long long)bits) - 1;
                const SelPart& P = sp[u];
                int X, Y;
                in_box(P, x, A.g.nx, 0, A.g.periodic[0], &X);
                in_box(P, y, A.g.ny, 1, A.g.periodic[1], &Y);
                const int bx = P.hi[0] - P.lo[0] + 1, by = P.hi[1] - P.lo[1] + 1;
                const unsigned short* col = vbox + (long long)P.pid * stride + (X - P.lo[0]) + bx * (Y - P.lo[1]);
                unsigned n[PSM_TZ];
#pragma unroll
                for (int lz = 0; lz < PSM_TZ; ++lz) {
                    const int z = tz * PSM_TZ + lz;
                    int Z;
                    n[lz] = 0u;
                    if (z < A.g.nz && in_box(P, z, A.g.nz, 2, A.g.periodic[2], &Z))
                        n[lz] = col[bx * by * (Z - P.lo[2])];
                }
#pragma unroll
                for (int lz = 0; lz < PSM_TZ; ++lz)
                    if (n[lz]) {
                        ++ne[lz];
                        unsigned v = (n[lz] << 8) | (unsigned)(255 - u);
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const unsigned hi = max(key[lz][q], v);
                            v = min(key[lz][q], v);
                            key[lz][q] = hi;
                        }
                    }
            }
    unsigned long long my_e = 0, my_d = 0;
    C* Bout = (C*)A.t.slot_B;
    const long long plane = A.g.ntiles * (long long)PSM_TILE;
    const double n3 = (double)(A.ns * A.ns * A.ns), tm = A.tau - 0.5;
#pragma unroll
    for (int lz = 0; lz < PSM_TZ; ++lz) {
        if (!xy_ok || tz * PSM_TZ + lz >= A.g.nz) continue;
        const int nk = ne[lz] < ms ? ne[lz] : ms;
        my_e += (unsigned long long)ne[lz];
        my_d += (unsigned long long)(ne[lz] - nk);
        // the kept keys reordered by local index: (u << 16) | count, empty last
        unsigned o[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            o[q] = q < nk ? ((255u - (key[lz][q] & 255u)) << 16) | (key[lz][q] >> 8) : 0xffffffffu;
#define PSM_CX(a, b) { const unsigned lo_ = min(o[a], o[b]), hi_ = max(o[a], o[b]); o[a] = lo_; o[b] = hi_; }
        PSM_CX(0, 1) PSM_CX(2, 3) PSM_CX(0, 2) PSM_CX(1, 3) PSM_CX(1, 2)
#undef PSM_CX
        const long long cell = t * (long long)PSM_TILE + lane + PSM_TX * (wid + PSM_TY * lz);
        unsigned lp = 0xffffffffu;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q < nk) lp = (lp & ~(0xffu << (8 * q))) | ((o[q] >> 16) << (8 * q));
        if (A.stream) __builtin_nontemporal_store(lp, &A.t.slot_lp[cell]);  // the LBM pass reads each once
        else A.t.slot_lp[cell] = lp;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q < nk) {
                const unsigned n = o[q] & 0xffffu;
                if (A.btab) {
                    if (A.stream) __builtin_nontemporal_store(((const C*)A.btab)[n], &Bout[q * plane + cell]);
                    else Bout[q * plane + cell] = ((const C*)A.btab)[n];
                    if (A.t.slot_beta) A.t.slot_beta[q * plane + cell] = A.betatab[n];
                } else {
                    const double beta = (double)n / n3;
                    Bout[q * plane + cell] = sel_B<C>(beta, tm);
                    if (A.t.slot_beta) A.t.slot_beta[q * plane + cell] = beta;
                }
            }
    }
    add_entry_counts(A, t, my_e, my_d, cnt_e, cnt_d);
}

// per tile: select the kept solids, the subdivision counts from the count boxes
template <typename C, bool SORT, bool SUB>
__global__ __launch_bounds__(VOX_T) void k_vox_select(VoxArgs A) {
    __shared__ SelPart sp[PSM_PMAX];
    __shared__ double off[32];
    __shared__ unsigned long long ks[SORT ? VOX_T : 1];
    __shared__ unsigned long long cnt_e, cnt_d;
    const long long t = blockIdx.x;
    if (t >= A.g.ntiles) return;
    const unsigned long long* keys = SORT ? sort_tile_list(A, t, ks) : nullptr;
    const TileRange R = tile_range(A, t);
    if (R.count <= 0) {
        if (threadIdx.x == 0 && A.t.tile_ed) A.t.tile_ed[2 * t] = A.t.tile_ed[2 * t + 1] = 0u;
        return;
    }
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) { cnt_e = 0; cnt_d = 0; }
    if (tid < A.ns) off[tid] = (double)(2 * tid + 1) / (double)(2 * A.ns);
    for (int u = tid; u < R.count; u += VOX_T) {
        int k = (int)((keys ? keys[u] : A.t.tile_list[R.s0 + u]) >> 32);
        if (k >= A.p.np) k = 0;
        sel_of(((const VoxPart*)A.vpart)[k], sp[u]);
    }
    __syncthreads();
    const double slo = off[0], shi = off[A.ns - 1];  // first and last sample offset
    const int x = R.tx * PSM_TX + lane, y = R.ty * PSM_TY + wid;
    const bool xy_ok = x < A.g.nx && y < A.g.ny;
    unsigned long long cm0, cm1;
    column_masks(A, sp, R.count, x, y, xy_ok, cm0, cm1);
    const unsigned short* vbox = A.vbox;
    const long long stride = A.box_stride;
    if constexpr (SUB) {
        select_counts<C>(A, sp, t, R.tz, x, y, xy_ok, cm0, cm1, vbox, stride, &cnt_e, &cnt_d);
        return;
    }
    select_slots<C, true, SelPart>(A, sp, t, R.tz, x, y, xy_ok, cm0, cm1, slo, shi, 0,
                          [&](const SelPart& P, int X, int Y, int Z) {
                              const int bx = P.hi[0] - P.lo[0] + 1, by = P.hi[1] - P.lo[1] + 1;
                              return (int)vbox[(long long)P.pid * stride + (X - P.lo[0]) +
                                               (long long)bx * ((Y - P.lo[1]) + (long long)by * (Z - P.lo[2]))];
                          },
                          &cnt_e, &cnt_d);
}

// consecutive blocks of the map stay on one XCD
__device__ inline long long xcd_block(long long nblocks) {
    const long long per = (nblocks + 7) / 8;
    return (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

// many domains in one launch: map[b] = (job, tile)
template <typename C>
__global__ __launch_bounds__(VOX_T) void k_voxelize_batch(const VoxArgs* __restrict__ jobs,
                                                          const int2* __restrict__ map, long long nmap) {
    const long long b = xcd_block(nmap);
    if (b >= nmap) return;
    const int2 m = map[b];
    voxelize_tile<C>(jobs[m.x], m.y);
}

// one wave per particle
__global__ __launch_bounds__(256) void k_reduce_hydro(VoxArgs A) {
    __shared__ double buf[4][64 * 6];
    const int k = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (k >= A.p.np) return;
    psm_reduce_hydro_wave(A.t, A.p, k, threadIdx.x & 63, buf[threadIdx.x >> 6]);
}

inline unsigned nblk(long long n, int t = 256) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }

}  // namespace

// the tile counters start at zero (creation) and are cleared again where the lists are ordered
hipError_t vox_register(const VoxArgs& A, int* scan_tmp, hipStream_t s) {
    hipError_t e;
    if (A.p.np > 0 && A.vpart) k_vox_parts<<<nblk(A.p.np), 256, 0, s>>>(A);
    const unsigned nbw = nblk((long long)VOX_REG_G * (A.p.np > 0 ? A.p.np : 1));
    k_vox_count<<<nbw, 256, 0, s>>>(A);
    if ((e = psm_scan2(A.t.vcount, A.t.voff, A.p.np, A.tile_count, A.t.tile_start, A.g.ntiles, scan_tmp, s)) !=
        hipSuccess)
        return e;
    if (A.p.np > 0) k_vox_scatter<<<nbw, 256, 0, s>>>(A);
    // small lattices: each tile's list is ordered by the first per-tile kernel
    // of vox_voxelize
    if (A.g.ntiles > VOX_SORT_IN_TILE_MAX) k_tile_sort<<<nblk(A.g.ntiles), 256, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t vox_voxelize(const VoxArgs& A, int ctype_double, hipStream_t s) {
    if (A.sf_method == 0 && A.p.np > 0) {
        if (A.ns == 10) k_vox_rows<10><<<(unsigned)A.p.np, VOX_T, 0, s>>>(A);
        else k_vox_rows<0><<<(unsigned)A.p.np, VOX_T, 0, s>>>(A);
    }
    return vox_select(A, ctype_double, s);
}

hipError_t vox_select(const VoxArgs& A, int ctype_double, hipStream_t s) {
    const unsigned nt = (unsigned)A.g.ntiles;
    const bool sort = A.g.ntiles <= VOX_SORT_IN_TILE_MAX;
    // (small lattices: the select kernel orders each tile's list)
    const bool sub = A.sf_method == 0;
    if (ctype_double) {
        if (sort) {
            if (sub) k_vox_select<double, true, true><<<nt, VOX_T, 0, s>>>(A);
            else k_vox_select<double, true, false><<<nt, VOX_T, 0, s>>>(A);
        } else {
            if (sub) k_vox_select<double, false, true><<<nt, VOX_T, 0, s>>>(A);
            else k_vox_select<double, false, false><<<nt, VOX_T, 0, s>>>(A);
        }
    } else {
        if (sort) {
            if (sub) k_vox_select<float, true, true><<<nt, VOX_T, 0, s>>>(A);
            else k_vox_select<float, true, false><<<nt, VOX_T, 0, s>>>(A);
        } else {
            if (sub) k_vox_select<float, false, true><<<nt, VOX_T, 0, s>>>(A);
            else k_vox_select<float, false, false><<<nt, VOX_T, 0, s>>>(A);
        }
    }
    return hipGetLastError();
}
hipError_t vox_register_batch(const VoxArgs* jobs, int njobs, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    k_vox_register_batch<<<(unsigned)njobs, VOX_RT, 0, s>>>(jobs);
    return hipGetLastError();
}

hipError_t vox_voxelize_batch(const VoxArgs* jobs, const int2* map, long long nmap, int ctype_double,
                              hipStream_t s) {
    if (nmap <= 0) return hipSuccess;
    const unsigned nb = (unsigned)(8 * ((nmap + 7) / 8));
    if (ctype_double) k_voxelize_batch<double><<<nb, VOX_T, 0, s>>>(jobs, map, nmap);
    else k_voxelize_batch<float><<<nb, VOX_T, 0, s>>>(jobs, map, nmap);
    return hipGetLastError();
}

hipError_t vox_reduce_hydro(const VoxArgs& A, hipStream_t s) {
    if (A.p.np == 0) return hipSuccess;
    k_reduce_hydro<<<nblk(64LL * A.p.np), 256, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t vox_fill_tables(void* btab, double* betatab, int ns, double tau, int ctype_double, hipStream_t s) {
    const int n3 = ns * ns * ns;
    const unsigned nb = (unsigned)((n3 + 1 + 255) / 256);
    if (ctype_double) k_fill_tables<double><<<nb, 256, 0, s>>>((double*)btab, betatab, n3, tau);
    else k_fill_tables<float><<<nb, 256, 0, s>>>((float*)btab, betatab, n3, tau);
    return hipGetLastError();
}

size_t vox_part_bytes() { return sizeof(VoxPart); }
size_t vox_box_cells_max() { return VOX_BOX_LDS; }

