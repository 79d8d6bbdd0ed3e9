// voxel.hip -- solid fractions of spheres and ellipsoids on lattice tiles
// (Sec. 2.4: subdivision and distance-based methods; Sec. 3.2.3: at most k
// solids per fluid cell) and the per-particle hydrodynamic reduction.
// Compiled with -ffp-contract=off: the subdivision sample test decides an
// integer count and is evaluated with separately rounded operations.
//
// Pipeline per coupled step:
//   k_vox_count    tiles touched by each particle's lattice box (count + tile histogram)
//   (scans)        emission offsets per particle, list offsets per tile
//   k_vox_scatter  counting-sort scatter of (pid, emission index) into tiles
//   k_tile_sort    order each tile's list by pid; inverse map emission -> position
//   k_voxelize     one workgroup per tile: beta of every (cell, particle), keep the
//                  max_solids largest (ties to the smaller pid), B_k, slots
//   k_reduce_hydro per particle: minus the sum of its tile partials (F, M)
#include <math.h>

#include "common.h"
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

// lattice box of particle k: unwrapped lo..hi per axis, clamped on walled axes
__device__ inline void lattice_box(const VoxArgs& A, int k, int lo[3], int hi[3]) {
    double e[3];
    half_extents(A, k, e);
    const int n[3] = {A.g.nx, A.g.ny, A.g.nz};
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
}

// distinct tile indices along one axis for the wrapped cell range lo..hi
__device__ inline int axis_tiles(int lo, int hi, int n, int T, int periodic, int* out) {
    int cnt = 0;
    int seg[2][2];
    int ns = 0;
    if (hi < lo) return 0;
    if (!periodic) {
        seg[ns][0] = lo; seg[ns][1] = hi; ++ns;
    } else if (lo < 0) {
        seg[ns][0] = lo + n; seg[ns][1] = n - 1; ++ns;
        seg[ns][0] = 0; seg[ns][1] = hi; ++ns;
    } else if (hi >= n) {
        seg[ns][0] = lo; seg[ns][1] = n - 1; ++ns;
        seg[ns][0] = 0; seg[ns][1] = hi - n; ++ns;
    } else {
        seg[ns][0] = lo; seg[ns][1] = hi; ++ns;
    }
    for (int s = 0; s < ns; ++s)
        for (int t = seg[s][0] / T; t <= seg[s][1] / T && cnt < VOX_AXIS_MAX; ++t) {
            bool dup = false;
            for (int u = 0; u < cnt; ++u) dup |= out[u] == t;
            if (!dup) out[cnt++] = t;
        }
    for (int u = 1; u < cnt; ++u)
        for (int v = u; v > 0 && out[v] < out[v - 1]; --v) {
            int t = out[v]; out[v] = out[v - 1]; out[v - 1] = t;
        }
    return cnt;
}

struct TileSet {
    int tx[VOX_AXIS_MAX], ty[VOX_AXIS_MAX], tz[VOX_AXIS_MAX];
    int nx, ny, nz;
};

__device__ inline void particle_tiles(const VoxArgs& A, int k, TileSet& S) {
    int lo[3], hi[3];
    lattice_box(A, k, lo, hi);
    S.nx = axis_tiles(lo[0], hi[0], A.g.nx, PSM_TX, A.g.periodic[0], S.tx);
    S.ny = axis_tiles(lo[1], hi[1], A.g.ny, PSM_TY, A.g.periodic[1], S.ty);
    S.nz = axis_tiles(lo[2], hi[2], A.g.nz, PSM_TZ, A.g.periodic[2], S.tz);
}

__global__ void k_vox_count(VoxArgs A) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.p.np) return;
    TileSet S;
    particle_tiles(A, k, S);
    A.t.vcount[k] = S.nx * S.ny * S.nz;
    for (int c = 0; c < S.nz; ++c)
        for (int b = 0; b < S.ny; ++b)
            for (int a = 0; a < S.nx; ++a) {
                long long t = S.tx[a] + (long long)A.g.ntx * (S.ty[b] + (long long)A.g.nty * S.tz[c]);
                atomicAdd(&A.tile_count[t], 1);
            }
}

__global__ void k_vox_scatter(VoxArgs A) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.p.np) return;
    TileSet S;
    particle_tiles(A, k, S);
    int e = A.t.voff[k];
    bool full = false;
    for (int c = 0; c < S.nz; ++c)
        for (int b = 0; b < S.ny; ++b)
            for (int a = 0; a < S.nx; ++a) {
                long long t = S.tx[a] + (long long)A.g.ntx * (S.ty[b] + (long long)A.g.nty * S.tz[c]);
                int slot = atomicAdd(&A.tile_fill[t], 1);
                long long at = (long long)A.t.tile_start[t] + slot;
                if (at < A.t.cap && e < A.t.cap)
                    A.t.tile_list[at] = ((unsigned long long)k << 32) | (unsigned)e;
                else
                    full = true;
                ++e;
            }
    if (full) atomicOr(&A.ctr->flags, (unsigned long long)PSM_FLAG_VREG);
}

__global__ void k_tile_sort(VoxArgs A) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= A.g.ntiles) return;
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

// per-particle data staged in LDS for a tile
struct VoxPart {
    double c[3];
    double ax[3];
    double R[9];
    double inv[3];
    double e[3];
    int lo[3], hi[3];
    int shape;
    int pid;
};

__device__ inline bool in_box(const VoxPart& P, int x, int n, int axis, int periodic, int* X) {
    int lo = P.lo[axis], hi = P.hi[axis];
    int v;
    if (periodic) {
        int d = x - lo;
        d %= n;
        if (d < 0) d += n;
        v = lo + d;
    } else {
        v = x;
    }
    *X = v;
    return v >= lo && v <= hi;
}

__device__ double beta_sphere(const VoxPart& P, int X, int Y, int Z, int ns, int method, double Rc) {
    const double R = P.ax[0];
    if (method == 1) {
        double dx = ((double)X + 0.5) - P.c[0], dy = ((double)Y + 0.5) - P.c[1], dz = ((double)Z + 0.5) - P.c[2];
        double dist = sqrt((dx * dx + dy * dy) + dz * dz);
        double delta = (R + Rc) - dist;
        if (delta < 0.0) return 0.0;
        if (delta > 2.0 * Rc) return 1.0;
        return delta / (2.0 * Rc);
    }
    const double R2 = R * R;
    // exact shortcuts: the cell box strictly inside / outside the sphere with a
    // margin far above the rounding of any sample's squared distance
    const int Xc[3] = {X, Y, Z};
    double maxr2 = 0.0, minr2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double dl = (double)Xc[a] - P.c[a];
        double dh = ((double)Xc[a] + 1.0) - P.c[a];
        double l2 = dl * dl, h2 = dh * dh;
        maxr2 += l2 > h2 ? l2 : h2;
        minr2 += dl > 0.0 ? l2 : (dh < 0.0 ? h2 : 0.0);
    }
    const double m = 1e-8 * (1.0 + R2);
    const int n3 = ns * ns * ns;
    if (maxr2 < R2 - m) return 1.0;
    if (minr2 > R2 + m) return 0.0;
    int cnt = 0;
    const double inv2ns = 1.0 / (double)(2 * ns);
    (void)inv2ns;
    for (int c = 0; c < ns; ++c) {
        double oz = (double)(2 * c + 1) / (double)(2 * ns);
        double dz = ((double)Z + oz) - P.c[2];
        double dz2 = dz * dz;
        for (int b = 0; b < ns; ++b) {
            double oy = (double)(2 * b + 1) / (double)(2 * ns);
            double dy = ((double)Y + oy) - P.c[1];
            double dy2 = dy * dy;
            for (int a = 0; a < ns; ++a) {
                double ox = (double)(2 * a + 1) / (double)(2 * ns);
                double dx = ((double)X + ox) - P.c[0];
                double r2 = (dx * dx + dy2) + dz2;
                cnt += (r2 < R2) ? 1 : 0;
            }
        }
    }
    return (double)cnt / (double)n3;
}

__device__ inline double ell_q(const VoxPart& P, double dx, double dy, double dz) {
    double p0 = (P.R[0] * dx + P.R[3] * dy) + P.R[6] * dz;
    double p1 = (P.R[1] * dx + P.R[4] * dy) + P.R[7] * dz;
    double p2 = (P.R[2] * dx + P.R[5] * dy) + P.R[8] * dz;
    return ((p0 * p0) * P.inv[0] + (p1 * p1) * P.inv[1]) + (p2 * p2) * P.inv[2];
}

__device__ double beta_ellipsoid(const VoxPart& P, int X, int Y, int Z, int ns) {
    const int Xc[3] = {X, Y, Z};
    double minr2 = 0.0;
    double amax = P.ax[0] > P.ax[1] ? P.ax[0] : P.ax[1];
    amax = amax > P.ax[2] ? amax : P.ax[2];
    for (int a = 0; a < 3; ++a) {
        double dl = (double)Xc[a] - P.c[a];
        double dh = ((double)Xc[a] + 1.0) - P.c[a];
        minr2 += dl > 0.0 ? dl * dl : (dh < 0.0 ? dh * dh : 0.0);
        // outside the ellipsoid's axis-aligned box by a margin
        if (dh < -P.e[a] - 1e-6 || dl > P.e[a] + 1e-6) return 0.0;
    }
    double rb = amax + 1e-6;
    if (minr2 > rb * rb) return 0.0;
    bool all_in = true;
    for (int corner = 0; corner < 8 && all_in; ++corner) {
        double dx = ((double)X + (double)(corner & 1)) - P.c[0];
        double dy = ((double)Y + (double)((corner >> 1) & 1)) - P.c[1];
        double dz = ((double)Z + (double)((corner >> 2) & 1)) - P.c[2];
        all_in = ell_q(P, dx, dy, dz) < 1.0 - 1e-9;
    }
    if (all_in) return 1.0;
    int cnt = 0;
    for (int c = 0; c < ns; ++c) {
        double dz = ((double)Z + (double)(2 * c + 1) / (double)(2 * ns)) - P.c[2];
        for (int b = 0; b < ns; ++b) {
            double dy = ((double)Y + (double)(2 * b + 1) / (double)(2 * ns)) - P.c[1];
            for (int a = 0; a < ns; ++a) {
                double dx = ((double)X + (double)(2 * a + 1) / (double)(2 * ns)) - P.c[0];
                cnt += (ell_q(P, dx, dy, dz) < 1.0) ? 1 : 0;
            }
        }
    }
    return (double)cnt / (double)(ns * ns * ns);
}

template <typename C>
__global__ __launch_bounds__(256) void k_voxelize(VoxArgs A) {
    __shared__ VoxPart sp[PSM_PMAX];
    __shared__ unsigned long long cnt_e, cnt_d;
    const long long t = blockIdx.x;
    if (t >= A.g.ntiles) return;
    long long s0 = A.t.tile_start[t], s1 = A.t.tile_start[t + 1];
    if (s1 > A.t.cap) s1 = A.t.cap;
    const int count = (int)(s1 - s0) < PSM_PMAX ? (int)(s1 - s0) : PSM_PMAX;
    const int tid = threadIdx.x;
    const int tx = (int)(t % A.g.ntx), ty = (int)((t / A.g.ntx) % A.g.nty), tz = (int)(t / ((long long)A.g.ntx * A.g.nty));
    const long long base = t * (long long)PSM_TILE;
    const int ms = A.ms;
    C* Bout = (C*)A.t.slot_B;
    const long long plane = A.g.ntiles * (long long)PSM_TILE;
    if (count <= 0) return;
    if (tid == 0) { cnt_e = 0; cnt_d = 0; }
    for (int u = tid; u < count; u += blockDim.x) {
        int k = (int)(A.t.tile_list[s0 + u] >> 32);
        if (k >= A.p.np) k = 0;
        VoxPart& P = sp[u];
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
    }
    __syncthreads();
    const int lx = tid & (PSM_TX - 1), ly = tid / PSM_TX;
    const int x = tx * PSM_TX + lx, y = ty * PSM_TY + ly;
    unsigned long long my_e = 0, my_d = 0;
    for (int lz = 0; lz < PSM_TZ; ++lz) {
        const int z = tz * PSM_TZ + lz;
        const long long l = lx + PSM_TX * (ly + PSM_TY * lz);
        double bb[PSM_SLOTS_MAX];
        int bl[PSM_SLOTS_MAX];
        int nk = 0;
        if (x < A.g.nx && y < A.g.ny && z < A.g.nz) {
            for (int u = 0; u < count; ++u) {
                const VoxPart& P = sp[u];
                int X, Y, Z;
                if (!in_box(P, x, A.g.nx, 0, A.g.periodic[0], &X)) continue;
                if (!in_box(P, y, A.g.ny, 1, A.g.periodic[1], &Y)) continue;
                if (!in_box(P, z, A.g.nz, 2, A.g.periodic[2], &Z)) continue;
                double beta = (P.shape == 0) ? beta_sphere(P, X, Y, Z, A.ns, A.sf_method, A.Rc)
                                             : beta_ellipsoid(P, X, Y, Z, A.ns);
                if (!(beta > 0.0)) continue;
                ++my_e;
                // keep the ms largest, ties to the earlier (smaller) pid
                if (nk < ms) {
                    int q = nk++;
                    while (q > 0 && bb[q - 1] < beta) { bb[q] = bb[q - 1]; bl[q] = bl[q - 1]; --q; }
                    bb[q] = beta; bl[q] = u;
                } else if (beta > bb[ms - 1]) {
                    ++my_d;
                    int q = ms - 1;
                    while (q > 0 && bb[q - 1] < beta) { bb[q] = bb[q - 1]; bl[q] = bl[q - 1]; --q; }
                    bb[q] = beta; bl[q] = u;
                } else {
                    ++my_d;
                }
            }
        }
        // kept slots ordered by pid (local index order is pid order)
        for (int u = 1; u < nk; ++u)
            for (int v = u; v > 0 && bl[v] < bl[v - 1]; --v) {
                int ti = bl[v]; bl[v] = bl[v - 1]; bl[v - 1] = ti;
                double tb = bb[v]; bb[v] = bb[v - 1]; bb[v - 1] = tb;
            }
        unsigned int lp = 0xffffffffu;
        for (int k = 0; k < nk; ++k) lp = (lp & ~(0xffu << (8 * k))) | ((unsigned)bl[k] << (8 * k));
        A.t.slot_lp[base + l] = lp;
        for (int k = 0; k < ms; ++k) {
            double beta = k < nk ? bb[k] : 0.0;
            double B = beta * (A.tau - 0.5) / ((1.0 - beta) + (A.tau - 0.5));
            Bout[k * plane + base + l] = (C)B;
            A.t.slot_beta[k * plane + base + l] = beta;
        }
    }
    if (my_e) atomicAdd(&cnt_e, my_e);
    if (my_d) atomicAdd(&cnt_d, my_d);
    __syncthreads();
    if (tid == 0) {
        if (cnt_e) atomicAdd(&A.ctr->entries, cnt_e);
        if (cnt_d) atomicAdd(&A.ctr->dropped, cnt_d);
    }
}

__global__ void k_reduce_hydro(VoxArgs A) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.p.np) return;
    double F[3] = {0.0, 0.0, 0.0}, M[3] = {0.0, 0.0, 0.0};
    int e0 = A.t.voff[k], e1 = A.t.voff[k + 1];
    for (int e = e0; e < e1 && e < A.t.cap; ++e) {
        long long s = A.t.vinv[e];
        if (s < 0 || s >= A.t.cap) continue;
        const double* P = A.t.partial + 6 * s;
        for (int c = 0; c < 3; ++c) {
            F[c] -= P[c];
            M[c] -= P[3 + c];
        }
    }
    for (int c = 0; c < 3; ++c) {
        A.p.fh[3 * k + c] = F[c];
        A.p.mh[3 * k + c] = M[c];
    }
}

inline unsigned nblk(long long n, int t = 256) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }

}  // namespace

hipError_t vox_register(const VoxArgs& A, int* scan_tmp, hipStream_t s) {
    hipError_t e;
    if ((e = psm_fill_int(A.tile_count, 0, A.g.ntiles, s)) != hipSuccess) return e;
    if ((e = psm_fill_int(A.tile_fill, 0, A.g.ntiles, s)) != hipSuccess) return e;
    if (A.p.np > 0) k_vox_count<<<nblk(A.p.np), 256, 0, s>>>(A);
    if ((e = psm_scan(A.t.vcount, A.t.voff, A.p.np, scan_tmp, s)) != hipSuccess) return e;
    if ((e = psm_scan(A.tile_count, A.t.tile_start, A.g.ntiles, scan_tmp, s)) != hipSuccess) return e;
    if (A.p.np > 0) k_vox_scatter<<<nblk(A.p.np), 256, 0, s>>>(A);
    k_tile_sort<<<nblk(A.g.ntiles), 256, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t vox_voxelize(const VoxArgs& A, int ctype_double, hipStream_t s) {
    if (ctype_double) k_voxelize<double><<<(unsigned)A.g.ntiles, 256, 0, s>>>(A);
    else k_voxelize<float><<<(unsigned)A.g.ntiles, 256, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t vox_reduce_hydro(const VoxArgs& A, hipStream_t s) {
    if (A.p.np == 0) return hipSuccess;
    k_reduce_hydro<<<nblk(A.p.np), 256, 0, s>>>(A);
    return hipGetLastError();
}
