// dem.hip -- DEM substep kernels (FP64).  Compiled with -ffp-contract=off so
// that the predicates deciding integer results (cell indices, contact flags)
// use separately rounded operations in a fixed order.
//
// Per substep (Sec. 3.2.1-3.2.2, Table 1):
//   k_predict          Verlet predictor of position and orientation (Eqs. advance-r ...)
//   k_reg_hist         DEM cells of each particle's axis-aligned box -> cell histogram
//   (scan)             cell offsets
//   k_reg_scatter      counting-sort scatter of particle ids into cells
//   k_cell_sort        order each cell's ids (deterministic lists)
//   k_pair_count/emit  per particle i the unique neighbours j > i sharing a cell,
//                      then wall candidates: the sorted unique pair list built per
//                      row, so no global sort or unique pass is needed
//   k_contacts         spring-dashpot + Coulomb per pair, history by binary search
//                      in the previous sorted list
//   k_dem_sum          per particle: second-member pairs (k, i) then first-member
//                      pairs (i, j), a fixed order
//   k_correct          Verlet corrector
#include <math.h>

#include "common.h"
#include "dem.h"

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

__device__ inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
__device__ inline void cross3(const double* a, const double* b, double* c) {
    double c0 = a[1] * b[2] - a[2] * b[1];
    double c1 = a[2] * b[0] - a[0] * b[2];
    double c2 = a[0] * b[1] - a[1] * b[0];
    c[0] = c0;
    c[1] = c1;
    c[2] = c2;
}

__device__ inline void min_image(const DemArgs& A, const double* a, const double* b, double* d) {
    for (int k = 0; k < 3; ++k) {
        double x = a[k] - b[k];
        if (A.g.periodic[k]) {
            double L = A.L[k];
            if (x > 0.5 * L) x -= L;
            else if (x < -0.5 * L) x += L;
        }
        d[k] = x;
    }
}

__device__ inline void half_extents(const DemArgs& A, int k, double e[3]) {
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

// DEM cells touched by particle k's box, sorted ascending; returns the count (<= 8)
__device__ int dem_cells(const DemArgs& A, int k, long long out[8]) {
    double e[3];
    half_extents(A, k, e);
    int list[3][2];
    int nl[3];
    for (int a = 0; a < 3; ++a) {
        double x = A.p.pos[3 * k + a];
        int lo = (int)floor((x - e[a]) / A.h[a]);
        int hi = (int)floor((x + e[a]) / A.h[a]);
        nl[a] = 0;
        for (int c = lo; c <= hi && nl[a] < 2; ++c) {
            int cw = c;
            if (A.g.periodic[a]) cw = ((c % A.nc[a]) + A.nc[a]) % A.nc[a];
            else cw = cw < 0 ? 0 : (cw > A.nc[a] - 1 ? A.nc[a] - 1 : cw);
            bool dup = false;
            for (int u = 0; u < nl[a]; ++u) dup |= (list[a][u] == cw);
            if (!dup) list[a][nl[a]++] = cw;
        }
    }
    int n = 0;
    for (int i = 0; i < nl[0]; ++i)
        for (int j = 0; j < nl[1]; ++j)
            for (int l = 0; l < nl[2]; ++l)
                out[n++] = (long long)list[0][i] +
                           (long long)A.nc[0] * ((long long)list[1][j] + (long long)A.nc[1] * list[2][l]);
    for (int u = 1; u < n; ++u)
        for (int v = u; v > 0 && out[v] < out[v - 1]; --v) {
            long long t = out[v];
            out[v] = out[v - 1];
            out[v - 1] = t;
        }
    return n;
}

__device__ inline double wall_dist(const DemArgs& A, int k, int f) {
    int a = f / 2;
    return (f % 2 == 0) ? A.p.pos[3 * k + a] : A.L[a] - A.p.pos[3 * k + a];
}

// is pid in the (pid-sorted) list of cell c?
__device__ inline bool cell_has(const DemArgs& A, long long c, int pid) {
    int lo = A.cell_start[c], hi = A.cell_start[c + 1];
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (A.cell_pid[mid] < pid) lo = mid + 1;
        else hi = mid;
    }
    return lo < A.cell_start[c + 1] && A.cell_pid[lo] == pid;
}

// unique neighbours of i sharing a cell, j > i (upper) or j < i (lower), ascending.
// Each j is taken from the first cell of i (ascending) that also holds j.
__device__ int neighbours(const DemArgs& A, int i, bool upper, int* nb, bool* overflow) {
    long long ci[8];
    int nci = dem_cells(A, i, ci);
    int n = 0;
    for (int u = 0; u < nci; ++u) {
        int s0 = A.cell_start[ci[u]], s1 = A.cell_start[ci[u] + 1];
        for (int s = s0; s < s1; ++s) {
            int j = A.cell_pid[s];
            if (upper ? (j <= i) : (j >= i)) continue;
            bool seen = false;
            for (int v = 0; v < u && !seen; ++v) seen = cell_has(A, ci[v], j);
            if (seen) continue;
            if (n >= PSM_MAXNB) {
                *overflow = true;
                continue;
            }
            int t = n++;
            while (t > 0 && nb[t - 1] > j) {
                nb[t] = nb[t - 1];
                --t;
            }
            nb[t] = j;
        }
    }
    return n;
}

// ---------------------------------------------------------------------------
// contact geometry (Sec. 2.1): spheres in closed form, ellipsoids by iterated
// equivalent spheres with the local curvature radius (Eq. local-curvature)
// ---------------------------------------------------------------------------
__device__ void ell_local(const double* c, const double* R, const double* ax, const double* p, double* rho,
                          double* n) {
    double d[3] = {p[0] - c[0], p[1] - c[1], p[2] - c[2]};
    double xb[3];
    for (int k = 0; k < 3; ++k) xb[k] = (R[0 + k] * d[0] + R[3 + k] * d[1]) + R[6 + k] * d[2];
    double a = ax[0], b = ax[1], cc = ax[2];
    *rho = b * cc * xb[0] * xb[0] / (a * a * a) + a * cc * xb[1] * xb[1] / (b * b * b) +
           a * b * xb[2] * xb[2] / (cc * cc * cc);
    double nb[3] = {xb[0] / (a * a), xb[1] / (b * b), xb[2] / (cc * cc)};
    double nw[3];
    for (int r = 0; r < 3; ++r) nw[r] = (R[3 * r] * nb[0] + R[3 * r + 1] * nb[1]) + R[3 * r + 2] * nb[2];
    double l = sqrt(dot3(nw, nw));
    for (int r = 0; r < 3; ++r) n[r] = nw[r] / l;
}

__device__ bool ell_line_hit(const double* c, const double* R, const double* ax, const double* s, const double* u,
                             bool far_positive, double* p) {
    double d[3] = {s[0] - c[0], s[1] - c[1], s[2] - c[2]};
    double y0[3], ud[3];
    for (int k = 0; k < 3; ++k) {
        y0[k] = (R[0 + k] * d[0] + R[3 + k] * d[1]) + R[6 + k] * d[2];
        ud[k] = (R[0 + k] * u[0] + R[3 + k] * u[1]) + R[6 + k] * u[2];
    }
    double qa = 0, qb = 0, qc = -1.0;
    for (int k = 0; k < 3; ++k) {
        double ia = 1.0 / (ax[k] * ax[k]);
        qa += ud[k] * ud[k] * ia;
        qb += y0[k] * ud[k] * ia;
        qc += y0[k] * y0[k] * ia;
    }
    double disc = qb * qb - qa * qc;
    if (disc < 0.0 || qa <= 0.0) return false;
    double sq = sqrt(disc);
    double t = far_positive ? (-qb + sq) / qa : (-qb - sq) / qa;
    for (int k = 0; k < 3; ++k) p[k] = s[k] + t * u[k];
    return true;
}

struct Geom {
    double delta, en[3], rci[3], rcj[3], rhoi, rhoj;
    bool sphere_law;
};

__device__ void ellipsoid_pair(const DemArgs& A, int i, int j, Geom& G) {
    const double* ci = A.p.pos + 3 * i;
    double dvec[3];
    min_image(A, ci, A.p.pos + 3 * j, dvec);
    double cj[3] = {ci[0] - dvec[0], ci[1] - dvec[1], ci[2] - dvec[2]};
    double Ri[9], Rj[9];
    quat_rbw(A.p.q + 4 * i, Ri);
    quat_rbw(A.p.q + 4 * j, Rj);
    const double* ai = A.p.semi + 3 * i;
    const double* aj = A.p.semi + 3 * j;
    double amin = ai[0];
    for (int k = 0; k < 3; ++k) {
        amin = ai[k] < amin ? ai[k] : amin;
        amin = aj[k] < amin ? aj[k] : amin;
    }
    double pi[3], pj[3];
    {
        double u[3] = {cj[0] - ci[0], cj[1] - ci[1], cj[2] - ci[2]};
        double l = sqrt(dot3(u, u));
        for (int k = 0; k < 3; ++k) u[k] /= l;
        ell_line_hit(ci, Ri, ai, ci, u, true, pi);
        double um[3] = {-u[0], -u[1], -u[2]};
        ell_line_hit(cj, Rj, aj, cj, um, true, pj);
    }
    for (int it = 0; it < 32; ++it) {
        double rhoi, rhoj, ni[3], nj[3], si[3], sj[3];
        ell_local(ci, Ri, ai, pi, &rhoi, ni);
        ell_local(cj, Rj, aj, pj, &rhoj, nj);
        for (int k = 0; k < 3; ++k) {
            si[k] = pi[k] - rhoi * ni[k];
            sj[k] = pj[k] - rhoj * nj[k];
        }
        double u[3] = {sj[0] - si[0], sj[1] - si[1], sj[2] - si[2]};
        double l = sqrt(dot3(u, u));
        if (!(l > 0.0)) break;
        for (int k = 0; k < 3; ++k) u[k] /= l;
        double npi[3], npj[3];
        if (!ell_line_hit(ci, Ri, ai, si, u, true, npi)) break;
        if (!ell_line_hit(cj, Rj, aj, sj, u, false, npj)) break;
        double dpi[3] = {npi[0] - pi[0], npi[1] - pi[1], npi[2] - pi[2]};
        double dpj[3] = {npj[0] - pj[0], npj[1] - pj[1], npj[2] - pj[2]};
        double conv = sqrt(dot3(dpi, dpi)) + sqrt(dot3(dpj, dpj));
        for (int k = 0; k < 3; ++k) {
            pi[k] = npi[k];
            pj[k] = npj[k];
        }
        if (conv < 1e-10 * amin) break;
    }
    double ni[3], nj[3], si[3], sj[3];
    ell_local(ci, Ri, ai, pi, &G.rhoi, ni);
    ell_local(cj, Rj, aj, pj, &G.rhoj, nj);
    for (int k = 0; k < 3; ++k) {
        si[k] = pi[k] - G.rhoi * ni[k];
        sj[k] = pj[k] - G.rhoj * nj[k];
    }
    double d[3] = {si[0] - sj[0], si[1] - sj[1], si[2] - sj[2]};
    double l = sqrt(dot3(d, d));
    G.delta = (G.rhoi + G.rhoj) - l;
    for (int k = 0; k < 3; ++k) {
        G.en[k] = d[k] / l;
        G.rci[k] = pi[k] - ci[k];
        G.rcj[k] = pj[k] - cj[k];
    }
}

__device__ void pair_geometry(const DemArgs& A, int i, int j, Geom& G) {
    const int np = A.p.np;
    G.sphere_law = false;
    if (j >= np) {
        int f = j - np, a = f / 2;
        double n[3] = {0.0, 0.0, 0.0};
        n[a] = (f % 2 == 0) ? 1.0 : -1.0;
        const double* c = A.p.pos + 3 * i;
        double dist = (f % 2 == 0) ? c[a] : A.L[a] - c[a];
        for (int k = 0; k < 3; ++k) {
            G.en[k] = n[k];
            G.rcj[k] = 0.0;
        }
        G.rhoj = 0.0;
        if (A.p.shape[i] == 0) {
            double R = A.p.semi[3 * i];
            G.delta = R - dist;
            for (int k = 0; k < 3; ++k) G.rci[k] = -R * n[k];
            G.rhoi = R;
            G.sphere_law = true;
        } else {
            double R[9];
            quat_rbw(A.p.q + 4 * i, R);
            const double* ax = A.p.semi + 3 * i;
            double nb[3];
            for (int k = 0; k < 3; ++k) nb[k] = (R[0 + k] * n[0] + R[3 + k] * n[1]) + R[6 + k] * n[2];
            double qf = (ax[0] * ax[0] * nb[0] * nb[0] + ax[1] * ax[1] * nb[1] * nb[1]) + ax[2] * ax[2] * nb[2] * nb[2];
            double sq = sqrt(qf);
            double Anb[3] = {ax[0] * ax[0] * nb[0], ax[1] * ax[1] * nb[1], ax[2] * ax[2] * nb[2]};
            double p[3];
            for (int r = 0; r < 3; ++r) {
                double An = (R[3 * r] * Anb[0] + R[3 * r + 1] * Anb[1]) + R[3 * r + 2] * Anb[2];
                p[r] = c[r] - An / sq;
            }
            G.delta = sq - dist;
            double nn[3];
            ell_local(c, R, ax, p, &G.rhoi, nn);
            for (int k = 0; k < 3; ++k) G.rci[k] = p[k] - c[k];
        }
        return;
    }
    double d[3];
    min_image(A, A.p.pos + 3 * i, A.p.pos + 3 * j, d);
    double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    if (A.p.shape[i] == 0 && A.p.shape[j] == 0) {
        double Ri = A.p.semi[3 * i], Rj = A.p.semi[3 * j];
        double dist = sqrt(r2);
        G.delta = (Ri + Rj) - dist;
        for (int k = 0; k < 3; ++k) {
            G.en[k] = d[k] / dist;
            G.rci[k] = -Ri * G.en[k];
            G.rcj[k] = Rj * G.en[k];
        }
        G.rhoi = Ri;
        G.rhoj = Rj;
        G.sphere_law = true;
        return;
    }
    double rs = A.p.rb[i] + A.p.rb[j];
    if (!(r2 < rs * rs)) {
        G.delta = -1.0;
        return;
    }
    ellipsoid_pair(A, i, j, G);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ void k_reg_hist(DemArgs A) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.p.np) return;
    long long c[8];
    int n = dem_cells(A, k, c);
    for (int u = 0; u < n; ++u) atomicAdd(&A.cell_count[c[u]], 1);
}

__global__ void k_reg_scatter(DemArgs A) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.p.np) return;
    long long c[8];
    int n = dem_cells(A, k, c);
    for (int u = 0; u < n; ++u) {
        int slot = atomicAdd(&A.cell_fill[c[u]], 1);
        long long at = (long long)A.cell_start[c[u]] + slot;
        if (at < A.reg_cap) A.cell_pid[at] = k;
    }
}

__global__ void k_cell_sort(DemArgs A) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= A.ncell) return;
    int s0 = A.cell_start[c], s1 = A.cell_start[c + 1];
    for (int u = s0 + 1; u < s1; ++u)
        for (int v = u; v > s0 && A.cell_pid[v] < A.cell_pid[v - 1]; --v) {
            int t = A.cell_pid[v];
            A.cell_pid[v] = A.cell_pid[v - 1];
            A.cell_pid[v - 1] = t;
        }
}

__global__ void k_pair_count(DemArgs A) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.p.np) return;
    int nb[PSM_MAXNB];
    bool ovf = false;
    int n = neighbours(A, i, true, nb, &ovf);
    for (int f = 0; f < 6; ++f)
        if (A.g.bc[f] != 0 && wall_dist(A, i, f) < A.p.rb[i]) ++n;
    if (ovf) atomicOr(&A.ctr->flags, (unsigned long long)PSM_FLAG_NEIGH);
    A.pcount[i] = n;
}

__global__ void k_pair_emit(DemArgs A) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.p.np) return;
    int nb[PSM_MAXNB];
    bool ovf = false;
    int n = neighbours(A, i, true, nb, &ovf);
    long long at = A.prow[i];
    const long long np = A.p.np;
    bool full = false;
    for (int u = 0; u < n; ++u) {
        if (at < A.pair_cap) A.pairs[at] = ((unsigned long long)i << 32) | (unsigned)nb[u];
        else full = true;
        ++at;
    }
    for (int f = 0; f < 6; ++f)
        if (A.g.bc[f] != 0 && wall_dist(A, i, f) < A.p.rb[i]) {
            if (at < A.pair_cap) A.pairs[at] = ((unsigned long long)i << 32) | (unsigned)(np + f);
            else full = true;
            ++at;
        }
    if (full) atomicOr(&A.ctr->flags, (unsigned long long)PSM_FLAG_PAIRS);
}

__device__ inline long long find_prev(const DemArgs& A, unsigned long long key, long long n) {
    long long lo = 0, hi = n;
    while (lo < hi) {
        long long mid = (lo + hi) >> 1;
        if (A.prev_pairs[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < n && A.prev_pairs[lo] == key) ? lo : -1;
}

// linear spring-dashpot with Coulomb cap and tangential history (Sec. 2.1):
// F_n = [k_n delta + gamma_n (v_j - v_i).e_n] e_n, gamma_n = -2 beta sqrt(k_n m*);
// v_rel = (v_i - v_j) - (rho_i w_i + rho_j w_j) x e_n, v_t its tangential part;
// history projected on the tangent plane then advanced by v_t dt;
// F_t = -k_t d_t - gamma_t v_t capped at mu |F_n| with the history reset.
__global__ void k_contacts(DemArgs A, const double* __restrict__ vv, const double* __restrict__ ww, double dth) {
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long n = A.prow[A.p.np];
    if (n > A.pair_cap) n = A.pair_cap;
    if (s >= n) return;
    long long nprev = A.prev_n ? *A.prev_n : 0;
    if (nprev > A.pair_cap) nprev = A.pair_cap;
    const int np = A.p.np;
    unsigned long long key = A.pairs[s];
    int i = (int)(key >> 32), j = (int)(key & 0xffffffffu);
    Geom G;
    pair_geometry(A, i, j, G);
    double* F = A.cF + 3 * s;
    double* Mi = A.cMi + 3 * s;
    double* Mj = A.cMj + 3 * s;
    double* h = A.hist + 3 * s;
    if (!(G.delta > 0.0)) {
        for (int k = 0; k < 3; ++k) F[k] = Mi[k] = Mj[k] = h[k] = 0.0;
        A.incontact[s] = 0;
        return;
    }
    A.incontact[s] = 1;
    double vi[3], wi[3], vj[3], wj[3], mstar;
    for (int k = 0; k < 3; ++k) {
        vi[k] = vv[3 * i + k];
        wi[k] = ww[3 * i + k];
    }
    if (j < np) {
        for (int k = 0; k < 3; ++k) {
            vj[k] = vv[3 * j + k];
            wj[k] = ww[3 * j + k];
        }
        mstar = A.p.mass[i] * A.p.mass[j] / (A.p.mass[i] + A.p.mass[j]);
    } else {
        int f = j - np;
        for (int k = 0; k < 3; ++k) {
            vj[k] = (A.g.bc[f] == 2) ? A.wall_u[f][k] : 0.0;
            wj[k] = 0.0;
        }
        mstar = A.p.mass[i];
    }
    const double kn = A.kn, kt = A.kt_ratio * kn;
    double gn = -2.0 * A.beta_e * sqrt(kn * mstar);
    double gt = A.gt_ratio * gn;
    double dv[3] = {vj[0] - vi[0], vj[1] - vi[1], vj[2] - vi[2]};
    double fn = kn * G.delta + gn * dot3(dv, G.en);
    double rw[3] = {G.rhoi * wi[0] + G.rhoj * wj[0], G.rhoi * wi[1] + G.rhoj * wj[1], G.rhoi * wi[2] + G.rhoj * wj[2]};
    double cr[3];
    cross3(rw, G.en, cr);
    double vrel[3] = {(vi[0] - vj[0]) - cr[0], (vi[1] - vj[1]) - cr[1], (vi[2] - vj[2]) - cr[2]};
    double vrn = dot3(vrel, G.en);
    double vt[3] = {vrel[0] - vrn * G.en[0], vrel[1] - vrn * G.en[1], vrel[2] - vrn * G.en[2]};
    double ho[3] = {0.0, 0.0, 0.0};
    long long ps = find_prev(A, key, nprev);
    if (ps >= 0)
        for (int k = 0; k < 3; ++k) ho[k] = A.prev_hist[3 * ps + k];
    double hp = dot3(ho, G.en);
    double ht[3];
    for (int k = 0; k < 3; ++k) ht[k] = (ho[k] - hp * G.en[k]) + vt[k] * dth;
    double ft[3];
    for (int k = 0; k < 3; ++k) ft[k] = -kt * ht[k] - gt * vt[k];
    double ftn = sqrt(dot3(ft, ft));
    double cap = A.mu * fabs(fn);
    if (ftn > cap) {
        double sc = cap / ftn;
        for (int k = 0; k < 3; ++k) ft[k] *= sc;
        if (kt > 0.0)
            for (int k = 0; k < 3; ++k) ht[k] = -(ft[k] + gt * vt[k]) / kt;
    }
    for (int k = 0; k < 3; ++k) {
        F[k] = fn * G.en[k] + ft[k];
        h[k] = ht[k];
    }
    if (G.sphere_law) {
        double T[3];
        cross3(G.en, ft, T);
        for (int k = 0; k < 3; ++k) {
            Mi[k] = -G.rhoi * T[k];
            Mj[k] = (j < np) ? -G.rhoj * T[k] : 0.0;
        }
    } else {
        double mF[3] = {-F[0], -F[1], -F[2]};
        cross3(G.rci, F, Mi);
        if (j < np) cross3(G.rcj, mF, Mj);
        else Mj[0] = Mj[1] = Mj[2] = 0.0;
    }
}

__device__ inline long long find_pair(const DemArgs& A, unsigned long long key, long long lo, long long hi) {
    long long end = hi;
    while (lo < hi) {
        long long mid = (lo + hi) >> 1;
        if (A.pairs[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < end && A.pairs[lo] == key) ? lo : -1;
}

__global__ void k_dem_sum(DemArgs A) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.p.np) return;
    double F[3] = {0.0, 0.0, 0.0}, M[3] = {0.0, 0.0, 0.0};
    int nb[PSM_MAXNB];
    bool ovf = false;
    int n = neighbours(A, i, false, nb, &ovf);
    long long cap = A.pair_cap;
    for (int u = 0; u < n; ++u) {
        int k = nb[u];
        long long lo = A.prow[k], hi = A.prow[k + 1];
        if (hi > cap) hi = cap;
        long long s = find_pair(A, ((unsigned long long)k << 32) | (unsigned)i, lo, hi);
        if (s < 0) continue;
        for (int c = 0; c < 3; ++c) {
            F[c] -= A.cF[3 * s + c];
            M[c] += A.cMj[3 * s + c];
        }
    }
    long long s0 = A.prow[i], s1 = A.prow[i + 1];
    if (s1 > cap) s1 = cap;
    for (long long s = s0; s < s1; ++s)
        for (int c = 0; c < 3; ++c) {
            F[c] += A.cF[3 * s + c];
            M[c] += A.cMi[3 * s + c];
        }
    for (int c = 0; c < 3; ++c) {
        A.p.fd[3 * i + c] = F[c];
        A.p.md[3 * i + c] = M[c];
    }
}

// q' = (1/2) [0, w] (x) q
__device__ inline void quat_rate(const double* w, const double* q, double* out) {
    out[0] = 0.5 * (-(w[0] * q[1] + w[1] * q[2] + w[2] * q[3]));
    out[1] = 0.5 * (q[0] * w[0] + (w[1] * q[3] - w[2] * q[2]));
    out[2] = 0.5 * (q[0] * w[1] + (w[2] * q[1] - w[0] * q[3]));
    out[3] = 0.5 * (q[0] * w[2] + (w[0] * q[2] - w[1] * q[1]));
}

// predictor: r += dt v + dt^2/2 a (wrapped), v^p = v + dt a, w^p = w + dt alpha,
// orientation advanced with w(t) by the triad predictor-corrector
__global__ void k_predict(DemArgs A, double dt, int write_kin) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.p.np) return;
    double hdt2 = 0.5 * dt * dt;
    double* x = A.p.pos + 3 * k;
    for (int c = 0; c < 3; ++c) {
        double xn = (x[c] + dt * A.p.v[3 * k + c]) + hdt2 * A.p.a[3 * k + c];
        if (A.g.periodic[c]) {
            double L = A.L[c];
            if (xn >= L) xn -= L;
            else if (xn < 0.0) xn += L;
            if (xn == L) xn = 0.0;
        }
        x[c] = xn;
        A.p.vp[3 * k + c] = A.p.v[3 * k + c] + dt * A.p.a[3 * k + c];
        A.p.wp[3 * k + c] = A.p.w[3 * k + c] + dt * A.p.al[3 * k + c];
    }
    double* q = A.p.q + 4 * k;
    double q0[4] = {q[0], q[1], q[2], q[3]};
    for (int c = 0; c < 4; ++c) A.p.qold[4 * k + c] = q0[c];
    double r1[4], qs[4], qm[4], r2[4], qn[4];
    quat_rate(A.p.w + 3 * k, q0, r1);
    for (int c = 0; c < 4; ++c) qs[c] = q0[c] + dt * r1[c];
    for (int c = 0; c < 4; ++c) qm[c] = 0.5 * (q0[c] + qs[c]);
    quat_rate(A.p.w + 3 * k, qm, r2);
    for (int c = 0; c < 4; ++c) qn[c] = q0[c] + dt * r2[c];
    double l = sqrt((qn[0] * qn[0] + qn[1] * qn[1]) + (qn[2] * qn[2] + qn[3] * qn[3]));
    for (int c = 0; c < 4; ++c) q[c] = qn[c] / l;
    if (write_kin) {
        for (int c = 0; c < 3; ++c) {
            A.p.kin[9 * k + c] = x[c];
            A.p.kin[9 * k + 3 + c] = A.p.vp[3 * k + c];
            A.p.kin[9 * k + 6 + c] = A.p.wp[3 * k + c];
        }
    }
}

// alpha = Rbw I^-1 [Rbw^T M - (Rbw^T w) x (I Rbw^T w)] at the substep start (as printed)
__device__ void angular_accel(const DemArgs& A, int k, const double* qo, const double* w, const double* M,
                              double* al) {
    double R[9];
    quat_rbw(qo, R);
    const double* I = A.p.inertia + 3 * k;
    double Mb[3], wb[3], Iw[3], g[3], ab[3];
    for (int c = 0; c < 3; ++c) {
        Mb[c] = (R[0 + c] * M[0] + R[3 + c] * M[1]) + R[6 + c] * M[2];
        wb[c] = (R[0 + c] * w[0] + R[3 + c] * w[1]) + R[6 + c] * w[2];
    }
    for (int c = 0; c < 3; ++c) Iw[c] = I[c] * wb[c];
    cross3(wb, Iw, g);
    for (int c = 0; c < 3; ++c) ab[c] = (Mb[c] - g[c]) / I[c];
    for (int r = 0; r < 3; ++r) al[r] = (R[3 * r] * ab[0] + R[3 * r + 1] * ab[1]) + R[3 * r + 2] * ab[2];
}

// corrector: a_new = (F_dem + F_hyd + F_ext)/m, F_ext = m (1 - rho0/rho_p) g;
// v += dt/2 (a + a_new); w += dt/2 (alpha + alpha_new)
__global__ void k_correct(DemArgs A, double dt) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.p.np) return;
    if (A.p.fixed[k]) {
        for (int c = 0; c < 3; ++c) A.p.a[3 * k + c] = A.p.al[3 * k + c] = 0.0;
        return;
    }
    double m = A.p.mass[k];
    double fb = 1.0 - 1.0 / A.p.dens[k];
    double M[3], an[3], aln[3];
    for (int c = 0; c < 3; ++c) {
        double fext = m * fb * A.gravity[c];
        an[c] = ((A.p.fd[3 * k + c] + A.p.fh[3 * k + c]) + fext) / m;
        M[c] = A.p.md[3 * k + c] + A.p.mh[3 * k + c];
    }
    angular_accel(A, k, A.p.qold + 4 * k, A.p.w + 3 * k, M, aln);
    for (int c = 0; c < 3; ++c) {
        A.p.v[3 * k + c] += 0.5 * dt * (A.p.a[3 * k + c] + an[c]);
        A.p.a[3 * k + c] = an[c];
        A.p.w[3 * k + c] += 0.5 * dt * (A.p.al[3 * k + c] + aln[c]);
        A.p.al[3 * k + c] = aln[c];
    }
}

// initial accelerations a(0) = (F_dem(0) + F_ext)/m, alpha(0) from M_dem(0)
__global__ void k_initial_accel(DemArgs A) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.p.np) return;
    double m = A.p.mass[k];
    double fb = 1.0 - 1.0 / A.p.dens[k];
    if (A.p.fixed[k]) {
        for (int c = 0; c < 3; ++c) A.p.a[3 * k + c] = A.p.al[3 * k + c] = 0.0;
    } else {
        double M[3];
        for (int c = 0; c < 3; ++c) {
            M[c] = A.p.md[3 * k + c];
            A.p.a[3 * k + c] = (A.p.fd[3 * k + c] + m * fb * A.gravity[c]) / m;
        }
        angular_accel(A, k, A.p.q + 4 * k, A.p.w + 3 * k, M, A.p.al + 3 * k);
    }
    for (int c = 0; c < 3; ++c) {
        A.p.vp[3 * k + c] = A.p.v[3 * k + c];
        A.p.wp[3 * k + c] = A.p.w[3 * k + c];
        A.p.kin[9 * k + c] = A.p.pos[3 * k + c];
        A.p.kin[9 * k + 3 + c] = A.p.v[3 * k + c];
        A.p.kin[9 * k + 6 + c] = A.p.w[3 * k + c];
    }
    for (int c = 0; c < 4; ++c) A.p.qold[4 * k + c] = A.p.q[4 * k + c];
}

__global__ void k_zero_d(double* p, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

inline unsigned nblk(long long n, int t = 256) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t dem_predict(const DemArgs& A, double dt, int write_kin, hipStream_t s) {
    if (A.p.np == 0) return hipSuccess;
    k_predict<<<nblk(A.p.np), 256, 0, s>>>(A, dt, write_kin);
    return hipGetLastError();
}

hipError_t dem_lists(const DemArgs& A, int* scan_tmp, hipStream_t s) {
    if (A.p.np == 0) return hipSuccess;
    hipError_t e;
    if ((e = psm_fill_int(A.cell_count, 0, A.ncell, s)) != hipSuccess) return e;
    if ((e = psm_fill_int(A.cell_fill, 0, A.ncell, s)) != hipSuccess) return e;
    k_reg_hist<<<nblk(A.p.np), 256, 0, s>>>(A);
    if ((e = psm_scan(A.cell_count, A.cell_start, A.ncell, scan_tmp, s)) != hipSuccess) return e;
    k_reg_scatter<<<nblk(A.p.np), 256, 0, s>>>(A);
    k_cell_sort<<<nblk(A.ncell), 256, 0, s>>>(A);
    k_pair_count<<<nblk(A.p.np), 128, 0, s>>>(A);
    if ((e = psm_scan(A.pcount, A.prow, A.p.np, scan_tmp, s)) != hipSuccess) return e;
    k_pair_emit<<<nblk(A.p.np), 128, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t dem_contacts(const DemArgs& A, const double* vv, const double* ww, double dth, hipStream_t s) {
    if (A.p.np == 0) return hipSuccess;
    k_contacts<<<nblk(A.pair_cap, 128), 128, 0, s>>>(A, vv, ww, dth);
    k_dem_sum<<<nblk(A.p.np, 128), 128, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t dem_correct(const DemArgs& A, double dt, hipStream_t s) {
    if (A.p.np == 0) return hipSuccess;
    k_correct<<<nblk(A.p.np), 256, 0, s>>>(A, dt);
    return hipGetLastError();
}

hipError_t dem_initial_accel(const DemArgs& A, hipStream_t s) {
    if (A.p.np == 0) return hipSuccess;
    k_initial_accel<<<nblk(A.p.np), 256, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t dem_zero(double* p, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_zero_d<<<nblk(n), 256, 0, s>>>(p, n);
    return hipGetLastError();
}
