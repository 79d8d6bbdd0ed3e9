// dem.hip -- DEM substep kernels (FP64).  Compiled with -ffp-contract=off so
// that the predicates deciding integer results (cell indices, pair lists) use
// separately rounded operations in a fixed order; only the ellipsoid
// iteration's helpers, an approximation refined to a tolerance, contract
// multiply-adds and use refined hardware reciprocal estimates.
//
// A substep (Sec. 3.2.1-3.2.2, Table 1), as per-index phases:
//   predict      Verlet predictor of position and orientation (Eqs. advance-r ...)
//                and the particle's DEM cells per axis (box of the particle)
//   cell list    counting sort of (cell, pid) registrations: histogram, scan,
//                scatter (each cell's list in arrival order; ordered by pid only
//                for a read-back)
//   pairs        per particle i the unique j > i sharing a cell (each j counted in
//                the lowest shared cell), then wall candidates; rows emitted and
//                ordered in place, so the list is sorted and unique without a
//                global sort
//   contacts     spring-dashpot + Coulomb per pair, history by binary search in the
//                previous sorted list (at the pair's own index on a kept list;
//                pairs out of contact at their last two evaluations write nothing)
//   sums         per particle: pairs where it is the second member (counting-sorted
//                columns, ascending pair index) then its own row, a fixed order
//   correct      Verlet corrector
// Large particle counts run each phase as a kernel.  Up to DEM_FUSED_MAX
// particles, one workgroup runs every substep of a coupled step in a single
// launch; there the candidate pairs come from testing all i < j for a shared
// cell, the same set in the same order as the cell list gives.
#include <math.h>

#include "common.h"
#include "dem.h"

#include "serve.h"

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

// half extents of the particle's axis-aligned box from its shape, semi-axes
// and orientation
__device__ inline void half_extents_of(int shape, const double s[3], const double q[4], double e[3]) {
    if (shape == 0) {
        e[0] = e[1] = e[2] = s[0];
        return;
    }
    double R[9];
    quat_rbw(q, R);
    for (int r = 0; r < 3; ++r) {
        double t0 = s[0] * R[3 * r + 0], t1 = s[1] * R[3 * r + 1], t2 = s[2] * R[3 * r + 2];
        e[r] = sqrt((t0 * t0 + t1 * t1) + t2 * t2);
    }
}

__device__ inline void half_extents(const DemArgs& A, int k, double e[3]) {
    const int shape = A.p.shape[k];
    const double s[3] = {A.p.semi[3 * k], A.p.semi[3 * k + 1], A.p.semi[3 * k + 2]};
    double q[4] = {1.0, 0.0, 0.0, 0.0};
    if (shape != 0)
        for (int c = 0; c < 4; ++c) q[c] = A.p.q[4 * k + c];
    half_extents_of(shape, s, q, e);
}

// ---------------------------------------------------------------------------
// registration cells: per axis the sorted DEM cells of the particle's box
// lo = floor((x - e)/h) .. hi = floor((x + e)/h), wrapped on periodic axes and
// clamped on walled ones (at most two per axis: h exceeds every diameter)
// ---------------------------------------------------------------------------
struct AxCells {
    int c[3][2];
    int n[3];
};

// Cell t (an integer-valued double: the floor of a coordinate over h) wrapped
// mod n on a periodic axis or clamped to [0, n-1] on a walled one.  The
// arithmetic stays in double until the result is in range, so a position of
// any finite size (a blown-up state) maps to a cell; NaN maps to cell 0.
__device__ inline int wrap_cell(double t, int n, int periodic) {
    if (t != t) return 0;
    const double dn = (double)n;
    if (periodic) {
        // one period off at most for a wrapped position (selects, exact);
        // any other offset takes the remainder
        double r = t < 0.0 ? t + dn : (t >= dn ? t - dn : t);
        if (r < 0.0 || r >= dn) {
            r = fmod(t, dn);
            if (r < 0.0) r += dn;
        }
        return (int)r;
    }
    return t < 0.0 ? 0 : (t > dn - 1.0 ? n - 1 : (int)t);
}

__device__ inline void axis_cells_at(const DemArgs& A, const double pos[3], const double e[3], AxCells& r) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double x = pos[a];
        const double lo = floor((x - e[a]) / A.h[a]);
        const double hi = floor((x + e[a]) / A.h[a]);
        const int per = A.g.periodic[a];
        int c0 = wrap_cell(lo, A.nc[a], per);
        int c1 = hi > lo ? wrap_cell(lo + 1.0, A.nc[a], per) : c0;
        if (c1 < c0) {
            int t = c0;
            c0 = c1;
            c1 = t;
        }
        r.c[a][0] = c0;
        r.c[a][1] = c1;
        r.n[a] = c1 == c0 ? 1 : 2;
    }
}

__device__ inline void axis_cells(const DemArgs& A, int k, AxCells& r) {
    double e[3];
    half_extents(A, k, e);
    const double pos[3] = {A.p.pos[3 * k], A.p.pos[3 * k + 1], A.p.pos[3 * k + 2]};
    axis_cells_at(A, pos, e, r);
}

__device__ inline void store_cells(const DemArgs& A, int k, const AxCells& r) {
    int* d = A.pc + 8 * k;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        d[2 * a] = r.c[a][0];
        d[2 * a + 1] = r.c[a][1];
    }
    d[6] = r.n[0] | (r.n[1] << 2) | (r.n[2] << 4);
}

__device__ inline void load_cells(const DemArgs& A, int k, AxCells& r) {
    const int* d = A.pc + 8 * k;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.c[a][0] = d[2 * a];
        r.c[a][1] = d[2 * a + 1];
    }
    r.n[0] = d[6] & 3;
    r.n[1] = (d[6] >> 2) & 3;
    r.n[2] = (d[6] >> 4) & 3;
}

__device__ inline long long cell_id(const DemArgs& A, int x, int y, int z) {
    return (long long)x + (long long)A.nc[0] * ((long long)y + (long long)A.nc[1] * z);
}

// lowest common cell along one axis, -1 if none
__device__ inline int axis_common(const AxCells& p, const AxCells& q, int a) {
    int best = -1;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
            if (u < p.n[a] && v < q.n[a] && p.c[a][u] == q.c[a][v] && (best < 0 || p.c[a][u] < best))
                best = p.c[a][u];
    return best;
}

__device__ inline bool share_cell(const AxCells& p, const AxCells& q) {
    return axis_common(p, q, 0) >= 0 && axis_common(p, q, 1) >= 0 && axis_common(p, q, 2) >= 0;
}

__device__ inline double wall_dist(const DemArgs& A, int k, int f) {
    int a = f / 2;
    return (f % 2 == 0) ? A.p.pos[3 * k + a] : A.L[a] - A.p.pos[3 * k + a];
}

__device__ inline int wall_count(const DemArgs& A, int i) {
    int n = 0;
#pragma unroll
    for (int f = 0; f < 6; ++f) n += (A.g.bc[f] != 0 && wall_dist(A, i, f) < A.p.rb[i]);
    return n;
}

// ---------------------------------------------------------------------------
// contact geometry (Sec. 2.1): spheres in closed form, ellipsoids by iterated
// equivalent spheres with the local curvature radius (Eq. local-curvature)
// ---------------------------------------------------------------------------
// An ellipsoid's constants for the iteration, formed once per evaluation: its
// rotation R (body to world), 1 / a_k^2, and the curvature-radius weights
// (b c / a^3, a c / b^3, a b / c^3), so that the iteration itself divides only
// where a quotient of two iterates is needed.  The iteration's two helpers
// contract multiply-adds (the file is otherwise compiled without): they form an
// approximation refined until it converges or the cap is met, and the
// contact decision on its result is not an exact predicate of the inputs.
// 1/sqrt(x) and 1/x from the hardware estimates refined by two Newton steps
// (within a few units in the last place of the rounded quotients)
__device__ inline double rsq_nr(double x) {
#pragma clang fp contract(fast)
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * (1.5 - h * y * y);
    y = y * (1.5 - h * y * y);
    return y;
}
// sqrt(x) for x >= 0 from the same estimate (0 at 0)
__device__ inline double sqrt_nr(double x) { return x > 0.0 ? x * rsq_nr(x) : 0.0; }
__device__ inline double rcp_nr(double x) {
#pragma clang fp contract(fast)
    double y = __builtin_amdgcn_rcp(x);
    y = y * (2.0 - x * y);
    y = y * (2.0 - x * y);
    return y;
}

struct EllShape {
    double R[9];
    double ia2[3];
    double kr[3];
};

__device__ inline void ell_shape(const double* q, const double* ax, EllShape& E) {
    quat_rbw(q, E.R);
    const double a = ax[0], b = ax[1], c = ax[2];
    E.ia2[0] = 1.0 / (a * a);
    E.ia2[1] = 1.0 / (b * b);
    E.ia2[2] = 1.0 / (c * c);
    E.kr[0] = b * c / (a * a * a);
    E.kr[1] = a * c / (b * b * b);
    E.kr[2] = a * b / (c * c * c);
}

// local curvature radius rho and unit outward normal n at surface point p
__device__ void ell_local(const double* c, const EllShape& E, const double* p, double* rho, double* n) {
#pragma clang fp contract(fast)
    const double* R = E.R;
    double d[3] = {p[0] - c[0], p[1] - c[1], p[2] - c[2]};
    double xb[3];
    for (int k = 0; k < 3; ++k) xb[k] = (R[0 + k] * d[0] + R[3 + k] * d[1]) + R[6 + k] * d[2];
    *rho = (E.kr[0] * xb[0] * xb[0] + E.kr[1] * xb[1] * xb[1]) + E.kr[2] * xb[2] * xb[2];
    double nb[3] = {xb[0] * E.ia2[0], xb[1] * E.ia2[1], xb[2] * E.ia2[2]};
    double nw[3];
    for (int r = 0; r < 3; ++r) nw[r] = (R[3 * r] * nb[0] + R[3 * r + 1] * nb[1]) + R[3 * r + 2] * nb[2];
    const double il = rsq_nr(dot3(nw, nw));
    for (int r = 0; r < 3; ++r) n[r] = nw[r] * il;
}

// intersection of the line s + t u with the surface: the root with the larger
// t when far_positive, else the smaller; false on a miss
__device__ bool ell_line_hit(const double* c, const EllShape& E, const double* s, const double* u, bool far_positive,
                             double* p) {
#pragma clang fp contract(fast)
    const double* R = E.R;
    double d[3] = {s[0] - c[0], s[1] - c[1], s[2] - c[2]};
    double y0[3], ud[3];
    for (int k = 0; k < 3; ++k) {
        y0[k] = (R[0 + k] * d[0] + R[3 + k] * d[1]) + R[6 + k] * d[2];
        ud[k] = (R[0 + k] * u[0] + R[3 + k] * u[1]) + R[6 + k] * u[2];
    }
    double qa = 0, qb = 0, qc = -1.0;
    for (int k = 0; k < 3; ++k) {
        qa += ud[k] * ud[k] * E.ia2[k];
        qb += y0[k] * ud[k] * E.ia2[k];
        qc += y0[k] * y0[k] * E.ia2[k];
    }
    double disc = qb * qb - qa * qc;
    if (disc < 0.0 || qa <= 0.0) return false;
    double sq = sqrt_nr(disc);
    double t = (far_positive ? -qb + sq : -qb - sq) * rcp_nr(qa);
    for (int k = 0; k < 3; ++k) p[k] = s[k] + t * u[k];
    return true;
}

struct Geom {
    double delta, en[3], rci[3], rcj[3], rhoi, rhoj;
    bool sphere_law;
    bool deferred;   // an ellipsoid pair within bounding-sphere reach left to the iteration kernel
};

__device__ void ellipsoid_pair(const DemArgs& A, int i, int j, Geom& G) {
    const double* ci = A.p.pos + 3 * i;
    double dvec[3];
    min_image(A, ci, A.p.pos + 3 * j, dvec);
    double cj[3] = {ci[0] - dvec[0], ci[1] - dvec[1], ci[2] - dvec[2]};
    const double* ai = A.p.semi + 3 * i;
    const double* aj = A.p.semi + 3 * j;
    EllShape Ei, Ej;
    ell_shape(A.p.q + 4 * i, ai, Ei);
    ell_shape(A.p.q + 4 * j, aj, Ej);
    double amin = ai[0];
    for (int k = 0; k < 3; ++k) {
        amin = ai[k] < amin ? ai[k] : amin;
        amin = aj[k] < amin ? aj[k] : amin;
    }
    double pi[3], pj[3];
    {
        double u[3] = {cj[0] - ci[0], cj[1] - ci[1], cj[2] - ci[2]};
        const double il = rsq_nr(dot3(u, u));
        for (int k = 0; k < 3; ++k) u[k] *= il;
        ell_line_hit(ci, Ei, ci, u, true, pi);
        double um[3] = {-u[0], -u[1], -u[2]};
        ell_line_hit(cj, Ej, cj, um, true, pj);
    }
    for (int it = 0; it < 32; ++it) {
        double rhoi, rhoj, ni[3], nj[3], si[3], sj[3];
        ell_local(ci, Ei, pi, &rhoi, ni);
        ell_local(cj, Ej, pj, &rhoj, nj);
        for (int k = 0; k < 3; ++k) {
            si[k] = pi[k] - rhoi * ni[k];
            sj[k] = pj[k] - rhoj * nj[k];
        }
        double u[3] = {sj[0] - si[0], sj[1] - si[1], sj[2] - si[2]};
        const double l2 = dot3(u, u);
        if (!(l2 > 0.0)) break;
        const double il = rsq_nr(l2);
        for (int k = 0; k < 3; ++k) u[k] *= il;
        double npi[3], npj[3];
        if (!ell_line_hit(ci, Ei, si, u, true, npi)) break;
        if (!ell_line_hit(cj, Ej, sj, u, false, npj)) break;
        double dpi[3] = {npi[0] - pi[0], npi[1] - pi[1], npi[2] - pi[2]};
        double dpj[3] = {npj[0] - pj[0], npj[1] - pj[1], npj[2] - pj[2]};
        double conv = sqrt_nr(dot3(dpi, dpi)) + sqrt_nr(dot3(dpj, dpj));
        for (int k = 0; k < 3; ++k) {
            pi[k] = npi[k];
            pj[k] = npj[k];
        }
        if (conv < 1e-10 * amin) break;
    }
    double ni[3], nj[3], si[3], sj[3];
    ell_local(ci, Ei, pi, &G.rhoi, ni);
    ell_local(cj, Ej, pj, &G.rhoj, nj);
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

// The same iteration with the pair on two adjacent lanes: side 0 evaluates
// ellipsoid i, side 1 ellipsoid j, and the lanes swap the sphere centres, the
// hit flags and the point moves they need of each other.  Every quantity both
// lanes branch on is formed from the same operands in the same order on both,
// so the two take each branch together and each exchange finds its partner
// active; the results are those of ellipsoid_pair, operation for operation.
// the partner lane's value (lanes 2k and 2k + 1 swap) by a DPP quad permutation
// [1, 0, 3, 2]: a register move, no LDS round trip.  Both lanes of a pair are
// always active together (they take the same branches).
__device__ inline int lane_swap_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true); }
__device__ inline double lane_swap(double v) {
    const int lo = lane_swap_i(__double2loint(v)), hi = lane_swap_i(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

__device__ void ellipsoid_pair2(const DemArgs& A, int i, int j, int side, Geom& G) {
    const double* ci = A.p.pos + 3 * i;
    double dvec[3];
    min_image(A, ci, A.p.pos + 3 * j, dvec);
    const double cj[3] = {ci[0] - dvec[0], ci[1] - dvec[1], ci[2] - dvec[2]};
    const int me = side ? j : i;
    const double c[3] = {side ? cj[0] : ci[0], side ? cj[1] : ci[1], side ? cj[2] : ci[2]};
    EllShape E;
    ell_shape(A.p.q + 4 * me, A.p.semi + 3 * me, E);
    const double* ai = A.p.semi + 3 * i;
    const double* aj = A.p.semi + 3 * j;
    double amin = ai[0];
    for (int k = 0; k < 3; ++k) {
        amin = ai[k] < amin ? ai[k] : amin;
        amin = aj[k] < amin ? aj[k] : amin;
    }
    double p[3];
    {
        double u[3] = {cj[0] - ci[0], cj[1] - ci[1], cj[2] - ci[2]};
        const double il = rsq_nr(dot3(u, u));
        for (int k = 0; k < 3; ++k) u[k] *= il;
        const double dir[3] = {side ? -u[0] : u[0], side ? -u[1] : u[1], side ? -u[2] : u[2]};
        ell_line_hit(c, E, c, dir, true, p);
    }
    for (int it = 0; it < 32; ++it) {
        double rho, n[3], sc[3], so[3];
        ell_local(c, E, p, &rho, n);
        for (int k = 0; k < 3; ++k) sc[k] = p[k] - rho * n[k];
        for (int k = 0; k < 3; ++k) so[k] = lane_swap(sc[k]);
        const double* si = side ? so : sc;
        const double* sj = side ? sc : so;
        double u[3] = {sj[0] - si[0], sj[1] - si[1], sj[2] - si[2]};
        const double l2 = dot3(u, u);
        if (!(l2 > 0.0)) break;
        const double il = rsq_nr(l2);
        for (int k = 0; k < 3; ++k) u[k] *= il;
        double np_[3];
        const int hit = ell_line_hit(c, E, sc, u, side == 0, np_) ? 1 : 0;
        const int hit_o = lane_swap_i(hit);
        if (!(hit && hit_o)) break;
        double dp[3] = {np_[0] - p[0], np_[1] - p[1], np_[2] - p[2]};
        const double m = sqrt_nr(dot3(dp, dp));
        const double mo = lane_swap(m);
        const double conv = side ? mo + m : m + mo;
        for (int k = 0; k < 3; ++k) p[k] = np_[k];
        if (conv < 1e-10 * amin) break;
    }
    double rho, n[3], sc[3], so[3], rc[3], ro[3];
    ell_local(c, E, p, &rho, n);
    for (int k = 0; k < 3; ++k) {
        sc[k] = p[k] - rho * n[k];
        rc[k] = p[k] - c[k];
    }
    for (int k = 0; k < 3; ++k) {
        so[k] = lane_swap(sc[k]);
        ro[k] = lane_swap(rc[k]);
    }
    const double rho_o = lane_swap(rho);
    const double* si = side ? so : sc;
    const double* sj = side ? sc : so;
    G.rhoi = side ? rho_o : rho;
    G.rhoj = side ? rho : rho_o;
    double d[3] = {si[0] - sj[0], si[1] - sj[1], si[2] - sj[2]};
    double l = sqrt(dot3(d, d));
    G.delta = (G.rhoi + G.rhoj) - l;
    for (int k = 0; k < 3; ++k) {
        G.en[k] = d[k] / l;
        G.rci[k] = side ? ro[k] : rc[k];
        G.rcj[k] = side ? rc[k] : ro[k];
    }
    G.sphere_law = false;
    G.deferred = false;
}

// ci, cj: centres; shi, shj: shapes; ri, rj: first semi-axes (loaded by the
// caller).  ELL = false compiles the sphere paths only (domains without
// ellipsoids), which keeps the register budget of the contact kernels small.
template <bool ELL>
__device__ void pair_geometry(const DemArgs& A, int i, int j, const double* ci, const double* cj, int shi, int shj,
                              double ri, double rj, Geom& G, bool defer = false) {
    const int np = A.p.np;
    G.sphere_law = false;
    G.deferred = false;
    if (j >= np) {
        int f = j - np, a = f / 2;
        // the wall normal and the centre's coordinate along it, by selects
        // (no indexing of register arrays)
        const double sgn = (f % 2 == 0) ? 1.0 : -1.0;
        const double n[3] = {a == 0 ? sgn : 0.0, a == 1 ? sgn : 0.0, a == 2 ? sgn : 0.0};
        const double* c = ci;
        const double ca = a == 0 ? c[0] : (a == 1 ? c[1] : c[2]);
        const double La = a == 0 ? A.L[0] : (a == 1 ? A.L[1] : A.L[2]);
        double dist = (f % 2 == 0) ? ca : La - ca;
        for (int k = 0; k < 3; ++k) {
            G.en[k] = n[k];
            G.rcj[k] = 0.0;
        }
        G.rhoj = 0.0;
        if (!ELL || shi == 0) {
            double R = ri;
            G.delta = R - dist;
            for (int k = 0; k < 3; ++k) G.rci[k] = -R * n[k];
            G.rhoi = R;
            G.sphere_law = true;
        } else {
            EllShape E;
            const double* ax = A.p.semi + 3 * i;
            ell_shape(A.p.q + 4 * i, ax, E);
            const double* R = E.R;
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
            ell_local(c, E, p, &G.rhoi, nn);
            for (int k = 0; k < 3; ++k) G.rci[k] = p[k] - c[k];
        }
        return;
    }
    double d[3];
    min_image(A, ci, cj, d);
    double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    if (!ELL || (shi == 0 && shj == 0)) {
        double Ri = ri, Rj = rj;
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
    if (defer) {
        G.deferred = true;
        return;
    }
    ellipsoid_pair(A, i, j, G);
}

// ---------------------------------------------------------------------------
// phases (one index each)
// ---------------------------------------------------------------------------
__device__ void ph_cells(const DemArgs& A, int k) {
    AxCells r;
    axis_cells(A, k, r);
    store_cells(A, k, r);
}

__device__ void ph_hist(const DemArgs& A, int k) {
    AxCells r;
    load_cells(A, k, r);
    for (int z = 0; z < r.n[2]; ++z)
        for (int y = 0; y < r.n[1]; ++y)
            for (int x = 0; x < r.n[0]; ++x) atomicAdd(&A.cell_count[cell_id(A, r.c[0][x], r.c[1][y], r.c[2][z])], 1);
}

__device__ void ph_scatter(const DemArgs& A, int k) {
    AxCells r;
    load_cells(A, k, r);
    for (int z = 0; z < r.n[2]; ++z)
        for (int y = 0; y < r.n[1]; ++y)
            for (int x = 0; x < r.n[0]; ++x) {
                const long long c = cell_id(A, r.c[0][x], r.c[1][y], r.c[2][z]);
                const int slot = atomicAdd(&A.cell_fill[c], 1);
                const long long at = (long long)A.cell_start[c] + slot;
                if (at < A.reg_cap) A.cell_pid[at] = k;
            }
}

__device__ void ph_cellsort(const DemArgs& A, long long c) {
    const int s0 = A.cell_start[c], s1 = A.cell_start[c + 1];
    for (int u = s0 + 1; u < s1; ++u)
        for (int v = u; v > s0 && A.cell_pid[v] < A.cell_pid[v - 1]; --v) {
            int t = A.cell_pid[v];
            A.cell_pid[v] = A.cell_pid[v - 1];
            A.cell_pid[v - 1] = t;
        }
}

// neighbours j > i through the cell lists; emit: write them (cell order) at out
__device__ int pairs_by_cells(const DemArgs& A, int i, unsigned long long* out, long long room) {
    AxCells ri;
    load_cells(A, i, ri);
    int n = 0;
    for (int z = 0; z < ri.n[2]; ++z)
        for (int y = 0; y < ri.n[1]; ++y)
            for (int x = 0; x < ri.n[0]; ++x) {
                const long long c = cell_id(A, ri.c[0][x], ri.c[1][y], ri.c[2][z]);
                const int s0 = A.cell_start[c], s1 = A.cell_start[c + 1];
                for (int s = s0; s < s1; ++s) {
                    const int j = A.cell_pid[s];
                    if (j <= i) continue;
                    AxCells rj;
                    load_cells(A, j, rj);
                    // count j in the lowest cell the two share
                    if (axis_common(ri, rj, 0) != ri.c[0][x] || axis_common(ri, rj, 1) != ri.c[1][y] ||
                        axis_common(ri, rj, 2) != ri.c[2][z])
                        continue;
                    if (out && n < room) out[n] = ((unsigned long long)i << 32) | (unsigned)j;
                    ++n;
                }
            }
    return n;
}

// neighbours j > i by testing every j (small particle counts), ascending
__device__ int pairs_all(const DemArgs& A, int i, unsigned long long* out, long long room) {
    AxCells ri;
    load_cells(A, i, ri);
    int n = 0;
    for (int j = i + 1; j < A.p.np; ++j) {
        AxCells rj;
        load_cells(A, j, rj);
        if (!share_cell(ri, rj)) continue;
        if (out && n < room) out[n] = ((unsigned long long)i << 32) | (unsigned)j;
        ++n;
    }
    return n;
}

__device__ inline void emit_walls(const DemArgs& A, int i, unsigned long long* out, long long room, int n0) {
    int n = n0;
    const unsigned long long np = (unsigned long long)A.p.np;
    for (int f = 0; f < 6; ++f)
        if (A.g.bc[f] != 0 && wall_dist(A, i, f) < A.p.rb[i]) {
            if (n < room) out[n] = ((unsigned long long)i << 32) | (unsigned)(np + f);
            ++n;
        }
}

__device__ inline long long find_prev(const PairBufs& B, unsigned long long key, long long n) {
    long long lo = 0, hi = n;
    while (lo < hi) {
        long long mid = (lo + hi) >> 1;
        if (B.prev_pairs[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < n && B.prev_pairs[lo] == key) ? lo : -1;
}

__device__ inline long long n_pairs(const DemArgs& A, const PairBufs& B) {
    long long n = B.prow[A.p.np];
    return n < A.pair_cap ? n : A.pair_cap;
}

// Spring-dashpot contact with a Coulomb limit and tangential history (Sec.
// 2.1; Hertz coefficients App. A), defined below.  same_list: the previous
// list holds the same keys in the same order, so the history of pair s sits
// at index s.  Returns whether the pair is in contact; out of contact, *gap
// (when given) receives the separation -delta.
__device__ bool contact_law(const DemArgs& A, const PairBufs& B, long long s, unsigned long long key, const Geom& G,
                            const double* __restrict__ vv, const double* __restrict__ ww, double dth, long long nprev,
                            bool same_list, double* gap);

// Geometry, then the law, of pair s.  With deferred non-null, an ellipsoid
// pair that needs the iteration is not evaluated: *deferred is set and the
// pair's outputs are left to the dense iteration kernel.
template <bool ELL>
__device__ bool ph_contact(const DemArgs& A, const PairBufs& B, long long s, const double* __restrict__ vv,
                           const double* __restrict__ ww, double dth, long long nprev, bool same_list = false,
                           double* gap = nullptr, bool* deferred = nullptr) {
    const int np = A.p.np;
    const unsigned long long key = B.pairs[s];
    const int i = (int)(key >> 32), j = (int)(key & 0xffffffffu);
    const bool wall = j >= np;
    // the geometry's inputs first; the kinematics, masses and history only for
    // pairs in contact (most candidate pairs are not)
    double ci[3], cj[3] = {0.0, 0.0, 0.0};
    const int shi = A.p.shape[i], shj = wall ? 0 : A.p.shape[j];
    const double ri = A.p.semi[3 * i], rj = wall ? 0.0 : A.p.semi[3 * j];
    for (int k = 0; k < 3; ++k) {
        ci[k] = A.p.pos[3 * i + k];
        if (!wall) cj[k] = A.p.pos[3 * j + k];
    }
    Geom G;
    pair_geometry<ELL>(A, i, j, ci, cj, shi, shj, ri, rj, G, deferred != nullptr);
    if (ELL && G.deferred) {
        *deferred = true;
        return false;
    }
    return contact_law(A, B, s, key, G, vv, ww, dth, nprev, same_list, gap);
}

// Spring and dashpot coefficients of a contact in contact: the linear law's
// constants (gamma_n = -2 beta sqrt(k_n m*)), or the Hertz law's from the
// material and the overlap (App. A: k_n = 4/3 Y* sqrt(R* delta), k_t = 8 G*
// sqrt(R* delta), gamma = -2 sqrt(5/6) beta sqrt(S m*) with S_n = 2 Y*
// sqrt(R* delta), S_t = 8 G* sqrt(R* delta); a wall has infinite radius and
// mass).
struct LawCoeffs {
    double kn, kt, gn, gt;
};

__device__ inline LawCoeffs law_coeffs(const DemArgs& A, const Geom& G, bool wall, double mstar) {
    LawCoeffs c;
    if (A.hertz) {
        const double Rs = wall ? G.rhoi : 1.0 / (1.0 / G.rhoi + 1.0 / G.rhoj);
        const double root = sqrt(Rs * G.delta);
        c.kn = 4.0 / 3.0 * A.ystar * root;
        c.kt = 8.0 * A.gstar * root;
        const double damp = -2.0 * sqrt(5.0 / 6.0) * A.beta_e;
        c.gn = damp * sqrt((2.0 * A.ystar * root) * mstar);
        c.gt = damp * sqrt((8.0 * A.gstar * root) * mstar);
    } else {
        c.kn = A.kn;
        c.kt = A.kt_ratio * A.kn;
        c.gn = -2.0 * A.beta_e * sqrt(c.kn * mstar);
        c.gt = A.gt_ratio * c.gn;
    }
    return c;
}

// Sliding: a tangential force above mu |F_n| is scaled down to it, and the
// spring displacement is reset to the one that force implies.
__device__ inline void coulomb_limit(const LawCoeffs& c, double limit, const double* ut, double* ft, double* xi) {
    const double mag = sqrt(dot3(ft, ft));
    if (!(mag > limit)) return;
    const double s = limit / mag;
    for (int k = 0; k < 3; ++k) ft[k] *= s;
    if (c.kt > 0.0)
        for (int k = 0; k < 3; ++k) xi[k] = -(ft[k] + c.gt * ut[k]) / c.kt;
}

// The contact law of pair s (key = B.pairs[s]) with its geometry G.  Out of
// contact every output is zero.  In contact, with n the unit normal from i
// towards j and d = v_i - v_j:
//   normal force   F_n = k_n delta - gamma_n (d . n), along n;
//   slip velocity  u = d - (rho_i w_i + rho_j w_j) x n, u_t its tangential part;
//   spring         xi = (h - (h . n) n) + u_t dt (the stored displacement h
//                  turned into the present tangent plane, then advanced);
//   friction       F_t = -k_t xi - gamma_t u_t, at most mu |F_n|;
// force on i: F_n n + F_t; moments: spheres -rho e_n x F_t on each, else the
// contact-point arms crossed with the force.  The arithmetic of each term is
// evaluated in the oracle's order (forces and history bit for bit on the
// same geometry).
__device__ bool contact_law(const DemArgs& A, const PairBufs& B, long long s, unsigned long long key, const Geom& G,
                            const double* __restrict__ vv, const double* __restrict__ ww, double dth, long long nprev,
                            bool same_list, double* gap) {
    const int np = A.p.np;
    const int i = (int)(key >> 32), j = (int)(key & 0xffffffffu);
    const bool wall = j >= np;
    double* out_f = A.cF + 3 * s;
    double* out_mi = A.cMi + 3 * s;
    double* out_mj = A.cMj + 3 * s;
    double* out_h = B.hist + 3 * s;
    // incontact[s]: bit 0 the pair is in contact at this evaluation, bit 1 it
    // was at the one before on the same list, or that is not known (a new
    // list).  A pair out of contact at both earlier evaluations on a kept list
    // already holds zero outputs and zero history in both buffers (the history
    // buffers alternate by substep), so it writes nothing.
    const unsigned char prev = same_list ? A.incontact[s] : (unsigned char)2;
    if (!(G.delta > 0.0)) {
        if (prev != 0) {
            for (int k = 0; k < 3; ++k) out_f[k] = out_mi[k] = out_mj[k] = out_h[k] = 0.0;
            A.incontact[s] = same_list ? (unsigned char)((prev & 1) << 1) : (unsigned char)2;
        }
        if (gap) *gap = -G.delta;
        return false;
    }
    A.incontact[s] = same_list ? (unsigned char)(1 | ((prev & 1) << 1)) : (unsigned char)3;
    // the partner's motion: a particle's, or the wall's (its velocity when it moves)
    double vi[3], wi[3], vj[3] = {0.0, 0.0, 0.0}, wj[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 3; ++k) {
        vi[k] = vv[3 * i + k];
        wi[k] = ww[3 * i + k];
    }
    double mstar;
    if (wall) {
        const int face = j - np;
        if (A.g.bc[face] == 2)
            for (int k = 0; k < 3; ++k) vj[k] = A.wall_u[face][k];
        mstar = A.p.mass[i];
    } else {
        for (int k = 0; k < 3; ++k) {
            vj[k] = vv[3 * j + k];
            wj[k] = ww[3 * j + k];
        }
        const double mi = A.p.mass[i], mj = A.p.mass[j];
        mstar = mi * mj / (mi + mj);
    }
    // the tangential displacement the pair carried out of the last substep
    double h[3] = {0.0, 0.0, 0.0};
    const long long at = same_list ? s : find_prev(B, key, nprev);
    if (at >= 0)
        for (int k = 0; k < 3; ++k) h[k] = B.prev_hist[3 * at + k];
    const LawCoeffs c = law_coeffs(A, G, wall, mstar);
    const double* n = G.en;
    double d[3], lever[3], spin[3], u[3];
    for (int k = 0; k < 3; ++k) {
        d[k] = vi[k] - vj[k];
        lever[k] = G.rhoi * wi[k] + G.rhoj * wj[k];
    }
    cross3(lever, n, spin);
    for (int k = 0; k < 3; ++k) u[k] = d[k] - spin[k];
    const double fnorm = c.kn * G.delta - c.gn * dot3(d, n);
    const double un = dot3(u, n), hn = dot3(h, n);
    double ut[3], xi[3], ft[3];
    for (int k = 0; k < 3; ++k) {
        ut[k] = u[k] - un * n[k];
        xi[k] = (h[k] - hn * n[k]) + ut[k] * dth;
    }
    for (int k = 0; k < 3; ++k) ft[k] = -c.kt * xi[k] - c.gt * ut[k];
    coulomb_limit(c, A.mu * fabs(fnorm), ut, ft, xi);
    for (int k = 0; k < 3; ++k) {
        out_f[k] = fnorm * n[k] + ft[k];
        out_h[k] = xi[k];
    }
    if (G.sphere_law) {
        double t[3];
        cross3(n, ft, t);
        for (int k = 0; k < 3; ++k) {
            out_mi[k] = -G.rhoi * t[k];
            out_mj[k] = wall ? 0.0 : -G.rhoj * t[k];
        }
    } else {
        const double back[3] = {-out_f[0], -out_f[1], -out_f[2]};
        cross3(G.rci, out_f, out_mi);
        if (wall) out_mj[0] = out_mj[1] = out_mj[2] = 0.0;
        else cross3(G.rcj, back, out_mj);
    }
    return true;
}

__device__ void ph_colhist(const DemArgs& A, const PairBufs& B, long long s) {
    const unsigned j = (unsigned)(B.pairs[s] & 0xffffffffu);
    if (j < (unsigned)A.p.np) atomicAdd(&A.col_count[j], 1);
}

__device__ void ph_colscatter(const DemArgs& A, const PairBufs& B, long long s) {
    const unsigned j = (unsigned)(B.pairs[s] & 0xffffffffu);
    if (j >= (unsigned)A.p.np) return;
    const int slot = atomicAdd(&A.col_fill[j], 1);
    const long long at = (long long)A.col_start[j] + slot;
    if (at < A.pair_cap) A.col_list[at] = (int)s;
}

__device__ void ph_colsort(const DemArgs& A, int j) {
    const int s0 = A.col_start[j], s1 = A.col_start[j + 1];
    for (int u = s0 + 1; u < s1; ++u)
        for (int v = u; v > s0 && A.col_list[v] < A.col_list[v - 1]; --v) {
            int t = A.col_list[v];
            A.col_list[v] = A.col_list[v - 1];
            A.col_list[v - 1] = t;
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
// Verlet predictor (Sec. 2.2): x += v dt + a dt^2/2, v^p = v + a dt,
// w^p = w + alpha dt, quaternion advanced by a midpoint step of q' = q (0, w)/2
// and renormalised.  Every input is loaded before the first store; the new
// position and orientation then give the particle's registration cells.
// one particle's integration state as the predictor reads it
struct PredIn {
    double x[3], v[3], a[3], w[3], al[3], q[4], sm[3];
    int shape;
};

__device__ inline void pred_load(const DemArgs& A, int k, PredIn& s) {
    s.shape = A.p.shape[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        s.x[c] = A.p.pos[3 * k + c];
        s.v[c] = A.p.v[3 * k + c];
        s.a[c] = A.p.a[3 * k + c];
        s.w[c] = A.p.w[3 * k + c];
        s.al[c] = A.p.al[3 * k + c];
        s.sm[c] = A.p.semi[3 * k + c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) s.q[c] = A.p.q[4 * k + c];
}

// The predictor on a loaded state: stores the new position, predicted
// velocities and orientation (and the previous one), and leaves the new
// position and orientation in s; q0 receives the orientation it started from.
__device__ inline void pred_core(const DemArgs& A, int k, double dt, int write_kin, PredIn& s, AxCells& cells,
                                 double* disp, double* q0) {
    const double hdt2 = 0.5 * dt * dt;
    double xn[3], vp[3], wp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double y = (s.x[c] + dt * s.v[c]) + hdt2 * s.a[c];
        if (A.g.periodic[c]) {
            double L = A.L[c];
            if (y >= L) y -= L;
            else if (y < 0.0) y += L;
            if (y == L) y = 0.0;
        }
        xn[c] = y;
        vp[c] = s.v[c] + dt * s.a[c];
        wp[c] = s.w[c] + dt * s.al[c];
    }
    // a centre that is not finite or more than a box length outside: blown up
    if (!(xn[0] >= -A.L[0] && xn[0] < 2.0 * A.L[0] && xn[1] >= -A.L[1] && xn[1] < 2.0 * A.L[1] &&
          xn[2] >= -A.L[2] && xn[2] < 2.0 * A.L[2]))
        atomicOr(&A.ctr->flags, (unsigned long long)PSM_FLAG_UNSTABLE);
    double r1[4], qs[4], qm[4], r2[4], qn[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) q0[c] = s.q[c];
    quat_rate(s.w, q0, r1);
    for (int c = 0; c < 4; ++c) qs[c] = q0[c] + dt * r1[c];
    for (int c = 0; c < 4; ++c) qm[c] = 0.5 * (q0[c] + qs[c]);
    quat_rate(s.w, qm, r2);
    for (int c = 0; c < 4; ++c) qn[c] = q0[c] + dt * r2[c];
    double l = sqrt((qn[0] * qn[0] + qn[1] * qn[1]) + (qn[2] * qn[2] + qn[3] * qn[3]));
    for (int c = 0; c < 4; ++c) qn[c] = qn[c] / l;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        A.p.pos[3 * k + c] = xn[c];
        A.p.vp[3 * k + c] = vp[c];
        A.p.wp[3 * k + c] = wp[c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        A.p.qold[4 * k + c] = q0[c];
        A.p.q[4 * k + c] = qn[c];
    }
    if (write_kin) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            A.p.kin[9 * k + c] = xn[c];
            A.p.kin[9 * k + 3 + c] = vp[c];
            A.p.kin[9 * k + 6 + c] = wp[c];
        }
    }
    double e[3];
    half_extents_of(s.shape, s.sm, qn, e);
    axis_cells_at(A, xn, e, cells);
    // an upper bound of the distance moved (L1 norm of the exact step)
    if (disp) {
        double d = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) d += fabs(dt * s.v[c]) + fabs(hdt2 * s.a[c]);
        *disp = d;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) s.x[c] = xn[c];
#pragma unroll
    for (int c = 0; c < 4; ++c) s.q[c] = qn[c];
}

__device__ void ph_predict(const DemArgs& A, int k, double dt, int write_kin, AxCells& cells,
                           double* disp = nullptr, double* xo = nullptr) {
    PredIn s;
    pred_load(A, k, s);
    double q0[4];
    pred_core(A, k, dt, write_kin, s, cells, disp, q0);
    if (xo)
#pragma unroll
        for (int c = 0; c < 3; ++c) xo[c] = s.x[c];
}

// alpha = Rbw I^-1 [Rbw^T M - (Rbw^T w) x (I Rbw^T w)] at the substep start (as printed)
__device__ void angular_accel_I(const double* I, const double* qo, const double* w, const double* M, double* al) {
    double R[9];
    quat_rbw(qo, R);
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

__device__ inline void angular_accel(const DemArgs& A, int k, const double* qo, const double* w, const double* M,
                                     double* al) {
    angular_accel_I(A.p.inertia + 3 * k, qo, w, M, al);
}

// corrector: a_new = (F_dem + F_hyd + F_ext)/m, F_ext = m (1 - rho0/rho_p) g;
// v += dt/2 (a + a_new); w += dt/2 (alpha + alpha_new)
// the corrector's inputs that stay fixed over the substeps of a step
struct CorrConst {
    double fh[3], mh[3], I[3];
    double m, dens;
    int fixed;
};

__device__ inline void corr_load_const(const DemArgs& A, int k, CorrConst& c) {
    c.fixed = A.p.fixed[k];
    c.m = A.p.mass[k];
    c.dens = A.p.dens[k];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        c.fh[q] = A.p.fh[3 * k + q];
        c.mh[q] = A.p.mh[3 * k + q];
        c.I[q] = A.p.inertia[3 * k + q];
    }
}

// The corrector on loaded values: v, a, w, al are read and replaced by the
// corrected ones, which are also stored.
__device__ inline void corr_core(const DemArgs& A, int k, double dt, const CorrConst& cc, const double* fd,
                                 const double* md, const double* qo, double* v, double* a, double* w, double* al) {
    if (cc.fixed) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            A.p.a[3 * k + c] = A.p.al[3 * k + c] = 0.0;
            a[c] = al[c] = 0.0;
        }
        return;
    }
    const double m = cc.m;
    const double fb = 1.0 - 1.0 / cc.dens;
    double M[3], an[3], aln[3];
    for (int c = 0; c < 3; ++c) {
        double fext = m * fb * A.gravity[c];
        an[c] = ((fd[c] + cc.fh[c]) + fext) / m;
        M[c] = md[c] + cc.mh[c];
    }
    angular_accel_I(cc.I, qo, w, M, aln);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        v[c] = v[c] + 0.5 * dt * (a[c] + an[c]);
        a[c] = an[c];
        w[c] = w[c] + 0.5 * dt * (al[c] + aln[c]);
        al[c] = aln[c];
        A.p.v[3 * k + c] = v[c];
        A.p.a[3 * k + c] = a[c];
        A.p.w[3 * k + c] = w[c];
        A.p.al[3 * k + c] = al[c];
    }
}

__device__ void ph_correct(const DemArgs& A, int k, double dt) {
    CorrConst cc;
    corr_load_const(A, k, cc);
    double fd[3], md[3], a[3], al[3], v[3], w[3], qo[4];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        fd[c] = A.p.fd[3 * k + c];
        md[c] = A.p.md[3 * k + c];
        a[c] = A.p.a[3 * k + c];
        al[c] = A.p.al[3 * k + c];
        v[c] = A.p.v[3 * k + c];
        w[c] = A.p.w[3 * k + c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) qo[c] = A.p.qold[4 * k + c];
    corr_core(A, k, dt, cc, fd, md, qo, v, a, w, al);
}

// initial accelerations a(0) = (F_dem(0) + F_ext)/m, alpha(0) from M_dem(0)
__device__ void ph_initial_accel(const DemArgs& A, int k) {
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


// ---------------------------------------------------------------------------
// kernels of the multi-launch path
// ---------------------------------------------------------------------------
#define GRID_LOOP(i, n) for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)

__global__ void k_predict(DemArgs A, double dt, int write_kin) {
    GRID_LOOP(k, A.p.np) {
        AxCells r;
        ph_predict(A, (int)k, dt, write_kin, r);
        store_cells(A, (int)k, r);
    }
}

// Multi-launch substeps keep the pair list while it is unchanged: the
// predictor also compares each particle's new cells and wall candidates with
// the stored ones (those of the last substep, so of the list) and raises
// list_flag[par]; the launch clears the other parity's flag for the next
// substep (every reader of it has finished: launches run in stream order).
__device__ inline void predict_keep_one(const DemArgs& A, int kk, double dt, int write_kin, int par) {
    const int* d = A.pc + 8 * kk;
    unsigned old[4];
#pragma unroll
    for (int a = 0; a < 3; ++a) old[a] = (unsigned)d[2 * a] | ((unsigned)d[2 * a + 1] << 16);
    old[3] = (unsigned)d[7];
    const double rbk = A.p.rb[kk];
    AxCells r;
    double xk[3];
    ph_predict(A, kk, dt, write_kin, r, nullptr, xk);
    store_cells(A, kk, r);
    unsigned wm = 0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int a = f / 2;
        const double wd = (f % 2 == 0) ? xk[a] : A.L[a] - xk[a];
        wm |= (A.g.bc[f] != 0 && wd < rbk) ? 1u << f : 0u;
    }
    A.pc[8 * kk + 7] = (int)wm;
    bool ch = wm != old[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) ch |= ((unsigned)r.c[a][0] | ((unsigned)r.c[a][1] << 16)) != old[a];
    if (ch) atomicOr(&A.list_flag[par], 1);
}

__global__ void k_predict_keep(DemArgs A, double dt, int write_kin, int par) {
    if (blockIdx.x == 0 && threadIdx.x == 0) A.list_flag[par ^ 1] = 0;
    GRID_LOOP(k, A.p.np) predict_keep_one(A, (int)k, dt, write_kin, par);
}

#define SUM_CHUNK 8

// The DEM sums of a substep, its corrector and the next substep's predictor,
// one thread per particle: the sums take the particle's column (pairs (k, i),
// ascending k), then its row, pairs in contact only, in the order of
// k_sum_wave; block 0 also clears the contacts' deferral queue (as k_sum_wave
// does) and the current parity's list flag (as k_predict_keep does).
__global__ __launch_bounds__(256) void k_sum_correct_predict(DemArgs A, PairBufs B, double dt, int write_kin,
                                                             int par) {
    if (blockIdx.x == 0 && threadIdx.x == 0) A.list_flag[par ^ 1] = 0;
    if (A.ell_cnt && blockIdx.x == 0 && threadIdx.x < DEM_ELL_SEGS) A.ell_cnt[threadIdx.x] = 0;
    const long long cap = A.pair_cap;
    GRID_LOOP(k, A.p.np) {
        const int i = (int)k;
        const long long c0 = A.col_start[i], c1 = A.col_start[i + 1];
        const long long s0 = B.prow[i];
        long long s1 = B.prow[i + 1];
        s1 = s1 < cap ? s1 : cap;
        double F[3] = {0.0, 0.0, 0.0}, M[3] = {0.0, 0.0, 0.0};
        // entries in chunks of SUM_CHUNK: the chunk's pair indices and contact
        // flags are loaded together, then the pairs in contact are added in
        // entry order (a flag per iteration would wait on each load in turn)
        for (long long u0 = c0; u0 < c1; u0 += SUM_CHUNK) {
            int sidx[SUM_CHUNK];
            unsigned char fl[SUM_CHUNK];
#pragma unroll
            for (int q = 0; q < SUM_CHUNK; ++q) sidx[q] = u0 + q < c1 ? A.col_list[u0 + q] : -1;
#pragma unroll
            for (int q = 0; q < SUM_CHUNK; ++q) fl[q] = sidx[q] >= 0 ? A.incontact[sidx[q]] : (unsigned char)0;
#pragma unroll
            for (int q = 0; q < SUM_CHUNK; ++q)
                if (fl[q] & 1) {
                    const long long s = sidx[q];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        F[c] -= A.cF[3 * s + c];
                        M[c] += A.cMj[3 * s + c];
                    }
                }
        }
        for (long long t0 = s0; t0 < s1; t0 += SUM_CHUNK) {
            unsigned char fl[SUM_CHUNK];
#pragma unroll
            for (int q = 0; q < SUM_CHUNK; ++q) fl[q] = t0 + q < s1 ? A.incontact[t0 + q] : (unsigned char)0;
#pragma unroll
            for (int q = 0; q < SUM_CHUNK; ++q)
                if (fl[q] & 1) {
                    const long long s = t0 + q;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        F[c] += A.cF[3 * s + c];
                        M[c] += A.cMi[3 * s + c];
                    }
                }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            A.p.fd[3 * i + c] = F[c];
            A.p.md[3 * i + c] = M[c];
        }
        ph_correct(A, i, dt);
        predict_keep_one(A, i, dt, write_kin, par);
    }
}

// The substep's decision, then its list work: a rebuild (something changed,
// or no list is kept) runs the cell histogram; one substep after a rebuild
// the kept list is copied into this buffer.  The list age has a word per
// substep parity: a substep reads the other parity's and writes its own, so
// every block reads the same age.  Block 0 writes the decision into
// list_flag[par] for the gated kernels that follow; the flag only rises to
// the decision itself, so a block that reads it after that write decides
// the same.
__global__ void k_list_decide(DemArgs A, PairBufs B, int par) {
    const int age = A.fused_age[par ^ 1];
    const int ch = A.list_flag[par] != 0 || age < 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        A.list_flag[par] = ch;
        A.fused_age[par] = ch ? 0 : age + 1;
    }
    if (ch) {
        GRID_LOOP(k, A.p.np) ph_hist(A, (int)k);
        GRID_LOOP(u, (long long)A.p.np / DEM_ROWS_PER_WG + 2) A.row_lb[u] = 0ull;  // k_rows' tickets, status
        return;
    }
    if (age != 0) return;
    long long n = *B.prev_n;
    n = n < A.pair_cap ? n : A.pair_cap;
    const int* prev_prow = B.prev_n - A.p.np;
    GRID_LOOP(u, n) B.pairs[u] = B.prev_pairs[u];
    GRID_LOOP(u, (long long)A.p.np + 1) B.prow[u] = prev_prow[u];
}
__global__ void k_cells(DemArgs A) { GRID_LOOP(k, A.p.np) ph_cells(A, (int)k); }
__global__ void k_hist(DemArgs A) {
    if (A.list_run && !*A.list_run) return;
    GRID_LOOP(k, A.p.np) ph_hist(A, (int)k);
    GRID_LOOP(u, (long long)A.p.np / DEM_ROWS_PER_WG + 2) A.row_lb[u] = 0ull;  // k_rows' tickets, status
}
// The scatter fills each cell's list in arrival order; the rows rank their
// partners by index, so nothing on the path needs the lists ordered.  The
// scan has consumed the cell counts: they are cleared here for the next list
// build (the fill counters by the rows kernel).
__global__ void k_scatter(DemArgs A) {
    if (A.list_run && !*A.list_run) return;
    GRID_LOOP(k, A.p.np) ph_scatter(A, (int)k);
    GRID_LOOP(c, A.ncell) A.cell_count[c] = 0;
}
// each cell's list in ascending particle order (for a read-back of the lists)
__global__ void k_cellsort(DemArgs A) { GRID_LOOP(c, A.ncell) ph_cellsort(A, c); }
// Candidate rows through the cell lists, one wave per particle i: the entries
// of i's registration cells are flattened over the lanes; a lane keeps
// partner j when j > i and the cell is the lowest the two share (each pair
// once).  Emission ranks the kept partners by j (ascending row), then the
// walls follow.
struct WaveCells {
    int start[8], size[8];   // list range of each registration cell (x bit 0, y bit 1, z bit 2)
    int total;
};

__device__ inline void wave_cells(const DemArgs& A, const AxCells& ri, WaveCells& W) {
    W.total = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int xq = q & 1, yq = (q >> 1) & 1, zq = q >> 2;
        int s0 = 0, n = 0;
        if (xq < ri.n[0] && yq < ri.n[1] && zq < ri.n[2]) {
            const long long c = cell_id(A, xq ? ri.c[0][1] : ri.c[0][0], yq ? ri.c[1][1] : ri.c[1][0],
                                        zq ? ri.c[2][1] : ri.c[2][0]);
            s0 = A.cell_start[c];
            n = A.cell_start[c + 1] - s0;
        }
        W.start[q] = s0;
        W.size[q] = n;
        W.total += n;
    }
}

// flat candidate f of i: partner j, or -1 when not kept
__device__ inline int wave_candidate(const DemArgs& A, int i, const AxCells& ri, const WaveCells& W, int f) {
    int q = 0, o = f;
#pragma unroll
    for (int u = 0; u < 7; ++u)
        if (q == u && o >= W.size[u]) {
            o -= W.size[u];
            q = u + 1;
        }
    int st = W.start[0];
#pragma unroll
    for (int u = 1; u < 8; ++u) st = q == u ? W.start[u] : st;
    const long long at = (long long)st + o;
    if (at >= A.reg_cap) return -1;
    const int j = A.cell_pid[at];
    if (j <= i) return -1;
    AxCells rj;
    load_cells(A, j, rj);
    // the cell's coordinates by selects (no indexing of register arrays)
    const int cx = (q & 1) ? ri.c[0][1] : ri.c[0][0];
    const int cy = (q & 2) ? ri.c[1][1] : ri.c[1][0];
    const int cz = (q & 4) ? ri.c[2][1] : ri.c[2][0];
    if (axis_common(ri, rj, 0) != cx || axis_common(ri, rj, 1) != cy || axis_common(ri, rj, 2) != cz) return -1;
    return j;
}


// Rows by groups of ROW_SEG lanes, several particles per wave: a row has a few
// dozen candidates, so a whole wave per row would leave most lanes idle while
// its chain of dependent loads (cells, cell lists, the partners' cells) runs.
#define ROW_SEG 16

// Rows in one pass (counts, offsets, emission).  Workgroups take chunks of
// DEM_ROWS_PER_WG consecutive particles in the order they start (a ticket);
// a group of ROW_SEG lanes finds a row's partners (up to ROW_KEEP kept in LDS),
// the chunk's counts are scanned, and the rows before the chunk come from the
// chunks before it: each publishes its own total and then its running sum in a
// status word (decoupled look-back), so a chunk waits only on chunks that
// started before it.  A wait past its bound raises PSM_FLAG_NEIGH (the step is
// reported as failed) instead of hanging.  Then each row is emitted: partners
// ascending (a partner's place is the number of partners below it), then the
// wall candidates; a row of more than ROW_KEEP partners is gathered again by
// one lane and ordered in place.  Every stored pair with a particle as second
// member counts in that particle's column (the column lists of the DEM sums).
#define ROW_KEEP 32
static_assert(DEM_ROWS_PER_WG == 64, "the chunk scan takes one wave");

__device__ inline unsigned long long row_wait(const unsigned long long* p, bool& ok) {
    unsigned long long v = 0;
    for (unsigned it = 0; ok; ++it) {
        v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v) break;
        if (it > (1u << 22)) ok = false;
        __builtin_amdgcn_s_sleep(1);
    }
    return v;
}

__global__ __launch_bounds__(256) void k_rows(DemArgs A, PairBufs B) {
    if (A.list_run && !*A.list_run) return;
    GRID_LOOP(c, A.ncell) A.cell_fill[c] = 0;  // the scatter's fill counters, for the next list build
    __shared__ int ticket_s;
    __shared__ int cnt_s[DEM_ROWS_PER_WG], wall_s[DEM_ROWS_PER_WG], off_s[DEM_ROWS_PER_WG + 1];
    __shared__ int kept_s[DEM_ROWS_PER_WG][ROW_KEEP];
    __shared__ long long base_s;
    const int tid = threadIdx.x, lane = tid & 63, sl = lane & (ROW_SEG - 1), sh = lane & ~(ROW_SEG - 1);
    const int grp = tid / ROW_SEG, ngrp = 256 / ROW_SEG;
    const unsigned long long seg = ((1ull << ROW_SEG) - 1ull) << sh;
    const unsigned long long lanes_below = ((1ull << sl) - 1ull) << sh;
    const int np = A.p.np;
    unsigned long long* st = A.row_lb;  // [0] tickets, [1 + c] status of chunk c
    if (tid == 0) ticket_s = (int)atomicAdd(&st[0], 1ull);
    __syncthreads();
    const int c = ticket_s;
    const int i0 = c * DEM_ROWS_PER_WG;
    // 1: each row's partners
    for (int r = grp; r < DEM_ROWS_PER_WG; r += ngrp) {
        const int i = i0 + r;
        int nk = 0, nw = 0;
        if (i < np) {
            AxCells ri;
            load_cells(A, i, ri);
            WaveCells W;
            wave_cells(A, ri, W);
            for (int f0 = 0; f0 < W.total; f0 += ROW_SEG) {
                const int f = f0 + sl;
                const int j = f < W.total ? wave_candidate(A, i, ri, W, f) : -1;
                const unsigned long long m = __ballot(j >= 0) & seg;
                const int pos = nk + __popcll(m & lanes_below);
                if (j >= 0 && pos < ROW_KEEP) kept_s[r][pos] = j;
                nk += __popcll(m);
            }
            nw = wall_count(A, i);
        }
        if (sl == 0) {
            cnt_s[r] = nk;
            wall_s[r] = nw;
        }
    }
    __syncthreads();
    // 2: offsets within the chunk
    if (tid < 64) {
        const int v = cnt_s[tid] + wall_s[tid];
        int x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        off_s[tid] = x - v;
        if (tid == 63) off_s[DEM_ROWS_PER_WG] = x;
    }
    __syncthreads();
    // 3: the rows of the chunks before this one
    if (tid == 0) {
        const unsigned long long T = (unsigned long long)off_s[DEM_ROWS_PER_WG];
        const unsigned long long AGG = 1ull << 62, INC = 2ull << 62, VAL = AGG - 1ull;
        long long ex = 0;
        bool ok = true;
        if (c > 0) {
            __hip_atomic_store(&st[1 + c], AGG | T, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int k = c - 1; k >= 0; --k) {
                const unsigned long long v = row_wait(&st[1 + k], ok);
                if (!ok) break;
                ex += (long long)(v & VAL);
                if ((v & ~VAL) == INC) break;
            }
            if (!ok) atomicOr(&A.ctr->flags, (unsigned long long)PSM_FLAG_NEIGH);
        }
        __hip_atomic_store(&st[1 + c], INC | (unsigned long long)(ex + (long long)T), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        base_s = ex;
    }
    __syncthreads();
    const long long base = base_s;
    if (tid < DEM_ROWS_PER_WG && i0 + tid < np) B.prow[i0 + tid] = (int)(base + off_s[tid]);
    if (tid == 0 && i0 + DEM_ROWS_PER_WG >= np) B.prow[np] = (int)(base + off_s[np - i0]);
    // 4: emission
    for (int r = grp; r < DEM_ROWS_PER_WG; r += ngrp) {
        const int i = i0 + r;
        if (i >= np) continue;
        const long long at = base + off_s[r];
        const long long room = A.pair_cap - at;
        const int nk = cnt_s[r];
        if (sl == 0 && room < (long long)(nk + wall_s[r])) atomicOr(&A.ctr->flags, (unsigned long long)PSM_FLAG_PAIRS);
        if (room <= 0) continue;
        unsigned long long* out = B.pairs + at;
        if (nk <= ROW_KEEP) {
            const int* kept = kept_s[r];
            for (int e = sl; e < nk; e += ROW_SEG) {
                const int j = kept[e];
                int below = 0;
                for (int v = 0; v < nk; ++v) below += kept[v] < j ? 1 : 0;
                if (below < room) {
                    out[below] = ((unsigned long long)i << 32) | (unsigned)j;
                    atomicAdd(&A.col_count[j], 1);
                }
            }
            if (sl == 0) emit_walls(A, i, out, room, nk);
        } else if (sl == 0) {
            // a long row: its partners again in cell order, ordered in place
            const int n = pairs_by_cells(A, i, out, room);
            emit_walls(A, i, out, room, n);
            const int m = n < room ? n : (int)room;
            for (int u = 1; u < m; ++u)
                for (int v = u; v > 0 && out[v] < out[v - 1]; --v) {
                    const unsigned long long t = out[v];
                    out[v] = out[v - 1];
                    out[v - 1] = t;
                }
            for (int e = 0; e < m; ++e) atomicAdd(&A.col_count[(int)(out[e] & 0xffffffffu)], 1);
        }
    }
}

// Contacts of the substep's pairs.  With ellipsoids, the pairs that need the
// iterated equivalent spheres (ellipsoid pairs within bounding-sphere reach,
// a small share of the candidates) are queued, one atomic per wave, and
// evaluated by k_contacts_ell with every lane busy: in place they would hold
// most waves for 32 iterations with a few lanes working.  Each pair writes
// only its own outputs, so the queue order does not matter.
template <bool ELL>
__global__ __launch_bounds__(256) void k_contacts(DemArgs A, PairBufs B, const double* vv, const double* ww, double dth) {
    long long nprev = B.prev_n ? *B.prev_n : 0;
    nprev = nprev < A.pair_cap ? nprev : A.pair_cap;
    const long long n = n_pairs(A, B);
    const bool same = A.list_run && !*A.list_run;  // a kept list: history at the pair's own index
    const bool defer = ELL && A.ell_list != nullptr;
    GRID_LOOP(s, n) {
        bool deferred = false;
        ph_contact<ELL>(A, B, s, vv, ww, dth, nprev, same, nullptr, defer ? &deferred : nullptr);
        if (ELL && defer) {
            const unsigned long long m = __ballot(deferred);
            if (m) {
                // the wave's segment: few waves share a counter, so its atomics do not queue up
                const int lane = threadIdx.x & 63, leader = __ffsll((long long)m) - 1;
                const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
                const int seg = (int)(wave % DEM_ELL_SEGS);
                unsigned base = 0;
                if (lane == leader) base = atomicAdd(&A.ell_cnt[seg], (unsigned)__popcll(m));
                base = __shfl(base, leader, 64);
                if (deferred)
                    A.ell_list[seg * A.ell_seg_cap + base + __popcll(m & ((1ull << lane) - 1ull))] = (int)s;
            }
        }
    }
}

// the queued ellipsoid pairs, two lanes each (ellipsoid_pair2), over the
// segments in order (the counters are cleared by k_sum_wave)
__global__ __launch_bounds__(64) void k_contacts_ell(DemArgs A, PairBufs B, const double* vv, const double* ww,
                                                     double dth) {
    __shared__ unsigned start[DEM_ELL_SEGS + 1];
    if (threadIdx.x == 0) {
        unsigned acc = 0;
        for (int g = 0; g < DEM_ELL_SEGS; ++g) {
            start[g] = acc;
            acc += A.ell_cnt[g];
        }
        start[DEM_ELL_SEGS] = acc;
    }
    __syncthreads();
    long long nprev = B.prev_n ? *B.prev_n : 0;
    nprev = nprev < A.pair_cap ? nprev : A.pair_cap;
    const bool same = A.list_run && !*A.list_run;
    // lanes 2q and 2q + 1 take queued pair q (the grid's stride is even, so
    // both lanes of a pair are always in the same pass)
    GRID_LOOP(w2, 2 * (long long)start[DEM_ELL_SEGS]) {
        const unsigned w = (unsigned)(w2 >> 1);
        const int side = (int)(w2 & 1);
        int lo = 0, hi = DEM_ELL_SEGS - 1;  // the segment holding flat index w
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (start[mid] <= w) lo = mid;
            else hi = mid - 1;
        }
        const long long s = (long long)A.ell_list[lo * A.ell_seg_cap + (w - start[lo])];
        const unsigned long long key = B.pairs[s];
        Geom G;
        ellipsoid_pair2(A, (int)(key >> 32), (int)(key & 0xffffffffu), side, G);
        if (side == 0) contact_law(A, B, s, key, G, vv, ww, dth, nprev, same, nullptr);
    }
}
__global__ void k_colhist(DemArgs A, PairBufs B) {
    if (A.list_run && !*A.list_run) return;
    const long long n = n_pairs(A, B);
    GRID_LOOP(s, n) ph_colhist(A, B, s);
}
__global__ void k_colscatter(DemArgs A, PairBufs B) {
    if (A.list_run && !*A.list_run) return;
    const long long n = n_pairs(A, B);
    GRID_LOOP(s, n) ph_colscatter(A, B, s);
}
// Orders each column list (pair indices with second member j) ascending, one
// wave per column: entries are distinct, so an entry's place is the number of
// entries below it; then clears the column's counters for the next build.
__device__ inline void sort_column(const DemArgs& A, int j, int lane) {
    const int s0 = A.col_start[j], n = A.col_start[j + 1] - s0;
    if (n > 64) {
        if (lane == 0) ph_colsort(A, j);
    } else if (n > 1) {
        const int v = lane < n ? A.col_list[s0 + lane] : 0x7fffffff;
        int below = 0;
        for (int u = 0; u < n; ++u) below += __shfl(v, u, 64) < v ? 1 : 0;
        if (lane < n) A.col_list[s0 + below] = v;
    }
    if (lane == 0) {
        A.col_count[j] = 0;
        A.col_fill[j] = 0;
    }
}

__global__ __launch_bounds__(256) void k_colsort(DemArgs A) {
    if (A.list_run && !*A.list_run) return;
    const int lane = threadIdx.x & 63;
    const long long nw = (long long)gridDim.x * (blockDim.x >> 6);
    for (long long jw = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; jw < A.p.np; jw += nw)
        sort_column(A, (int)jw, lane);
}
// F_dem, M_dem of particle i, one wave per particle: pairs (k, i) by ascending
// k (its column list), then its own row, as the pairs are ordered.  The lanes
// fetch the particle's entries
// with their in-contact flags and forces at once; lane 0 adds the terms of
// the pairs in contact in that order.  A pair out of contact holds zero forces,
// whose terms leave a sum unchanged.
// DEM sums of every particle, one wave per particle
__global__ __launch_bounds__(256) void k_sum_wave(DemArgs A, PairBufs B) {
    const int lane = threadIdx.x & 63;
    if (A.ell_cnt && blockIdx.x == 0 && threadIdx.x < DEM_ELL_SEGS)
        A.ell_cnt[threadIdx.x] = 0;  // the contacts' deferral queue, for the next substep
    const long long nw = (long long)gridDim.x * (blockDim.x >> 6);
    const long long cap = A.pair_cap;
    for (long long w = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < A.p.np; w += nw) {
        const int i = (int)w;
        const long long c0 = A.col_start[i], nc = A.col_start[i + 1] - c0;
        const long long s0 = B.prow[i];
        long long s1 = B.prow[i + 1];
        s1 = s1 < cap ? s1 : cap;
        const long long ne = nc + (s1 > s0 ? s1 - s0 : 0);
        double F[3] = {0.0, 0.0, 0.0}, M[3] = {0.0, 0.0, 0.0};
        for (long long b = 0; b < ne; b += 64) {
            const long long e = b + lane;
            double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            bool in = false;
            if (e < ne) {
                const bool col = e < nc;
                const long long s = col ? (long long)A.col_list[c0 + e] : s0 + (e - nc);
                in = (A.incontact[s] & 1) != 0;
                if (in) {
                    const double* Mo = col ? A.cMj : A.cMi;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        v[c] = A.cF[3 * s + c];
                        v[3 + c] = Mo[3 * s + c];
                    }
                }
            }
            for (unsigned long long m = __ballot(in); m; m &= m - 1) {
                const int j = __ffsll((long long)m) - 1;
                double t[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) t[c] = __shfl(v[c], j, 64);
                if (b + j < nc) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        F[c] -= t[c];
                        M[c] += t[3 + c];
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        F[c] += t[c];
                        M[c] += t[3 + c];
                    }
                }
            }
        }
        if (lane == 0)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                A.p.fd[3 * i + c] = F[c];
                A.p.md[3 * i + c] = M[c];
            }
    }
}
__global__ void k_correct(DemArgs A, double dt) { GRID_LOOP(k, A.p.np) ph_correct(A, (int)k, dt); }

// after the LBM-PSM pass: each particle's hydrodynamic sums (one wave), then
// its corrector (lane 0, which stored the sums)
// the hydrodynamic sums and the corrector, HYD_G lanes per particle: the lanes
// fetch HYD_G partials at a time into the group's LDS buffer and the group's
// first lane adds them in emission order (a particle of the multi-launch path
// touches a few tiles, so a whole wave per particle would idle most lanes)
#define HYD_G 16
__global__ __launch_bounds__(256) void k_hydro_correct(DemArgs A, TileArgs T, double dt) {
    __shared__ double buf[256 / HYD_G][HYD_G * 6];
    const int k = (int)(((long long)blockIdx.x * blockDim.x + threadIdx.x) / HYD_G);
    const int lane = threadIdx.x & 63, gl = lane & (HYD_G - 1), sh = lane & ~(HYD_G - 1);
    if (k >= A.p.np) return;
    double* b = buf[threadIdx.x / HYD_G];
    const int e0 = T.voff[k], e1 = T.voff[k + 1];
    double F[3] = {0.0, 0.0, 0.0}, M[3] = {0.0, 0.0, 0.0};
    for (int b0 = e0; b0 < e1 && b0 < T.cap; b0 += HYD_G) {
        const int e = b0 + gl;
        bool ok = false;
        if (e < e1 && e < T.cap) {
            const long long s = T.vinv[e];
            ok = s >= 0 && s < T.cap;
            if (ok)
#pragma unroll
                for (int c = 0; c < 6; ++c) b[6 * gl + c] = T.partial[6 * s + c];
        }
        const unsigned okm = (unsigned)((__ballot(ok) >> sh) & ((1ull << HYD_G) - 1ull));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (gl == 0) {
            const int m = e1 - b0 < HYD_G ? e1 - b0 : HYD_G;
            for (int j = 0; j < m; ++j)
                if ((okm >> j) & 1u)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        F[c] -= b[6 * j + c];
                        M[c] -= b[6 * j + 3 + c];
                    }
        }
        // the buffer is refilled only after the group's first lane has read it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (gl == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            A.p.fh[3 * k + c] = F[c];
            A.p.mh[3 * k + c] = M[c];
        }
        ph_correct(A, k, dt);
    }
}
__global__ void k_initial_accel(DemArgs A) { GRID_LOOP(k, A.p.np) ph_initial_accel(A, (int)k); }

__global__ void k_zero_d(double* p, long long n) { GRID_LOOP(i, n) p[i] = 0.0; }

// ---------------------------------------------------------------------------
// fused single-workgroup substeps
// ---------------------------------------------------------------------------
#define FUSED_T 512

#define FUSED_PREV_LDS 3072   // previous pair keys staged in LDS for the history search
#define FUSED_CELLS 8192      // DEM grids up to this many cells keep their cell list in LDS
#define FUSED_COLS 8192       // pair lists up to this length keep their column lists in LDS
// the saved skip state (bytes): a header (pairs, list age), the column ends,
// separations, movement bounds, column lists and quiet counters
#define FZ_CNT 16
#define FZ_GAP (FZ_CNT + 4 * (DEM_FUSED_MAX + 2))
#define FZ_DACC (FZ_GAP + 8 * FUSED_PREV_LDS)
#define FZ_COL (FZ_DACC + 8 * DEM_FUSED_MAX)
#define FZ_QUIET (FZ_COL + 2 * FUSED_COLS)
#define FZ_BYTES (FZ_QUIET + FUSED_PREV_LDS)
#define FUSED_SKIP_EPS 1e-9   // separation margin above the rounding of positions and distances

__device__ inline unsigned pack_axis(const AxCells& r, int a) {
    return (unsigned)r.c[a][0] | ((unsigned)r.c[a][1] << 16);
}

// the two particles' cells meet along one axis (packed low/high cell pairs)
__device__ inline bool axis_meet(unsigned p, unsigned q) {
    const unsigned p0 = p & 0xffffu, p1 = p >> 16, q0 = q & 0xffffu, q1 = q >> 16;
    return p0 == q0 || p0 == q1 || p1 == q0 || p1 == q1;
}

__device__ inline long long find_key(const unsigned long long* keys, unsigned long long key, long long n) {
    long long lo = 0, hi = n;
    while (lo < hi) {
        long long mid = (lo + hi) >> 1;
        if (keys[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < n && keys[lo] == key) ? lo : -1;
}

// registration cell q (x bit 0, y bit 1, z bit 2) of a particle with packed
// per-axis cells; -1 when that axis has one cell only.  Ascending q is
// ascending cell id.
__device__ inline int reg_cell(const DemArgs& A, unsigned px, unsigned py, unsigned pz, int q) {
    const unsigned x0 = px & 0xffffu, x1 = px >> 16, y0 = py & 0xffffu, y1 = py >> 16, z0 = pz & 0xffffu,
                   z1 = pz >> 16;
    if (((q & 1) && x1 == x0) || ((q & 2) && y1 == y0) || ((q & 4) && z1 == z0)) return -1;
    const int x = (int)((q & 1) ? x1 : x0), y = (int)((q & 2) ? y1 : y0), z = (int)((q & 4) ? z1 : z0);
    return x + A.nc[0] * (y + A.nc[1] * z);
}

// Row of particle i from the LDS cell lists: the partners j > i registered in
// any of i's cells, merged from the (ascending) per-cell lists in ascending j,
// each once.  The head of every cell's list stays in a register; a merge step
// takes the smallest head and advances every list that holds it.  After the
// scatter, cst[c] holds the end of cell c's list and cst[c - 1] its start.
template <bool EMIT>
__device__ int merged_row(const DemArgs& A, int i, const unsigned* cells_s, const int* cst,
                          const unsigned short* cpid, unsigned long long* out, long long room) {
    const unsigned px = cells_s[3 * i], py = cells_s[3 * i + 1], pz = cells_s[3 * i + 2];
    constexpr int NONE = 0x7fffffff;
    int cur[8], end[8], head[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int c = reg_cell(A, px, py, pz, q);
        cur[q] = c > 0 ? cst[c - 1] : 0;
        end[q] = c >= 0 ? cst[c] : 0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) head[q] = cur[q] < end[q] ? (int)cpid[cur[q]] : NONE;
    int n = 0;
    for (;;) {
        int best = head[0];
#pragma unroll
        for (int q = 1; q < 8; ++q) best = head[q] < best ? head[q] : best;
        if (best == NONE) break;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (head[q] == best) {
                ++cur[q];
                head[q] = cur[q] < end[q] ? (int)cpid[cur[q]] : NONE;
            }
        if (best > i) {
            if (EMIT && n < room) out[n] = ((unsigned long long)i << 32) | (unsigned)best;
            ++n;
        }
    }
    return n;
}

// All substeps of a coupled step for up to DEM_FUSED_MAX particles in one
// workgroup, every list in LDS:
//   cells    per-axis cells of each particle, a counting-sorted cell list
//            (ids ascending per cell) when the grid has at most FUSED_CELLS cells;
//   rows     partners j > i merged from i's cell lists (ascending, unique), then
//            wall candidates; offsets by a workgroup scan;
//   contacts the previous list's keys in LDS for the history search;
//   sums     column lists (pairs by second member, ascending pair index) built in
//            LDS, then each particle sums its column and its own row.
// Larger grids test every i < j for a shared cell (64 partners per ballot);
// longer pair lists search each (k, i) pair in row k.
// The pair list is a function of the particles' cells and wall candidates
// alone: a substep in which none of them changed keeps the list (and the
// column lists) of the last rebuild.  One substep after a rebuild the list is
// copied into the other buffer; from then on both buffers hold it.  History
// is then found at the pair's own index.
// Sphere pairs of a kept list (up to FUSED_PREV_LDS) also carry their last
// separation and each particle the distance it has moved since (an upper
// bound): a pair out of contact at its last two evaluations whose separation
// exceeds the two particles' movement since by FUSED_SKIP_EPS is still out of
// contact, and its outputs and both history buffers already hold zeros, so it
// is not evaluated again.  These live in the cell-list space, which a kept
// list does not use.
// The list also outlives the launch: A.fused_age records how long it had been
// kept when the launch ended (pc holds the cells, with the wall candidates in
// its last word); the next launch keeps it when nothing changed and rebuilds
// only its LDS state (column lists, staged keys, separations).  Every other
// writer of the lists or particles resets A.fused_age to -1.  For sphere
// lists the launch also saves that LDS state (A.fz, with the list's length and
// age) and the next launch restores it when its list is that one: its first
// substeps then skip quiet pairs and keep the column lists like any later one.
template <bool ELL>
__device__ __attribute__((always_inline)) void dem_fused_body(const DemArgs& A, const PairSet& P, int cur, const int nsub, const double dt,
                               const int stop_before_correct) {
    __shared__ unsigned cells_s[3 * DEM_FUSED_MAX];
    __shared__ int cnt_s[DEM_FUSED_MAX + 1];
    __shared__ __align__(16) int cst_s[FUSED_CELLS + 1];
    __shared__ __align__(16) unsigned short cpid_s[8 * DEM_FUSED_MAX];
    __shared__ unsigned long long prev_s[FUSED_PREV_LDS];
    __shared__ unsigned short col_s[FUSED_COLS];
    __shared__ unsigned char wmask_s[DEM_FUSED_MAX];
    __shared__ unsigned char inc_s[FUSED_COLS];  // pair in contact (lists up to FUSED_COLS)
    const int np = A.p.np, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nw = FUSED_T / 64;
    const unsigned long long lanes_below = (1ull << lane) - 1ull;
    const bool lds_cells = A.ncell <= FUSED_CELLS;
    const int ncell = (int)A.ncell;
    // kept-list state in the cell-list space
    double* gapb_s = reinterpret_cast<double*>(cst_s);                                // [FUSED_PREV_LDS]
    unsigned char* quiet_s = reinterpret_cast<unsigned char*>(cpid_s);                // [FUSED_PREV_LDS]
    double* dacc_s = reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(cpid_s) + 4096);  // [np]
    static_assert(FUSED_PREV_LDS * 8 <= (FUSED_CELLS + 1) * 4, "separations exceed the cell-list space");
    static_assert(FUSED_PREV_LDS <= 4096 && 4096 + DEM_FUSED_MAX * 8 <= 8 * DEM_FUSED_MAX * 2,
                  "movement bounds exceed the cell-list space");
    const int age0 = *A.fused_age;  // the last launch's list age, -1: none
    int age = 0;                     // substeps since the list was last rebuilt
    bool keys_lds = false;           // the kept list's keys are staged in prev_s
    // the last launch's skip state, when it belongs to the list of buffer cur
    bool restored = false;
    if (!ELL && A.fz && age0 >= 0) {
        const int* hdr = reinterpret_cast<const int*>(A.fz);
        long long nk = (cur ? P.prow[1] : P.prow[0])[np];
        nk = nk < A.pair_cap ? nk : A.pair_cap;
        restored = hdr[0] >= 0 && hdr[0] == nk && hdr[1] == age0 && nk <= FUSED_PREV_LDS && nk <= FUSED_COLS;
        if (restored) {
            const unsigned long long* keys = cur ? P.pairs[1] : P.pairs[0];
            const int* zc = reinterpret_cast<const int*>(A.fz + FZ_CNT);
            const double* zg = reinterpret_cast<const double*>(A.fz + FZ_GAP);
            const double* zd = reinterpret_cast<const double*>(A.fz + FZ_DACC);
            const unsigned short* zl = reinterpret_cast<const unsigned short*>(A.fz + FZ_COL);
            const unsigned char* zq = A.fz + FZ_QUIET;
            for (int k = tid; k <= np; k += FUSED_T) cnt_s[k] = zc[k];
            for (int k = tid; k < np; k += FUSED_T) dacc_s[k] = zd[k];
            for (int s = tid; s < (int)nk; s += FUSED_T) {
                prev_s[s] = keys[s];
                gapb_s[s] = zg[s];
                quiet_s[s] = zq[s];
                col_s[s] = zl[s];
            }
            keys_lds = true;
        }
    }
    long long save_n = -1;  // the last substep's list length when its skip state is complete
    // With at most one particle per thread (and LDS column lists) each thread
    // runs its particle's sums, corrector and next predictor back to back on
    // the state it holds in registers: no barrier and no load between them
    // (the same arithmetic as the stored-state path).
    // Predictor of particle k for substep psub on its loaded state; returns
    // whether its cells or wall candidates differ from those the kept list
    // was built from.
    auto predict_k = [&](int k, int psub, PredIn& st, double rbk, double* q0) __attribute__((always_inline)) -> int {
        unsigned old[4];
        if (psub == 0) {
            const int* d = A.pc + 8 * k;
#pragma unroll
            for (int a = 0; a < 3; ++a) old[a] = (unsigned)d[2 * a] | ((unsigned)d[2 * a + 1] << 16);
            old[3] = (unsigned)d[7];
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) old[a] = cells_s[3 * k + a];
            old[3] = wmask_s[k];
        }
        const int pl = psub == nsub - 1 ? 1 : 0;
        AxCells r;
        double dsp;
        pred_core(A, k, dt, pl, st, r, &dsp, q0);
        const double xk[3] = {st.x[0], st.x[1], st.x[2]};
        if (!ELL) dacc_s[k] += dsp;  // reset by the first substep, which starts fresh
        store_cells(A, k, r);
        unsigned wm = 0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int a = f / 2;
            const double wd = (f % 2 == 0) ? xk[a] : A.L[a] - xk[a];
            wm |= (A.g.bc[f] != 0 && wd < rbk) ? 1u << f : 0u;
        }
        A.pc[8 * k + 7] = (int)wm;
        int ch = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const unsigned pk = pack_axis(r, a);
            ch |= pk != old[a];
            cells_s[3 * k + a] = pk;
        }
        ch |= wm != old[3];
        wmask_s[k] = (unsigned char)wm;
        return ch;
    };
    int changed_next = 0;  // predictors of the next substep run after the sums
    bool tail_done = false;  // ... in the previous substep
    // With one particle per thread the thread's particle state stays in
    // registers from its predictor to its corrector and on to the next
    // predictor: every value the corrector and the predictor read back is one
    // they wrote (the hydrodynamic force and the particle constants do not
    // change within a launch).  Its row range is kept while the list is.
    const bool own = np <= FUSED_T;
    PredIn own_ps;
    CorrConst own_cs;
    double own_qo[4], own_rb = 0.0;
    long long own_r0 = 0, own_r1 = 0;
    bool own_rows = false;
    for (int sub = 0; sub < nsub; ++sub) {
        const bool last = sub == nsub - 1;
        const int c = cur ^ 1;
        PairBufs B;
        // buffer pointers by selects (the pair set is not indexed)
        B.pairs = c ? P.pairs[1] : P.pairs[0];
        B.prow = c ? P.prow[1] : P.prow[0];
        B.hist = c ? P.hist[1] : P.hist[0];
        B.prev_pairs = c ? P.pairs[0] : P.pairs[1];
        B.prev_hist = c ? P.hist[0] : P.hist[1];
        const int* prev_prow = c ? P.prow[0] : P.prow[1];
        B.prev_n = prev_prow + np;
        int changed = sub == 0 && age0 < 0;
        if (!tail_done) {
            for (int k = tid; k < np; k += FUSED_T) {
                PredIn st;
                pred_load(A, k, st);
                const double rbk = A.p.rb[k];
                double q0[4];
                changed |= predict_k(k, sub, st, rbk, q0);
                if (own) {
                    own_ps = st;
                    corr_load_const(A, k, own_cs);
#pragma unroll
                    for (int q = 0; q < 4; ++q) own_qo[q] = q0[q];
                    own_rb = rbk;
                }
            }
        } else {
            changed = changed_next;
        }
        const bool rebuild = __syncthreads_or(changed) != 0;
        age = rebuild ? 0 : (sub == 0 ? age0 + 1 : age + 1);
        // LDS state (column lists, staged keys, separations) is built afresh
        // with a new list and at the start of a launch that restored none
        const bool fresh = rebuild || (sub == 0 && !restored);
        if (fresh) keys_lds = false;
        if (rebuild) own_rows = false;
        if (!rebuild) {
            // the previous list is this list: one substep after the rebuild it
            // is copied into this buffer, later this buffer already holds it
            if (age == 1) {
                long long n = *B.prev_n;
                n = n < A.pair_cap ? n : A.pair_cap;
                for (long long u = tid; u < n; u += FUSED_T) B.pairs[u] = B.prev_pairs[u];
                for (int u = tid; u <= np; u += FUSED_T) B.prow[u] = prev_prow[u];
            }
        } else if (lds_cells) {
            // counting sort of the registrations by cell
            for (int u = tid; u <= ncell; u += FUSED_T) cst_s[u] = 0;
            __syncthreads();
            for (int k = tid; k < np; k += FUSED_T) {
                const unsigned px = cells_s[3 * k], py = cells_s[3 * k + 1], pz = cells_s[3 * k + 2];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int cc = reg_cell(A, px, py, pz, q);
                    if (cc >= 0) atomicAdd(&cst_s[cc], 1);
                }
            }
            __syncthreads();
            psm_block_scan<FUSED_T>(cst_s, cst_s, ncell);
            for (int k = tid; k < np; k += FUSED_T) {
                const unsigned px = cells_s[3 * k], py = cells_s[3 * k + 1], pz = cells_s[3 * k + 2];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int cc = reg_cell(A, px, py, pz, q);
                    if (cc >= 0) cpid_s[atomicAdd(&cst_s[cc], 1)] = (unsigned short)k;
                }
            }
            __syncthreads();
            for (int cc = tid; cc < ncell; cc += FUSED_T) {
                const int s0 = cc > 0 ? cst_s[cc - 1] : 0, s1 = cst_s[cc];
                for (int u = s0 + 1; u < s1; ++u)
                    for (int v = u; v > s0 && cpid_s[v] < cpid_s[v - 1]; --v) {
                        const unsigned short t = cpid_s[v];
                        cpid_s[v] = cpid_s[v - 1];
                        cpid_s[v - 1] = t;
                    }
            }
            __syncthreads();
            for (int i = tid; i < np; i += FUSED_T)
                cnt_s[i] = merged_row<false>(A, i, cells_s, cst_s, cpid_s, nullptr, 0) + wall_count(A, i);
        } else {
            // row sizes: partners j > i sharing a cell (64 per ballot), plus walls
            for (int i = wid; i < np; i += nw) {
                const unsigned pi0 = cells_s[3 * i], pi1 = cells_s[3 * i + 1], pi2 = cells_s[3 * i + 2];
                int cnt = 0;
                for (int j0 = i + 1; j0 < np; j0 += 64) {
                    const int j = j0 + lane;
                    const bool ok = j < np && axis_meet(pi0, cells_s[3 * j]) && axis_meet(pi1, cells_s[3 * j + 1]) &&
                                    axis_meet(pi2, cells_s[3 * j + 2]);
                    cnt += __popcll(__ballot(ok));
                }
                if (lane == 0) cnt_s[i] = cnt + wall_count(A, i);
            }
        }
        if (rebuild) {
            __syncthreads();
            psm_block_scan<FUSED_T>(cnt_s, B.prow, np);
            // rows: ascending j, then walls
            if (lds_cells) {
                for (int i = tid; i < np; i += FUSED_T) {
                    const long long at = B.prow[i];
                    const long long room = A.pair_cap - at;
                    long long e = at;
                    if (room > 0) e += merged_row<true>(A, i, cells_s, cst_s, cpid_s, B.pairs + at, room);
                    for (int f = 0; f < 6; ++f)
                        if (A.g.bc[f] != 0 && wall_dist(A, i, f) < A.p.rb[i]) {
                            if (e < A.pair_cap) B.pairs[e] = ((unsigned long long)i << 32) | (unsigned)(np + f);
                            ++e;
                        }
                    if (e > A.pair_cap) atomicOr(&A.ctr->flags, (unsigned long long)PSM_FLAG_PAIRS);
                }
            } else {
                for (int i = wid; i < np; i += nw) {
                    const unsigned pi0 = cells_s[3 * i], pi1 = cells_s[3 * i + 1], pi2 = cells_s[3 * i + 2];
                    long long at = B.prow[i];
                    for (int j0 = i + 1; j0 < np; j0 += 64) {
                        const int j = j0 + lane;
                        const bool ok = j < np && axis_meet(pi0, cells_s[3 * j]) && axis_meet(pi1, cells_s[3 * j + 1]) &&
                                        axis_meet(pi2, cells_s[3 * j + 2]);
                        const unsigned long long m = __ballot(ok);
                        const long long pos = at + __popcll(m & lanes_below);
                        if (ok && pos < A.pair_cap) B.pairs[pos] = ((unsigned long long)i << 32) | (unsigned)j;
                        at += __popcll(m);
                    }
                    if (lane == 0) {
                        for (int f = 0; f < 6; ++f)
                            if (A.g.bc[f] != 0 && wall_dist(A, i, f) < A.p.rb[i]) {
                                if (at < A.pair_cap) B.pairs[at] = ((unsigned long long)i << 32) | (unsigned)(np + f);
                                ++at;
                            }
                        if (at > A.pair_cap) atomicOr(&A.ctr->flags, (unsigned long long)PSM_FLAG_PAIRS);
                    }
                }
            }
        }
        long long nprev = *B.prev_n;
        nprev = nprev < A.pair_cap ? nprev : A.pair_cap;
        const bool prev_in_lds = rebuild && nprev <= FUSED_PREV_LDS;
        if (prev_in_lds)
            for (long long u = tid; u < nprev; u += FUSED_T) prev_s[u] = B.prev_pairs[u];
        __syncthreads();
        const long long npairs = n_pairs(A, B);
        const bool lds_cols = npairs <= FUSED_COLS;
        {
            PairBufs BL = B;
            if (prev_in_lds) BL.prev_pairs = prev_s;
            if (!rebuild && keys_lds) BL.pairs = prev_s;
            // separations tracked for sphere lists whose keys LDS holds when kept
            const bool track = !ELL && npairs <= FUSED_PREV_LDS;
            const bool skip_ok = track && !fresh && age >= 2 && keys_lds;
            if (fresh && track)
                for (int k = tid; k < np; k += FUSED_T) dacc_s[k] = 0.0;
            for (long long s = tid; s < npairs; s += FUSED_T) {
                int pi = 0, pj = 0;
                if (skip_ok) {
                    const unsigned long long key = prev_s[s];
                    pi = (int)(key >> 32);
                    pj = (int)(key & 0xffffffffu);
                    if (quiet_s[s] >= 2) {
                        const double mv = dacc_s[pi] + (pj < np ? dacc_s[pj] : 0.0);
                        if (gapb_s[s] - mv > FUSED_SKIP_EPS) {
                            if (lds_cols) inc_s[s] = 0;
                            continue;
                        }
                    }
                }
                double gp = 0.0;
                const bool in = ph_contact<ELL>(A, BL, s, A.p.vp, A.p.wp, dt, nprev, !rebuild, track ? &gp : nullptr);
                if (lds_cols) inc_s[s] = in ? 1 : 0;
                if (track) {
                    if (fresh) {
                        quiet_s[s] = in ? 0 : 1;
                        gapb_s[s] = gp;
                    } else {
                        if (!skip_ok) {
                            const unsigned long long key = prev_s[s];
                            pi = (int)(key >> 32);
                            pj = (int)(key & 0xffffffffu);
                        }
                        const int q = quiet_s[s];
                        quiet_s[s] = in ? 0 : (q < 2 ? q + 1 : 2);
                        gapb_s[s] = gp + (dacc_s[pi] + (pj < np ? dacc_s[pj] : 0.0));
                    }
                }
            }
        }
        if (fresh && lds_cols) {
            // column lists: pairs by second member, ascending pair index
            for (int k = tid; k <= np; k += FUSED_T) cnt_s[k] = 0;
            __syncthreads();
            // the history search is done: prev_s takes this list's keys for
            // the substeps that keep it
            keys_lds = npairs <= FUSED_PREV_LDS;
            if (keys_lds)
                for (int s = tid; s < (int)npairs; s += FUSED_T) prev_s[s] = B.pairs[s];
            for (int s = tid; s < (int)npairs; s += FUSED_T) {
                const unsigned j = (unsigned)(B.pairs[s] & 0xffffffffu);
                if (j < (unsigned)np) atomicAdd(&cnt_s[j], 1);
            }
            __syncthreads();
            psm_block_scan<FUSED_T>(cnt_s, cnt_s, np);
            for (int s = tid; s < (int)npairs; s += FUSED_T) {
                const unsigned j = (unsigned)(B.pairs[s] & 0xffffffffu);
                if (j < (unsigned)np) col_s[atomicAdd(&cnt_s[j], 1)] = (unsigned short)s;
            }
            __syncthreads();
            for (int k = tid; k < np; k += FUSED_T) {
                const int s0 = k > 0 ? cnt_s[k - 1] : 0, s1 = cnt_s[k];
                for (int u = s0 + 1; u < s1; ++u)
                    for (int v = u; v > s0 && col_s[v] < col_s[v - 1]; --v) {
                        const unsigned short t = col_s[v];
                        col_s[v] = col_s[v - 1];
                        col_s[v - 1] = t;
                    }
            }
        }
        save_n = (!ELL && lds_cols && keys_lds && npairs <= FUSED_PREV_LDS) ? npairs : -1;
        __syncthreads();
        // DEM sums: pairs (k, i) for ascending k, then the own row
        const bool tail = !ELL && own && lds_cols;  // ellipsoids: registers go to the contacts
        for (int i = tid; i < np; i += FUSED_T) {
            double F[3] = {0.0, 0.0, 0.0}, M[3] = {0.0, 0.0, 0.0};
            if (lds_cols) {
                const int s0 = i > 0 ? cnt_s[i - 1] : 0, s1 = cnt_s[i];
                for (int u = s0; u < s1; ++u) {
                    const long long s = col_s[u];
                    if (!inc_s[s]) continue;  // zero terms leave a sum unchanged
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        F[q] -= A.cF[3 * s + q];
                        M[q] += A.cMj[3 * s + q];
                    }
                }
            } else {
                const unsigned pi0 = cells_s[3 * i], pi1 = cells_s[3 * i + 1], pi2 = cells_s[3 * i + 2];
                for (int k = 0; k < i; ++k) {
                    if (!(axis_meet(pi0, cells_s[3 * k]) && axis_meet(pi1, cells_s[3 * k + 1]) &&
                          axis_meet(pi2, cells_s[3 * k + 2])))
                        continue;
                    const long long lo = B.prow[k];
                    long long hi = B.prow[k + 1];
                    hi = hi < A.pair_cap ? hi : A.pair_cap;
                    if (hi <= lo) continue;
                    const long long s =
                        lo + find_key(B.pairs + lo, ((unsigned long long)k << 32) | (unsigned)i, hi - lo);
                    if (s < lo) continue;
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        F[q] -= A.cF[3 * s + q];
                        M[q] += A.cMj[3 * s + q];
                    }
                }
            }
            if (!own_rows) {
                own_r0 = B.prow[i];
                own_r1 = B.prow[i + 1];
                own_r1 = own_r1 < A.pair_cap ? own_r1 : A.pair_cap;
                own_rows = own;
            }
            for (long long s = own_r0; s < own_r1; ++s) {
                if (lds_cols && !inc_s[s]) continue;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    F[q] += A.cF[3 * s + q];
                    M[q] += A.cMi[3 * s + q];
                }
            }
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                A.p.fd[3 * i + q] = F[q];
                A.p.md[3 * i + q] = M[q];
            }
            if (tail) {
                // this thread's particle: corrector, then the next predictor
                if (!(last && stop_before_correct))
                    corr_core(A, i, dt, own_cs, F, M, own_qo, own_ps.v, own_ps.a, own_ps.w, own_ps.al);
                if (!last) changed_next = predict_k(i, sub + 1, own_ps, own_rb, own_qo);
            }
        }
        if (!tail) {
            __syncthreads();
            if (!(last && stop_before_correct)) {
                for (int k = tid; k < np; k += FUSED_T) ph_correct(A, k, dt);
                __syncthreads();
            }
        }
        tail_done = tail && !last;
        cur = c;
    }
    if (tid == 0 && nsub > 0) *A.fused_age = age;
    if (!ELL && A.fz && nsub > 0) {
        // the kept list's skip state for the next launch
        __syncthreads();
        if (save_n >= 0) {
            int* zc = reinterpret_cast<int*>(A.fz + FZ_CNT);
            double* zg = reinterpret_cast<double*>(A.fz + FZ_GAP);
            double* zd = reinterpret_cast<double*>(A.fz + FZ_DACC);
            unsigned short* zl = reinterpret_cast<unsigned short*>(A.fz + FZ_COL);
            unsigned char* zq = A.fz + FZ_QUIET;
            for (int k = tid; k <= np; k += FUSED_T) zc[k] = cnt_s[k];
            for (int k = tid; k < np; k += FUSED_T) zd[k] = dacc_s[k];
            for (int s = tid; s < (int)save_n; s += FUSED_T) {
                zg[s] = gapb_s[s];
                zq[s] = quiet_s[s];
                zl[s] = col_s[s];
            }
        }
        if (tid == 0) {
            int* hdr = reinterpret_cast<int*>(A.fz);
            hdr[0] = (int)save_n;
            hdr[1] = age;
        }
    }
}

template <bool ELL>
__global__ __launch_bounds__(FUSED_T) void k_dem_fused(DemArgs A, PairSet P, int cur, int nsub, double dt,
                                                       int stop_before_correct) {
    dem_fused_body<ELL>(A, P, cur, nsub, dt, stop_before_correct);
}

// one workgroup per domain of a serving batch: the fused substeps (the last
// one stops before the corrector when the fluid is coupled), or for a domain
// without DEM the kinematics the LBM-PSM pass reads
template <bool ELL>
__global__ __launch_bounds__(FUSED_T) void k_dem_fused_batch(const DemJob* __restrict__ jobs, SrvDyn dyn) {
    const DemJob& J = jobs[blockIdx.x];
    if (J.dem) {
        dem_fused_body<ELL>(J.A, J.P, srv_bit(dyn.cur, blockIdx.x), J.nsub, J.dt, J.fluid);
    } else if (J.fluid) {
        const PartArgs& p = J.A.p;
        for (int k = threadIdx.x; k < p.np; k += FUSED_T)
            for (int c = 0; c < 3; ++c) {
                p.vp[3 * k + c] = p.v[3 * k + c];
                p.wp[3 * k + c] = p.w[3 * k + c];
                p.kin[9 * k + c] = p.pos[3 * k + c];
                p.kin[9 * k + 3 + c] = p.vp[3 * k + c];
                p.kin[9 * k + 6 + c] = p.wp[3 * k + c];
            }
    }
}

// hydrodynamic sums, then the corrector, per particle of each domain
__global__ __launch_bounds__(256) void k_dem_finish_batch(const DemJob* __restrict__ jobs) {
    const DemJob& J = jobs[blockIdx.x];
    if (!J.fluid) return;
    for (int k = threadIdx.x; k < J.A.p.np; k += 256) {
        psm_reduce_hydro(J.t, J.A.p, k);
        if (J.dem) ph_correct(J.A, k, J.dt);
    }
}

inline unsigned nblk(long long n, int t = 256) {
    long long b = (n + t - 1) / t;
    b = b < 1 ? 1 : (b > 65535 ? 65535 : b);
    return (unsigned)b;
}

// The list kernels loop over their items with a grid stride; on the substeps
// that keep the list they return at once, so their grids stay small (a launch
// dispatches every workgroup even when each returns at once).
constexpr unsigned DEM_LIST_GRID_MAX = 512;
inline unsigned nblk_list(long long n) {
    const unsigned b = nblk(n);
    return b < DEM_LIST_GRID_MAX ? b : DEM_LIST_GRID_MAX;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t dem_predict(const DemArgs& A, double dt, int write_kin, hipStream_t s) {
    if (A.p.np == 0) return hipSuccess;
    k_predict<<<nblk(A.p.np), 256, 0, s>>>(A, dt, write_kin);
    return hipGetLastError();
}

hipError_t dem_predict_keep(const DemArgs& A, double dt, int write_kin, int par, hipStream_t s) {
    if (A.p.np == 0) return hipSuccess;
    k_predict_keep<<<nblk(A.p.np), 256, 0, s>>>(A, dt, write_kin, par);
    return hipGetLastError();
}

// the multi-launch list build of a substep, its kernels skipped (on the
// device) when the list is kept; A.list_run is list_flag + par
hipError_t dem_lists_kept(const DemArgs& A, const PairBufs& B, int par, int* scan_tmp, hipStream_t s) {
    if (A.p.np == 0) return hipSuccess;
    hipError_t e;
    k_list_decide<<<nblk_list(A.pair_cap > A.p.np ? A.pair_cap : A.p.np), 256, 0, s>>>(A, B, par);
    if ((e = psm_scan(A.cell_count, A.cell_start, A.ncell, scan_tmp, s, A.list_run)) != hipSuccess) return e;
    k_scatter<<<nblk_list(A.p.np > A.ncell ? A.p.np : A.ncell), 256, 0, s>>>(A);
    k_rows<<<(unsigned)((A.p.np + DEM_ROWS_PER_WG - 1) / DEM_ROWS_PER_WG), 256, 0, s>>>(A, B);
    return hipGetLastError();
}

// the column lists of the current rows from their column counts (counted by
// the row emission, or by dem_count_columns); list_run gates them as the rows
hipError_t dem_columns(const DemArgs& A, const PairBufs& B, int* scan_tmp, hipStream_t s) {
    hipError_t e;
    if ((e = psm_scan(A.col_count, A.col_start, A.p.np, scan_tmp, s, A.list_run)) != hipSuccess) return e;
    k_colscatter<<<nblk_list(A.pair_cap), 256, 0, s>>>(A, B);
    k_colsort<<<nblk_list(64LL * A.p.np), 256, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t dem_lists(const DemArgs& A, const PairBufs& B, int* scan_tmp, hipStream_t s) {
    if (A.p.np == 0) return hipSuccess;
    hipError_t e;
    // the cell and column counters start at zero (creation) and the sort kernels clear them again
    k_cells<<<nblk(A.p.np), 256, 0, s>>>(A);
    k_hist<<<nblk(A.p.np), 256, 0, s>>>(A);
    if ((e = psm_scan(A.cell_count, A.cell_start, A.ncell, scan_tmp, s)) != hipSuccess) return e;
    k_scatter<<<nblk_list(A.p.np > A.ncell ? A.p.np : A.ncell), 256, 0, s>>>(A);
    k_rows<<<(unsigned)((A.p.np + DEM_ROWS_PER_WG - 1) / DEM_ROWS_PER_WG), 256, 0, s>>>(A, B);
    return dem_columns(A, B, scan_tmp, s);
}

hipError_t dem_sort_cells(const DemArgs& A, hipStream_t s) {
    if (A.p.np == 0) return hipSuccess;
    k_cellsort<<<nblk_list(A.ncell), 256, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t dem_count_columns(const DemArgs& A, const PairBufs& B, hipStream_t s) {
    k_colhist<<<nblk_list(A.pair_cap), 256, 0, s>>>(A, B);
    return hipGetLastError();
}

hipError_t dem_contacts(const DemArgs& A, const PairBufs& B, const double* vv, const double* ww, double dth,
                        int* scan_tmp, hipStream_t s, bool sums) {
    if (A.p.np == 0) return hipSuccess;
    // a grid for the pairs the list can hold, capped (the kernel strides over the rest)
    unsigned nbc = nblk(A.pair_cap, 128);
    nbc = nbc < DEM_CONTACT_GRID_MAX ? nbc : DEM_CONTACT_GRID_MAX;
    if (A.ellipsoids) {
        k_contacts<true><<<nbc, 128, 0, s>>>(A, B, vv, ww, dth);
        if (A.ell_list) {
            const unsigned nb = nblk(2 * A.pair_cap, 64);
            k_contacts_ell<<<nb < 4096 ? nb : 4096, 64, 0, s>>>(A, B, vv, ww, dth);
        }
    } else {
        k_contacts<false><<<nbc, 128, 0, s>>>(A, B, vv, ww, dth);
    }
    if (sums) k_sum_wave<<<nblk(64LL * A.p.np), 256, 0, s>>>(A, B);
    return hipGetLastError();
}

hipError_t dem_sums(const DemArgs& A, const PairBufs& B, hipStream_t s) {
    if (A.p.np == 0) return hipSuccess;
    k_sum_wave<<<nblk(64LL * A.p.np), 256, 0, s>>>(A, B);
    return hipGetLastError();
}

hipError_t dem_sum_correct_predict(const DemArgs& A, const PairBufs& B, double dt, int write_kin, int par,
                                   hipStream_t s) {
    if (A.p.np == 0) return hipSuccess;
    k_sum_correct_predict<<<nblk(A.p.np), 256, 0, s>>>(A, B, dt, write_kin, par);
    return hipGetLastError();
}

hipError_t dem_hydro_correct(const DemArgs& A, const TileArgs& T, double dt, hipStream_t s) {
    if (A.p.np == 0) return hipSuccess;
    k_hydro_correct<<<(unsigned)(((long long)HYD_G * A.p.np + 255) / 256), 256, 0, s>>>(A, T, dt);
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

hipError_t dem_fused_batch(const DemJob* jobs, int njobs, const SrvDyn& dyn, int ellipsoids, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    if (ellipsoids) k_dem_fused_batch<true><<<(unsigned)njobs, FUSED_T, 0, s>>>(jobs, dyn);
    else k_dem_fused_batch<false><<<(unsigned)njobs, FUSED_T, 0, s>>>(jobs, dyn);
    return hipGetLastError();
}

hipError_t dem_finish_batch(const DemJob* jobs, int njobs, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    k_dem_finish_batch<<<(unsigned)njobs, 256, 0, s>>>(jobs);
    return hipGetLastError();
}

size_t dem_fused_save_bytes() { return FZ_BYTES; }

hipError_t dem_fused(const DemArgs& A, const PairSet& P, int cur, int nsub, double dt, int stop_before_correct,
                     hipStream_t s) {
    if (A.p.np == 0 || nsub <= 0) return hipSuccess;
    if (A.p.np > DEM_FUSED_MAX || A.nc[0] > 65535 || A.nc[1] > 65535 || A.nc[2] > 65535) return hipErrorInvalidValue;
    if (A.ellipsoids) k_dem_fused<true><<<1, FUSED_T, 0, s>>>(A, P, cur, nsub, dt, stop_before_correct);
    else k_dem_fused<false><<<1, FUSED_T, 0, s>>>(A, P, cur, nsub, dt, stop_before_correct);
    return hipGetLastError();
}
