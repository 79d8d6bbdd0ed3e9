/*
 * oracle.c -- plain FP64 CPU oracle of the coupled LBM-PSM-DEM time step
 * (arXiv 2512.04997, "LEDDS").  TEST INFRASTRUCTURE ONLY: see oracle.h.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -fPIC -shared.
 * Floating point is FP64 throughout; reductions are serial in a fixed order
 * (cells ascending, pairs ascending), so results do not depend on the thread
 * count.
 *
 * Each function cites the passage of the paper it follows (section and
 * equation names).  Where the paper is silent or garbled, the reading taken
 * is named in the comment with a tag Gnn; the same tags are listed in the
 * design notes of the repository.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* D3Q19 lattice (Sec. 2.3, "The lattice Boltzmann method"): textbook weights  */
/* ------------------------------------------------------------------------- */
static const int CX[19] = {0, 1, 0, 0, 1, 1, 1, 1, 0, 0, -1, 0, 0, -1, -1, -1, -1, 0, 0};
static const int CY[19] = {0, 0, 1, 0, 1, -1, 0, 0, 1, 1, 0, -1, 0, -1, 1, 0, 0, -1, -1};
static const int CZ[19] = {0, 0, 0, 1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 0, 0, -1, 1, -1, 1};
static double W[19];
static int OPP[19];

static void lattice_init(void) {
    for (int i = 0; i < 19; ++i) {
        W[i] = (i == 0) ? 1.0 / 3.0 : (((i - 1) % 9) < 3 ? 1.0 / 18.0 : 1.0 / 36.0);
        OPP[i] = (i == 0) ? 0 : (i <= 9 ? i + 9 : i - 9);
    }
}

static char g_err[256];
struct or_domain;
static void dem_initial_accel(struct or_domain* D);
const char* or_error(void) { return g_err; }

/* ------------------------------------------------------------------------- */
/* Domain                                                                      */
/* ------------------------------------------------------------------------- */
struct or_domain {
    or_desc d;
    int64_t N;
    double *f, *fn;
    /* particles */
    int32_t np;
    int32_t* shape;
    uint8_t* fixed;
    double *semi, *dens, *mass, *inertia, *rb;
    double *pos, *q, *qold, *v, *w, *vp, *wp, *a, *al;
    double *fh, *mh, *fd, *md;
    double *fh1, *mh1, *fd1, *md1; /* per-component L1 norms of the summands: per-cell momentum-exchange
                                      terms for F_hyd, M_hyd; pair terms for F_dem, M_dem */
    double *fhr, *mhr, *fhg, *mhg; /* per-component rounding scales of F_hyd, M_hyd (parity bars): the
                                      magnitudes the momentum-exchange terms are formed from, as populations
                                      (fhr, mhr) and as deviations from the weights (fhg, mhg) */
    /* DEM lists */
    int64_t nreg, cap_reg;
    uint64_t* reg;
    int64_t npairs, cap_pairs;
    uint64_t* pairs;
    double* hist;
    double *cF, *cMi, *cMj; /* per pair force on i, torque on i, torque on j */
    uint8_t* incontact;
    int64_t ncontacts;
    /* solids */
    int32_t* slot_pid; /* N * max_solids, -1 empty, ascending pid */
    double* slot_beta;
    int64_t nentries, overflow;
    /* DEM parameters */
    int32_t nc[3];
    double h[3];
    int32_t nsub;
    double dt, beta_e, Rc;
    double ystar, gstar;      /* Hertz: Y* and G* of a contact (App. A), one material */
    int64_t step;
};

static int periodic_axis(const or_domain* D, int a) { return D->d.bc[2 * a] == 0; }
static int extent(const or_domain* D, int a) { return a == 0 ? D->d.nx : (a == 1 ? D->d.ny : D->d.nz); }

/* quaternion (w,x,y,z) -> rotation matrix Rbw (body -> world), row-major.
 * Written with a fixed parenthesisation. */
static void quat_to_rbw(const double* q, double R[9]) {
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

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* c) {
    double c0 = a[1] * b[2] - a[2] * b[1];
    double c1 = a[2] * b[0] - a[0] * b[2];
    double c2 = a[0] * b[1] - a[1] * b[0];
    c[0] = c0; c[1] = c1; c[2] = c2;
}

/* minimum-image difference a - b on periodic axes */
static void min_image(const or_domain* D, const double* a, const double* b, double* d) {
    for (int k = 0; k < 3; ++k) {
        double L = (double)extent(D, k);
        double x = a[k] - b[k];
        if (periodic_axis(D, k)) {
            if (x > 0.5 * L) x -= L;
            else if (x < -0.5 * L) x += L;
        }
        d[k] = x;
    }
}

/* ------------------------------------------------------------------------- */
/* Particle properties: mass, inertia (Sec. 2.2 inertia tensors), bounds      */
/* ------------------------------------------------------------------------- */
static void particle_props(or_domain* D, int k) {
    const double* s = D->semi + 3 * k;
    double V = (D->shape[k] == 0) ? 4.0 / 3.0 * M_PI * s[0] * s[0] * s[0]
                                  : 4.0 / 3.0 * M_PI * s[0] * s[1] * s[2];
    double m = D->dens[k] * D->d.rho0 * V;
    D->mass[k] = m;
    if (D->shape[k] == 0) {
        double I = 0.4 * m * s[0] * s[0];
        D->inertia[3 * k] = D->inertia[3 * k + 1] = D->inertia[3 * k + 2] = I;
        D->rb[k] = s[0];
    } else {
        D->inertia[3 * k + 0] = m / 5.0 * (s[1] * s[1] + s[2] * s[2]);
        D->inertia[3 * k + 1] = m / 5.0 * (s[0] * s[0] + s[2] * s[2]);
        D->inertia[3 * k + 2] = m / 5.0 * (s[0] * s[0] + s[1] * s[1]);
        double r = s[0];
        if (s[1] > r) r = s[1];
        if (s[2] > r) r = s[2];
        D->rb[k] = r;
    }
}

/* Axis-aligned half extents of a particle (sphere: R; ellipsoid: exact box of
 * the rotated ellipsoid, e_x = sqrt(sum_k (a_k Rbw[x][k])^2)). */
static void half_extents(const or_domain* D, int k, double e[3]) {
    const double* s = D->semi + 3 * k;
    if (D->shape[k] == 0) {
        e[0] = e[1] = e[2] = s[0];
        return;
    }
    double R[9];
    quat_to_rbw(D->q + 4 * k, R);
    for (int r = 0; r < 3; ++r) {
        double t0 = s[0] * R[3 * r + 0], t1 = s[1] * R[3 * r + 1], t2 = s[2] * R[3 * r + 2];
        e[r] = sqrt((t0 * t0 + t1 * t1) + t2 * t2);
    }
}

/* ------------------------------------------------------------------------- */
/* Creation                                                                    */
/* ------------------------------------------------------------------------- */
static void* xcalloc(size_t n, size_t s) {
    void* p = calloc(n ? n : 1, s);
    if (!p) {
        fprintf(stderr, "oracle: out of memory\n");
        abort();
    }
    return p;
}

/* n_sub automatic rule (G16): n_sub = max(1, ceil(20 / t_c,min)),
 * t_c = pi sqrt(m*_min / k_n) / sqrt(1 - beta_e^2). */
static int32_t auto_nsub(const or_domain* D) {
    if (D->np == 0 || D->d.kn <= 0.0) return 1;
    double m1 = INFINITY, m2 = INFINITY;
    for (int k = 0; k < D->np; ++k) {
        double m = D->mass[k];
        if (m < m1) { m2 = m1; m1 = m; }
        else if (m < m2) m2 = m;
    }
    double ms = (D->np >= 2) ? m1 * m2 / (m1 + m2) : m1;
    double tc = M_PI * sqrt(ms / D->d.kn) / sqrt(1.0 - D->beta_e * D->beta_e);
    int32_t n = (int32_t)ceil(20.0 / tc);
    return n < 1 ? 1 : n;
}

or_domain* or_create(const or_desc* d, int32_t np, const int32_t* shape, const double* semi,
                     const double* dens, const double* pos, const double* quat, const double* vel,
                     const double* omega, const uint8_t* fixed) {
    lattice_init();
    g_err[0] = 0;
    if (d->nx < 1 || d->ny < 1 || d->nz < 1 || d->tau <= 0.5 || np < 0) {
        snprintf(g_err, sizeof g_err, "invalid lattice or tau");
        return NULL;
    }
    for (int a = 0; a < 3; ++a) {
        int p0 = d->bc[2 * a] == 0, p1 = d->bc[2 * a + 1] == 0;
        if (p0 != p1) {
            snprintf(g_err, sizeof g_err, "axis %d: periodic on one face only", a);
            return NULL;
        }
    }
    if (d->max_solids < 1 || d->max_solids > 4 || d->sf_subdiv < 1) {
        snprintf(g_err, sizeof g_err, "invalid max_solids or sf_subdiv");
        return NULL;
    }
    if (d->collision < 0 || d->collision > 1 || d->trt_magic < 0.0) {
        snprintf(g_err, sizeof g_err, "invalid collision operator");
        return NULL;
    }
    if (d->contact_law < 0 || d->contact_law > 1 ||
        (d->contact_law == 1 && (!(d->young > 0.0) || !(d->poisson >= 0.0 && d->poisson < 0.5)))) {
        snprintf(g_err, sizeof g_err, "invalid contact law or material");
        return NULL;
    }
    if (d->contact_law == 1 && np > 0 && d->dem_on && d->n_sub < 1) {
        snprintf(g_err, sizeof g_err, "the Hertz law needs n_sub >= 1");
        return NULL;
    }
    if (np > 0 && (d->restitution <= 0.0 || d->restitution > 1.0)) {
        snprintf(g_err, sizeof g_err, "restitution must be in (0,1]");
        return NULL;
    }
    or_domain* D = (or_domain*)xcalloc(1, sizeof(or_domain));
    D->d = *d;
    D->N = (int64_t)d->nx * d->ny * d->nz;
    D->np = np;
    D->f = (double*)xcalloc((size_t)(19 * D->N), sizeof(double));
    D->fn = (double*)xcalloc((size_t)(19 * D->N), sizeof(double));
    /* initialisation at equilibrium f = f^eq(rho0, 0) (Sec. 2.3) */
    for (int i = 0; i < 19; ++i)
        for (int64_t c = 0; c < D->N; ++c) D->f[i * D->N + c] = W[i] * d->rho0;

    D->shape = (int32_t*)xcalloc(np, sizeof(int32_t));
    D->fixed = (uint8_t*)xcalloc(np, 1);
#define ALLOC3(p) p = (double*)xcalloc(3 * (size_t)np, sizeof(double))
    ALLOC3(D->semi); ALLOC3(D->inertia); ALLOC3(D->pos); ALLOC3(D->v); ALLOC3(D->w);
    ALLOC3(D->vp); ALLOC3(D->wp); ALLOC3(D->a); ALLOC3(D->al); ALLOC3(D->fh); ALLOC3(D->mh);
    ALLOC3(D->fd); ALLOC3(D->md);
    ALLOC3(D->fh1); ALLOC3(D->mh1); ALLOC3(D->fd1); ALLOC3(D->md1);
    ALLOC3(D->fhr); ALLOC3(D->mhr); ALLOC3(D->fhg); ALLOC3(D->mhg);
#undef ALLOC3
    D->dens = (double*)xcalloc(np, sizeof(double));
    D->mass = (double*)xcalloc(np, sizeof(double));
    D->rb = (double*)xcalloc(np, sizeof(double));
    D->q = (double*)xcalloc(4 * (size_t)np, sizeof(double));
    D->qold = (double*)xcalloc(4 * (size_t)np, sizeof(double));
    double e = d->restitution > 0 ? d->restitution : 1.0;
    D->beta_e = log(e) / sqrt(log(e) * log(e) + M_PI * M_PI); /* App. A */
    if (d->contact_law == 1) {
        /* App. A with both bodies of the one material:
         * Y* = ((1 - nu_i^2)/E_i + (1 - nu_j^2)/E_j)^-1,
         * G* = (2 (2 - nu_i)(1 + nu_i)/E_i + 2 (2 - nu_j)(1 + nu_j)/E_j)^-1 */
        double E = d->young, nu = d->poisson;
        D->ystar = 1.0 / ((1.0 - nu * nu) / E + (1.0 - nu * nu) / E);
        D->gstar = 1.0 / (2.0 * (2.0 - nu) * (1.0 + nu) / E + 2.0 * (2.0 - nu) * (1.0 + nu) / E);
    }
    D->Rc = cbrt(3.0 / (4.0 * M_PI));                          /* Sec. 2.4 distance method */
    double dmax = 0.0;
    for (int k = 0; k < np; ++k) {
        D->shape[k] = shape[k];
        for (int c = 0; c < 3; ++c) {
            D->semi[3 * k + c] = (shape[k] == 0) ? semi[3 * k] : semi[3 * k + c];
            D->pos[3 * k + c] = pos[3 * k + c];
            D->v[3 * k + c] = vel[3 * k + c];
            D->w[3 * k + c] = omega[3 * k + c];
        }
        double qn = sqrt(quat[4 * k] * quat[4 * k] + quat[4 * k + 1] * quat[4 * k + 1] +
                         quat[4 * k + 2] * quat[4 * k + 2] + quat[4 * k + 3] * quat[4 * k + 3]);
        for (int c = 0; c < 4; ++c) D->q[4 * k + c] = quat[4 * k + c] / qn;
        D->dens[k] = dens[k];
        D->fixed[k] = fixed ? fixed[k] : 0;
        particle_props(D, k);
        if (2.0 * D->rb[k] > dmax) dmax = 2.0 * D->rb[k];
        if (d->sf_method == 1 && shape[k] != 0) {
            snprintf(g_err, sizeof g_err, "distance solid fraction is for spheres only");
            or_destroy(D);
            return NULL;
        }
    }
    /* periodic axes must be wide enough for a particle's box not to wrap onto itself */
    for (int a = 0; a < 3; ++a) {
        if (!periodic_axis(D, a)) continue;
        for (int k = 0; k < np; ++k)
            if (2.0 * (D->rb[k] + D->Rc + 1.0) + 1.0 > (double)extent(D, a)) {
                snprintf(g_err, sizeof g_err, "periodic axis %d too short for particle %d", a, k);
                or_destroy(D);
                return NULL;
            }
    }
    /* DEM grid (G31): n_c = floor(L / (1.1 d_max)), h = L / n_c */
    for (int a = 0; a < 3; ++a) {
        double L = (double)extent(D, a);
        int32_t n;
        if (d->dem_cell > 0.0) n = (int32_t)floor(L / d->dem_cell);
        else n = (dmax > 0.0) ? (int32_t)floor(L / (1.1 * dmax)) : 1;
        if (n < 1) n = 1;
        if (np > 0 && periodic_axis(D, a) && n < 2) {
            snprintf(g_err, sizeof g_err, "periodic axis %d has fewer than 2 DEM cells", a);
            or_destroy(D);
            return NULL;
        }
        D->nc[a] = n;
        D->h[a] = L / (double)n;
        /* a particle box must span at most two DEM cells per axis */
        if (n > 1 && !(D->h[a] > dmax)) {
            snprintf(g_err, sizeof g_err, "DEM cell %g smaller than the largest diameter %g", D->h[a], dmax);
            or_destroy(D);
            return NULL;
        }
    }
    D->nsub = d->n_sub > 0 ? d->n_sub : auto_nsub(D);
    D->dt = 1.0 / (double)D->nsub;
    D->slot_pid = (int32_t*)xcalloc((size_t)(D->N * d->max_solids), sizeof(int32_t));
    D->slot_beta = (double*)xcalloc((size_t)(D->N * d->max_solids), sizeof(double));
    for (int64_t c = 0; c < D->N * d->max_solids; ++c) D->slot_pid[c] = -1;
    D->cap_reg = 16;
    D->reg = (uint64_t*)xcalloc(D->cap_reg, sizeof(uint64_t));
    D->cap_pairs = 16;
    D->pairs = (uint64_t*)xcalloc(D->cap_pairs, sizeof(uint64_t));
    D->hist = (double*)xcalloc(3 * D->cap_pairs, sizeof(double));
    D->cF = (double*)xcalloc(3 * D->cap_pairs, sizeof(double));
    D->cMi = (double*)xcalloc(3 * D->cap_pairs, sizeof(double));
    D->cMj = (double*)xcalloc(3 * D->cap_pairs, sizeof(double));
    D->incontact = (uint8_t*)xcalloc(D->cap_pairs, 1);

    /* initial accelerations (G33): a(0) = (F_dem(0) + F_ext)/m with zero history and
     * no history increment; alpha(0) from M_dem(0); F_hyd(0) = 0. */
    dem_initial_accel(D);
    return D;
}

void or_destroy(or_domain* D) {
    if (!D) return;
    free(D->f); free(D->fn); free(D->shape); free(D->fixed); free(D->semi); free(D->dens);
    free(D->mass); free(D->inertia); free(D->rb); free(D->pos); free(D->q); free(D->qold);
    free(D->v); free(D->w); free(D->vp); free(D->wp); free(D->a); free(D->al); free(D->fh);
    free(D->mh); free(D->fd); free(D->md); free(D->reg); free(D->pairs); free(D->hist);
    free(D->cF); free(D->cMi); free(D->cMj); free(D->incontact); free(D->slot_pid);
    free(D->slot_beta);
    free(D->fh1); free(D->mh1); free(D->fd1); free(D->md1);
    free(D->fhr); free(D->mhr); free(D->fhg); free(D->mhg);
    free(D);
}

int32_t or_nsub(const or_domain* D) { return D->nsub; }
void or_dem_grid(const or_domain* D, int32_t nc[3], double h[3]) {
    for (int a = 0; a < 3; ++a) { nc[a] = D->nc[a]; h[a] = D->h[a]; }
}
double or_mass(const or_domain* D, int32_t k) { return D->mass[k]; }

/* ------------------------------------------------------------------------- */
/* Solid fraction (Sec. 2.4, subdivision and distance-based methods)          */
/* ------------------------------------------------------------------------- */

/* Subdivision method, sphere (G5, G27): samples at (X + (2m+1)/(2 ns), ...),
 * strict inside test |s - r_k|^2 < R^2 with a fixed evaluation order. */
double or_beta_subdiv_sphere(double cx, double cy, double cz, double R, int32_t X, int32_t Y,
                             int32_t Z, int32_t ns) {
    double R2 = R * R;
    int64_t cnt = 0;
    for (int c = 0; c < ns; ++c) {
        double oz = (double)(2 * c + 1) / (double)(2 * ns);
        double dz = ((double)Z + oz) - cz;
        for (int b = 0; b < ns; ++b) {
            double oy = (double)(2 * b + 1) / (double)(2 * ns);
            double dy = ((double)Y + oy) - cy;
            for (int a = 0; a < ns; ++a) {
                double ox = (double)(2 * a + 1) / (double)(2 * ns);
                double dx = ((double)X + ox) - cx;
                double r2 = (dx * dx + dy * dy) + dz * dz;
                if (r2 < R2) ++cnt;
            }
        }
    }
    return (double)cnt / (double)((int64_t)ns * ns * ns);
}

/* Subdivision method, ellipsoid: sample s is inside when, with p = Rbw^T (s - c)
 * (each component summed left to right), sum_k (p_k p_k) inv_a2_k < 1. */
static double beta_subdiv_ellipsoid(const double* c, const double* R, const double* ax, int32_t X,
                                    int32_t Y, int32_t Z, int32_t ns) {
    double inv0 = 1.0 / (ax[0] * ax[0]), inv1 = 1.0 / (ax[1] * ax[1]), inv2 = 1.0 / (ax[2] * ax[2]);
    int64_t cnt = 0;
    for (int cc = 0; cc < ns; ++cc) {
        double dz = ((double)Z + (double)(2 * cc + 1) / (double)(2 * ns)) - c[2];
        for (int b = 0; b < ns; ++b) {
            double dy = ((double)Y + (double)(2 * b + 1) / (double)(2 * ns)) - c[1];
            for (int a = 0; a < ns; ++a) {
                double dx = ((double)X + (double)(2 * a + 1) / (double)(2 * ns)) - c[0];
                double p0 = (R[0] * dx + R[3] * dy) + R[6] * dz;
                double p1 = (R[1] * dx + R[4] * dy) + R[7] * dz;
                double p2 = (R[2] * dx + R[5] * dy) + R[8] * dz;
                double s = ((p0 * p0) * inv0 + (p1 * p1) * inv1) + (p2 * p2) * inv2;
                if (s < 1.0) ++cnt;
            }
        }
    }
    return (double)cnt / (double)((int64_t)ns * ns * ns);
}

/* Distance-based method (spheres): delta = R + R_c - |r_k - r_j|, r_j = cell centre
 * (G28), R_c = (3/(4 pi))^(1/3); beta = 0, 1 or delta/(2 R_c). */
double or_beta_distance(double cx, double cy, double cz, double R, int32_t X, int32_t Y, int32_t Z) {
    double Rc = cbrt(3.0 / (4.0 * M_PI));
    double dx = ((double)X + 0.5) - cx, dy = ((double)Y + 0.5) - cy, dz = ((double)Z + 0.5) - cz;
    double dist = sqrt((dx * dx + dy * dy) + dz * dz);
    double delta = (R + Rc) - dist;
    if (delta < 0.0) return 0.0;
    if (delta > 2.0 * Rc) return 1.0;
    return delta / (2.0 * Rc);
}

typedef struct {
    int64_t cell;
    int32_t pid;
    double beta;
} entry_t;

static int entry_cmp(const void* A, const void* B) {
    const entry_t* a = (const entry_t*)A;
    const entry_t* b = (const entry_t*)B;
    if (a->cell != b->cell) return a->cell < b->cell ? -1 : 1;
    if (a->beta != b->beta) return a->beta > b->beta ? -1 : 1; /* larger beta first */
    return a->pid < b->pid ? -1 : (a->pid > b->pid);
}

/* Voxelisation (Table 1, "Compute solid fractions"): for every particle and
 * every lattice cell of its (unwrapped) bounding box, beta_kj; keep per cell the
 * max_solids largest entries, ties to the smaller pid, dropped ones counted
 * (G20); kept slots ordered by pid. */
void or_stage_voxelize(or_domain* D) {
    int ns = D->d.sf_subdiv;
    int np = D->np;
    int64_t* cnt = (int64_t*)xcalloc(np + 1, sizeof(int64_t));
    entry_t** per = (entry_t**)xcalloc(np, sizeof(entry_t*));
    int dims[3] = {D->d.nx, D->d.ny, D->d.nz};
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < np; ++k) {
        double e[3];
        half_extents(D, k, e);
        const double* c = D->pos + 3 * k;
        double R[9];
        quat_to_rbw(D->q + 4 * k, R);
        int32_t lo[3], hi[3];
        /* a centre more than one box length outside the domain (a state that
         * has blown up) or not finite has no entries */
        int far = 0;
        for (int a = 0; a < 3; ++a)
            far |= !(c[a] >= -(double)dims[a] && c[a] < 2.0 * (double)dims[a]);
        if (far) {
            per[k] = NULL;
            cnt[k] = 0;
            continue;
        }
        for (int a = 0; a < 3; ++a) {
            double E = e[a] + 1e-6;
            if (D->d.sf_method == 1) E += D->Rc;
            lo[a] = (int32_t)floor(c[a] - E);
            hi[a] = (int32_t)floor(c[a] + E);
            if (!periodic_axis(D, a)) {
                if (lo[a] < 0) lo[a] = 0;
                if (hi[a] > dims[a] - 1) hi[a] = dims[a] - 1;
            }
        }
        int64_t cap = (int64_t)(hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
        if (cap < 0) cap = 0;
        entry_t* out = (entry_t*)xcalloc(cap, sizeof(entry_t));
        int64_t n = 0;
        for (int32_t Z = lo[2]; Z <= hi[2]; ++Z)
            for (int32_t Y = lo[1]; Y <= hi[1]; ++Y)
                for (int32_t X = lo[0]; X <= hi[0]; ++X) {
                    double beta;
                    if (D->d.sf_method == 1)
                        beta = or_beta_distance(c[0], c[1], c[2], D->semi[3 * k], X, Y, Z);
                    else if (D->shape[k] == 0)
                        beta = or_beta_subdiv_sphere(c[0], c[1], c[2], D->semi[3 * k], X, Y, Z, ns);
                    else
                        beta = beta_subdiv_ellipsoid(c, R, D->semi + 3 * k, X, Y, Z, ns);
                    if (beta > 0.0) {
                        int32_t xw = ((X % dims[0]) + dims[0]) % dims[0];
                        int32_t yw = ((Y % dims[1]) + dims[1]) % dims[1];
                        int32_t zw = ((Z % dims[2]) + dims[2]) % dims[2];
                        out[n].cell = (int64_t)xw + (int64_t)dims[0] * ((int64_t)yw + (int64_t)dims[1] * zw);
                        out[n].pid = k;
                        out[n].beta = beta;
                        ++n;
                    }
                }
        per[k] = out;
        cnt[k] = n;
    }
    int64_t tot = 0;
    for (int k = 0; k < np; ++k) tot += cnt[k];
    entry_t* all = (entry_t*)xcalloc(tot, sizeof(entry_t));
    int64_t o = 0;
    for (int k = 0; k < np; ++k) {
        if (cnt[k]) memcpy(all + o, per[k], cnt[k] * sizeof(entry_t));
        o += cnt[k];
        free(per[k]);
    }
    free(per);
    free(cnt);
    qsort(all, tot, sizeof(entry_t), entry_cmp);
    int ms = D->d.max_solids;
    for (int64_t c = 0; c < D->N * ms; ++c) { D->slot_pid[c] = -1; D->slot_beta[c] = 0.0; }
    D->nentries = tot;
    D->overflow = 0;
    for (int64_t s = 0; s < tot;) {
        int64_t t = s;
        while (t < tot && all[t].cell == all[s].cell) ++t;
        int64_t keep = (t - s) < ms ? (t - s) : ms;
        D->overflow += (t - s) - keep;
        /* order the kept slots by pid (insertion sort on <= 4 items) */
        entry_t kept[4];
        for (int64_t u = 0; u < keep; ++u) kept[u] = all[s + u];
        for (int64_t u = 1; u < keep; ++u)
            for (int64_t v = u; v > 0 && kept[v].pid < kept[v - 1].pid; --v) {
                entry_t tmp = kept[v]; kept[v] = kept[v - 1]; kept[v - 1] = tmp;
            }
        for (int64_t u = 0; u < keep; ++u) {
            D->slot_pid[all[s].cell * ms + u] = kept[u].pid;
            D->slot_beta[all[s].cell * ms + u] = kept[u].beta;
        }
        s = t;
    }
    free(all);
}

int64_t or_get_solid(const or_domain* D, int64_t cap, uint32_t* cell, uint32_t* pid, double* beta) {
    int ms = D->d.max_solids;
    int64_t n = 0;
    for (int64_t c = 0; c < D->N; ++c)
        for (int u = 0; u < ms; ++u) {
            int32_t p = D->slot_pid[c * ms + u];
            if (p < 0) continue;
            if (n < cap) {
                cell[n] = (uint32_t)c;
                pid[n] = (uint32_t)p;
                beta[n] = D->slot_beta[c * ms + u];
            }
            ++n;
        }
    return n;
}

/* ------------------------------------------------------------------------- */
/* LBM with PSM (Sec. 2.3-2.4)                                                 */
/* ------------------------------------------------------------------------- */

/* second-order equilibrium, Eq. (equilibrium), c_s^2 = 1/3 (G1) */
void or_feq(double rho, const double u[3], double feq[19]) {
    if (W[0] == 0.0) lattice_init();
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < 19; ++i) {
        double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
        feq[i] = W[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* B_k = beta (tau - 1/2) / ((1 - beta) + (tau - 1/2)), Eq. (bk) */
static double b_weight(double beta, double tau) {
    return beta * (tau - 0.5) / ((1.0 - beta) + (tau - 0.5));
}

/* Collision of one cell with PSM, Eqs. (psm1), (lbePS) with the BGK fluid
 * operator Eq. (BGK) or the TRT operator Eq. (TRT), and the solid operator
 * Omega^s; Guo forcing (G26) with the
 * (1 - B_tot) factor.  Pk receives B_k sum_i Omega^s_{i,k} c_i per slot.
 * Mk (may be NULL) receives per slot the magnitudes that term is formed from,
 * the bound of its rounding error up to a factor of a few machine epsilons:
 * for component a, B_k [sum_i |c_ia| (|f_ibar| + |feq_ibar(u)| + |f_i| +
 * |feq_i(u_k)|) + sum_i |f_i|] (the last sum for the moments behind u) in
 * Mk[6 s + a], and the same of the deviations from the weights (f - w,
 * f^eq - w), the quantities a shifted storage rounds, in Mk[6 s + 3 + a]. */
static void collide_cell(const or_domain* D, const double f[19], int32_t nslot, const double* B,
                         const double* uk, const double F[3], double fpost[19], double* Pk, double* Mk);

void or_collide_cell(const or_domain* D, const double f[19], int32_t nslot, const double* B,
                     const double* uk, const double F[3], double fpost[19], double* Pk) {
    collide_cell(D, f, nslot, B, uk, F, fpost, Pk, NULL);
}

static void collide_cell(const or_domain* D, const double f[19], int32_t nslot, const double* B,
                         const double* uk, const double F[3], double fpost[19], double* Pk, double* Mk) {
    if (W[0] == 0.0) lattice_init();
    double tau = D->d.tau;
    double rho = 0.0, m[3] = {0, 0, 0};
    for (int i = 0; i < 19; ++i) {
        rho += f[i];
        m[0] += f[i] * CX[i];
        m[1] += f[i] * CY[i];
        m[2] += f[i] * CZ[i];
    }
    int forcing = (F[0] != 0.0 || F[1] != 0.0 || F[2] != 0.0);
    double u[3];
    for (int k = 0; k < 3; ++k) u[k] = (m[k] + (forcing ? 0.5 * F[k] : 0.0)) / rho;
    double feq[19];
    or_feq(rho, u, feq);
    double Bsum = 0.0;
    for (int s = 0; s < nslot; ++s) Bsum += B[s];
    double Btot = Bsum < 1.0 ? Bsum : 1.0; /* Eq. (btot) */
    /* Guo source: w_i [3 (c_i - u) + 9 (c_i . u) c_i] . F, times its relaxation
     * prefactor (BGK) or split below (TRT) */
    double G[19] = {0};
    if (forcing) {
        for (int i = 0; i < 19; ++i) {
            double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
            double t0 = 3.0 * (CX[i] - u[0]) + 9.0 * cu * CX[i];
            double t1 = 3.0 * (CY[i] - u[1]) + 9.0 * cu * CY[i];
            double t2 = 3.0 * (CZ[i] - u[2]) + 9.0 * cu * CZ[i];
            G[i] = t0 * F[0] + t1 * F[1] + t2 * F[2];
        }
    }
    if (D->d.collision == 0) {
        /* BGK, Eq. (BGK); Guo prefactor 1 - 1/(2 tau) */
        double cu_pref = 1.0 - 1.0 / (2.0 * tau);
        for (int i = 0; i < 19; ++i) {
            double Si = cu_pref * W[i] * G[i];
            fpost[i] = f[i] - (1.0 - Btot) * (f[i] - feq[i]) / tau + (1.0 - Btot) * Si;
        }
    } else {
        double S[19];
        for (int i = 0; i < 19; ++i) S[i] = W[i] * G[i];
        /* TRT, Eqs. (trt_populations), (TRT): f+- = (f_i +- f_ibar)/2 and the same
         * split of f^eq relax with dt/tau+ = 1/tau and dt/tau-; the Guo source is
         * split the same way, each part with its own prefactor 1 - (dt/tau+-)/2 */
        double wp = 1.0 / tau, wm;
        if (D->d.trt_magic > 0.0) wm = 1.0 / (D->d.trt_magic / (tau - 0.5) + 0.5);
        else wm = 8.0 * (2.0 - wp) / (8.0 - wp);
        for (int i = 0; i < 19; ++i) {
            int o = OPP[i];
            double fp = 0.5 * (f[i] + f[o]), fm = 0.5 * (f[i] - f[o]);
            double ep = 0.5 * (feq[i] + feq[o]), em = 0.5 * (feq[i] - feq[o]);
            double Sp = 0.5 * (S[i] + S[o]), Sm = 0.5 * (S[i] - S[o]);
            double omega = -wp * (fp - ep) - wm * (fm - em);
            double src = (1.0 - 0.5 * wp) * Sp + (1.0 - 0.5 * wm) * Sm;
            fpost[i] = f[i] + (1.0 - Btot) * omega + (1.0 - Btot) * src;
        }
    }
    for (int s = 0; s < nslot; ++s) {
        double feqk[19];
        or_feq(rho, uk + 3 * s, feqk);
        double P[3] = {0, 0, 0};
        for (int i = 0; i < 19; ++i) {
            int o = OPP[i];
            double Os = (f[o] - feq[o]) - (f[i] - feqk[i]);
            fpost[i] += B[s] * Os;
            P[0] += Os * CX[i];
            P[1] += Os * CY[i];
            P[2] += Os * CZ[i];
        }
        for (int k = 0; k < 3; ++k) Pk[3 * s + k] = B[s] * P[k];
        if (Mk) {
            double a64[3] = {0, 0, 0}, a32[3] = {0, 0, 0}, r64 = 0.0, r32 = 0.0;
            for (int i = 0; i < 19; ++i) {
                int o = OPP[i];
                double m64 = fabs(f[o]) + fabs(feq[o]) + fabs(f[i]) + fabs(feqk[i]);
                double m32 = fabs(f[o] - W[o]) + fabs(feq[o] - W[o]) + fabs(f[i] - W[i]) + fabs(feqk[i] - W[i]);
                const int c[3] = {CX[i], CY[i], CZ[i]};
                for (int k = 0; k < 3; ++k)
                    if (c[k] != 0) {
                        a64[k] += m64;
                        a32[k] += m32;
                    }
                r64 += fabs(f[i]);
                r32 += fabs(f[i] - W[i]);
            }
            for (int k = 0; k < 3; ++k) {
                Mk[6 * s + k] = B[s] * (a64[k] + r64);
                Mk[6 * s + 3 + k] = B[s] * (a32[k] + r32);
            }
        }
    }
}

/* fluid force density at a cell: constant body force plus Kolmogorov sine (G26) */
static void cell_force(const or_domain* D, int x, int y, int z, double F[3]) {
    F[0] = D->d.body_force[0];
    F[1] = D->d.body_force[1];
    F[2] = D->d.body_force[2];
    if (D->d.kolm_amp != 0.0) {
        int ax = D->d.kolm_axis, dir = D->d.kolm_dir;
        int coord = ax == 0 ? x : (ax == 1 ? y : z);
        double L = (double)extent(D, ax);
        F[dir] += D->d.kolm_amp * sin(2.0 * M_PI * ((double)coord + 0.5) / L);
    }
}

/* One LBM step (Eq. collAndStream): collide every cell with PSM, then push the
 * post-collision populations to their neighbours; a link leaving through a
 * walled face is bounced back halfway into the own cell with the moving-wall
 * term -2 w_i rho_w (c_i . u_w)/c_s^2, rho_w = rho0 (G25).  Hydrodynamic force
 * and torque (Eqs. forceSF, torqueSF) are accumulated serially, cells ascending. */
void or_stage_lbm(or_domain* D) {
    const int nx = D->d.nx, ny = D->d.ny, nz = D->d.nz;
    const int64_t N = D->N;
    const int ms = D->d.max_solids;
    double* Pcell = (double*)xcalloc((size_t)(N * ms * 3), sizeof(double));
    double* Tcell = (double*)xcalloc((size_t)(N * ms * 3), sizeof(double));
    /* rounding scales per (cell, slot): force r, torque r, force g, torque g */
    double* Rcell = (double*)xcalloc((size_t)(N * ms * 12), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((int64_t)nx * ny));
        double f[19], fp[19], F[3];
        for (int i = 0; i < 19; ++i) f[i] = D->f[i * N + c];
        cell_force(D, x, y, z, F);
        int32_t nsl = 0;
        double B[4], uk[12], rjk[12];
        for (int u = 0; u < ms; ++u) {
            int32_t p = D->slot_pid[c * ms + u];
            if (p < 0) continue;
            B[nsl] = b_weight(D->slot_beta[c * ms + u], D->d.tau);
            /* solid surface velocity u_k = v_k + w_k x (r_j - r_k) (G4), min image */
            double rj[3] = {x + 0.5, y + 0.5, z + 0.5}, d[3], wx[3];
            min_image(D, rj, D->pos + 3 * p, d);
            cross3(D->wp + 3 * p, d, wx);
            for (int k = 0; k < 3; ++k) {
                uk[3 * nsl + k] = D->vp[3 * p + k] + wx[k];
                rjk[3 * nsl + k] = d[k];
            }
            ++nsl;
        }
        double P[12], M[24];
        collide_cell(D, f, nsl, B, uk, F, fp, P, M);
        for (int s = 0; s < nsl; ++s) {
            double T[3];
            const double* d = rjk + 3 * s;
            cross3(d, P + 3 * s, T);
            for (int k = 0; k < 3; ++k) {
                Pcell[(c * ms + s) * 3 + k] = P[3 * s + k];
                Tcell[(c * ms + s) * 3 + k] = T[k];
            }
            /* a torque component d_a P_b - d_b P_a rounds like |d_a| M_b + |d_b| M_a */
            double* R = Rcell + (c * ms + s) * 12;
            for (int v = 0; v < 2; ++v) {
                const double* m = M + 6 * s + 3 * v;
                for (int k = 0; k < 3; ++k) {
                    int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
                    R[6 * v + k] = m[k];
                    R[6 * v + 3 + k] = fabs(d[k1]) * m[k2] + fabs(d[k2]) * m[k1];
                }
            }
        }
        for (int i = 0; i < 19; ++i) {
            int dst[3] = {x + CX[i], y + CY[i], z + CZ[i]};
            int dims[3] = {nx, ny, nz};
            int hit = -1;
            for (int a = 0; a < 3 && hit < 0; ++a) {
                int face = -1;
                if (dst[a] < 0) face = 2 * a;
                else if (dst[a] >= dims[a]) face = 2 * a + 1;
                if (face < 0) continue;
                if (D->d.bc[face] != 0) hit = face;
            }
            if (hit >= 0) {
                const double* uw = D->d.wall_u[hit];
                double cu = CX[i] * uw[0] + CY[i] * uw[1] + CZ[i] * uw[2];
                double corr = (D->d.bc[hit] == 2) ? 6.0 * W[i] * D->d.rho0 * cu : 0.0;
                D->fn[OPP[i] * N + c] = fp[i] - corr;
            } else {
                for (int a = 0; a < 3; ++a) dst[a] = (dst[a] + dims[a]) % dims[a];
                int64_t dc = dst[0] + (int64_t)nx * (dst[1] + (int64_t)ny * dst[2]);
                D->fn[i * N + dc] = fp[i];
            }
        }
    }
    for (int k = 0; k < 3 * D->np; ++k) {
        D->fh[k] = D->mh[k] = D->fh1[k] = D->mh1[k] = 0.0;
        D->fhr[k] = D->mhr[k] = D->fhg[k] = D->mhg[k] = 0.0;
    }
    for (int64_t c = 0; c < N; ++c) {
        int s = 0;
        for (int u = 0; u < ms; ++u) {
            int32_t p = D->slot_pid[c * ms + u];
            if (p < 0) continue;
            for (int k = 0; k < 3; ++k) {
                D->fh[3 * p + k] -= Pcell[(c * ms + s) * 3 + k];
                D->mh[3 * p + k] -= Tcell[(c * ms + s) * 3 + k];
                D->fh1[3 * p + k] += fabs(Pcell[(c * ms + s) * 3 + k]);
                D->mh1[3 * p + k] += fabs(Tcell[(c * ms + s) * 3 + k]);
                const double* R = Rcell + (c * ms + s) * 12;
                D->fhr[3 * p + k] += R[k];
                D->mhr[3 * p + k] += R[3 + k];
                D->fhg[3 * p + k] += R[6 + k];
                D->mhg[3 * p + k] += R[9 + k];
            }
            ++s;
        }
    }
    free(Pcell);
    free(Tcell);
    free(Rcell);
    double* t = D->f;
    D->f = D->fn;
    D->fn = t;
}

/* ------------------------------------------------------------------------- */
/* DEM: uniform grid, candidate pairs (Sec. 3.2.1, Figs. uniform grid and     */
/* collision scheme)                                                           */
/* ------------------------------------------------------------------------- */
static int u64_cmp(const void* A, const void* B) {
    uint64_t a = *(const uint64_t*)A, b = *(const uint64_t*)B;
    return a < b ? -1 : (a > b);
}

/* Cell index t (an integer-valued double, floor of a coordinate over h) wrapped
 * on a periodic axis (remainder mod n, exact in double) or clamped to
 * [0, n-1] on a walled one.  Done in double so that a position of any finite
 * magnitude maps to a cell without an out-of-range integer conversion; a NaN
 * coordinate maps to cell 0. */
static int32_t wrap_cell(double t, int32_t n, int periodic) {
    if (t != t) return 0;
    if (periodic) {
        double r = fmod(t, (double)n);
        if (r < 0.0) r += (double)n;
        return (int32_t)r;
    }
    if (t < 0.0) return 0;
    if (t > (double)(n - 1)) return n - 1;
    return (int32_t)t;
}

/* DEM cells touched by particle k's axis-aligned box: per axis
 * lo = floor((x - e)/h) .. hi = floor((x + e)/h) (at most two cells, as h
 * exceeds every diameter), wrapped on periodic axes and clamped on walled
 * ones.  Returns the number of cells (<= 8) in out[]. */
static int registrations(const or_domain* D, int k, int64_t* out) {
    double e[3];
    half_extents(D, k, e);
    int32_t list[3][2];
    int nl[3];
    for (int a = 0; a < 3; ++a) {
        double x = D->pos[3 * k + a];
        double lo = floor((x - e[a]) / D->h[a]);
        double hi = floor((x + e[a]) / D->h[a]);
        double cand[2] = {lo, lo + 1.0};
        int nc = hi > lo ? 2 : 1;
        nl[a] = 0;
        for (int u = 0; u < nc; ++u) {
            int32_t cw = wrap_cell(cand[u], D->nc[a], periodic_axis(D, a));
            int dup = 0;
            for (int v = 0; v < nl[a]; ++v) dup |= (list[a][v] == cw);
            if (!dup) list[a][nl[a]++] = cw;
        }
    }
    int n = 0;
    for (int i = 0; i < nl[0]; ++i)
        for (int j = 0; j < nl[1]; ++j)
            for (int l = 0; l < nl[2]; ++l)
                out[n++] = (int64_t)list[0][i] + (int64_t)D->nc[0] * ((int64_t)list[1][j] + (int64_t)D->nc[1] * list[2][l]);
    return n;
}

static void ensure_pairs(or_domain* D, int64_t n) {
    if (n <= D->cap_pairs) return;
    int64_t c = D->cap_pairs;
    while (c < n) c *= 2;
    D->pairs = (uint64_t*)realloc(D->pairs, c * sizeof(uint64_t));
    D->hist = (double*)realloc(D->hist, 3 * c * sizeof(double));
    D->cF = (double*)realloc(D->cF, 3 * c * sizeof(double));
    D->cMi = (double*)realloc(D->cMi, 3 * c * sizeof(double));
    D->cMj = (double*)realloc(D->cMj, 3 * c * sizeof(double));
    D->incontact = (uint8_t*)realloc(D->incontact, c);
    D->cap_pairs = c;
}

/* Builds the sorted registration keys (cell << 32 | pid) and the sorted unique
 * candidate pairs (i << 32 | j), i < j sharing a DEM cell, plus wall
 * candidates (i << 32 | (np + face)) when the centre is closer to a walled face
 * than the bounding radius (walls as static particles, Sec. 2.1).  The new
 * pair list is returned; the caller keeps the previous list for the history. */
static int64_t build_lists(or_domain* D, uint64_t** out_pairs) {
    int np = D->np;
    int64_t ncell = (int64_t)D->nc[0] * D->nc[1] * D->nc[2];
    /* bucket grid: count, then fill (pids ascending within a cell) */
    int64_t* regc = (int64_t*)xcalloc((size_t)np * 27, sizeof(int64_t));
    int* nreg = (int*)xcalloc(np, sizeof(int));
    int64_t tot = 0;
    for (int k = 0; k < np; ++k) {
        nreg[k] = registrations(D, k, regc + 27 * k);
        tot += nreg[k];
    }
    if (tot > D->cap_reg) {
        D->cap_reg = tot;
        D->reg = (uint64_t*)realloc(D->reg, tot * sizeof(uint64_t));
    }
    int64_t* count = (int64_t*)xcalloc(ncell + 1, sizeof(int64_t));
    for (int k = 0; k < np; ++k)
        for (int u = 0; u < nreg[k]; ++u) count[regc[27 * k + u] + 1]++;
    for (int64_t c = 0; c < ncell; ++c) count[c + 1] += count[c];
    int32_t* bucket = (int32_t*)xcalloc(tot, sizeof(int32_t));
    int64_t* fill = (int64_t*)xcalloc(ncell, sizeof(int64_t));
    for (int k = 0; k < np; ++k)
        for (int u = 0; u < nreg[k]; ++u) {
            int64_t c = regc[27 * k + u];
            bucket[count[c] + fill[c]++] = k;
        }
    D->nreg = 0;
    for (int64_t c = 0; c < ncell; ++c)
        for (int64_t s = count[c]; s < count[c + 1]; ++s)
            D->reg[D->nreg++] = ((uint64_t)c << 32) | (uint32_t)bucket[s];
    /* per-cell pairs n(n-1)/2 */
    int64_t npair = 0;
    for (int64_t c = 0; c < ncell; ++c) {
        int64_t n = count[c + 1] - count[c];
        npair += n * (n - 1) / 2;
    }
    int64_t nwall = 0;
    for (int k = 0; k < np; ++k)
        for (int f = 0; f < 6; ++f) nwall += (D->d.bc[f] != 0);
    uint64_t* P = (uint64_t*)xcalloc(npair + nwall, sizeof(uint64_t));
    int64_t o = 0;
    for (int64_t c = 0; c < ncell; ++c)
        for (int64_t s = count[c]; s < count[c + 1]; ++s)
            for (int64_t t = s + 1; t < count[c + 1]; ++t)
                P[o++] = ((uint64_t)bucket[s] << 32) | (uint32_t)bucket[t];
    for (int k = 0; k < np; ++k)
        for (int f = 0; f < 6; ++f) {
            if (D->d.bc[f] == 0) continue;
            int a = f / 2;
            double dist = (f % 2 == 0) ? D->pos[3 * k + a] : (double)extent(D, a) - D->pos[3 * k + a];
            if (dist < D->rb[k]) P[o++] = ((uint64_t)k << 32) | (uint32_t)(np + f);
        }
    qsort(P, o, sizeof(uint64_t), u64_cmp);
    int64_t m = 0;
    for (int64_t s = 0; s < o; ++s)
        if (m == 0 || P[s] != P[m - 1]) P[m++] = P[s];
    free(regc); free(nreg); free(count); free(bucket); free(fill);
    *out_pairs = P;
    return m;
}

void or_stage_lists(or_domain* D) {
    uint64_t* P;
    int64_t n = build_lists(D, &P);
    ensure_pairs(D, n);
    memcpy(D->pairs, P, n * sizeof(uint64_t));
    D->npairs = n;
    free(P);
}

int64_t or_brute_pairs(or_domain* D, int64_t cap, uint64_t* keys) {
    int np = D->np;
    int64_t* rc = (int64_t*)xcalloc((size_t)np * 27, sizeof(int64_t));
    int* nr = (int*)xcalloc(np, sizeof(int));
    for (int k = 0; k < np; ++k) nr[k] = registrations(D, k, rc + 27 * k);
    int64_t n = 0;
    for (int i = 0; i < np; ++i) {
        for (int j = i + 1; j < np; ++j) {
            int share = 0;
            for (int u = 0; u < nr[i] && !share; ++u)
                for (int v = 0; v < nr[j]; ++v)
                    if (rc[27 * i + u] == rc[27 * j + v]) { share = 1; break; }
            if (share) {
                if (n < cap) keys[n] = ((uint64_t)i << 32) | (uint32_t)j;
                ++n;
            }
        }
        for (int f = 0; f < 6; ++f) {
            if (D->d.bc[f] == 0) continue;
            int a = f / 2;
            double dist = (f % 2 == 0) ? D->pos[3 * i + a] : (double)extent(D, a) - D->pos[3 * i + a];
            if (dist < D->rb[i]) {
                if (n < cap) keys[n] = ((uint64_t)i << 32) | (uint32_t)(np + f);
                ++n;
            }
        }
    }
    free(rc);
    free(nr);
    return n;
}

/* ------------------------------------------------------------------------- */
/* Contact geometry (Sec. 2.1)                                                 */
/* ------------------------------------------------------------------------- */

/* local curvature radius, Eq. (local-curvature) (G24), and unit outward normal
 * at surface point p of ellipsoid (c, Rbw, semi-axes ax) */
static void ell_local(const double* c, const double* R, const double* ax, const double* p,
                      double* rho, double* n) {
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

/* intersection of the line s + t u with the ellipsoid surface; the root with
 * the larger t when far_positive, else the smaller; returns 0 on a miss */
static int ell_line_hit(const double* c, const double* R, const double* ax, const double* s,
                        const double* u, int far_positive, double* p) {
    double d[3] = {s[0] - c[0], s[1] - c[1], s[2] - c[2]};
    double y0[3], ud[3];
    for (int k = 0; k < 3; ++k) {
        y0[k] = (R[0 + k] * d[0] + R[3 + k] * d[1]) + R[6 + k] * d[2];
        ud[k] = (R[0 + k] * u[0] + R[3 + k] * u[1]) + R[6 + k] * u[2];
    }
    double A = 0, B = 0, C = -1.0;
    for (int k = 0; k < 3; ++k) {
        double ia = 1.0 / (ax[k] * ax[k]);
        A += ud[k] * ud[k] * ia;
        B += y0[k] * ud[k] * ia;
        C += y0[k] * y0[k] * ia;
    }
    double disc = B * B - A * C;
    if (disc < 0.0 || A <= 0.0) return 0;
    double sq = sqrt(disc);
    double t = far_positive ? (-B + sq) / A : (-B - sq) / A;
    for (int k = 0; k < 3; ++k) p[k] = s[k] + t * u[k];
    return 1;
}

/* Ellipsoid pair contact by iterated equivalent spheres (Sec. 2.1; G23):
 * start where the centre segment crosses each surface; at each point take the
 * curvature radius rho and normal n, sphere centre s = p - rho n; the new
 * points are where the line through both sphere centres leaves each surface
 * towards the other body; stop on |dp_i| + |dp_j| < 1e-10 a_min or 32
 * iterations, or keep the previous points when a line misses.  Then
 * delta = rho_i + rho_j - |s_i - s_j|, e_n = (s_i - s_j)/|s_i - s_j|. */
static int ellipsoid_pair(const or_domain* D, int i, int j, double* delta, double en[3],
                          double rci[3], double rcj[3], double* rhoi_out, double* rhoj_out,
                          int* iters) {
    const double* ci = D->pos + 3 * i;
    double dvec[3];
    min_image(D, ci, D->pos + 3 * j, dvec);
    double cj[3] = {ci[0] - dvec[0], ci[1] - dvec[1], ci[2] - dvec[2]};
    double Ri[9], Rj[9];
    quat_to_rbw(D->q + 4 * i, Ri);
    quat_to_rbw(D->q + 4 * j, Rj);
    const double* ai = D->semi + 3 * i;
    const double* aj = D->semi + 3 * j;
    double amin = ai[0];
    for (int k = 0; k < 3; ++k) {
        if (ai[k] < amin) amin = ai[k];
        if (aj[k] < amin) amin = aj[k];
    }
    double pi[3], pj[3];
    {
        double u[3] = {cj[0] - ci[0], cj[1] - ci[1], cj[2] - ci[2]};
        double l = sqrt(dot3(u, u));
        for (int k = 0; k < 3; ++k) u[k] /= l;
        ell_line_hit(ci, Ri, ai, ci, u, 1, pi);
        double um[3] = {-u[0], -u[1], -u[2]};
        ell_line_hit(cj, Rj, aj, cj, um, 1, pj);
    }
    int it = 0;
    for (; it < 32; ++it) {
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
        if (!ell_line_hit(ci, Ri, ai, si, u, 1, npi)) break;
        if (!ell_line_hit(cj, Rj, aj, sj, u, 0, npj)) break;
        double dpi[3] = {npi[0] - pi[0], npi[1] - pi[1], npi[2] - pi[2]};
        double dpj[3] = {npj[0] - pj[0], npj[1] - pj[1], npj[2] - pj[2]};
        double conv = sqrt(dot3(dpi, dpi)) + sqrt(dot3(dpj, dpj));
        for (int k = 0; k < 3; ++k) { pi[k] = npi[k]; pj[k] = npj[k]; }
        if (conv < 1e-10 * amin) { ++it; break; }
    }
    double rhoi, rhoj, ni[3], nj[3], si[3], sj[3];
    ell_local(ci, Ri, ai, pi, &rhoi, ni);
    ell_local(cj, Rj, aj, pj, &rhoj, nj);
    for (int k = 0; k < 3; ++k) {
        si[k] = pi[k] - rhoi * ni[k];
        sj[k] = pj[k] - rhoj * nj[k];
    }
    double d[3] = {si[0] - sj[0], si[1] - sj[1], si[2] - sj[2]};
    double l = sqrt(dot3(d, d));
    *delta = (rhoi + rhoj) - l;
    for (int k = 0; k < 3; ++k) {
        en[k] = d[k] / l;
        rci[k] = pi[k] - ci[k];
        rcj[k] = pj[k] - cj[k];
    }
    *rhoi_out = rhoi;
    *rhoj_out = rhoj;
    if (iters) *iters = it;
    return 1;
}

/* geometry of pair (i, j): j < np a particle, j >= np the wall face j - np.
 * Returns 1 if the geometry was evaluated (pre-filter passed). */
static int pair_geometry(const or_domain* D, int i, int j, double* delta, double en[3], double rci[3],
                         double rcj[3], double* rhoi, double* rhoj, int* sphere_law, int* iters) {
    int np = D->np;
    if (iters) *iters = 0;
    if (j >= np) {
        /* wall (plane) contact; inward normal n */
        int f = j - np, a = f / 2;
        double n[3] = {0, 0, 0};
        n[a] = (f % 2 == 0) ? 1.0 : -1.0;
        const double* c = D->pos + 3 * i;
        double dist = (f % 2 == 0) ? c[a] : (double)extent(D, a) - c[a];
        for (int k = 0; k < 3; ++k) { en[k] = n[k]; rcj[k] = 0.0; }
        *rhoj = 0.0;
        if (D->shape[i] == 0) {
            double R = D->semi[3 * i];
            *delta = R - dist;
            for (int k = 0; k < 3; ++k) rci[k] = -R * n[k];
            *rhoi = R;
            *sphere_law = 1;
        } else {
            /* deepest point p = c - A n / sqrt(n^T A n), A = Rbw diag(a^2) Rbw^T */
            double R[9];
            quat_to_rbw(D->q + 4 * i, R);
            const double* ax = D->semi + 3 * i;
            double nb[3];
            for (int k = 0; k < 3; ++k) nb[k] = (R[0 + k] * n[0] + R[3 + k] * n[1]) + R[6 + k] * n[2];
            double qf = (ax[0] * ax[0] * nb[0] * nb[0] + ax[1] * ax[1] * nb[1] * nb[1]) +
                        ax[2] * ax[2] * nb[2] * nb[2];
            double sq = sqrt(qf);
            double An_b[3] = {ax[0] * ax[0] * nb[0], ax[1] * ax[1] * nb[1], ax[2] * ax[2] * nb[2]};
            double p[3];
            for (int r = 0; r < 3; ++r) {
                double An = (R[3 * r] * An_b[0] + R[3 * r + 1] * An_b[1]) + R[3 * r + 2] * An_b[2];
                p[r] = c[r] - An / sq;
            }
            *delta = sq - dist;
            double nn[3];
            ell_local(c, R, ax, p, rhoi, nn);
            for (int k = 0; k < 3; ++k) rci[k] = p[k] - c[k];
            *sphere_law = 0;
        }
        return 1;
    }
    double d[3];
    min_image(D, D->pos + 3 * i, D->pos + 3 * j, d);
    double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    if (D->shape[i] == 0 && D->shape[j] == 0) {
        double Ri = D->semi[3 * i], Rj = D->semi[3 * j];
        double dist = sqrt(r2);
        *delta = (Ri + Rj) - dist; /* Eq. (distanceSpheres) */
        for (int k = 0; k < 3; ++k) {
            en[k] = d[k] / dist;
            rci[k] = -Ri * en[k];
            rcj[k] = Rj * en[k];
        }
        *rhoi = Ri;
        *rhoj = Rj;
        *sphere_law = 1;
        return 1;
    }
    /* bounding-sphere pre-filter */
    double rs = D->rb[i] + D->rb[j];
    if (!(r2 < rs * rs)) {
        *delta = -1.0;
        *sphere_law = 0;
        return 0;
    }
    *sphere_law = 0;
    ellipsoid_pair(D, i, j, delta, en, rci, rcj, rhoi, rhoj, iters);
    return 1;
}

int32_t or_contact_geometry(const or_domain* D, int32_t i, int32_t j, double* delta, double en[3],
                            double rci[3], double rcj[3], int32_t* iters) {
    double ri, rj;
    int sl, it = 0;
    int ok = pair_geometry(D, i, j, delta, en, rci, rcj, &ri, &rj, &sl, &it);
    if (iters) *iters = it;
    return ok;
}

/* ------------------------------------------------------------------------- */
/* Contact law: linear spring-dashpot + Coulomb (Sec. 2.1, Eqs. fnScal,       */
/* relative_velocity, trangential-history, coulombCoeff, torque; G2, G3, G22, */
/* G30)                                                                        */
/* ------------------------------------------------------------------------- */
static uint64_t* g_prev_keys;
static double* g_prev_hist;
static int64_t g_prev_n;

static int find_prev(uint64_t key) {
    int64_t lo = 0, hi = g_prev_n;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (g_prev_keys[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < g_prev_n && g_prev_keys[lo] == key) ? (int)lo : -1;
}

/* Evaluates every pair of the current list with the previous list's history
 * (binary search, Sec. 3.2.2), velocities vv/ww, history increment dth, and
 * accumulates F_dem, M_dem in pair order. */
static void dem_contacts(or_domain* D, const double* vv, const double* ww, double dth,
                         const uint64_t* prev_keys, const double* prev_hist, int64_t prev_n) {
    int np = D->np;
    g_prev_keys = (uint64_t*)prev_keys;
    g_prev_hist = (double*)prev_hist;
    g_prev_n = prev_n;
    D->ncontacts = 0;
    for (int k = 0; k < 3 * np; ++k) { D->fd[k] = 0.0; D->md[k] = 0.0; D->fd1[k] = 0.0; D->md1[k] = 0.0; }
    for (int64_t p = 0; p < D->npairs; ++p) {
        uint64_t key = D->pairs[p];
        int i = (int)(key >> 32), j = (int)(key & 0xffffffffu);
        double delta, en[3], rci[3], rcj[3], rhoi, rhoj;
        int sphere_law;
        double kn = D->d.kn, kt = D->d.kt_ratio * D->d.kn;  /* linear law; Hertz below */
        pair_geometry(D, i, j, &delta, en, rci, rcj, &rhoi, &rhoj, &sphere_law, NULL);
        double *F = D->cF + 3 * p, *Mi = D->cMi + 3 * p, *Mj = D->cMj + 3 * p, *h = D->hist + 3 * p;
        if (!(delta > 0.0)) {
            for (int k = 0; k < 3; ++k) F[k] = Mi[k] = Mj[k] = h[k] = 0.0;
            D->incontact[p] = 0;
            continue;
        }
        D->incontact[p] = 1;
        D->ncontacts++;
        double vi[3], wi[3], vj[3], wj[3], mstar;
        for (int k = 0; k < 3; ++k) { vi[k] = vv[3 * i + k]; wi[k] = ww[3 * i + k]; }
        if (j < np) {
            for (int k = 0; k < 3; ++k) { vj[k] = vv[3 * j + k]; wj[k] = ww[3 * j + k]; }
            mstar = D->mass[i] * D->mass[j] / (D->mass[i] + D->mass[j]);
        } else {
            int f = j - np;
            for (int k = 0; k < 3; ++k) {
                vj[k] = (D->d.bc[f] == 2) ? D->d.wall_u[f][k] : 0.0;
                wj[k] = 0.0;
            }
            mstar = D->mass[i];
        }
        double gn, gt;
        if (D->d.contact_law == 1) {
            /* Hertz (App. A): k_n = 4/3 Y* sqrt(R* d), k_t = 8 G* sqrt(R* d),
             * gamma = -2 sqrt(5/6) beta sqrt(S m*), S_n = 2 Y* sqrt(R* d),
             * S_t = 8 G* sqrt(R* d); R* = (1/R_i + 1/R_j)^-1 with the local
             * equivalent-sphere radii; a wall has infinite radius and mass */
            double Rs = (j < np) ? 1.0 / (1.0 / rhoi + 1.0 / rhoj) : rhoi;
            double sq = sqrt(Rs * delta);
            kn = 4.0 / 3.0 * D->ystar * sq;
            kt = 8.0 * D->gstar * sq;
            double Sn = 2.0 * D->ystar * sq, St = 8.0 * D->gstar * sq;
            gn = -2.0 * sqrt(5.0 / 6.0) * D->beta_e * sqrt(Sn * mstar);
            gt = -2.0 * sqrt(5.0 / 6.0) * D->beta_e * sqrt(St * mstar);
        } else {
            gn = -2.0 * D->beta_e * sqrt(kn * mstar);
            gt = D->d.gt_ratio * gn;
        }
        /* normal: F_n = [k_n delta + gamma_n (v_j - v_i).e_n] e_n (G2) */
        double dv[3] = {vj[0] - vi[0], vj[1] - vi[1], vj[2] - vi[2]};
        double fn = kn * delta + gn * dot3(dv, en);
        /* relative surface velocity and its tangential part (G3) */
        double rw[3] = {rhoi * wi[0] + rhoj * wj[0], rhoi * wi[1] + rhoj * wj[1], rhoi * wi[2] + rhoj * wj[2]};
        double cr[3];
        cross3(rw, en, cr);
        double vrel[3] = {(vi[0] - vj[0]) - cr[0], (vi[1] - vj[1]) - cr[1], (vi[2] - vj[2]) - cr[2]};
        double vrn = dot3(vrel, en);
        double vt[3] = {vrel[0] - vrn * en[0], vrel[1] - vrn * en[1], vrel[2] - vrn * en[2]};
        /* tangential history: project the previous displacement, then integrate (G22) */
        double ho[3] = {0, 0, 0};
        int pi_ = find_prev(key);
        if (pi_ >= 0)
            for (int k = 0; k < 3; ++k) ho[k] = g_prev_hist[3 * pi_ + k];
        double hp = dot3(ho, en);
        double ht[3];
        for (int k = 0; k < 3; ++k) ht[k] = (ho[k] - hp * en[k]) + vt[k] * dth;
        double ft[3];
        for (int k = 0; k < 3; ++k) ft[k] = -kt * ht[k] - gt * vt[k];
        double ftn = sqrt(dot3(ft, ft));
        double cap = D->d.mu * fabs(fn);
        if (ftn > cap) {
            double sc = cap / ftn;
            for (int k = 0; k < 3; ++k) ft[k] *= sc;
            if (kt > 0.0)
                for (int k = 0; k < 3; ++k) ht[k] = -(ft[k] + gt * vt[k]) / kt;
        }
        for (int k = 0; k < 3; ++k) {
            F[k] = fn * en[k] + ft[k];
            h[k] = ht[k];
        }
        if (sphere_law) {
            /* spheres: M_i = -R_i e_n x F_t, M_j = -R_j e_n x F_t */
            double T[3];
            cross3(en, ft, T);
            for (int k = 0; k < 3; ++k) {
                Mi[k] = -rhoi * T[k];
                Mj[k] = (j < np) ? -rhoj * T[k] : 0.0;
            }
        } else {
            /* general: M = rc x F on i, rc_j x (-F) on j (G32) */
            double mF[3] = {-F[0], -F[1], -F[2]};
            cross3(rci, F, Mi);
            if (j < np) cross3(rcj, mF, Mj);
            else Mj[0] = Mj[1] = Mj[2] = 0.0;
        }
    }
    /* per-particle sums, pairs ascending (Sec. 3.2.2, both pair members) */
    for (int64_t p = 0; p < D->npairs; ++p) {
        uint64_t key = D->pairs[p];
        int i = (int)(key >> 32), j = (int)(key & 0xffffffffu);
        for (int k = 0; k < 3; ++k) {
            D->fd[3 * i + k] += D->cF[3 * p + k];
            D->md[3 * i + k] += D->cMi[3 * p + k];
            D->fd1[3 * i + k] += fabs(D->cF[3 * p + k]);
            D->md1[3 * i + k] += fabs(D->cMi[3 * p + k]);
        }
        if (j < np)
            for (int k = 0; k < 3; ++k) {
                D->fd[3 * j + k] -= D->cF[3 * p + k];
                D->md[3 * j + k] += D->cMj[3 * p + k];
                D->fd1[3 * j + k] += fabs(D->cF[3 * p + k]);
                D->md1[3 * j + k] += fabs(D->cMj[3 * p + k]);
            }
    }
}

/* ------------------------------------------------------------------------- */
/* Integration (Sec. 2.2, Eqs. advance-r .. advance-omega; G6, G17, G18)      */
/* ------------------------------------------------------------------------- */

/* alpha = Rbw I^-1 [Rbw^T M - (Rbw^T w) x (I Rbw^T w)] with the rotation and the
 * angular velocity at the start of the substep */
static void angular_accel(const or_domain* D, int k, const double* qold, const double* w,
                          const double* M, double* al) {
    double R[9];
    quat_to_rbw(qold, R);
    const double* I = D->inertia + 3 * k;
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

/* q' = (1/2) [0, w] (x) q (world-frame w) */
static void quat_rate(const double* w, const double* q, double* out) {
    out[0] = 0.5 * (-(w[0] * q[1] + w[1] * q[2] + w[2] * q[3]));
    out[1] = 0.5 * (q[0] * w[0] + (w[1] * q[3] - w[2] * q[2]));
    out[2] = 0.5 * (q[0] * w[1] + (w[2] * q[1] - w[0] * q[3]));
    out[3] = 0.5 * (q[0] * w[2] + (w[0] * q[2] - w[1] * q[1]));
}

/* predictor: r += dt v + dt^2/2 a (wrapped on periodic axes), v^p = v + dt a,
 * w^p = w + dt alpha, orientation predictor-corrector mirroring the triad
 * update with w(t) */
static void dem_predict(or_domain* D) {
    double dt = D->dt, hdt2 = 0.5 * dt * dt;
    for (int k = 0; k < D->np; ++k) {
        double* x = D->pos + 3 * k;
        for (int c = 0; c < 3; ++c) {
            x[c] = (x[c] + dt * D->v[3 * k + c]) + hdt2 * D->a[3 * k + c];
            if (periodic_axis(D, c)) {
                double L = (double)extent(D, c);
                if (x[c] >= L) x[c] -= L;
                else if (x[c] < 0.0) x[c] += L;
                if (x[c] == L) x[c] = 0.0;
            }
            D->vp[3 * k + c] = D->v[3 * k + c] + dt * D->a[3 * k + c];
            D->wp[3 * k + c] = D->w[3 * k + c] + dt * D->al[3 * k + c];
        }
        double* q = D->q + 4 * k;
        for (int c = 0; c < 4; ++c) D->qold[4 * k + c] = q[c];
        double r1[4], qs[4], qm[4], r2[4];
        quat_rate(D->w + 3 * k, q, r1);
        for (int c = 0; c < 4; ++c) qs[c] = q[c] + dt * r1[c];
        for (int c = 0; c < 4; ++c) qm[c] = 0.5 * (q[c] + qs[c]);
        quat_rate(D->w + 3 * k, qm, r2);
        double qn[4];
        for (int c = 0; c < 4; ++c) qn[c] = q[c] + dt * r2[c];
        double l = sqrt((qn[0] * qn[0] + qn[1] * qn[1]) + (qn[2] * qn[2] + qn[3] * qn[3]));
        for (int c = 0; c < 4; ++c) q[c] = qn[c] / l;
    }
}

/* corrector: a(t+dt) = (F_dem + F_hyd + F_ext)/m, F_ext = m (1 - rho0/rho_p) g
 * (G7); v += dt/2 (a + a_new); alpha per G18; w += dt/2 (alpha + alpha_new) */
static void dem_correct(or_domain* D) {
    double dt = D->dt;
    for (int k = 0; k < D->np; ++k) {
        if (D->fixed[k]) {
            for (int c = 0; c < 3; ++c) D->a[3 * k + c] = D->al[3 * k + c] = 0.0;
            continue;
        }
        double m = D->mass[k];
        double fb = 1.0 - 1.0 / D->dens[k];
        double M[3], an[3], aln[3];
        for (int c = 0; c < 3; ++c) {
            double fext = m * fb * D->d.gravity[c];
            an[c] = ((D->fd[3 * k + c] + D->fh[3 * k + c]) + fext) / m;
            M[c] = D->md[3 * k + c] + D->mh[3 * k + c];
        }
        angular_accel(D, k, D->qold + 4 * k, D->w + 3 * k, M, aln);
        for (int c = 0; c < 3; ++c) {
            D->v[3 * k + c] += 0.5 * dt * (D->a[3 * k + c] + an[c]);
            D->a[3 * k + c] = an[c];
            D->w[3 * k + c] += 0.5 * dt * (D->al[3 * k + c] + aln[c]);
            D->al[3 * k + c] = aln[c];
        }
    }
}

static void dem_initial_accel(or_domain* D) {
    if (D->np == 0) return;
    or_stage_lists(D);
    dem_contacts(D, D->v, D->w, 0.0, NULL, NULL, 0);
    for (int k = 0; k < D->np; ++k) {
        double m = D->mass[k];
        double fb = 1.0 - 1.0 / D->dens[k];
        double M[3];
        for (int c = 0; c < 3; ++c) M[c] = D->md[3 * k + c];
        if (D->fixed[k]) {
            for (int c = 0; c < 3; ++c) D->a[3 * k + c] = D->al[3 * k + c] = 0.0;
        } else {
            for (int c = 0; c < 3; ++c) D->a[3 * k + c] = (D->fd[3 * k + c] + m * fb * D->d.gravity[c]) / m;
            angular_accel(D, k, D->q + 4 * k, D->w + 3 * k, M, D->al + 3 * k);
        }
        for (int c = 0; c < 3; ++c) {
            D->vp[3 * k + c] = D->v[3 * k + c];
            D->wp[3 * k + c] = D->w[3 * k + c];
        }
        for (int c = 0; c < 4; ++c) D->qold[4 * k + c] = D->q[4 * k + c];
    }
    /* the initial list carries no history into the first substep */
    for (int64_t p = 0; p < 3 * D->npairs; ++p) D->hist[p] = 0.0;
}

/* ------------------------------------------------------------------------- */
/* Coupled step (Fig. flowchart; G21): per DEM substep predict, cell list,     */
/* pairs, contacts, DEM sums; in the last substep voxelise, LBM-PSM and        */
/* hydrodynamic sums before the corrector.                                     */
/* ------------------------------------------------------------------------- */
static void coupled_step(or_domain* D) {
    if (D->d.dem_on && D->np > 0) {
        for (int s = 1; s <= D->nsub; ++s) {
            dem_predict(D);
            /* fixed particles keep their prescribed velocities */
            int64_t pn = D->npairs;
            uint64_t* pk = (uint64_t*)xcalloc(pn, sizeof(uint64_t));
            double* ph = (double*)xcalloc(3 * pn, sizeof(double));
            memcpy(pk, D->pairs, pn * sizeof(uint64_t));
            memcpy(ph, D->hist, 3 * pn * sizeof(double));
            or_stage_lists(D);
            dem_contacts(D, D->vp, D->wp, D->dt, pk, ph, pn);
            free(pk);
            free(ph);
            if (s == D->nsub && D->d.fluid_on) {
                or_stage_voxelize(D);
                or_stage_lbm(D);
            }
            dem_correct(D);
        }
    } else if (D->d.fluid_on) {
        for (int k = 0; k < 3 * D->np; ++k) { D->vp[k] = D->v[k]; D->wp[k] = D->w[k]; }
        or_stage_voxelize(D);
        or_stage_lbm(D);
    }
    D->step++;
}

/* contact forces of the current pair list, with that list and its history as
 * the previous substep's, predicted velocities and one substep of history */
void or_stage_contacts(or_domain* D) {
    int64_t pn = D->npairs;
    uint64_t* pk = (uint64_t*)xcalloc(pn, sizeof(uint64_t));
    double* ph = (double*)xcalloc(3 * pn, sizeof(double));
    memcpy(pk, D->pairs, pn * sizeof(uint64_t));
    memcpy(ph, D->hist, 3 * pn * sizeof(double));
    dem_contacts(D, D->vp, D->wp, D->dt, pk, ph, pn);
    free(pk);
    free(ph);
}

void or_step(or_domain* D, int64_t n) {
    for (int64_t s = 0; s < n; ++s) coupled_step(D);
}

/* ------------------------------------------------------------------------- */
/* Accessors                                                                   */
/* ------------------------------------------------------------------------- */
void or_get_populations(const or_domain* D, double* f) { memcpy(f, D->f, 19 * D->N * sizeof(double)); }
void or_set_populations(or_domain* D, const double* f) { memcpy(D->f, f, 19 * D->N * sizeof(double)); }

void or_get_fields(const or_domain* D, double* rho, double* u) {
    /* rho = sum f, rho u = sum f c (Eqs. rho, momentum); with forcing the
     * velocity carries the half-force shift used by the collision */
    for (int64_t c = 0; c < D->N; ++c) {
        double r = 0, m[3] = {0, 0, 0};
        for (int i = 0; i < 19; ++i) {
            double fi = D->f[i * D->N + c];
            r += fi;
            m[0] += fi * CX[i];
            m[1] += fi * CY[i];
            m[2] += fi * CZ[i];
        }
        int nx = D->d.nx, ny = D->d.ny;
        int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((int64_t)nx * ny));
        double F[3];
        cell_force(D, x, y, z, F);
        rho[c] = r;
        for (int k = 0; k < 3; ++k) u[3 * c + k] = (m[k] + 0.5 * F[k]) / r;
    }
}

void or_get_particles(const or_domain* D, double* pos, double* quat, double* vel, double* omega,
                      double* acc, double* alpha, double* fh, double* mh, double* fd, double* md) {
    size_t n3 = 3 * (size_t)D->np * sizeof(double);
    if (pos) memcpy(pos, D->pos, n3);
    if (quat) memcpy(quat, D->q, 4 * (size_t)D->np * sizeof(double));
    if (vel) memcpy(vel, D->v, n3);
    if (omega) memcpy(omega, D->w, n3);
    if (acc) memcpy(acc, D->a, n3);
    if (alpha) memcpy(alpha, D->al, n3);
    if (fh) memcpy(fh, D->fh, n3);
    if (mh) memcpy(mh, D->mh, n3);
    if (fd) memcpy(fd, D->fd, n3);
    if (md) memcpy(md, D->md, n3);
}

void or_set_particles(or_domain* D, const double* pos, const double* quat, const double* vel,
                      const double* omega, const double* acc, const double* alpha, const double* fh,
                      const double* mh) {
    size_t n3 = 3 * (size_t)D->np * sizeof(double);
    if (pos) memcpy(D->pos, pos, n3);
    if (quat) memcpy(D->q, quat, 4 * (size_t)D->np * sizeof(double));
    if (vel) memcpy(D->v, vel, n3);
    if (omega) memcpy(D->w, omega, n3);
    if (acc) memcpy(D->a, acc, n3);
    if (alpha) memcpy(D->al, alpha, n3);
    if (fh) memcpy(D->fh, fh, n3);
    if (mh) memcpy(D->mh, mh, n3);
}

void or_get_rounding_scales(const or_domain* D, double* fhr, double* mhr, double* fhg, double* mhg) {
    size_t n3 = 3 * (size_t)D->np * sizeof(double);
    if (fhr) memcpy(fhr, D->fhr, n3);
    if (mhr) memcpy(mhr, D->mhr, n3);
    if (fhg) memcpy(fhg, D->fhg, n3);
    if (mhg) memcpy(mhg, D->mhg, n3);
}

void or_get_scales(const or_domain* D, double* fh1, double* mh1, double* fd1, double* md1) {
    size_t n3 = 3 * (size_t)D->np * sizeof(double);
    if (fh1) memcpy(fh1, D->fh1, n3);
    if (mh1) memcpy(mh1, D->mh1, n3);
    if (fd1) memcpy(fd1, D->fd1, n3);
    if (md1) memcpy(md1, D->md1, n3);
}

void or_get_predicted(const or_domain* D, double* vp, double* wp) {
    memcpy(vp, D->vp, 3 * (size_t)D->np * sizeof(double));
    memcpy(wp, D->wp, 3 * (size_t)D->np * sizeof(double));
}
void or_set_predicted(or_domain* D, const double* vp, const double* wp) {
    memcpy(D->vp, vp, 3 * (size_t)D->np * sizeof(double));
    memcpy(D->wp, wp, 3 * (size_t)D->np * sizeof(double));
}

int64_t or_get_pairs(const or_domain* D, int64_t cap, uint64_t* keys, double* hist) {
    int64_t n = D->npairs < cap ? D->npairs : cap;
    if (keys) memcpy(keys, D->pairs, n * sizeof(uint64_t));
    if (hist) memcpy(hist, D->hist, 3 * n * sizeof(double));
    return D->npairs;
}

void or_set_pairs(or_domain* D, int64_t n, const uint64_t* keys, const double* hist) {
    ensure_pairs(D, n);
    memcpy(D->pairs, keys, n * sizeof(uint64_t));
    memcpy(D->hist, hist, 3 * n * sizeof(double));
    D->npairs = n;
}

int64_t or_get_cells(const or_domain* D, int64_t cap, uint64_t* keys) {
    int64_t n = D->nreg < cap ? D->nreg : cap;
    if (keys) memcpy(keys, D->reg, n * sizeof(uint64_t));
    return D->nreg;
}

int64_t or_get_contacts(const or_domain* D, int64_t cap, uint64_t* keys, double* force, double* mi,
                        double* mj) {
    int64_t n = 0;
    for (int64_t p = 0; p < D->npairs; ++p) {
        if (!D->incontact[p]) continue;
        if (n < cap) {
            keys[n] = D->pairs[p];
            for (int k = 0; k < 3; ++k) {
                force[3 * n + k] = D->cF[3 * p + k];
                mi[3 * n + k] = D->cMi[3 * p + k];
                mj[3 * n + k] = D->cMj[3 * p + k];
            }
        }
        ++n;
    }
    return n;
}

void or_counters(const or_domain* D, int64_t out[6]) {
    out[0] = D->npairs;
    out[1] = D->ncontacts;
    out[2] = D->nentries;
    out[3] = D->overflow;
    out[4] = D->nreg;
    out[5] = D->step;
}

void or_set_threads(int32_t n) {
#ifdef _OPENMP
    omp_set_num_threads(n);
#else
    (void)n;
#endif
}
int32_t or_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
