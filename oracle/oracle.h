/*
 * oracle.h -- plain FP64 CPU oracle of the coupled LBM-PSM-DEM time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code: only tests/, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code with the HIP library.
 *
 * The oracle is a definition, not an optimised algorithm: two population
 * arrays with push streaming, a plain bucket grid for the cell list,
 * qsort + unique for pairs, serial fixed-order reductions.
 *
 * Conventions (lattice units, dx = dt = 1):
 *   node (x,y,z) has centre (x+1/2, y+1/2, z+1/2), the domain is [0,N)^3,
 *   walls sit on the planes 0 and N of walled axes (halfway bounce-back);
 *   D3Q19 ordering: 0 rest, 1..9 = (1,0,0),(0,1,0),(0,0,1),(1,1,0),(1,-1,0),
 *   (1,0,1),(1,0,-1),(0,1,1),(0,1,-1), 10..18 their negatives;
 *   populations are stored f[i*N + cell], cell = x + nx*(y + ny*z);
 *   quaternions are (w,x,y,z) and rotate body-frame vectors into the world.
 */
#ifndef PSM_ORACLE_H
#define PSM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;
    double tau, rho0;
    int32_t bc[6];            /* faces -x,+x,-y,+y,-z,+z: 0 periodic, 1 no-slip, 2 moving */
    double wall_u[6][3];      /* wall velocity per face (moving walls) */
    double body_force[3];     /* constant fluid force density (Guo forcing) */
    double kolm_amp;          /* Kolmogorov forcing amplitude */
    int32_t kolm_axis;        /* coordinate the sine depends on */
    int32_t kolm_dir;         /* force component it drives */
    double gravity[3];        /* acceleration on particles (net of buoyancy applied inside) */
    int32_t sf_method;        /* 0 subdivision, 1 distance (spheres only) */
    int32_t sf_subdiv;        /* samples per direction (10) */
    int32_t fluid_on, dem_on, n_sub;   /* n_sub = 0: automatic rule */
    double dem_cell;          /* 0: automatic DEM grid */
    double kn, restitution, mu, kt_ratio, gt_ratio;
    int32_t max_solids;       /* solids kept per fluid cell (2) */
    int32_t collision;        /* fluid operator: 0 BGK, 1 TRT (Sec. 2.3, Eq. TRT) */
    double trt_magic;         /* TRT: 0 = the paper's tau^- rule; > 0 = magic parameter Lambda */
    int32_t contact_law;      /* 0 linear spring-dashpot (k_n given), 1 Hertz from the material (App. A) */
    double young, poisson;    /* Hertz: Young's modulus and Poisson's ratio of particles and walls */
} or_desc;

typedef struct or_domain or_domain;

/* Returns NULL on invalid input; or_error() then holds a message. */
or_domain* or_create(const or_desc* d, int32_t np, const int32_t* shape,
                     const double* semi, const double* dens, const double* pos,
                     const double* quat, const double* vel, const double* omega,
                     const uint8_t* fixed);
const char* or_error(void);
void or_destroy(or_domain* D);

/* n coupled steps. */
void or_step(or_domain* D, int64_t n);
int32_t or_nsub(const or_domain* D);
void or_dem_grid(const or_domain* D, int32_t nc[3], double h[3]);
double or_mass(const or_domain* D, int32_t k);

/* state access (canonical populations, pre-collision at the current time) */
void or_get_populations(const or_domain* D, double* f);
void or_set_populations(or_domain* D, const double* f);
void or_get_fields(const or_domain* D, double* rho, double* u);
void or_get_particles(const or_domain* D, double* pos, double* quat, double* vel,
                      double* omega, double* acc, double* alpha, double* fh,
                      double* mh, double* fd, double* md);
void or_set_particles(or_domain* D, const double* pos, const double* quat,
                      const double* vel, const double* omega, const double* acc,
                      const double* alpha, const double* fh, const double* mh);
void or_get_predicted(const or_domain* D, double* vp, double* wp);
/* scales of the last hydrodynamic and DEM sums against which force parity is
 * measured: for F_hyd / M_hyd the per-component L1 norm of the population-level
 * summands of the momentum exchange (|f| and |f^eq| terms times |c_i|, times
 * |r_j - r_k| for the torque), which bounds their rounding; for F_dem / M_dem
 * the L1 norm of the pair forces and torques */
void or_get_scales(const or_domain* D, double* fh1, double* mh1, double* fd1, double* md1);
/* rounding scales of the last LBM-PSM step's F_hyd and M_hyd [3 np] each:
 * the population magnitudes the momentum-exchange terms are formed from
 * (fhr, mhr) and the same of the deviations f - w (fhg, mhg) */
void or_get_rounding_scales(const or_domain* D, double* fhr, double* mhr, double* fhg, double* mhg);
int64_t or_get_pairs(const or_domain* D, int64_t cap, uint64_t* keys, double* hist);
void or_set_pairs(or_domain* D, int64_t n, const uint64_t* keys, const double* hist);
int64_t or_get_cells(const or_domain* D, int64_t cap, uint64_t* keys);
int64_t or_get_solid(const or_domain* D, int64_t cap, uint32_t* cell, uint32_t* pid, double* beta);
int64_t or_get_contacts(const or_domain* D, int64_t cap, uint64_t* keys, double* force,
                        double* mi, double* mj);
void or_counters(const or_domain* D, int64_t out[6]); /* pairs, contacts, entries, overflow, regs, step */

/* stage-level entry points used by the pins and by per-stage parity */
void or_stage_lists(or_domain* D);      /* cell registrations + candidate pairs from current positions */
void or_stage_voxelize(or_domain* D);   /* solid fractions and slots from current positions */
void or_stage_lbm(or_domain* D);        /* one LBM-PSM step with the current slots and v^p, w^p */
void or_stage_contacts(or_domain* D);   /* contacts of the current list, its history as the previous */
void or_set_predicted(or_domain* D, const double* vp, const double* wp);

/* brute-force candidate pairs (all i<j with intersecting registrations), sorted */
int64_t or_brute_pairs(or_domain* D, int64_t cap, uint64_t* keys);

/* single-cell collision helpers for the algebraic pins */
void or_feq(double rho, const double u[3], double feq[19]);
void or_collide_cell(const or_domain* D, const double f[19], int32_t nslot,
                     const double* B, const double* uk, const double F[3],
                     double fpost[19], double* Pk /* 3*nslot */);

/* geometry helpers exposed for pins */
double or_beta_subdiv_sphere(double cx, double cy, double cz, double R,
                             int32_t X, int32_t Y, int32_t Z, int32_t ns);
double or_beta_distance(double cx, double cy, double cz, double R,
                        int32_t X, int32_t Y, int32_t Z);
/* ellipsoid-ellipsoid / sphere-sphere contact geometry between particles i, j */
int32_t or_contact_geometry(const or_domain* D, int32_t i, int32_t j, double* delta,
                            double en[3], double rci[3], double rcj[3], int32_t* iters);

void or_set_threads(int32_t n);
int32_t or_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
