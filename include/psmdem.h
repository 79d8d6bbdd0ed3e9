/*
 * psmdem.h -- C ABI of the MI355X (gfx950) coupled LBM-PSM-DEM time step.
 *
 * The library advances a fully coupled lattice Boltzmann / discrete element
 * system as formulated in arXiv 2512.04997 ("LEDDS"):
 *   - D3Q19 BGK collide-and-stream (Sec. 2.3, Eqs. collAndStream, BGK,
 *     equilibrium) with partially-saturated-method weighting (Sec. 2.4, Eqs.
 *     psm1, lbePS, bk, btot), halfway and moving-wall bounce-back (Sec. 2.3);
 *   - solid fractions of spheres and ellipsoids by subdivision or, for
 *     spheres, by the distance formula (Sec. 2.4, Eq. naiveSolidFrac);
 *   - hydrodynamic force and torque per particle (Sec. 2.4, Eqs. forceSF,
 *     torqueSF);
 *   - DEM: uniform-grid cell list and candidate pairs (Sec. 3.2.1), linear
 *     spring-dashpot contacts with Coulomb friction and tangential history
 *     (Sec. 2.1, Eqs. spring_dashpot_easy, fnScal, relative_velocity,
 *     trangential-history, coulombCoeff, torque), walls as static particles,
 *     ellipsoid contact by iterated equivalent spheres (Eq. local-curvature);
 *   - Verlet integration of translation and rotation (Sec. 2.2, Eqs.
 *     advance-r .. advance-omega) with DEM sub-stepping (Sec. 2.3);
 *   in the coupled order of the workflow figure (Sec. 3.2).
 *
 * Units are lattice units (dx = dt = 1).  Node (x,y,z) has centre
 * (x+1/2, y+1/2, z+1/2); the domain is [0,nx) x [0,ny) x [0,nz); walls lie on
 * the planes 0 and n of walled axes.  D3Q19 order: 0 rest, 1..9 =
 * (1,0,0),(0,1,0),(0,0,1),(1,1,0),(1,-1,0),(1,0,1),(1,0,-1),(0,1,1),(0,1,-1),
 * 10..18 their negatives.  Cell index = x + nx*(y + ny*z).  Quaternions are
 * (w,x,y,z) and rotate body-frame vectors into the world frame.
 *
 * Conventions of every call:
 *   - all functions return psmdem_status (0 = OK, < 0 = error) and never
 *     abort; psmdem_last_error() returns a thread-local message;
 *   - host pointers are plain host memory owned by the caller; inputs are
 *     copied before the call returns; outputs are written before it returns;
 *   - device memory is owned by the library (allocated through the optional
 *     allocator callback, else hipMalloc) and freed by psmdem_destroy;
 *   - work is enqueued on the HIP stream given at creation (NULL = the
 *     default stream); psmdem_step is asynchronous, every read_* call
 *     synchronises the stream first;
 *   - device flags (PSMDEM_E_UNSTABLE, PSMDEM_E_CAPACITY) are raised by the
 *     kernels and reported by psmdem_sync and by every read_* call, which
 *     still writes its outputs (for inspection) and then returns the flag;
 *     they stay set until a write_* call rewrites the state.
 */
#ifndef PSMDEM_H
#define PSMDEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PSMDEM_OK = 0,
    PSMDEM_E_INVALID = -1,   /* bad argument or configuration */
    PSMDEM_E_NOMEM = -2,     /* device allocation failed */
    PSMDEM_E_CAPACITY = -3,  /* a device list outgrew its capacity; results of the step are invalid */
    PSMDEM_E_UNSTABLE = -4,  /* the state has blown up: a cell density that is not a positive finite
                                number (checked by every LBM-PSM pass), or a particle centre that is not
                                finite or lies more than one box length outside the domain (checked by
                                every DEM predictor and every voxelisation, which then gives that
                                particle no solid fractions) */
    PSMDEM_E_HIP = -5,       /* a HIP runtime call failed */
    PSMDEM_E_STATE = -6,     /* call not valid in the current state */
    PSMDEM_E_NODEVICE = -7   /* no gfx950 device available */
} psmdem_status;

typedef enum { PSMDEM_BC_PERIODIC = 0, PSMDEM_BC_NOSLIP = 1, PSMDEM_BC_MOVING = 2 } psmdem_bc;

/* Population storage.  All modes store shifted populations f_i - w_i.
 * FP64: stored and computed in double.  FP32: float storage and arithmetic.
 * BF16 / FP16: 16-bit storage (round to nearest even), float arithmetic.
 * Particle kinematics and force/torque sums are double in every mode. */
typedef enum {
    PSMDEM_FP64 = 0,
    PSMDEM_FP32 = 1,
    PSMDEM_BF16_SHIFTED = 2,
    PSMDEM_FP16_SHIFTED = 3
} psmdem_precision;

typedef enum { PSMDEM_SF_SUBDIVISION = 0, PSMDEM_SF_DISTANCE = 1 } psmdem_sf;

/* Fluid collision operator inside the PSM step, Eq. (lbePS).  BGK: Eq. (BGK).
 * TRT, Eqs. (trt_populations), (TRT): the even and odd parts of f - f^eq relax
 * with dt/tau+ = 1/tau and dt/tau-; the Guo source is split into its even and
 * odd parts the same way, each scaled by 1 - (dt/tau+-)/2. */
typedef enum { PSMDEM_BGK = 0, PSMDEM_TRT = 1 } psmdem_collision;

/* Contact law, Sec. 2.1 and App. A.  LINEAR: F_n = [k_n d + gamma_n (v_j - v_i).e_n] e_n
 * with the given k_n, gamma_n = -2 beta sqrt(k_n m*), beta = ln e / sqrt(ln^2 e + pi^2),
 * k_t = kt_ratio k_n, gamma_t = gt_ratio gamma_n.  HERTZ: the same force form with
 * k_n = 4/3 Y* sqrt(R* d), k_t = 8 G* sqrt(R* d), gamma = -2 sqrt(5/6) beta sqrt(S m*),
 * S_n = 2 Y* sqrt(R* d), S_t = 8 G* sqrt(R* d), R* = (1/R_i + 1/R_j)^-1 (local equivalent
 * sphere radii for ellipsoids), Y* and G* from one material (young, poisson) shared by the
 * particles and the walls; a wall has infinite radius and mass.  The contact time then
 * depends on the impact speed, so n_sub must be given (> 0). */
typedef enum { PSMDEM_LINEAR = 0, PSMDEM_HERTZ = 1 } psmdem_contact_law;
typedef enum { PSMDEM_SPHERE = 0, PSMDEM_ELLIPSOID = 1 } psmdem_shape;

typedef struct {
    int32_t nx, ny, nz;         /* lattice extents (>= 1) */
    double tau;                 /* relaxation time (tau+ of TRT), tau = 3 nu + 1/2 (Eq. tau), > 1/2 */
    double rho0;                /* reference density (1): initial density, wall density */
    int32_t bc[6];              /* faces -x,+x,-y,+y,-z,+z: psmdem_bc; both faces of an axis
                                   periodic or neither */
    double wall_u[6][3];        /* wall velocity of PSMDEM_BC_MOVING faces */
    double body_force[3];       /* constant fluid force density (Guo forcing) */
    double kolm_amp;            /* Kolmogorov forcing: component kolm_dir of the force
                                   density gets kolm_amp sin(2 pi (c + 1/2) / n_axis),
                                   c the coordinate along kolm_axis */
    int32_t kolm_axis, kolm_dir;
    double gravity[3];          /* acceleration on particles; F_ext = m (1 - rho0/rho_p) g */
    int32_t precision;          /* psmdem_precision */
    int32_t sf_method;          /* psmdem_sf (distance: spheres only) */
    int32_t sf_subdiv;          /* subdivision samples per direction (10), 1..32 */
    int32_t fluid_on, dem_on;   /* LBM and DEM usable independently or coupled */
    int32_t n_sub;              /* DEM substeps per LBM step; 0 = automatic:
                                   max(1, ceil(20 / t_c)) from the stiffest contact */
    double dem_cell;            /* DEM grid spacing; 0 = automatic (>= 1.1 x largest diameter) */
    double kn;                  /* normal stiffness of the linear law */
    double restitution;         /* coefficient of restitution in (0, 1] */
    double mu;                  /* Coulomb friction coefficient */
    double kt_ratio, gt_ratio;  /* k_t / k_n and gamma_t / gamma_n */
    int32_t max_solids;         /* solids kept per fluid cell (2), 1..4 */
    int64_t pair_capacity;      /* candidate-pair capacity; 0 = automatic */
    int32_t collision;          /* fluid operator: psmdem_collision (BGK, 0, when zeroed) */
    double trt_magic;           /* TRT only: 0 = the paper's rule dt/tau- = 8 (2 - w) / (8 - w),
                                   w = dt/tau+ (Sec. 2.3), which is the magic parameter
                                   Lambda = (tau+ - 1/2)(tau- - 1/2) = 3/16; > 0 sets Lambda */
    int32_t contact_law;        /* psmdem_contact_law (linear, 0, when zeroed) */
    double young, poisson;      /* Hertz: Young's modulus (> 0) and Poisson's ratio (in [0, 1/2)) of the
                                   particles and the walls, in lattice units */
} psmdem_desc;

typedef struct {
    int32_t n;                    /* number of particles (may be 0) */
    const int32_t* shape;         /* [n] psmdem_shape */
    const double* semi_axes;      /* [3n] radius (sphere: first entry) or semi-axes */
    const double* density_ratio;  /* [n] rho_p / rho0 */
    const double* pos;            /* [3n] centres */
    const double* quat;           /* [4n] orientation (w,x,y,z); NULL = identity */
    const double* vel;            /* [3n] NULL = 0 */
    const double* omega;          /* [3n] world-frame angular velocity; NULL = 0 */
    const uint8_t* fixed;         /* [n] 1 = velocities prescribed (not integrated); NULL = 0 */
} psmdem_particles;

/* Optional allocator: returns device memory of at least `bytes` bytes, or
 * NULL.  Used for every device allocation of a domain. */
typedef void* (*psmdem_alloc_fn)(size_t bytes, void* ctx);
typedef void (*psmdem_free_fn)(void* ptr, size_t bytes, void* ctx);

typedef struct psmdem_domain psmdem_domain;

typedef struct {
    int64_t n_pairs;         /* candidate pairs of the last substep */
    int64_t n_contacts;      /* pairs with positive overlap */
    int64_t n_registrations; /* DEM cell registrations */
    int64_t n_entries;       /* (cell, particle) solid-fraction entries with beta > 0 */
    int64_t n_dropped;       /* entries beyond max_solids in a cell (dropped, Sec. 3.2.3 limit) */
    int64_t n_solid_tiles;   /* lattice tiles holding any particle */
    int64_t step;            /* coupled steps taken */
    int64_t flags;           /* bit 0 pair capacity, bit 1 tile particle list, bit 2 neighbour list,
                                bit 3 tile registrations, bit 4 unstable */
} psmdem_counters_t;

typedef struct {
    int32_t n_sub;          /* DEM substeps per coupled step */
    int32_t dem_cells[3];   /* DEM grid */
    double dem_h[3];        /* DEM cell size */
    int64_t n_cells;        /* lattice cells */
    int32_t n_particles;
    int32_t precision;
    int64_t device_bytes;   /* device memory held by the domain */
    int32_t tile[3];        /* lattice tile used by the LBM and voxelisation kernels */
} psmdem_info_t;

/* --- life cycle ----------------------------------------------------------- */

/* Creates a domain: validates the description, allocates device memory,
 * initialises f = f^eq(rho0, 0) (Sec. 2.3), and evaluates the initial DEM
 * forces (a(0) = (F_dem + F_ext)/m, zero tangential history).  stream is a
 * hipStream_t (NULL: default stream).  alloc/free may be NULL. */
psmdem_status psmdem_create(const psmdem_desc* desc, const psmdem_particles* parts, void* stream,
                            psmdem_alloc_fn alloc, psmdem_free_fn free_fn, void* alloc_ctx,
                            psmdem_domain** out);
void psmdem_destroy(psmdem_domain* d);

/* Enqueues n coupled steps (one LBM step with n_sub DEM substeps each). */
psmdem_status psmdem_step(psmdem_domain* d, int64_t n);
/* Waits for the stream and reports the device flags: PSMDEM_E_UNSTABLE, else
 * PSMDEM_E_CAPACITY, else PSMDEM_OK. */
psmdem_status psmdem_sync(psmdem_domain* d);

/* --- stages (one stage on the current state; for per-stage checks) ------- */
typedef enum {
    PSMDEM_STAGE_LISTS = 0,     /* cell registrations and candidate pairs from current positions */
    PSMDEM_STAGE_VOXELIZE = 1,  /* solid fractions and per-cell slots from current positions */
    PSMDEM_STAGE_LBM = 2,       /* one LBM-PSM step with current slots and predicted velocities,
                                   and the hydrodynamic force and torque */
    PSMDEM_STAGE_CONTACTS = 3   /* contact forces with the current pair list and history as the
                                   previous list, predicted velocities, one substep of history */
} psmdem_stage_t;
psmdem_status psmdem_stage(psmdem_domain* d, int32_t stage);

/* --- state access (all synchronise the stream) ---------------------------- */
/* f: [19 * n_cells] double, f[i * n_cells + cell], pre-collision populations at
 * the current time in the canonical layout (the in-place storage is decoded). */
psmdem_status psmdem_read_populations(psmdem_domain* d, double* f);
psmdem_status psmdem_write_populations(psmdem_domain* d, const double* f);
/* Density and velocity of the populations at the current time (Sec. 2.3,
 * Eqs. for rho and rho u; with forcing, u includes the half-force shift):
 * rho [n_cells], u [3 n_cells] (x, y, z per cell); either may be NULL.  The
 * moments are formed on the device, chunk by chunk, in a staging block the
 * library allocates for the call through the domain's allocator (32 bytes
 * per cell of a chunk of at most 2^22 cells; PSMDEM_E_NOMEM when it cannot). */
psmdem_status psmdem_read_fields(psmdem_domain* d, double* rho, double* u);
/* The same read-out for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation): identical outputs, staged through a file-scope device array
 * of 2^20 cells x 4 doubles (32 MiB, one per device, held until the process
 * ends), any lattice size in chunks of 2^20 cells.  Calls no allocating
 * routine.  Every call on a device shares that device's array, and each chunk
 * overwrites what it reads back (nothing has to start at zero): calls that
 * overlap on one device (from several host threads) race. */
psmdem_status psmdem_read_fields_noalloc(psmdem_domain* d, double* rho, double* u);
/* particle arrays [3n] (quat [4n]); any pointer may be NULL */
psmdem_status psmdem_read_particles(psmdem_domain* d, double* pos, double* quat, double* vel,
                                   double* omega, double* acc, double* alpha, double* f_hyd,
                                   double* m_hyd, double* f_dem, double* m_dem);
psmdem_status psmdem_write_particles(psmdem_domain* d, const double* pos, const double* quat,
                                    const double* vel, const double* omega, const double* acc,
                                    const double* alpha, const double* f_hyd, const double* m_hyd);
/* predicted velocities v^p, w^p of the last substep ([3n] each) */
psmdem_status psmdem_read_predicted(psmdem_domain* d, double* vp, double* wp);
psmdem_status psmdem_write_predicted(psmdem_domain* d, const double* vp, const double* wp);
/* sorted candidate pairs (i << 32 | j; j >= n for wall face j - n) and their
 * tangential history [3 cap]; *n receives the count (may exceed cap) */
psmdem_status psmdem_read_pairs(psmdem_domain* d, int64_t cap, uint64_t* keys, double* hist,
                               int64_t* n);
psmdem_status psmdem_write_pairs(psmdem_domain* d, int64_t n, const uint64_t* keys,
                                const double* hist);
/* pairs in contact with force on i [3], torque on i [3], torque on j [3] */
psmdem_status psmdem_read_contacts(psmdem_domain* d, int64_t cap, uint64_t* keys, double* force,
                                  double* m_i, double* m_j, int64_t* n);
/* sorted DEM cell registrations (cell << 32 | pid) */
psmdem_status psmdem_read_cells(psmdem_domain* d, int64_t cap, uint64_t* keys, int64_t* n);
/* kept solid slots sorted by (cell, pid) with their solid fraction beta */
psmdem_status psmdem_read_solid(psmdem_domain* d, int64_t cap, uint32_t* cell, uint32_t* pid,
                               double* beta, int64_t* n);
psmdem_status psmdem_counters(psmdem_domain* d, psmdem_counters_t* out);
psmdem_status psmdem_info(psmdem_domain* d, psmdem_info_t* out);

/* Average device time per launch of each kernel family over the last
 * psmdem_step call when timing is on (HIP events on the domain stream).
 * PSMDEM_T_HYDRO covers the per-particle hydrodynamic sums after the LBM-PSM
 * pass, which with the DEM on run in one launch with the step's final
 * corrector; PSMDEM_T_DEM covers the substeps before it. */
psmdem_status psmdem_set_timing(psmdem_domain* d, int32_t on);
psmdem_status psmdem_timing(psmdem_domain* d, int32_t which, double* avg_ms, int64_t* launches);
typedef enum { PSMDEM_T_LBM = 0, PSMDEM_T_VOXEL = 1, PSMDEM_T_DEM = 2, PSMDEM_T_HYDRO = 3 } psmdem_timer;

/* --- checkpoint and restore ------------------------------------------------ */
/* The whole state of a domain as one host byte image: a header (step, AA
 * parity, DEM buffer index) and every device block of the domain (in-place
 * populations, particle state, both pair lists with their tangential history,
 * the kept-list and skip state of the DEM substeps, tile lists, solid slots,
 * counters and device flags).  A domain created from the same description and
 * particle count that receives the image continues bit for bit as the saved
 * one would have: n steps, a checkpoint, n more steps equal 2n steps.
 * psmdem_read_state: *used receives the image size; with buf NULL only the
 * size is reported (PSMDEM_OK); a buffer shorter than the image gives
 * PSMDEM_E_INVALID.  Otherwise the image is written to buf (caller-owned host
 * memory) and the device flags are returned as by the read_* calls.
 * psmdem_write_state: n must be the image size and the image must come from a
 * domain of the same layout (description and particle count), else
 * PSMDEM_E_INVALID with nothing changed; the device flags are restored with
 * the image. */
psmdem_status psmdem_read_state(psmdem_domain* d, void* buf, size_t cap, size_t* used);
psmdem_status psmdem_write_state(psmdem_domain* d, const void* buf, size_t n);

/* Device bytes psmdem_create would allocate for this description and particle
 * set (the memory model used for admission by the serving loop).  Touches no
 * device. */
psmdem_status psmdem_footprint(const psmdem_desc* desc, const psmdem_particles* parts, int64_t* bytes);

/* --- ensemble serving: continuous batching of many domains ---------------- */
/* A server advances many independent domains ("jobs") together.  Each
 * psmdem_server_iterate call
 *   1. marks jobs done whose last step the device has finished,
 *   2. admits queued jobs in arrival order while a slot is free and the
 *      footprints of the held jobs plus the next one fit hbm_budget (the job
 *      is created on the admission stream, so the steps already enqueued keep
 *      running meanwhile),
 *   3. enqueues one coupled step of every active job as six batched launches
 *      on the compute stream: fused DEM substeps (one workgroup per job), tile
 *      registration (one workgroup per job), voxelisation and the two LBM-PSM
 *      passes (one workgroup per lattice tile of every job), hydrodynamic sums
 *      and the corrector (one workgroup per job),
 *   4. retires the jobs that reached their step count (their memory stays
 *      held, and readable, until psmdem_server_release).
 * The host runs at most max_inflight steps ahead of the device.  A job's
 * result is the one psmdem_step gives on the same domain, bit for bit: the
 * batched launches run the single-domain device code on each job's own data,
 * in the same order (the voxelisation in a one-workgroup form that counts the
 * same samples).  Jobs must have the fluid on, the server's precision, at
 * most 2048 particles when the DEM is on, and at most 8192 lattice tiles of
 * 64 x 4 x 4 cells.  Calls on one server are not thread-safe. */
typedef struct psmdem_server psmdem_server;

typedef struct {
    int32_t max_jobs;       /* active slots, 1..128 */
    int64_t hbm_budget;     /* device bytes the held jobs may occupy together (0: unlimited) */
    int32_t max_inflight;   /* coupled steps enqueued ahead of the device (0: 2) */
    int32_t precision;      /* psmdem_precision of every job */
} psmdem_server_desc;

typedef enum {
    PSMDEM_JOB_QUEUED = 0,
    PSMDEM_JOB_ACTIVE = 1,
    PSMDEM_JOB_FINISHING = 2,   /* every step enqueued, device not finished yet */
    PSMDEM_JOB_DONE = 3,        /* results readable */
    PSMDEM_JOB_FAILED = 4       /* creation failed (psmdem_server_job reports the status) */
} psmdem_job_state;

typedef struct {
    int32_t state;          /* psmdem_job_state */
    int32_t slot;           /* active slot, -1 when not active */
    int64_t steps;          /* requested coupled steps */
    int64_t steps_done;     /* coupled steps enqueued so far */
    int64_t footprint;      /* device bytes (psmdem_footprint) */
    int32_t status;         /* creation status of a failed job */
    double t_submit;        /* psmdem_clock() at submission */
    double t_admit;         /* at admission (0 before) */
    double t_done;          /* when the server saw the device finish the last step (0 before) */
} psmdem_job_info_t;

/* Seconds of a monotonic host clock (the clock of the job times). */
double psmdem_clock(void);

/* stream: compute stream; admit_stream: stream of job creation (NULL: the
 * compute stream).  alloc/free as for psmdem_create, used for every job and
 * for the server's tables (memory is allocated while admit_stream's work is
 * the only work that may touch it). */
psmdem_status psmdem_server_create(const psmdem_server_desc* desc, void* stream, void* admit_stream,
                                   psmdem_alloc_fn alloc, psmdem_free_fn free_fn, void* alloc_ctx,
                                   psmdem_server** out);
/* Waits for the device and frees every job. */
void psmdem_server_destroy(psmdem_server* s);
/* Queues a job of `steps` coupled steps; inputs are copied.  *job receives
 * its id (> 0).  Refuses, with PSMDEM_E_INVALID, jobs the server cannot run
 * (precision, fluid off, particle or tile limits) and jobs whose footprint
 * alone exceeds the budget (they could never be admitted). */
psmdem_status psmdem_server_submit(psmdem_server* s, const psmdem_desc* desc, const psmdem_particles* parts,
                                   int64_t steps, int64_t* job);
/* One serving iteration (steps 1-4 above); either output may be NULL. */
psmdem_status psmdem_server_iterate(psmdem_server* s, int32_t* n_active, int32_t* n_queued);
/* Waits for the enqueued steps; finishing jobs become done. */
psmdem_status psmdem_server_drain(psmdem_server* s);
psmdem_status psmdem_server_job(psmdem_server* s, int64_t job, psmdem_job_info_t* out);
/* The domain of a done job, for the psmdem_read_* calls (owned by the
 * server; valid until the job is released; do not step it). */
psmdem_status psmdem_server_domain(psmdem_server* s, int64_t job, psmdem_domain** out);
/* Frees a job's memory; a queued job is dropped, an active one cancelled
 * (waits for the device). */
psmdem_status psmdem_server_release(psmdem_server* s, int64_t job);

const char* psmdem_last_error(void);
const char* psmdem_version(void);

#ifdef __cplusplus
}
#endif
#endif
