// psmdem.hip -- domain object, coupled-step orchestration and the C ABI
// declared in include/psmdem.h.
//
// Coupled step (workflow figure, Sec. 3.2; substeps per Sec. 2.3): for each of
// n_sub DEM substeps: predictor, cell list, candidate pairs, contacts, DEM
// sums; in the last substep, with the fluid on, solid fractions, the LBM-PSM
// step and the hydrodynamic sums run before the corrector.  Every launch is
// enqueued on the domain stream; nothing is copied back inside a step.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "dem.h"
#include "domain.h"
#include "lbm.h"
#include "voxel.h"

static thread_local char g_err[512] = "";

void psm_set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

PsmErr psm_hip_fail(hipError_t e, const char* what, const char* file, int line) {
    psm_set_error("HIP error %s (%d) in %s at %s:%d", hipGetErrorString(e), (int)e, what, file, line);
    return PsmErr{PSMDEM_E_HIP};
}

namespace {

__global__ void k_kin(PartArgs p, int copy_vw) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= p.np) return;
    for (int c = 0; c < 3; ++c) {
        if (copy_vw) {
            p.vp[3 * k + c] = p.v[3 * k + c];
            p.wp[3 * k + c] = p.w[3 * k + c];
        }
        p.kin[9 * k + c] = p.pos[3 * k + c];
        p.kin[9 * k + 3 + c] = p.vp[3 * k + c];
        p.kin[9 * k + 6 + c] = p.wp[3 * k + c];
    }
}

inline unsigned nblk(long long n, int t = 256) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }

const int CX[19] = {0, 1, 0, 0, 1, 1, 1, 1, 0, 0, -1, 0, 0, -1, -1, -1, -1, 0, 0};
const int CY[19] = {0, 0, 1, 0, 1, -1, 0, 0, 1, 1, 0, -1, 0, -1, 1, 0, 0, -1, -1};
const int CZ[19] = {0, 0, 0, 1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 0, 0, -1, 1, -1, 1};
inline int OPP(int i) { return i == 0 ? 0 : (i <= 9 ? i + 9 : i - 9); }
inline double WT(int i) { return i == 0 ? 1.0 / 3.0 : (((i - 1) % 9) < 3 ? 1.0 / 18.0 : 1.0 / 36.0); }

size_t storage_bytes(int prec) { return prec == 0 ? 8 : (prec == 1 ? 4 : 2); }

double decode(const unsigned char* raw, int prec, long long idx) {
    switch (prec) {
        case 0: return ((const double*)raw)[idx];
        case 1: return (double)((const float*)raw)[idx];
        case 2: {
            unsigned u = ((unsigned)((const unsigned short*)raw)[idx]) << 16;
            float f;
            memcpy(&f, &u, 4);
            return (double)f;
        }
        default: return (double)((const _Float16*)raw)[idx];
    }
}

void encode(unsigned char* raw, int prec, long long idx, double v) {
    switch (prec) {
        case 0: ((double*)raw)[idx] = v; break;
        case 1: ((float*)raw)[idx] = (float)v; break;
        case 2: {
            float f = (float)v;
            unsigned u;
            memcpy(&u, &f, 4);
            if ((u & 0x7fffffffu) > 0x7f800000u) u = (u >> 16) | 0x40u;
            else u = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
            ((unsigned short*)raw)[idx] = (unsigned short)u;
            break;
        }
        default: ((_Float16*)raw)[idx] = (_Float16)(float)v; break;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// stages
// ---------------------------------------------------------------------------
static int run_voxelize(psmdem_domain* D) {
    // without particles the tile lists stay empty as created: every tile is fluid
    if (D->np == 0) {
        D->voxelized = true;
        return 0;
    }
    VoxArgs V = D->vox_args();
    V.t.slot_beta = nullptr;  // only the read-back needs beta itself (B drives the step)
    int tk = D->timed_begin(PSMDEM_T_VOXEL);
    PSM_CHECK(vox_register(V, D->scan_tmp, D->s));
    PSM_CHECK(vox_voxelize(V, D->prec == 0, D->s));
    D->timed_end(tk);
    D->voxelized = true;
    D->tile_counts = true;
    D->beta_fresh = false;
    return 0;
}

// beta of the kept slots into t.slot_beta when the last voxelisation left it
// out: the same selection again from that voxelisation's particle records
// and count boxes, which stay until the next one
static int fresh_beta(psmdem_domain* D) {
    if (D->beta_fresh || !D->voxelized) return 0;
    PSM_CHECK(vox_select(D->vox_args(), D->prec == 0, D->s));
    PSM_CHECK(hipStreamSynchronize(D->s));
    D->beta_fresh = true;
    return 0;
}

// the LBM-PSM pass, then the hydrodynamic sums unless the caller runs them
// with the DEM corrector (dem_hydro_correct)
static int run_lbm(psmdem_domain* D, bool hydro = true) {
    LbmArgs A = D->lbm_args();
    int tk = D->timed_begin(PSMDEM_T_LBM);
    PSM_CHECK(lbm_step(A, D->prec, (int)(D->step & 1), D->s));
    D->timed_end(tk);
    if (!hydro) return 0;
    VoxArgs V = D->vox_args();
    tk = D->timed_begin(PSMDEM_T_HYDRO);
    PSM_CHECK(vox_reduce_hydro(V, D->s));
    D->timed_end(tk);
    return 0;
}

// the single-workgroup DEM may keep its pair list across launches; any other
// writer of the lists, cells or particle state makes its next launch rebuild
static int forget_fused_list(psmdem_domain* D) {
    if (D->np > 0) PSM_CHECK(hipMemsetAsync(D->fused_age, 0xff, 2 * sizeof(int), D->s));
    if (D->fz) PSM_CHECK(hipMemsetAsync(D->fz, 0xff, sizeof(int), D->s));
    return 0;
}

static int run_lists(psmdem_domain* D) {
    if (int rc = forget_fused_list(D)) return rc;
    DemArgs A = D->dem_args();
    PairBufs B = D->pair_bufs(1);
    PSM_CHECK(dem_lists(A, B, D->scan_tmp, D->s));
    return 0;
}

static int coupled_step(psmdem_domain* D) {
    int rc;
    if (D->d.dem_on && D->np > 0 && D->np <= DEM_FUSED_MAX && D->nc[0] < 65536 && D->nc[1] < 65536 &&
        D->nc[2] < 65536) {
        // every DEM substep in one workgroup launch; with the fluid on, the last
        // substep stops after the DEM sums and the corrector follows the coupling
        const bool couple = D->d.fluid_on != 0;
        DemArgs A = D->dem_args();
        int tk = D->timed_begin(PSMDEM_T_DEM);
        PSM_CHECK(dem_fused(A, D->pair_set(), D->cur, D->nsub, D->dt, couple ? 1 : 0, D->s));
        D->timed_end(tk);
        D->cur ^= (D->nsub & 1);
        if (couple) {
            if ((rc = run_voxelize(D))) return rc;
            if ((rc = run_lbm(D, false))) return rc;
            tk = D->timed_begin(PSMDEM_T_HYDRO);
            PSM_CHECK(dem_hydro_correct(A, D->t, D->dt, D->s));
            D->timed_end(tk);
        }
    } else if (D->d.dem_on && D->np > 0) {
        // a substep's corrector and the next substep's predictor share a launch
        for (int sub = 1; sub <= D->nsub; ++sub) {
            const bool last = sub == D->nsub;
            int tk = D->timed_begin(PSMDEM_T_DEM);
            // the list is rebuilt only when some particle's cells or wall
            // candidates changed (decided on the device, list_flag[par])
            const int par = (int)(D->dem_sub++ & 1);
            DemArgs A = D->dem_args();
            A.list_run = A.list_flag + par;
            if (sub == 1) PSM_CHECK(dem_predict_keep(A, D->dt, last ? 1 : 0, par, D->s));
            D->cur ^= 1;
            PairBufs B = D->pair_bufs(1);
            PSM_CHECK(dem_lists_kept(A, B, par, D->scan_tmp, D->s));
            PSM_CHECK(dem_columns(A, B, D->scan_tmp, D->s));
            PSM_CHECK(dem_contacts(A, B, D->p.vp, D->p.wp, D->dt, D->scan_tmp, D->s, false));
            // a substep that is followed by another runs its sums with the
            // corrector and the next predictor
            if (last) PSM_CHECK(dem_sums(A, B, D->s));
            if (last && D->d.fluid_on) {
                D->timed_end(tk);
                if ((rc = run_voxelize(D))) return rc;
                if ((rc = run_lbm(D, false))) return rc;
                tk = D->timed_begin(PSMDEM_T_HYDRO);
                PSM_CHECK(dem_hydro_correct(A, D->t, D->dt, D->s));
            } else if (last) {
                PSM_CHECK(dem_correct(A, D->dt, D->s));
            } else {
                PSM_CHECK(dem_sum_correct_predict(A, B, D->dt, sub + 1 == D->nsub ? 1 : 0, (int)(D->dem_sub & 1),
                                                  D->s));
            }
            D->timed_end(tk);
        }
    } else if (D->d.fluid_on) {
        if (D->np > 0) k_kin<<<nblk(D->np), 256, 0, D->s>>>(D->p, 1);
        if ((rc = run_voxelize(D))) return rc;
        if ((rc = run_lbm(D))) return rc;
    }
    D->step++;
    return 0;
}

// ---------------------------------------------------------------------------
// creation
// ---------------------------------------------------------------------------
static int validate(const psmdem_desc* d, const psmdem_particles* P) {
    if (!d) { psm_set_error("desc is NULL"); return 0; }
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) { psm_set_error("lattice extents must be >= 1"); return 0; }
    if (!(d->tau > 0.5)) { psm_set_error("tau must exceed 1/2"); return 0; }
    for (int a = 0; a < 3; ++a) {
        int p0 = d->bc[2 * a] == 0, p1 = d->bc[2 * a + 1] == 0;
        if (p0 != p1) { psm_set_error("axis %d: periodic on one face only", a); return 0; }
        for (int f = 0; f < 2; ++f)
            if (d->bc[2 * a + f] < 0 || d->bc[2 * a + f] > 2) { psm_set_error("invalid boundary code"); return 0; }
    }
    if (d->precision < 0 || d->precision > 3) { psm_set_error("invalid precision"); return 0; }
    if (d->sf_method < 0 || d->sf_method > 1) { psm_set_error("invalid sf_method"); return 0; }
    if (d->sf_subdiv < 1 || d->sf_subdiv > 32) { psm_set_error("sf_subdiv must be in 1..32"); return 0; }
    if (d->max_solids < 1 || d->max_solids > PSM_SLOTS_MAX) { psm_set_error("max_solids must be in 1..4"); return 0; }
    if (d->collision < 0 || d->collision > 1) { psm_set_error("invalid collision operator"); return 0; }
    if (d->collision == 1 && !(d->trt_magic >= 0.0 && d->trt_magic < 1e6)) {
        psm_set_error("trt_magic must be 0 (the paper's rule) or a positive magic parameter"); return 0;
    }
    if (d->kolm_amp != 0.0 && (d->kolm_axis < 0 || d->kolm_axis > 2 || d->kolm_dir < 0 || d->kolm_dir > 2)) {
        psm_set_error("invalid Kolmogorov axis"); return 0;
    }
    if (d->contact_law < 0 || d->contact_law > 1) { psm_set_error("invalid contact_law"); return 0; }
    if (d->contact_law == 1 && (!(d->young > 0.0) || !(d->poisson >= 0.0 && d->poisson < 0.5))) {
        psm_set_error("the Hertz law needs young > 0 and poisson in [0, 1/2)"); return 0;
    }
    if (d->contact_law == 1 && P && P->n > 0 && d->dem_on && d->n_sub < 1) {
        psm_set_error("the Hertz law needs n_sub >= 1 (its contact time depends on the impact speed)"); return 0;
    }
    if (P && P->n < 0) { psm_set_error("negative particle count"); return 0; }
    if (P && P->n > 0) {
        if (!P->shape || !P->semi_axes || !P->density_ratio || !P->pos) {
            psm_set_error("particle arrays missing"); return 0;
        }
        if (!(d->restitution > 0.0 && d->restitution <= 1.0)) { psm_set_error("restitution must be in (0,1]"); return 0; }
        if (d->kn < 0.0 || d->mu < 0.0) { psm_set_error("kn and mu must be >= 0"); return 0; }
        for (int k = 0; k < P->n; ++k) {
            if (P->shape[k] != 0 && P->shape[k] != 1) { psm_set_error("invalid shape of particle %d", k); return 0; }
            if (P->shape[k] == 1 && d->sf_method == 1) {
                psm_set_error("distance solid fraction is for spheres only"); return 0;
            }
            int na = P->shape[k] == 0 ? 1 : 3;
            for (int a = 0; a < na; ++a)
                if (!(P->semi_axes[3 * k + a] > 0.0)) { psm_set_error("semi-axes must be > 0"); return 0; }
            if (!(P->density_ratio[k] > 0.0)) { psm_set_error("density ratio must be > 0"); return 0; }
        }
    }
    return 1;
}

psmdem_status psm_domain_create(const psmdem_desc* desc, const psmdem_particles* parts, void* stream,
                                psmdem_alloc_fn alloc, psmdem_free_fn free_fn, void* alloc_ctx, bool dry,
                                psmdem_domain** out, size_t* bytes) {
    if (!out && !dry) { psm_set_error("out is NULL"); return PSMDEM_E_INVALID; }
    if (out) *out = nullptr;
    if (!validate(desc, parts)) return PSMDEM_E_INVALID;
    int ndev = 0;
    if (!dry && (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)) {
        psm_set_error("no HIP device");
        return PSMDEM_E_NODEVICE;
    }
    psmdem_domain* D = new psmdem_domain();
    D->dry = dry;
    if (!dry && hipGetDevice(&D->dev) != hipSuccess) D->dev = 0;
    D->d = *desc;
    D->s = (hipStream_t)stream;
    D->alloc = alloc;
    D->freef = free_fn;
    D->actx = alloc_ctx;
    const psmdem_desc& d = D->d;
    D->prec = d.precision;
    D->np = parts ? parts->n : 0;
    const int np = D->np;
    D->N = (long long)d.nx * d.ny * d.nz;
    GeoArgs& g = D->geo;
    g.nx = d.nx; g.ny = d.ny; g.nz = d.nz; g.N = D->N;
    g.ntx = (d.nx + PSM_TX - 1) / PSM_TX;
    g.nty = (d.ny + PSM_TY - 1) / PSM_TY;
    g.ntz = (d.nz + PSM_TZ - 1) / PSM_TZ;
    g.ntiles = (long long)g.ntx * g.nty * g.ntz;
    for (int a = 0; a < 3; ++a) g.periodic[a] = d.bc[2 * a] == 0;
    for (int f = 0; f < 6; ++f) g.bc[f] = d.bc[f];
    D->L[0] = d.nx; D->L[1] = d.ny; D->L[2] = d.nz;
    for (int f = 0; f < 6; ++f)
        for (int i = 0; i < 19; ++i) {
            double cu = CX[i] * d.wall_u[f][0] + CY[i] * d.wall_u[f][1] + CZ[i] * d.wall_u[f][2];
            D->wall_corr[f][i] = (d.bc[f] == 2) ? 6.0 * WT(i) * d.rho0 * cu : 0.0;
        }
    double e = d.restitution > 0 ? d.restitution : 1.0;
    D->beta_e = log(e) / sqrt(log(e) * log(e) + M_PI * M_PI);
    if (d.contact_law == 1) {
        // App. A with both bodies of the one material
        const double E = d.young, nu = d.poisson;
        D->ystar = 1.0 / ((1.0 - nu * nu) / E + (1.0 - nu * nu) / E);
        D->gstar = 1.0 / (2.0 * (2.0 - nu) * (1.0 + nu) / E + 2.0 * (2.0 - nu) * (1.0 + nu) / E);
    }
    D->Rc = cbrt(3.0 / (4.0 * M_PI));

    // host particle properties
    std::vector<double> semi(3 * (size_t)np), mass(np), inertia(3 * (size_t)np), rb(np), dens(np);
    std::vector<double> pos(3 * (size_t)np), q(4 * (size_t)np), v(3 * (size_t)np, 0.0), w(3 * (size_t)np, 0.0);
    std::vector<unsigned char> fixed(np, 0);
    D->h_shape.assign(np, 0);
    double dmax = 0.0;
    for (int k = 0; k < np; ++k) {
        int sh = parts->shape[k];
        D->h_shape[k] = sh;
        for (int a = 0; a < 3; ++a) {
            semi[3 * k + a] = sh == 0 ? parts->semi_axes[3 * k] : parts->semi_axes[3 * k + a];
            pos[3 * k + a] = parts->pos[3 * k + a];
            if (parts->vel) v[3 * k + a] = parts->vel[3 * k + a];
            if (parts->omega) w[3 * k + a] = parts->omega[3 * k + a];
        }
        double qq[4] = {1.0, 0.0, 0.0, 0.0};
        if (parts->quat)
            for (int c = 0; c < 4; ++c) qq[c] = parts->quat[4 * k + c];
        double qn = sqrt(qq[0] * qq[0] + qq[1] * qq[1] + qq[2] * qq[2] + qq[3] * qq[3]);
        if (!(qn > 0.0)) { delete D; psm_set_error("zero quaternion for particle %d", k); return PSMDEM_E_INVALID; }
        for (int c = 0; c < 4; ++c) q[4 * k + c] = qq[c] / qn;
        dens[k] = parts->density_ratio[k];
        fixed[k] = parts->fixed ? parts->fixed[k] : 0;
        const double* s3 = &semi[3 * k];
        double V = sh == 0 ? 4.0 / 3.0 * M_PI * s3[0] * s3[0] * s3[0] : 4.0 / 3.0 * M_PI * s3[0] * s3[1] * s3[2];
        double m = dens[k] * d.rho0 * V;
        mass[k] = m;
        if (sh == 0) {
            inertia[3 * k] = inertia[3 * k + 1] = inertia[3 * k + 2] = 0.4 * m * s3[0] * s3[0];
            rb[k] = s3[0];
        } else {
            inertia[3 * k + 0] = m / 5.0 * (s3[1] * s3[1] + s3[2] * s3[2]);
            inertia[3 * k + 1] = m / 5.0 * (s3[0] * s3[0] + s3[2] * s3[2]);
            inertia[3 * k + 2] = m / 5.0 * (s3[0] * s3[0] + s3[1] * s3[1]);
            rb[k] = std::max(s3[0], std::max(s3[1], s3[2]));
        }
        dmax = std::max(dmax, 2.0 * rb[k]);
    }
    double rbmax = dmax / 2.0;
    for (int a = 0; a < 3; ++a)
        if (g.periodic[a] && np > 0 && 2.0 * (rbmax + D->Rc + 1.0) + 1.0 > D->L[a]) {
            delete D;
            psm_set_error("periodic axis %d too short for the largest particle", a);
            return PSMDEM_E_INVALID;
        }
    // tiles one particle box may touch per axis
    {
        const int T[3] = {PSM_TX, PSM_TY, PSM_TZ};
        for (int a = 0; a < 3; ++a) {
            int span = (int)ceil(2.0 * (rbmax + D->Rc + 1e-6)) + 2;
            if (span / T[a] + 3 > VOX_AXIS_MAX) {
                delete D;
                psm_set_error("particles too large for the lattice tiles");
                return PSMDEM_E_INVALID;
            }
        }
    }
    // DEM grid: n_c = floor(L / (1.1 d_max)), h = L / n_c
    for (int a = 0; a < 3; ++a) {
        int n;
        if (d.dem_cell > 0.0) n = (int)floor(D->L[a] / d.dem_cell);
        else n = dmax > 0.0 ? (int)floor(D->L[a] / (1.1 * dmax)) : 1;
        if (n < 1) n = 1;
        if (np > 0 && g.periodic[a] && n < 2) {
            delete D;
            psm_set_error("periodic axis %d has fewer than 2 DEM cells", a);
            return PSMDEM_E_INVALID;
        }
        D->nc[a] = n;
        D->h[a] = D->L[a] / (double)n;
        if (n > 1 && !(D->h[a] > dmax)) {
            delete D;
            psm_set_error("DEM cell smaller than the largest diameter");
            return PSMDEM_E_INVALID;
        }
    }
    D->ncell = (long long)D->nc[0] * D->nc[1] * D->nc[2];
    if (d.n_sub > 0) {
        D->nsub = d.n_sub;
    } else if (np == 0 || d.kn <= 0.0) {
        D->nsub = 1;
    } else {
        std::vector<double> ms(mass);
        std::sort(ms.begin(), ms.end());
        double mst = np >= 2 ? ms[0] * ms[1] / (ms[0] + ms[1]) : ms[0];
        double tc = M_PI * sqrt(mst / d.kn) / sqrt(1.0 - D->beta_e * D->beta_e);
        D->nsub = std::max(1, (int)ceil(20.0 / tc));
    }
    D->dt = 1.0 / (double)D->nsub;

    // ---- device allocation
    bool ok = true;
    auto A = [&](size_t n) {
        void* p_ = D->dalloc(n);
        ok = ok && p_ != nullptr;
        return p_;
    };
    D->f = A(19 * (size_t)D->N * storage_bytes(D->prec));
    PartArgs& P = D->p;
    P.np = np;
    P.shape = (int*)A(sizeof(int) * std::max(np, 1));
    P.fixed = (unsigned char*)A(std::max(np, 1));
    double** d3[] = {&P.semi, &P.inertia, &P.pos, &P.v, &P.w, &P.vp, &P.wp, &P.a, &P.al, &P.fh, &P.mh, &P.fd, &P.md};
    for (double** pp : d3) *pp = (double*)A(sizeof(double) * 3 * std::max(np, 1));
    P.mass = (double*)A(sizeof(double) * std::max(np, 1));
    P.rb = (double*)A(sizeof(double) * std::max(np, 1));
    P.dens = (double*)A(sizeof(double) * std::max(np, 1));
    P.q = (double*)A(sizeof(double) * 4 * std::max(np, 1));
    P.qold = (double*)A(sizeof(double) * 4 * std::max(np, 1));
    P.kin = (double*)A(sizeof(double) * 9 * std::max(np, 1));
    D->reg_cap = 8LL * std::max(np, 1);
    D->pc = (int*)A(sizeof(int) * 8 * std::max(np, 1));
    D->fused_age = (int*)A(2 * sizeof(int));
    // the fused DEM kernel's saved skip state (domains it runs)
    D->fz = np > 0 && np <= DEM_FUSED_MAX ? (unsigned char*)A(dem_fused_save_bytes()) : nullptr;
    D->list_flag = (int*)A(2 * sizeof(int));
    D->cell_count = (int*)A(sizeof(int) * D->ncell);
    D->cell_fill = (int*)A(sizeof(int) * D->ncell);
    D->cell_start = (int*)A(sizeof(int) * (D->ncell + 1));
    D->cell_pid = (int*)A(sizeof(int) * D->reg_cap);
    D->pair_cap = d.pair_capacity > 0 ? d.pair_capacity : 32LL * np + 1024;
    D->row_lb = (unsigned long long*)A(sizeof(unsigned long long) * (np / DEM_ROWS_PER_WG + 2));
    for (int b = 0; b < 2; ++b) {
        D->prow[b] = (int*)A(sizeof(int) * (np + 1));
        D->pairs[b] = (unsigned long long*)A(sizeof(unsigned long long) * D->pair_cap);
        D->hist[b] = (double*)A(sizeof(double) * 3 * D->pair_cap);
    }
    D->cF = (double*)A(sizeof(double) * 3 * D->pair_cap);
    D->cMi = (double*)A(sizeof(double) * 3 * D->pair_cap);
    D->cMj = (double*)A(sizeof(double) * 3 * D->pair_cap);
    D->incontact = (unsigned char*)A(D->pair_cap);
    bool any_ell = false;
    for (int k = 0; k < np; ++k) any_ell = any_ell || D->h_shape[k] != 0;
    if (any_ell) {
        D->ell_seg_cap = dem_ell_seg_cap(D->pair_cap);
        D->ell_list = (int*)A(sizeof(int) * (size_t)(DEM_ELL_SEGS * D->ell_seg_cap));
        D->ell_cnt = (unsigned*)A(sizeof(unsigned) * DEM_ELL_SEGS);
    }
    D->col_count = (int*)A(sizeof(int) * std::max(np, 1));
    D->col_fill = (int*)A(sizeof(int) * std::max(np, 1));
    D->col_start = (int*)A(sizeof(int) * (np + 1));
    D->col_list = (int*)A(sizeof(int) * D->pair_cap);
    // tiles
    long long per_particle = 1;
    {
        const int T[3] = {PSM_TX, PSM_TY, PSM_TZ};
        for (int a = 0; a < 3; ++a) {
            int span = (int)ceil(2.0 * (rbmax + D->Rc + 1e-6)) + 2;
            per_particle *= std::min<long long>(span / T[a] + 3, VOX_AXIS_MAX);
        }
    }
    TileArgs& t = D->t;
    t.cap = std::max<long long>(1, per_particle * np);
    t.tile_start = (int*)A(sizeof(int) * (g.ntiles + 1));
    t.tile_list = (unsigned long long*)A(sizeof(unsigned long long) * t.cap);
    t.vcount = (int*)A(sizeof(int) * std::max(np, 1));
    t.voff = (int*)A(sizeof(int) * (np + 1));
    t.vinv = (int*)A(sizeof(int) * t.cap);
    const long long plane = g.ntiles * (long long)PSM_TILE;
    t.slot_lp = (unsigned*)A(sizeof(unsigned) * plane);
    t.slot_B = A((D->prec == 0 ? 8 : 4) * (size_t)plane * d.max_solids);
    t.slot_beta = (double*)A(sizeof(double) * (size_t)plane * d.max_solids);
    t.tile_ed = (unsigned*)A(sizeof(unsigned) * 2 * (size_t)g.ntiles);
    t.partial = (double*)A(sizeof(double) * 6 * t.cap);
    D->tile_count = (int*)A(sizeof(int) * g.ntiles);
    D->tile_fill = (int*)A(sizeof(int) * g.ntiles);
    if (np > 0) D->vpart = A(vox_part_bytes() * (size_t)np);
    if (np > 0 && d.sf_method == 0) {
        const size_t nt = (size_t)d.sf_subdiv * d.sf_subdiv * d.sf_subdiv + 1;
        D->btab = A((D->prec == 0 ? 8 : 4) * nt);
        D->betatab = (double*)A(sizeof(double) * nt);
    }
    // subdivision method: one count box per particle, sized for the largest
    // lattice box (per axis at most floor(2 r_b + 2e-6) + 2 cells)
    if (np > 0 && d.sf_method == 0) {
        const long long side = (long long)floor(2.0 * rbmax + 2e-6) + 2;
        if (side * side > (long long)vox_box_cells_max()) {  // (the tile limit above keeps it far below)
            delete D;
            psm_set_error("particles too large for the solid-fraction count boxes");
            return PSMDEM_E_INVALID;
        }
        D->box_stride = side * side * side;
        D->vbox = (unsigned short*)A(sizeof(unsigned short) * (size_t)D->box_stride * np);
    }
    long long scan_n = std::max<long long>(std::max<long long>(D->ncell, g.ntiles), np + 1);
    D->scan_tmp = (int*)A(sizeof(int) * psm_scan_tmp_ints(scan_n));
    D->ctr = (DevCounters*)A(sizeof(DevCounters));
    D->wall_corr_d = (double*)A(sizeof(double) * 6 * 19);
    if (d.kolm_amp != 0.0) {
        int n_ax = d.kolm_axis == 0 ? d.nx : (d.kolm_axis == 1 ? d.ny : d.nz);
        std::vector<double> prof(n_ax);
        for (int c = 0; c < n_ax; ++c) prof[c] = d.kolm_amp * sin(2.0 * M_PI * ((double)c + 0.5) / (double)n_ax);
        D->kolm_prof = (double*)A(sizeof(double) * n_ax);
        if (ok && !dry &&
            hipMemcpy(D->kolm_prof, prof.data(), sizeof(double) * n_ax, hipMemcpyHostToDevice) != hipSuccess)
            ok = false;
    }
    if (!ok) {
        delete D;
        psm_set_error("device allocation failed");
        return PSMDEM_E_NOMEM;
    }
    if (dry) {
        if (bytes) *bytes = D->bytes;
        delete D;
        return PSMDEM_OK;
    }
    int rc = 0;
    auto H2D = [&](void* dst, const void* src, size_t n) {
        if (n && (hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, D->s) != hipSuccess ||
                  hipStreamSynchronize(D->s) != hipSuccess))
            rc = PSMDEM_E_HIP;
    };
    if (np > 0) {
        std::vector<int> shp(D->h_shape);
        H2D((void*)P.shape, shp.data(), sizeof(int) * np);
        H2D((void*)P.fixed, fixed.data(), np);
        H2D(P.semi, semi.data(), sizeof(double) * 3 * np);
        H2D(P.inertia, inertia.data(), sizeof(double) * 3 * np);
        H2D(P.pos, pos.data(), sizeof(double) * 3 * np);
        H2D(P.v, v.data(), sizeof(double) * 3 * np);
        H2D(P.w, w.data(), sizeof(double) * 3 * np);
        H2D(P.mass, mass.data(), sizeof(double) * np);
        H2D(P.rb, rb.data(), sizeof(double) * np);
        H2D(P.dens, dens.data(), sizeof(double) * np);
        H2D(P.q, q.data(), sizeof(double) * 4 * np);
        std::vector<double> zero(3 * (size_t)np, 0.0);
        for (double* z : {P.a, P.al, P.fh, P.mh, P.fd, P.md, P.vp, P.wp}) H2D(z, zero.data(), sizeof(double) * 3 * np);
    }
    {
        std::vector<int> z(np + 1, 0);
        for (int b = 0; b < 2; ++b) H2D(D->prow[b], z.data(), sizeof(int) * (np + 1));
        H2D(D->t.voff, z.data(), sizeof(int) * (np + 1));
        std::vector<int> zt(g.ntiles + 1, 0);
        H2D(D->t.tile_start, zt.data(), sizeof(int) * (g.ntiles + 1));
        DevCounters c0{};
        H2D(D->ctr, &c0, sizeof c0);
        H2D(D->wall_corr_d, D->wall_corr, sizeof(double) * 6 * 19);
        // registration lists start out valid (particle 0, entry 0)
        if (hipMemsetAsync(D->t.tile_list, 0, sizeof(unsigned long long) * D->t.cap, D->s) != hipSuccess ||
            hipMemsetAsync(D->tile_count, 0, sizeof(int) * g.ntiles, D->s) != hipSuccess ||
            hipMemsetAsync(D->cell_count, 0, sizeof(int) * D->ncell, D->s) != hipSuccess ||
            hipMemsetAsync(D->cell_fill, 0, sizeof(int) * D->ncell, D->s) != hipSuccess ||
            hipMemsetAsync(D->col_count, 0, sizeof(int) * std::max(np, 1), D->s) != hipSuccess ||
            hipMemsetAsync(D->col_fill, 0, sizeof(int) * std::max(np, 1), D->s) != hipSuccess ||
            hipMemsetAsync(D->tile_fill, 0, sizeof(int) * g.ntiles, D->s) != hipSuccess ||
            hipMemsetAsync(D->t.vinv, 0, sizeof(int) * D->t.cap, D->s) != hipSuccess ||
            hipMemsetAsync(D->t.slot_lp, 0xff, sizeof(unsigned) * g.ntiles * (size_t)PSM_TILE, D->s) != hipSuccess ||
            hipMemsetAsync(D->t.tile_ed, 0, sizeof(unsigned) * 2 * (size_t)g.ntiles, D->s) != hipSuccess ||
            hipMemsetAsync(D->cell_pid, 0, sizeof(int) * D->reg_cap, D->s) != hipSuccess ||
            hipMemsetAsync(D->fused_age, 0xff, 2 * sizeof(int), D->s) != hipSuccess ||
            (D->fz && hipMemsetAsync(D->fz, 0xff, sizeof(int), D->s) != hipSuccess) ||
            hipMemsetAsync(D->list_flag, 0, 2 * sizeof(int), D->s) != hipSuccess ||
            (D->ell_cnt && hipMemsetAsync(D->ell_cnt, 0, sizeof(unsigned) * DEM_ELL_SEGS, D->s) != hipSuccess) ||
            hipStreamSynchronize(D->s) != hipSuccess)
            rc = PSMDEM_E_HIP;
    }
    if (rc) {
        delete D;
        psm_set_error("initial copies failed");
        return PSMDEM_E_HIP;
    }
    if (D->btab && vox_fill_tables(D->btab, D->betatab, d.sf_subdiv, d.tau, D->prec == 0, D->s) != hipSuccess) {
        delete D;
        psm_set_error("init kernel failed");
        return PSMDEM_E_HIP;
    }
    if (lbm_init(D->f, D->prec, D->N, d.rho0, D->s) != hipSuccess) {
        delete D;
        psm_set_error("init kernel failed");
        return PSMDEM_E_HIP;
    }
    if (np > 0) {
        // initial DEM forces: zero history, no increment (a(0) from F_dem(0) + F_ext)
        D->cur = 0;
        DemArgs A0 = D->dem_args();
        PairBufs B0 = D->pair_bufs(0);
        if (dem_lists(A0, B0, D->scan_tmp, D->s) != hipSuccess ||
            dem_contacts(A0, B0, P.v, P.w, 0.0, D->scan_tmp, D->s) != hipSuccess ||
            dem_initial_accel(A0, D->s) != hipSuccess || dem_zero(D->hist[0], 3 * D->pair_cap, D->s) != hipSuccess) {
            delete D;
            psm_set_error("initial DEM evaluation failed");
            return PSMDEM_E_HIP;
        }
    }
    if (hipStreamSynchronize(D->s) != hipSuccess) {
        delete D;
        psm_set_error("device error during creation: %s", hipGetErrorString(hipGetLastError()));
        return PSMDEM_E_HIP;
    }
    if (bytes) *bytes = D->bytes;
    *out = D;
    return PSMDEM_OK;
}

extern "C" psmdem_status psmdem_create(const psmdem_desc* desc, const psmdem_particles* parts, void* stream,
                                       psmdem_alloc_fn alloc, psmdem_free_fn free_fn, void* alloc_ctx,
                                       psmdem_domain** out) {
    return psm_domain_create(desc, parts, stream, alloc, free_fn, alloc_ctx, false, out, nullptr);
}

extern "C" psmdem_status psmdem_footprint(const psmdem_desc* desc, const psmdem_particles* parts, int64_t* bytes) {
    if (!bytes) { psm_set_error("bytes is NULL"); return PSMDEM_E_INVALID; }
    size_t b = 0;
    psmdem_status rc = psm_domain_create(desc, parts, nullptr, nullptr, nullptr, nullptr, true, nullptr, &b);
    *bytes = rc == PSMDEM_OK ? (int64_t)b : 0;
    return rc;
}

extern "C" void psmdem_destroy(psmdem_domain* d) { delete d; }

extern "C" psmdem_status psmdem_step(psmdem_domain* d, int64_t n) {
    if (!d || n < 0) { psm_set_error("invalid arguments"); return PSMDEM_E_INVALID; }
    if (d->timing) {
        for (int k = 0; k < 4; ++k) { d->t_ms[k] = 0; d->t_n[k] = 0; }
    }
    for (int64_t k = 0; k < n; ++k) {
        int rc = coupled_step(d);
        if (rc) return (psmdem_status)rc;
    }
    if (d->timing) {
        if (hipStreamSynchronize(d->s) != hipSuccess) return psm_hip_fail(hipGetLastError(), "sync", __FILE__, __LINE__);
        d->collect_timing();
    }
    return PSMDEM_OK;
}

// Waits for the stream and reports the device flags: PSMDEM_E_UNSTABLE when
// the state has blown up, else PSMDEM_E_CAPACITY when a device list outgrew
// its capacity.  The flags stay set until a write_* call rewrites the state.
psmdem_status psm_sync_flags(psmdem_domain* d) {
    PSM_CHECK(hipStreamSynchronize(d->s));
    DevCounters c{};
    PSM_CHECK(hipMemcpy(&c, d->ctr, sizeof c, hipMemcpyDeviceToHost));
    if (c.flags & PSM_FLAG_UNSTABLE) {
        psm_set_error("unstable: a cell density is not a positive finite number or a particle centre is not finite "
                      "or lies more than one box length outside the domain (flags 0x%llx)",
                      (unsigned long long)c.flags);
        return PSMDEM_E_UNSTABLE;
    }
    if (c.flags & PSM_FLAG_CAPACITY_MASK) {
        psm_set_error("device capacity exceeded (flags 0x%llx: 1 pairs, 2 tile list, 4 neighbours, 8 tile registrations)",
                      (unsigned long long)c.flags);
        return PSMDEM_E_CAPACITY;
    }
    return PSMDEM_OK;
}

// a status of sync_flags that stops a read (the device flags do not: the
// outputs are still written and the flag is returned)
bool psm_read_fails(psmdem_status st) { return st != PSMDEM_OK && st != PSMDEM_E_CAPACITY && st != PSMDEM_E_UNSTABLE; }

// the state is being rewritten: the device flags of the old one are dropped
static psmdem_status clear_flags(psmdem_domain* d) {
    PSM_CHECK(hipStreamSynchronize(d->s));
    const unsigned long long z = 0;
    PSM_CHECK(hipMemcpy(&d->ctr->flags, &z, sizeof z, hipMemcpyHostToDevice));
    return PSMDEM_OK;
}

extern "C" psmdem_status psmdem_sync(psmdem_domain* d) {
    if (!d) return PSMDEM_E_INVALID;
    return psm_sync_flags(d);
}

extern "C" psmdem_status psmdem_stage(psmdem_domain* d, int32_t stage) {
    if (!d) return PSMDEM_E_INVALID;
    int rc = forget_fused_list(d);
    if (rc) return (psmdem_status)rc;
    switch (stage) {
        case PSMDEM_STAGE_LISTS:
            d->cur ^= 1;
            rc = run_lists(d);
            break;
        case PSMDEM_STAGE_VOXELIZE:
            rc = run_voxelize(d);
            break;
        case PSMDEM_STAGE_LBM:
            if (d->np > 0) k_kin<<<nblk(d->np), 256, 0, d->s>>>(d->p, 0);
            rc = run_lbm(d);
            if (!rc) d->step++;
            break;
        case PSMDEM_STAGE_CONTACTS: {
            // the current list, with its own history as the previous list
            int prev = d->cur;
            d->cur ^= 1;
            size_t nb = sizeof(unsigned long long) * d->pair_cap;
            if (hipMemcpyAsync(d->pairs[d->cur], d->pairs[prev], nb, hipMemcpyDeviceToDevice, d->s) != hipSuccess ||
                hipMemcpyAsync(d->prow[d->cur], d->prow[prev], sizeof(int) * (d->np + 1), hipMemcpyDeviceToDevice, d->s) != hipSuccess)
                return psm_hip_fail(hipGetLastError(), "copy", __FILE__, __LINE__);
            DemArgs A = d->dem_args();
            PairBufs B = d->pair_bufs(1);
            if (dem_count_columns(A, B, d->s) != hipSuccess || dem_columns(A, B, d->scan_tmp, d->s) != hipSuccess ||
                dem_contacts(A, B, d->p.vp, d->p.wp, d->dt, d->scan_tmp, d->s) != hipSuccess)
                return psm_hip_fail(hipGetLastError(), "contacts", __FILE__, __LINE__);
            break;
        }
        default:
            psm_set_error("unknown stage %d", stage);
            return PSMDEM_E_INVALID;
    }
    if (rc) return (psmdem_status)rc;
    return psm_sync_flags(d);
}

// ---------------------------------------------------------------------------
// populations: decode the in-place storage on the host
// ---------------------------------------------------------------------------
static void host_face(const psmdem_domain* D, int x, int y, int z, int dx, int dy, int dz, long long* cell, int* face) {
    const int c[3] = {x, y, z}, dd[3] = {dx, dy, dz};
    const int n[3] = {D->d.nx, D->d.ny, D->d.nz};
    int r[3];
    *face = -1;
    for (int a = 0; a < 3; ++a) {
        int v = c[a] + dd[a];
        if (v < 0 || v >= n[a]) {
            if (D->geo.periodic[a]) v = (v + n[a]) % n[a];
            else if (*face < 0) *face = v < 0 ? 2 * a : 2 * a + 1;
        }
        r[a] = v;
    }
    *cell = (long long)r[0] + (long long)n[0] * ((long long)r[1] + (long long)n[1] * r[2]);
}

extern "C" psmdem_status psmdem_read_populations(psmdem_domain* d, double* fout) {
    if (!d || !fout) return PSMDEM_E_INVALID;
    const psmdem_status st = psm_sync_flags(d);
    if (psm_read_fails(st)) return st;
    const long long N = d->N;
    const size_t sb = storage_bytes(d->prec);
    std::vector<unsigned char> raw(19 * (size_t)N * sb);
    PSM_CHECK(hipMemcpy(raw.data(), d->f, raw.size(), hipMemcpyDeviceToHost));
    const bool odd = (d->step & 1) != 0;
    for (long long c = 0; c < N; ++c) {
        int x = (int)(c % d->d.nx), y = (int)((c / d->d.nx) % d->d.ny), z = (int)(c / ((long long)d->d.nx * d->d.ny));
        for (int i = 0; i < 19; ++i) {
            double gi;
            if (!odd) {
                gi = decode(raw.data(), d->prec, (long long)i * N + c);
            } else {
                long long src;
                int face;
                host_face(d, x, y, z, -CX[i], -CY[i], -CZ[i], &src, &face);
                if (face >= 0) gi = decode(raw.data(), d->prec, (long long)i * N + c) + d->wall_corr[face][i];
                else gi = decode(raw.data(), d->prec, (long long)OPP(i) * N + src);
            }
            fout[(long long)i * N + c] = gi + WT(i);
        }
    }
    return st;
}

extern "C" psmdem_status psmdem_write_populations(psmdem_domain* d, const double* fin) {
    if (!d || !fin) return PSMDEM_E_INVALID;
    if (psmdem_status cs = clear_flags(d)) return cs;
    const long long N = d->N;
    const size_t sb = storage_bytes(d->prec);
    std::vector<unsigned char> raw(19 * (size_t)N * sb);
    const bool odd = (d->step & 1) != 0;
    for (long long c = 0; c < N; ++c) {
        int x = (int)(c % d->d.nx), y = (int)((c / d->d.nx) % d->d.ny), z = (int)(c / ((long long)d->d.nx * d->d.ny));
        for (int i = 0; i < 19; ++i) {
            double gi = fin[(long long)i * N + c] - WT(i);
            if (!odd) {
                encode(raw.data(), d->prec, (long long)i * N + c, gi);
            } else {
                long long src;
                int face;
                host_face(d, x, y, z, -CX[i], -CY[i], -CZ[i], &src, &face);
                if (face >= 0) encode(raw.data(), d->prec, (long long)i * N + c, gi - d->wall_corr[face][i]);
                else encode(raw.data(), d->prec, (long long)OPP(i) * N + src, gi);
            }
        }
    }
    PSM_CHECK(hipMemcpy(d->f, raw.data(), raw.size(), hipMemcpyHostToDevice));
    return PSMDEM_OK;
}

// ---------------------------------------------------------------------------
// particles, pairs, cells, solid slots
// ---------------------------------------------------------------------------
extern "C" psmdem_status psmdem_read_particles(psmdem_domain* d, double* pos, double* quat, double* vel, double* omega,
                                              double* acc, double* alpha, double* f_hyd, double* m_hyd, double* f_dem,
                                              double* m_dem) {
    if (!d) return PSMDEM_E_INVALID;
    const psmdem_status st = psm_sync_flags(d);
    if (psm_read_fails(st)) return st;
    size_t n3 = sizeof(double) * 3 * d->np;
    if (d->np == 0) return st;
    struct { double* h; double* dv; size_t n; } m[] = {
        {pos, d->p.pos, n3}, {quat, d->p.q, sizeof(double) * 4 * d->np}, {vel, d->p.v, n3}, {omega, d->p.w, n3},
        {acc, d->p.a, n3}, {alpha, d->p.al, n3}, {f_hyd, d->p.fh, n3}, {m_hyd, d->p.mh, n3},
        {f_dem, d->p.fd, n3}, {m_dem, d->p.md, n3}};
    for (auto& x : m)
        if (x.h) PSM_CHECK(hipMemcpy(x.h, x.dv, x.n, hipMemcpyDeviceToHost));
    return st;
}

extern "C" psmdem_status psmdem_write_particles(psmdem_domain* d, const double* pos, const double* quat,
                                               const double* vel, const double* omega, const double* acc,
                                               const double* alpha, const double* f_hyd, const double* m_hyd) {
    if (!d) return PSMDEM_E_INVALID;
    if (int rc = forget_fused_list(d)) return (psmdem_status)rc;
    if (psmdem_status cs = clear_flags(d)) return cs;
    if (d->np == 0) return PSMDEM_OK;
    size_t n3 = sizeof(double) * 3 * d->np;
    struct { const double* h; double* dv; size_t n; } m[] = {
        {pos, d->p.pos, n3}, {quat, d->p.q, sizeof(double) * 4 * d->np}, {vel, d->p.v, n3}, {omega, d->p.w, n3},
        {acc, d->p.a, n3}, {alpha, d->p.al, n3}, {f_hyd, d->p.fh, n3}, {m_hyd, d->p.mh, n3}};
    for (auto& x : m)
        if (x.h) PSM_CHECK(hipMemcpy(x.dv, x.h, x.n, hipMemcpyHostToDevice));
    if (quat) PSM_CHECK(hipMemcpy(d->p.qold, quat, sizeof(double) * 4 * d->np, hipMemcpyHostToDevice));
    return PSMDEM_OK;
}

extern "C" psmdem_status psmdem_read_predicted(psmdem_domain* d, double* vp, double* wp) {
    if (!d) return PSMDEM_E_INVALID;
    const psmdem_status st = psm_sync_flags(d);
    if (psm_read_fails(st)) return st;
    if (d->np == 0) return st;
    if (vp) PSM_CHECK(hipMemcpy(vp, d->p.vp, sizeof(double) * 3 * d->np, hipMemcpyDeviceToHost));
    if (wp) PSM_CHECK(hipMemcpy(wp, d->p.wp, sizeof(double) * 3 * d->np, hipMemcpyDeviceToHost));
    return st;
}

extern "C" psmdem_status psmdem_write_predicted(psmdem_domain* d, const double* vp, const double* wp) {
    if (!d) return PSMDEM_E_INVALID;
    if (int rc = forget_fused_list(d)) return (psmdem_status)rc;
    PSM_CHECK(hipStreamSynchronize(d->s));
    if (d->np == 0) return PSMDEM_OK;
    if (vp) PSM_CHECK(hipMemcpy(d->p.vp, vp, sizeof(double) * 3 * d->np, hipMemcpyHostToDevice));
    if (wp) PSM_CHECK(hipMemcpy(d->p.wp, wp, sizeof(double) * 3 * d->np, hipMemcpyHostToDevice));
    return PSMDEM_OK;
}

static psmdem_status pair_count(psmdem_domain* d, int64_t* n) {
    int v = 0;
    if (d->np > 0) PSM_CHECK(hipMemcpy(&v, d->prow[d->cur] + d->np, sizeof(int), hipMemcpyDeviceToHost));
    *n = v;
    return PSMDEM_OK;
}

extern "C" psmdem_status psmdem_read_pairs(psmdem_domain* d, int64_t cap, uint64_t* keys, double* hist, int64_t* n) {
    if (!d || !n) return PSMDEM_E_INVALID;
    const psmdem_status st = psm_sync_flags(d);
    if (psm_read_fails(st)) return st;
    int64_t np_ = 0;
    if (psmdem_status pc = pair_count(d, &np_)) return pc;
    *n = np_;
    int64_t m = std::min<int64_t>(std::min<int64_t>(np_, cap), d->pair_cap);
    if (m > 0 && keys) PSM_CHECK(hipMemcpy(keys, d->pairs[d->cur], sizeof(uint64_t) * m, hipMemcpyDeviceToHost));
    if (m > 0 && hist) PSM_CHECK(hipMemcpy(hist, d->hist[d->cur], sizeof(double) * 3 * m, hipMemcpyDeviceToHost));
    return st;
}

extern "C" psmdem_status psmdem_write_pairs(psmdem_domain* d, int64_t n, const uint64_t* keys, const double* hist) {
    if (!d || n < 0 || (n > 0 && (!keys || !hist))) return PSMDEM_E_INVALID;
    if (n > d->pair_cap) { psm_set_error("pair list exceeds the capacity"); return PSMDEM_E_CAPACITY; }
    if (int rc = forget_fused_list(d)) return (psmdem_status)rc;
    if (psmdem_status cs = clear_flags(d)) return cs;
    // rebuild row offsets from the sorted keys
    std::vector<int> row(d->np + 1, 0);
    for (int64_t s = 0; s < n; ++s) {
        uint64_t i = keys[s] >> 32;
        if ((s > 0 && keys[s] <= keys[s - 1]) || i >= (uint64_t)d->np) {
            psm_set_error("pair keys must be sorted, unique and index existing particles");
            return PSMDEM_E_INVALID;
        }
        row[i + 1]++;
    }
    for (int k = 0; k < d->np; ++k) row[k + 1] += row[k];
    if (d->np > 0) PSM_CHECK(hipMemcpy(d->prow[d->cur], row.data(), sizeof(int) * (d->np + 1), hipMemcpyHostToDevice));
    if (n > 0) {
        PSM_CHECK(hipMemcpy(d->pairs[d->cur], keys, sizeof(uint64_t) * n, hipMemcpyHostToDevice));
        PSM_CHECK(hipMemcpy(d->hist[d->cur], hist, sizeof(double) * 3 * n, hipMemcpyHostToDevice));
    }
    return PSMDEM_OK;
}

extern "C" psmdem_status psmdem_read_contacts(psmdem_domain* d, int64_t cap, uint64_t* keys, double* force, double* m_i,
                                             double* m_j, int64_t* n) {
    if (!d || !n) return PSMDEM_E_INVALID;
    const psmdem_status st = psm_sync_flags(d);
    if (psm_read_fails(st)) return st;
    int64_t np_ = 0;
    if (psmdem_status pc = pair_count(d, &np_)) return pc;
    np_ = std::min<int64_t>(np_, d->pair_cap);
    std::vector<uint64_t> k(np_);
    std::vector<unsigned char> ic(np_);
    std::vector<double> F(3 * np_), Mi(3 * np_), Mj(3 * np_);
    if (np_ > 0) {
        PSM_CHECK(hipMemcpy(k.data(), d->pairs[d->cur], sizeof(uint64_t) * np_, hipMemcpyDeviceToHost));
        PSM_CHECK(hipMemcpy(ic.data(), d->incontact, np_, hipMemcpyDeviceToHost));
        PSM_CHECK(hipMemcpy(F.data(), d->cF, sizeof(double) * 3 * np_, hipMemcpyDeviceToHost));
        PSM_CHECK(hipMemcpy(Mi.data(), d->cMi, sizeof(double) * 3 * np_, hipMemcpyDeviceToHost));
        PSM_CHECK(hipMemcpy(Mj.data(), d->cMj, sizeof(double) * 3 * np_, hipMemcpyDeviceToHost));
    }
    int64_t m = 0;
    for (int64_t s = 0; s < np_; ++s) {
        if (!(ic[s] & 1)) continue;
        if (m < cap) {
            if (keys) keys[m] = k[s];
            for (int c = 0; c < 3; ++c) {
                if (force) force[3 * m + c] = F[3 * s + c];
                if (m_i) m_i[3 * m + c] = Mi[3 * s + c];
                if (m_j) m_j[3 * m + c] = Mj[3 * s + c];
            }
        }
        ++m;
    }
    *n = m;
    return st;
}

extern "C" psmdem_status psmdem_read_cells(psmdem_domain* d, int64_t cap, uint64_t* keys, int64_t* n) {
    if (!d || !n) return PSMDEM_E_INVALID;
    const psmdem_status st = psm_sync_flags(d);
    if (psm_read_fails(st)) return st;
    *n = 0;
    if (d->np == 0) return st;
    PSM_CHECK(dem_sort_cells(d->dem_args(), d->s));
    PSM_CHECK(hipStreamSynchronize(d->s));
    std::vector<int> start(d->ncell + 1);
    PSM_CHECK(hipMemcpy(start.data(), d->cell_start, sizeof(int) * (d->ncell + 1), hipMemcpyDeviceToHost));
    long long tot = std::min<long long>(start[d->ncell], d->reg_cap);
    std::vector<int> pid(std::max<long long>(tot, 1));
    if (tot > 0) PSM_CHECK(hipMemcpy(pid.data(), d->cell_pid, sizeof(int) * tot, hipMemcpyDeviceToHost));
    int64_t m = 0;
    for (long long c = 0; c < d->ncell; ++c)
        for (int s = start[c]; s < start[c + 1] && s < tot; ++s) {
            if (m < cap && keys) keys[m] = ((uint64_t)c << 32) | (uint32_t)pid[s];
            ++m;
        }
    *n = m;
    return st;
}

extern "C" psmdem_status psmdem_read_solid(psmdem_domain* d, int64_t cap, uint32_t* cell, uint32_t* pid, double* beta,
                                          int64_t* n) {
    if (!d || !n) return PSMDEM_E_INVALID;
    const psmdem_status st = psm_sync_flags(d);
    if (psm_read_fails(st)) return st;
    *n = 0;
    if (!d->voxelized) return st;
    if (int rc = fresh_beta(d)) return (psmdem_status)rc;
    const GeoArgs& g = d->geo;
    const long long plane = g.ntiles * (long long)PSM_TILE;
    const int ms = d->d.max_solids;
    std::vector<int> ts(g.ntiles + 1);
    PSM_CHECK(hipMemcpy(ts.data(), d->t.tile_start, sizeof(int) * (g.ntiles + 1), hipMemcpyDeviceToHost));
    long long tot = std::min<long long>(ts[g.ntiles], d->t.cap);
    std::vector<unsigned long long> tl(std::max<long long>(tot, 1));
    if (tot > 0) PSM_CHECK(hipMemcpy(tl.data(), d->t.tile_list, sizeof(unsigned long long) * tot, hipMemcpyDeviceToHost));
    std::vector<unsigned> lp(plane);
    std::vector<double> bt((size_t)plane * ms);
    PSM_CHECK(hipMemcpy(lp.data(), d->t.slot_lp, sizeof(unsigned) * plane, hipMemcpyDeviceToHost));
    PSM_CHECK(hipMemcpy(bt.data(), d->t.slot_beta, sizeof(double) * plane * ms, hipMemcpyDeviceToHost));
    int64_t m = 0;
    for (long long c = 0; c < d->N; ++c) {
        int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / ((long long)g.nx * g.ny));
        long long t = x / PSM_TX + (long long)g.ntx * (y / PSM_TY + (long long)g.nty * (z / PSM_TZ));
        if (ts[t + 1] <= ts[t]) continue;
        long long l = (x % PSM_TX) + PSM_TX * ((y % PSM_TY) + PSM_TY * (z % PSM_TZ));
        unsigned w = lp[t * PSM_TILE + l];
        for (int k = 0; k < ms; ++k) {
            unsigned b = (w >> (8 * k)) & 0xffu;
            if (b == 0xffu) break;
            long long at = ts[t] + b;
            if (at >= tot) break;
            if (m < cap) {
                if (cell) cell[m] = (uint32_t)c;
                if (pid) pid[m] = (uint32_t)(tl[at] >> 32);
                if (beta) beta[m] = bt[(size_t)k * plane + t * PSM_TILE + l];
            }
            ++m;
        }
    }
    *n = m;
    return st;
}

extern "C" psmdem_status psmdem_counters(psmdem_domain* d, psmdem_counters_t* out) {
    if (!d || !out) return PSMDEM_E_INVALID;
    PSM_CHECK(hipStreamSynchronize(d->s));
    DevCounters c{};
    PSM_CHECK(hipMemcpy(&c, d->ctr, sizeof c, hipMemcpyDeviceToHost));
    memset(out, 0, sizeof *out);
    int64_t npairs = 0;
    psmdem_status st = pair_count(d, &npairs);
    if (st) return st;
    out->n_pairs = npairs;
    npairs = std::min<int64_t>(npairs, d->pair_cap);
    if (npairs > 0) {
        std::vector<unsigned char> ic(npairs);
        PSM_CHECK(hipMemcpy(ic.data(), d->incontact, npairs, hipMemcpyDeviceToHost));
        for (auto v : ic) out->n_contacts += v & 1;
    }
    if (d->np > 0) {
        int r = 0;
        PSM_CHECK(hipMemcpy(&r, d->cell_start + d->ncell, sizeof(int), hipMemcpyDeviceToHost));
        out->n_registrations = r;
    }
    std::vector<int> ts(d->geo.ntiles + 1);
    PSM_CHECK(hipMemcpy(ts.data(), d->t.tile_start, sizeof(int) * ts.size(), hipMemcpyDeviceToHost));
    for (long long t = 0; t < d->geo.ntiles; ++t) out->n_solid_tiles += ts[t + 1] > ts[t];
    out->n_entries = (int64_t)c.entries;
    out->n_dropped = (int64_t)c.dropped;
    if (d->t.tile_ed && d->np > 0 && d->tile_counts) {
        // the per-tile words of the last selection
        std::vector<unsigned> ed(2 * (size_t)d->geo.ntiles);
        PSM_CHECK(hipMemcpy(ed.data(), d->t.tile_ed, sizeof(unsigned) * ed.size(), hipMemcpyDeviceToHost));
        int64_t e = 0, dr = 0;
        for (size_t k = 0; k < ed.size(); k += 2) {
            e += ed[k];
            dr += ed[k + 1];
        }
        out->n_entries = e;
        out->n_dropped = dr;
    }
    out->step = d->step;
    out->flags = (int64_t)c.flags;
    return PSMDEM_OK;
}

extern "C" psmdem_status psmdem_info(psmdem_domain* d, psmdem_info_t* out) {
    if (!d || !out) return PSMDEM_E_INVALID;
    out->n_sub = d->nsub;
    for (int a = 0; a < 3; ++a) {
        out->dem_cells[a] = d->nc[a];
        out->dem_h[a] = d->h[a];
    }
    out->n_cells = d->N;
    out->n_particles = d->np;
    out->precision = d->prec;
    out->device_bytes = (int64_t)d->bytes;
    out->tile[0] = PSM_TX;
    out->tile[1] = PSM_TY;
    out->tile[2] = PSM_TZ;
    return PSMDEM_OK;
}

// ---------------------------------------------------------------------------
// checkpoint: a header, then every device block of the domain in allocation
// order (the in-place populations with their parity, particle state, both
// pair lists and histories, the kept-list and skip state, tile lists, slots,
// counters and flags), so a restored domain continues bit for bit
// ---------------------------------------------------------------------------
namespace {
struct StateHeader {
    char magic[8];          // "PSMDEMS1"
    uint64_t layout;        // FNV-1a of the block sizes and the domain shape
    uint64_t nblocks;
    uint64_t payload;       // bytes of the blocks after the header
    int64_t step;
    int64_t dem_sub;
    int32_t cur;
    int32_t voxelized;
};
const char kStateMagic[8] = {'P', 'S', 'M', 'D', 'E', 'M', 'S', '1'};

uint64_t fnv(uint64_t h, const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    return h;
}

uint64_t state_layout(const psmdem_domain* d) {
    uint64_t h = 14695981039346656037ull;
    const int64_t shape[8] = {d->d.nx, d->d.ny, d->d.nz, d->np, d->prec, d->nsub, d->d.max_solids,
                              (int64_t)d->blocks.size()};
    h = fnv(h, shape, sizeof shape);
    for (const auto& b : d->blocks) {
        const uint64_t n = b.second;
        h = fnv(h, &n, sizeof n);
    }
    return h;
}
}  // namespace

extern "C" psmdem_status psmdem_read_state(psmdem_domain* d, void* buf, size_t cap, size_t* used) {
    if (!d || !used) { psm_set_error("invalid arguments"); return PSMDEM_E_INVALID; }
    const size_t need = sizeof(StateHeader) + d->bytes;
    *used = need;
    if (!buf) return PSMDEM_OK;
    if (cap < need) {
        psm_set_error("state buffer holds %zu bytes, %zu needed", cap, need);
        return PSMDEM_E_INVALID;
    }
    const psmdem_status st = psm_sync_flags(d);
    if (psm_read_fails(st)) return st;
    if (int rc = fresh_beta(d)) return (psmdem_status)rc;  // a state always holds beta
    StateHeader h{};
    memcpy(h.magic, kStateMagic, 8);
    h.layout = state_layout(d);
    h.nblocks = d->blocks.size();
    h.payload = d->bytes;
    h.step = d->step;
    h.dem_sub = d->dem_sub;
    h.cur = d->cur;
    h.voxelized = d->voxelized ? 1 : 0;
    unsigned char* o = (unsigned char*)buf;
    memcpy(o, &h, sizeof h);
    o += sizeof h;
    for (const auto& b : d->blocks) {
        PSM_CHECK(hipMemcpy(o, b.first, b.second, hipMemcpyDeviceToHost));
        o += b.second;
    }
    return st;
}

extern "C" psmdem_status psmdem_write_state(psmdem_domain* d, const void* buf, size_t n) {
    if (!d || !buf) { psm_set_error("invalid arguments"); return PSMDEM_E_INVALID; }
    StateHeader h{};
    if (n < sizeof h) { psm_set_error("state buffer too short"); return PSMDEM_E_INVALID; }
    memcpy(&h, buf, sizeof h);
    if (memcmp(h.magic, kStateMagic, 8) != 0) { psm_set_error("not a psmdem state"); return PSMDEM_E_INVALID; }
    if (h.layout != state_layout(d) || h.nblocks != d->blocks.size() || h.payload != d->bytes ||
        n != sizeof h + d->bytes) {
        psm_set_error("the state was saved from a domain of another description or particle count");
        return PSMDEM_E_INVALID;
    }
    PSM_CHECK(hipStreamSynchronize(d->s));
    const unsigned char* in = (const unsigned char*)buf + sizeof h;
    for (const auto& b : d->blocks) {
        PSM_CHECK(hipMemcpy(b.first, in, b.second, hipMemcpyHostToDevice));
        in += b.second;
    }
    d->step = h.step;
    d->dem_sub = h.dem_sub;
    d->cur = h.cur;
    d->voxelized = h.voxelized != 0;
    d->beta_fresh = true;
    return PSMDEM_OK;
}

extern "C" psmdem_status psmdem_set_timing(psmdem_domain* d, int32_t on) {
    if (!d) return PSMDEM_E_INVALID;
    d->timing = on != 0;
    return PSMDEM_OK;
}

extern "C" psmdem_status psmdem_timing(psmdem_domain* d, int32_t which, double* avg_ms, int64_t* launches) {
    if (!d || which < 0 || which > 3) return PSMDEM_E_INVALID;
    if (avg_ms) *avg_ms = d->t_n[which] ? d->t_ms[which] / (double)d->t_n[which] : 0.0;
    if (launches) *launches = d->t_n[which];
    return PSMDEM_OK;
}

extern "C" const char* psmdem_last_error(void) { return g_err; }
extern "C" const char* psmdem_version(void) { return "psmdem 0.1 gfx950"; }
