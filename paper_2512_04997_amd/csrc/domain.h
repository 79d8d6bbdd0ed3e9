// domain.h -- the domain object behind psmdem_domain* (internal).
#pragma once
#include <stdint.h>

#include <utility>
#include <vector>

#include "common.h"
#include "dem.h"
#include "lbm.h"
#include "voxel.h"

struct psmdem_domain {
    psmdem_desc d;
    hipStream_t s = nullptr;
    int dev = 0;        // device current at creation (the device of the stream)
    psmdem_alloc_fn alloc = nullptr;
    psmdem_free_fn freef = nullptr;
    void* actx = nullptr;
    std::vector<std::pair<void*, size_t>> blocks;
    size_t bytes = 0;

    int np = 0;
    long long N = 0;
    GeoArgs geo{};
    double L[3];
    int prec = 0;
    void* f = nullptr;
    double wall_corr[6][19];
    double* kolm_prof = nullptr;
    double* wall_corr_d = nullptr;

    // particles
    PartArgs p{};
    std::vector<int> h_shape;
    // DEM
    int nsub = 1;
    double dt = 1.0, beta_e = 0.0, Rc = 0.0;
    double ystar = 0.0, gstar = 0.0;  // Hertz: Y*, G*
    int nc[3];
    double h[3];
    long long ncell = 1;
    int *cell_count = nullptr, *cell_start = nullptr, *cell_fill = nullptr, *cell_pid = nullptr;
    int* pc = nullptr;
    int* fused_age = nullptr;
    unsigned char* fz = nullptr;
    int* list_flag = nullptr;
    long long dem_sub = 0;  // multi-launch substeps run (their parity indexes list_flag)
    int *col_count = nullptr, *col_fill = nullptr, *col_start = nullptr, *col_list = nullptr;
    long long reg_cap = 0;
    unsigned long long* row_lb = nullptr;
    int* prow[2] = {nullptr, nullptr};
    unsigned long long* pairs[2] = {nullptr, nullptr};
    double* hist[2] = {nullptr, nullptr};
    double *cF = nullptr, *cMi = nullptr, *cMj = nullptr;
    unsigned char* incontact = nullptr;
    int* ell_list = nullptr;
    unsigned* ell_cnt = nullptr;
    long long ell_seg_cap = 0;
    long long pair_cap = 0;
    int cur = 0;
    // voxel / tiles
    TileArgs t{};
    int* tile_count = nullptr;
    int* tile_fill = nullptr;
    unsigned short* vbox = nullptr;
    long long box_stride = 0;
    void* vpart = nullptr;
    void* btab = nullptr;         // subdivision method: B per inside-sample count (compute type)
    double* betatab = nullptr;    // and beta
    int* scan_tmp = nullptr;
    DevCounters* ctr = nullptr;

    int64_t step = 0;
    bool voxelized = false;
    bool tile_counts = false;  // the entry counts of the last voxelisation are in t.tile_ed
    bool beta_fresh = true;    // t.slot_beta holds the last voxelisation's beta (a stepping
                               // voxelisation leaves it to the read-back, which reselects)

    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev;
    double t_ms[4] = {0, 0, 0, 0};
    long long t_n[4] = {0, 0, 0, 0};

    bool dry = false;   // plan only: sum the allocation sizes, touch no device

    void* dalloc(size_t n) {
        if (n == 0) n = 16;
        n = (n + 255) & ~(size_t)255;
        void* ptr = nullptr;
        if (dry) {
            bytes += n;
            return (void*)(uintptr_t)256;
        }
        if (alloc) {
            ptr = alloc(n, actx);
        } else if (hipMalloc(&ptr, n) != hipSuccess) {
            ptr = nullptr;
        }
        if (ptr) {
            blocks.push_back({ptr, n});
            bytes += n;
        }
        return ptr;
    }
    // a device block for the duration of one call (not part of the domain)
    void* talloc(size_t n) {
        n = (n + 255) & ~(size_t)255;
        void* ptr = nullptr;
        if (alloc) ptr = alloc(n, actx);
        else if (hipMalloc(&ptr, n) != hipSuccess) ptr = nullptr;
        return ptr;
    }
    void tfree(void* ptr, size_t n) {
        n = (n + 255) & ~(size_t)255;
        if (freef) freef(ptr, n, actx);
        else if (!alloc) (void)hipFree(ptr);
    }
    ~psmdem_domain() {
        if (dry) return;
        if (s) (void)hipStreamSynchronize(s);
        else (void)hipDeviceSynchronize();
        for (auto& b : blocks) {
            if (freef) freef(b.first, b.second, actx);
            else if (!alloc) (void)hipFree(b.first);
        }
        for (auto e : ev) (void)hipEventDestroy(e);
    }

    DemArgs dem_args() {
        DemArgs A{};
        A.g = geo;
        A.p = p;
        for (int a = 0; a < 3; ++a) {
            A.L[a] = L[a];
            A.nc[a] = nc[a];
            A.h[a] = h[a];
            A.gravity[a] = d.gravity[a];
        }
        A.ncell = ncell;
        A.pc = pc;
        A.fused_age = fused_age;
        A.fz = fz;
        A.list_flag = list_flag;
        A.list_run = nullptr;
        A.cell_count = cell_count;
        A.cell_start = cell_start;
        A.cell_fill = cell_fill;
        A.cell_pid = cell_pid;
        A.reg_cap = reg_cap;
        A.row_lb = row_lb;
        A.cF = cF;
        A.cMi = cMi;
        A.cMj = cMj;
        A.incontact = incontact;
        A.col_count = col_count;
        A.col_fill = col_fill;
        A.col_start = col_start;
        A.col_list = col_list;
        A.pair_cap = pair_cap;
        A.kn = d.kn;
        A.beta_e = beta_e;
        A.mu = d.mu;
        A.kt_ratio = d.kt_ratio;
        A.gt_ratio = d.gt_ratio;
        A.hertz = d.contact_law == PSMDEM_HERTZ;
        A.ystar = ystar;
        A.gstar = gstar;
        for (int f_ = 0; f_ < 6; ++f_)
            for (int c = 0; c < 3; ++c) A.wall_u[f_][c] = d.wall_u[f_][c];
        A.ellipsoids = 0;
        for (int sh : h_shape) A.ellipsoids |= sh != 0;
        A.ell_list = ell_list;
        A.ell_cnt = ell_cnt;
        A.ell_seg_cap = ell_seg_cap;
        A.ctr = ctr;
        return A;
    }

    // current list = buffer cur, previous = the other one (or none)
    PairBufs pair_bufs(int use_prev) {
        PairBufs B{};
        B.pairs = pairs[cur];
        B.prow = prow[cur];
        B.hist = hist[cur];
        B.prev_pairs = pairs[cur ^ 1];
        B.prev_hist = hist[cur ^ 1];
        B.prev_n = use_prev ? prow[cur ^ 1] + np : nullptr;
        return B;
    }

    PairSet pair_set() {
        PairSet P{};
        for (int b = 0; b < 2; ++b) {
            P.pairs[b] = pairs[b];
            P.prow[b] = prow[b];
            P.hist[b] = hist[b];
        }
        return P;
    }

    VoxArgs vox_args() {
        VoxArgs A{};
        A.g = geo;
        A.p = p;
        A.t = t;
        A.tile_count = tile_count;
        A.tile_fill = tile_fill;
        A.sf_method = d.sf_method;
        A.ns = d.sf_subdiv;
        A.Rc = Rc;
        A.tau = d.tau;
        A.ms = d.max_solids;
        A.vbox = vbox;
        A.box_stride = box_stride;
        A.vpart = vpart;
        A.btab = btab;
        A.betatab = betatab;
        // the LBM pass's rule for streaming accesses (large lattices with line-aligned rows)
        const long long sb = prec == 0 ? 8 : (prec == 1 ? 4 : 2);
        A.stream = 19ll * N * sb > (192ll << 20) && geo.nx % 64 == 0 && sb >= 4;
        A.ctr = ctr;
        return A;
    }

    LbmArgs lbm_args() {
        LbmArgs A{};
        A.g = geo;
        A.f = f;
        A.omega = 1.0 / d.tau;
        A.omega_m = A.omega;
        if (d.collision == PSMDEM_TRT) {
            // Lambda = (1/w+ - 1/2)(1/w- - 1/2); the paper's rule is Lambda = 3/16
            if (d.trt_magic > 0.0) A.omega_m = 1.0 / (d.trt_magic / (d.tau - 0.5) + 0.5);
            else A.omega_m = 8.0 * (2.0 - A.omega) / (8.0 - A.omega);
        }
        A.forcing = (d.body_force[0] != 0.0 || d.body_force[1] != 0.0 || d.body_force[2] != 0.0 ||
                     d.kolm_amp != 0.0);
        for (int a = 0; a < 3; ++a) {
            A.F[a] = d.body_force[a];
            A.L[a] = L[a];
        }
        A.kolm_axis = d.kolm_axis;
        A.kolm_dir = d.kolm_dir;
        A.kolm_prof = kolm_prof;
        A.wall_corr = wall_corr_d;
        A.t = t;
        A.kin = p.kin;
        A.np = np;
        A.ms = d.max_solids;
        A.flags = &ctr->flags;
        return A;
    }

    int timed_begin(int which) {
        if (!timing) return -1;
        hipEvent_t a, b;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        ev.push_back(a);
        ev.push_back(b);
        (void)hipEventRecord(a, s);
        pending.push_back({which, (int)ev.size() - 2});
        return (int)ev.size() - 1;
    }
    void timed_end(int idx) {
        if (idx >= 0) (void)hipEventRecord(ev[idx], s);
    }
    std::vector<std::pair<int, int>> pending;
    void collect_timing() {
        for (auto& pr : pending) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[pr.second], ev[pr.second + 1]) == hipSuccess) {
                t_ms[pr.first] += ms;
                t_n[pr.first] += 1;
            }
        }
        pending.clear();
        for (auto e : ev) (void)hipEventDestroy(e);
        ev.clear();
    }
};


// creation; with dry set nothing touches the device and *bytes receives the
// device bytes the domain would allocate (the admission memory model)
psmdem_status psm_domain_create(const psmdem_desc* desc, const psmdem_particles* parts, void* stream,
                                psmdem_alloc_fn alloc, psmdem_free_fn free_fn, void* alloc_ctx, bool dry,
                                psmdem_domain** out, size_t* bytes);
// waits for the domain stream and reports the device flags (unstable, then
// capacity); psm_read_fails: a status that stops a read (the flags do not)
psmdem_status psm_sync_flags(psmdem_domain* d);
bool psm_read_fails(psmdem_status st);
