// server.hip -- ensemble serving: continuous batching of many independent
// domains at coupled-step granularity (the psmdem_server_* calls of
// include/psmdem.h).
//
// Jobs wait in a FIFO queue.  Between steps the head of the queue is admitted
// while a slot is free and the held footprints plus its own fit the budget;
// the job's domain is created on the admission stream, so the steps already on
// the compute stream keep the device busy meanwhile.  Every active job then
// takes one coupled step through six batched launches that read per-job
// argument tables (uploaded only when the active set changes) and a per-slot
// parity block passed by value.  A job that reached its step count leaves the
// tables; an event after its last step tells when its results are readable.
#include <math.h>
#include <string.h>
#include <time.h>

#include <deque>
#include <map>
#include <vector>

#include "domain.h"
#include "serve.h"

namespace {

double now_s() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

struct Job {
    int64_t id = 0;
    psmdem_desc desc{};
    // host copy of the particle set until admission
    int n = 0;
    std::vector<int32_t> shape;
    std::vector<double> semi, dens, pos, quat, vel, omega;
    std::vector<uint8_t> fixed;
    bool has_quat = false, has_vel = false, has_omega = false, has_fixed = false;

    int64_t steps = 0, steps_done = 0;
    int state = PSMDEM_JOB_QUEUED;
    int slot = -1;
    int status = 0;
    size_t footprint = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    psmdem_domain* D = nullptr;
    hipEvent_t done_ev = nullptr;

    psmdem_particles parts() const {
        psmdem_particles P{};
        P.n = n;
        P.shape = shape.data();
        P.semi_axes = semi.data();
        P.density_ratio = dens.data();
        P.pos = pos.data();
        P.quat = has_quat ? quat.data() : nullptr;
        P.vel = has_vel ? vel.data() : nullptr;
        P.omega = has_omega ? omega.data() : nullptr;
        P.fixed = has_fixed ? fixed.data() : nullptr;
        return P;
    }
    void drop_host_copy() {
        std::vector<int32_t>().swap(shape);
        for (auto* v : {&semi, &dens, &pos, &quat, &vel, &omega}) std::vector<double>().swap(*v);
        std::vector<uint8_t>().swap(fixed);
    }
};

}  // namespace

struct psmdem_server {
    psmdem_server_desc d{};
    hipStream_t s = nullptr, sa = nullptr;
    psmdem_alloc_fn alloc = nullptr;
    psmdem_free_fn freef = nullptr;
    void* actx = nullptr;

    int64_t next_id = 1;
    std::map<int64_t, Job*> jobs;
    std::deque<Job*> queue;
    std::vector<Job*> active;    // slot order
    size_t held = 0;             // footprints of admitted, unreleased jobs
    bool dirty = true;

    // device tables (capacity SRV_MAX_JOBS) and tile maps
    DemJob* dem_tab = nullptr;
    VoxArgs* vox_tab = nullptr;
    LbmArgs* lbm_tab = nullptr;
    int2* map_d = nullptr;       // [all | ms <= 2 | ms > 2]
    long long map_cap = 0;
    long long n_all = 0, n_ms2 = 0, n_ms4 = 0;
    size_t tab_bytes = 0;
    // pinned staging of the uploads, two in rotation
    unsigned char* stage[2] = {nullptr, nullptr};
    size_t stage_cap[2] = {0, 0};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    int stage_next = 0;
    // throttle: events of the last steps
    std::deque<hipEvent_t> inflight;
    std::vector<hipEvent_t> ev_pool;

    void* dalloc(size_t n) {
        void* p = nullptr;
        if (alloc) p = alloc(n, actx);
        else if (hipMalloc(&p, n) != hipSuccess) p = nullptr;
        return p;
    }
    void dfree(void* p, size_t n) {
        if (!p) return;
        if (freef) freef(p, n, actx);
        else if (!alloc) (void)hipFree(p);
    }
    hipEvent_t get_event() {
        if (!ev_pool.empty()) {
            hipEvent_t e = ev_pool.back();
            ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }
    void put_event(hipEvent_t e) {
        if (e) ev_pool.push_back(e);
    }
};

namespace {

// a job's domain freed after the device has finished with it
void free_job_domain(psmdem_server* S, Job* J) {
    if (J->D) {
        psmdem_destroy(J->D);
        J->D = nullptr;
        S->held -= J->footprint;
    }
    if (J->done_ev) {
        S->put_event(J->done_ev);
        J->done_ev = nullptr;
    }
}

// the device has finished the job: later reads synchronise the admission
// stream only, not the compute stream that runs the other jobs
void mark_done(psmdem_server* S, Job* J) {
    J->state = PSMDEM_JOB_DONE;
    J->t_done = now_s();
    if (J->D) J->D->s = S->sa;
}

void observe_done(psmdem_server* S, bool wait) {
    for (auto& kv : S->jobs) {
        Job* J = kv.second;
        if (J->state != PSMDEM_JOB_FINISHING) continue;
        hipError_t e = wait ? hipEventSynchronize(J->done_ev) : hipEventQuery(J->done_ev);
        if (e == hipSuccess) mark_done(S, J);
    }
}

int admit(psmdem_server* S) {
    while (!S->queue.empty() && (int)S->active.size() < S->d.max_jobs) {
        Job* J = S->queue.front();
        if (S->d.hbm_budget > 0 && S->held + J->footprint > (size_t)S->d.hbm_budget) break;
        psmdem_particles P = J->parts();
        psmdem_domain* D = nullptr;
        size_t bytes = 0;
        psmdem_status rc = psm_domain_create(&J->desc, &P, S->sa, S->alloc, S->freef, S->actx, false, &D, &bytes);
        if (rc == PSMDEM_E_NOMEM) break;  // retried once memory frees up
        S->queue.pop_front();
        if (rc != PSMDEM_OK) {
            J->state = PSMDEM_JOB_FAILED;
            J->status = rc;
            J->drop_host_copy();
            continue;
        }
        D->s = S->s;  // created and synchronised on the admission stream; steps run on the compute stream
        J->D = D;
        J->footprint = bytes;
        S->held += bytes;
        J->state = PSMDEM_JOB_ACTIVE;
        J->t_admit = now_s();
        J->drop_host_copy();
        S->active.push_back(J);
        S->dirty = true;
    }
    return 0;
}

// rebuild and upload the argument tables and tile maps of the active set
int upload_tables(psmdem_server* S) {
    const int na = (int)S->active.size();
    std::vector<DemJob> dem(na);
    std::vector<VoxArgs> vox(na);
    std::vector<LbmArgs> lbm(na);
    std::vector<int2> m_all, m2, m4;
    for (int i = 0; i < na; ++i) {
        psmdem_domain* D = S->active[i]->D;
        S->active[i]->slot = i;
        DemJob& J = dem[i];
        J = DemJob{};
        J.A = D->dem_args();
        J.P = D->pair_set();
        J.t = D->t;
        J.dt = D->dt;
        J.nsub = D->nsub;
        J.dem = (D->d.dem_on && D->np > 0) ? 1 : 0;
        J.fluid = 1;
        vox[i] = D->vox_args();
        vox[i].vpart = nullptr;  // the one-workgroup voxelisation forms its own particle records
        vox[i].t.tile_ed = nullptr;  // and counts its entries in the job's step counters
        lbm[i] = D->lbm_args();
        const int nt = (int)D->geo.ntiles;
        std::vector<int2>& mp = D->d.max_solids <= 2 ? m2 : m4;
        for (int t = 0; t < nt; ++t) {
            m_all.push_back(make_int2(i, t));
            mp.push_back(make_int2(i, t));
        }
    }
    S->n_all = (long long)m_all.size();
    S->n_ms2 = (long long)m2.size();
    S->n_ms4 = (long long)m4.size();
    const long long nmap = S->n_all + S->n_ms2 + S->n_ms4;
    if (nmap > S->map_cap) {
        // the old map may still be read by enqueued steps
        PSM_CHECK(hipStreamSynchronize(S->s));
        S->dfree(S->map_d, sizeof(int2) * (size_t)S->map_cap);
        long long cap = std::max<long long>(nmap, 2 * S->map_cap);
        S->map_d = (int2*)S->dalloc(sizeof(int2) * (size_t)cap);
        if (!S->map_d) {
            S->map_cap = 0;
            psm_set_error("device allocation of the tile map failed");
            return PSMDEM_E_NOMEM;
        }
        S->map_cap = cap;
    }
    const size_t b_dem = sizeof(DemJob) * na, b_vox = sizeof(VoxArgs) * na, b_lbm = sizeof(LbmArgs) * na;
    const size_t b_map = sizeof(int2) * (size_t)nmap;
    const size_t total = b_dem + b_vox + b_lbm + b_map;
    const int k = S->stage_next;
    S->stage_next ^= 1;
    PSM_CHECK(hipEventSynchronize(S->stage_ev[k]));  // the upload that last used this buffer is done
    if (S->stage_cap[k] < total) {
        if (S->stage[k]) PSM_CHECK(hipHostFree(S->stage[k]));
        S->stage[k] = nullptr;
        S->stage_cap[k] = 0;
        size_t cap = std::max(total, (size_t)1 << 20);
        PSM_CHECK(hipHostMalloc((void**)&S->stage[k], cap, hipHostMallocDefault));
        S->stage_cap[k] = cap;
    }
    unsigned char* h = S->stage[k];
    memcpy(h, dem.data(), b_dem);
    memcpy(h + b_dem, vox.data(), b_vox);
    memcpy(h + b_dem + b_vox, lbm.data(), b_lbm);
    int2* hm = (int2*)(h + b_dem + b_vox + b_lbm);
    if (S->n_all) memcpy(hm, m_all.data(), sizeof(int2) * S->n_all);
    if (S->n_ms2) memcpy(hm + S->n_all, m2.data(), sizeof(int2) * S->n_ms2);
    if (S->n_ms4) memcpy(hm + S->n_all + S->n_ms2, m4.data(), sizeof(int2) * S->n_ms4);
    // stream-ordered after every enqueued step that still reads the old tables
    if (b_dem) PSM_CHECK(hipMemcpyAsync(S->dem_tab, h, b_dem, hipMemcpyHostToDevice, S->s));
    if (b_vox) PSM_CHECK(hipMemcpyAsync(S->vox_tab, h + b_dem, b_vox, hipMemcpyHostToDevice, S->s));
    if (b_lbm) PSM_CHECK(hipMemcpyAsync(S->lbm_tab, h + b_dem + b_vox, b_lbm, hipMemcpyHostToDevice, S->s));
    if (b_map) PSM_CHECK(hipMemcpyAsync(S->map_d, hm, b_map, hipMemcpyHostToDevice, S->s));
    PSM_CHECK(hipEventRecord(S->stage_ev[k], S->s));
    S->dirty = false;
    return 0;
}

int enqueue_step(psmdem_server* S) {
    const int na = (int)S->active.size();
    SrvDyn dyn;
    memset(&dyn, 0, sizeof dyn);
    for (int i = 0; i < na; ++i) {
        psmdem_domain* D = S->active[i]->D;
        srv_set(dyn.cur, i, D->cur);
        srv_set(dyn.odd, i, (int)(D->step & 1));
    }
    const int prec = S->d.precision;
    const int2* m_all = S->map_d;
    const int2* m2 = S->map_d + S->n_all;
    const int2* m4 = m2 + S->n_ms2;
    int ell = 0;
    for (int i = 0; i < na; ++i) ell |= S->active[i]->D->dem_args().ellipsoids;
    PSM_CHECK(dem_fused_batch(S->dem_tab, na, dyn, ell, S->s));
    PSM_CHECK(vox_register_batch(S->vox_tab, na, S->s));
    PSM_CHECK(vox_voxelize_batch(S->vox_tab, m_all, S->n_all, prec == 0, S->s));
    PSM_CHECK(lbm_step_batch(S->lbm_tab, dyn, m_all, S->n_all, 0, prec, S->s));
    PSM_CHECK(lbm_step_batch(S->lbm_tab, dyn, m2, S->n_ms2, 2, prec, S->s));
    PSM_CHECK(lbm_step_batch(S->lbm_tab, dyn, m4, S->n_ms4, 4, prec, S->s));
    PSM_CHECK(dem_finish_batch(S->dem_tab, na, S->s));
    for (int i = 0; i < na; ++i) {
        Job* J = S->active[i];
        psmdem_domain* D = J->D;
        if (D->d.dem_on && D->np > 0) D->cur ^= (D->nsub & 1);
        D->step++;
        D->voxelized = true;
        D->tile_counts = false;  // the batch counts entries in the step counters
        D->beta_fresh = true;    // and stores beta
        J->steps_done++;
    }
    return 0;
}

// jobs with every step enqueued leave the active set; an event after their
// last step tells when the device has finished them
int retire(psmdem_server* S) {
    std::vector<Job*> keep;
    for (Job* J : S->active) {
        if (J->steps_done < J->steps) {
            keep.push_back(J);
            continue;
        }
        J->done_ev = S->get_event();
        if (!J->done_ev) { psm_set_error("event creation failed"); return PSMDEM_E_HIP; }
        PSM_CHECK(hipEventRecord(J->done_ev, S->s));
        J->state = PSMDEM_JOB_FINISHING;
        J->slot = -1;
        S->dirty = true;
    }
    S->active.swap(keep);
    return 0;
}

int throttle(psmdem_server* S) {
    hipEvent_t e = S->get_event();
    if (!e) { psm_set_error("event creation failed"); return PSMDEM_E_HIP; }
    PSM_CHECK(hipEventRecord(e, S->s));
    S->inflight.push_back(e);
    const size_t lim = (size_t)(S->d.max_inflight > 0 ? S->d.max_inflight : 2);
    while (S->inflight.size() > lim) {
        hipEvent_t o = S->inflight.front();
        S->inflight.pop_front();
        PSM_CHECK(hipEventSynchronize(o));
        S->put_event(o);
    }
    return 0;
}

}  // namespace

extern "C" double psmdem_clock(void) { return now_s(); }

extern "C" psmdem_status psmdem_server_create(const psmdem_server_desc* desc, void* stream, void* admit_stream,
                                              psmdem_alloc_fn alloc, psmdem_free_fn free_fn, void* alloc_ctx,
                                              psmdem_server** out) {
    if (!out || !desc) { psm_set_error("desc or out is NULL"); return PSMDEM_E_INVALID; }
    *out = nullptr;
    if (desc->max_jobs < 1 || desc->max_jobs > SRV_MAX_JOBS) {
        psm_set_error("max_jobs must be in 1..%d", SRV_MAX_JOBS);
        return PSMDEM_E_INVALID;
    }
    if (desc->precision < 0 || desc->precision > 3) { psm_set_error("invalid precision"); return PSMDEM_E_INVALID; }
    if (desc->hbm_budget < 0 || desc->max_inflight < 0) {
        psm_set_error("negative budget or in-flight limit");
        return PSMDEM_E_INVALID;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        psm_set_error("no HIP device");
        return PSMDEM_E_NODEVICE;
    }
    psmdem_server* S = new psmdem_server();
    S->d = *desc;
    S->s = (hipStream_t)stream;
    S->sa = admit_stream ? (hipStream_t)admit_stream : S->s;
    S->alloc = alloc;
    S->freef = free_fn;
    S->actx = alloc_ctx;
    S->tab_bytes = (sizeof(DemJob) + sizeof(VoxArgs) + sizeof(LbmArgs)) * SRV_MAX_JOBS;
    S->dem_tab = (DemJob*)S->dalloc(sizeof(DemJob) * SRV_MAX_JOBS);
    S->vox_tab = (VoxArgs*)S->dalloc(sizeof(VoxArgs) * SRV_MAX_JOBS);
    S->lbm_tab = (LbmArgs*)S->dalloc(sizeof(LbmArgs) * SRV_MAX_JOBS);
    bool ok = S->dem_tab && S->vox_tab && S->lbm_tab;
    for (int k = 0; k < 2 && ok; ++k) ok = hipEventCreateWithFlags(&S->stage_ev[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        psmdem_server_destroy(S);
        psm_set_error("server allocation failed");
        return PSMDEM_E_NOMEM;
    }
    *out = S;
    return PSMDEM_OK;
}

extern "C" void psmdem_server_destroy(psmdem_server* S) {
    if (!S) return;
    (void)hipStreamSynchronize(S->s);
    if (S->sa != S->s) (void)hipStreamSynchronize(S->sa);
    for (auto& kv : S->jobs) {
        free_job_domain(S, kv.second);
        delete kv.second;
    }
    S->dfree(S->dem_tab, sizeof(DemJob) * SRV_MAX_JOBS);
    S->dfree(S->vox_tab, sizeof(VoxArgs) * SRV_MAX_JOBS);
    S->dfree(S->lbm_tab, sizeof(LbmArgs) * SRV_MAX_JOBS);
    S->dfree(S->map_d, sizeof(int2) * (size_t)S->map_cap);
    for (int k = 0; k < 2; ++k) {
        if (S->stage[k]) (void)hipHostFree(S->stage[k]);
        if (S->stage_ev[k]) (void)hipEventDestroy(S->stage_ev[k]);
    }
    for (hipEvent_t e : S->inflight) (void)hipEventDestroy(e);
    for (hipEvent_t e : S->ev_pool) (void)hipEventDestroy(e);
    delete S;
}

extern "C" psmdem_status psmdem_server_submit(psmdem_server* S, const psmdem_desc* desc,
                                              const psmdem_particles* parts, int64_t steps, int64_t* job) {
    if (!S || !desc || !job || steps < 0) { psm_set_error("invalid arguments"); return PSMDEM_E_INVALID; }
    *job = 0;
    if (desc->precision != S->d.precision) {
        psm_set_error("job precision differs from the server's");
        return PSMDEM_E_INVALID;
    }
    if (!desc->fluid_on) { psm_set_error("serving runs coupled jobs (fluid_on = 1)"); return PSMDEM_E_INVALID; }
    const int n = parts ? parts->n : 0;
    if (desc->dem_on && n > DEM_FUSED_MAX) {
        psm_set_error("serving jobs hold at most %d particles", DEM_FUSED_MAX);
        return PSMDEM_E_INVALID;
    }
    const long long ntiles = (long long)((desc->nx + PSM_TX - 1) / PSM_TX) * ((desc->ny + PSM_TY - 1) / PSM_TY) *
                             ((desc->nz + PSM_TZ - 1) / PSM_TZ);
    if (desc->nx < 1 || desc->ny < 1 || desc->nz < 1 || ntiles > 8192) {
        psm_set_error("serving jobs hold at most 8192 lattice tiles");
        return PSMDEM_E_INVALID;
    }
    int64_t fp = 0;
    psmdem_status rc = psmdem_footprint(desc, parts, &fp);
    if (rc != PSMDEM_OK) return rc;
    if (S->d.hbm_budget > 0 && fp > S->d.hbm_budget) {
        psm_set_error("job footprint %lld B exceeds the budget of %lld B: it could never be admitted",
                      (long long)fp, (long long)S->d.hbm_budget);
        return PSMDEM_E_INVALID;
    }
    Job* J = new Job();
    J->id = S->next_id++;
    J->desc = *desc;
    J->n = n;
    J->steps = steps;
    J->footprint = (size_t)fp;
    J->t_submit = now_s();
    if (n > 0) {
        J->shape.assign(parts->shape, parts->shape + n);
        J->semi.assign(parts->semi_axes, parts->semi_axes + 3 * (size_t)n);
        J->dens.assign(parts->density_ratio, parts->density_ratio + n);
        J->pos.assign(parts->pos, parts->pos + 3 * (size_t)n);
        if ((J->has_quat = parts->quat != nullptr)) J->quat.assign(parts->quat, parts->quat + 4 * (size_t)n);
        if ((J->has_vel = parts->vel != nullptr)) J->vel.assign(parts->vel, parts->vel + 3 * (size_t)n);
        if ((J->has_omega = parts->omega != nullptr)) J->omega.assign(parts->omega, parts->omega + 3 * (size_t)n);
        if ((J->has_fixed = parts->fixed != nullptr)) J->fixed.assign(parts->fixed, parts->fixed + n);
    }
    S->jobs[J->id] = J;
    S->queue.push_back(J);
    *job = J->id;
    return PSMDEM_OK;
}

extern "C" psmdem_status psmdem_server_iterate(psmdem_server* S, int32_t* n_active, int32_t* n_queued) {
    if (!S) return PSMDEM_E_INVALID;
    int rc;
    observe_done(S, false);
    if ((rc = admit(S))) return (psmdem_status)rc;
    // jobs of zero steps finish at admission
    if ((rc = retire(S))) return (psmdem_status)rc;
    if (!S->active.empty()) {
        if (S->dirty && (rc = upload_tables(S))) return (psmdem_status)rc;
        if ((rc = enqueue_step(S))) return (psmdem_status)rc;
        if ((rc = retire(S))) return (psmdem_status)rc;
        if ((rc = throttle(S))) return (psmdem_status)rc;
    }
    observe_done(S, false);
    if (n_active) *n_active = (int32_t)S->active.size();
    if (n_queued) *n_queued = (int32_t)S->queue.size();
    return PSMDEM_OK;
}

extern "C" psmdem_status psmdem_server_drain(psmdem_server* S) {
    if (!S) return PSMDEM_E_INVALID;
    PSM_CHECK(hipStreamSynchronize(S->s));
    observe_done(S, true);
    return PSMDEM_OK;
}

extern "C" psmdem_status psmdem_server_job(psmdem_server* S, int64_t job, psmdem_job_info_t* out) {
    if (!S || !out) return PSMDEM_E_INVALID;
    auto it = S->jobs.find(job);
    if (it == S->jobs.end()) { psm_set_error("unknown job %lld", (long long)job); return PSMDEM_E_INVALID; }
    const Job* J = it->second;
    out->state = J->state;
    out->slot = J->slot;
    out->steps = J->steps;
    out->steps_done = J->steps_done;
    out->footprint = (int64_t)J->footprint;
    out->status = J->status;
    out->t_submit = J->t_submit;
    out->t_admit = J->t_admit;
    out->t_done = J->t_done;
    return PSMDEM_OK;
}

extern "C" psmdem_status psmdem_server_domain(psmdem_server* S, int64_t job, psmdem_domain** out) {
    if (!S || !out) return PSMDEM_E_INVALID;
    *out = nullptr;
    auto it = S->jobs.find(job);
    if (it == S->jobs.end()) { psm_set_error("unknown job %lld", (long long)job); return PSMDEM_E_INVALID; }
    Job* J = it->second;
    if (J->state == PSMDEM_JOB_FINISHING) {
        PSM_CHECK(hipEventSynchronize(J->done_ev));
        mark_done(S, J);
    }
    if (J->state != PSMDEM_JOB_DONE) { psm_set_error("job %lld is not done", (long long)job); return PSMDEM_E_STATE; }
    *out = J->D;
    return PSMDEM_OK;
}

extern "C" psmdem_status psmdem_server_release(psmdem_server* S, int64_t job) {
    if (!S) return PSMDEM_E_INVALID;
    auto it = S->jobs.find(job);
    if (it == S->jobs.end()) { psm_set_error("unknown job %lld", (long long)job); return PSMDEM_E_INVALID; }
    Job* J = it->second;
    switch (J->state) {
        case PSMDEM_JOB_QUEUED:
            for (auto q = S->queue.begin(); q != S->queue.end(); ++q)
                if (*q == J) {
                    S->queue.erase(q);
                    break;
                }
            break;
        case PSMDEM_JOB_ACTIVE: {
            // enqueued steps still read the job's memory
            PSM_CHECK(hipStreamSynchronize(S->s));
            std::vector<Job*> keep;
            for (Job* A : S->active)
                if (A != J) keep.push_back(A);
            S->active.swap(keep);
            S->dirty = true;
            break;
        }
        case PSMDEM_JOB_FINISHING:
            PSM_CHECK(hipEventSynchronize(J->done_ev));
            break;
        default:
            break;
    }
    if (J->D) J->D->s = S->sa;  // nothing left on the compute stream: no wait for it on destruction
    free_job_domain(S, J);
    S->jobs.erase(it);
    delete J;
    return PSMDEM_OK;
}
