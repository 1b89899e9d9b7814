// The GPU backend of the SIP server (sip_server_* / sip_batch_* in
// include/sip.h; the request scheduler is sip_sched.cpp).
//
// The paper's redesigned solver owns its coefficients and reuses one
// factorisation for every later iteration and time step (Sec. 4.1); the
// server generalises that to many blocks and many right-hand sides on one
// GPU.  This backend keeps, in device memory, each resident system's
// coefficients and factors and each running request's b, x, y, face words
// and partial sums, and runs the scheduler's steps as kernel launches on the
// server's own stream:
//   - a request's arrays (coefficients, b, x0) are read on the server's
//     stream only after an event recorded on the caller's stream at submit;
//   - new systems are factorised in one batched launch per factor precision;
//   - while no new request arrives, all admitted requests of one arithmetic
//     run in one persistent launch (k_persist): every request iterates at its
//     own pace (its forward and backward sweeps follow each other as its own
//     finalisers publish them), so small blocks do not wait for the largest
//     one; a launch ends when every request in it has stopped or has been
//     asked to pause at its next iteration boundary, which the host does when
//     queued requests wait, when a stopped request has waited long enough to
//     be retired, or to give another launch group its turn;
//   - while requests keep arriving, all admitted requests advance together in
//     epochs of `epoch_iters` iterations, each a batched forward launch and a
//     batched backward launch over one merged ticket order (an epoch boundary
//     admits new requests without draining a persistent launch);
//     SIP_SERVER_PERSISTENT=1 / 0 forces one mode.
// Every request's arithmetic depends only on its own data and tile order, so
// a result is the same alone and in any mix.
#include "sip_internal.h"
#include "sip_runtime.h"
#include "sip_sched.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <thread>
#include <vector>

using namespace sipk;

namespace {

constexpr int MAX_SLOTS = SERVER_MAX_SLOTS;
constexpr int MAX_PAIRS = 1024;   // pairs of requests swept together

struct GpuResident final : Resident {
    Geom g{};
    int fp32 = 0;          // factors stored in FP32
    int arith = 0;         // sweep arithmetic (sip_precision)
    double alpha = 0.92;
    int sym = 0;           // sweeps read the symmetric coefficient storage
    double *A = nullptr;
    void *LU = nullptr;
};

struct GpuReq;

// Two requests of one resident system swept together (FP32 factors): b and x
// of both interleaved, their own face words and three control blocks (the
// sweep's, one per request).  Each request stops at its own tolerance; the
// pair's buffers go when both have.
struct Pair {
    GpuReq *r[2] = {nullptr, nullptr};
    GpuResident *sys = nullptr;
    int idx = -1;             // control blocks pctl[3 idx .. 3 idx + 2]
    double *bx = nullptr;     // b pairs, then x pairs
    void *y = nullptr;
    uint64_t *face = nullptr;
    double *part = nullptr;
    bool done[2] = {false, false};
    size_t held = 0;          // budget bytes of a finished member, released with the pair
};

struct GpuReq final : Req {
    double *bx = nullptr;
    void *y = nullptr;
    uint64_t *face = nullptr;
    double *part = nullptr;
    Pair *pair = nullptr;    // swept together with another request
    int pm = 0;              // which of the pair
    hipEvent_t ready = nullptr;   // recorded on the caller's stream at submit
    ~GpuReq() override
    {
        if (ready) (void)hipEventDestroy(ready);
    }
};

GpuResident *gsys(const Req *q) { return static_cast<GpuResident *>(q->sys); }

size_t slot_bytes(const Geom &g, int fp32)
{
    const size_t E = (size_t)g.elems;
    return E * (2 * 8 + (fp32 ? 4 : 8)) + (size_t)g.ntiles * g.steps * FACE_WORDS * 8 + (size_t)g.ntiles * 16;
}

size_t resident_bytes(const Geom &g, int fp32) { return (size_t)g.elems * (7 * 8 + 7 * (fp32 ? 4 : 8)); }

sip_status dev_alloc(void **p, size_t n, hipStream_t s)
{
    hipError_t e = hipMallocAsync(p, n ? n : 1, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return set_error(SIP_ENOMEM, "device allocation of %zu bytes failed", n);
    }
    return SIP_OK;
}

void dev_free(void *p, hipStream_t s)
{
    if (p) (void)hipFreeAsync(p, s);
}

// x behind b in the request's buffer, in the precision of the sweeps
void *x_of(const GpuResident *s, const GpuReq *q)
{
    return s->arith == ARITH_F32 ? (void *)((float *)q->bx + s->g.elems) : (void *)(q->bx + s->g.elems);
}

// x pairs behind the b pairs, in the precision of the sweeps
void *pair_x(const Pair *p)
{
    const size_t E = (size_t)p->sys->g.elems;
    return p->sys->arith == ARITH_F32 ? (void *)((float *)p->bx + 2 * E) : (void *)(p->bx + 2 * E);
}

Job job_of(const GpuResident *s, const GpuReq *q, Ctl *ctl, int fw)
{
    Job J{};
    J.g = s->g;
    J.A = s->A;
    J.LU = s->LU;
    J.b = q->bx;
    J.x = x_of(s, q);
    J.y = q->y;
    J.face = q->face;
    J.part = q->part;
    J.hist = nullptr;   // served requests keep no residual history
    J.ctl = ctl + q->slot;
    J.alpha = s->alpha;
    J.fw = fw;
    J.sym = fw == FACE_WORDS ? 0 : s->sym;   // the factorisation reads the full coefficients
    return J;
}

class GpuBackend final : public Backend {
public:
    sip_server_config cfg{};
    int device = 0;
    int num_cu = 256;   // compute units of the device
    hipStream_t stream = nullptr;
    uint64_t timeout_ticks = 0;
    uint32_t torture = 0;   // schedule_seed() at creation: a new random order every launch group
    uint64_t steps = 0;     // steps run (varies the race-testing orders)
    std::chrono::steady_clock::time_point t0;
    // The sweeps of an epoch as a captured graph.  Its kernels read the job
    // list and ticket orders from device buffers uploaded before every epoch,
    // so the graph stays valid while the launch parameters (buffer addresses,
    // tile counts, plans, epoch length) stay the same; it is captured the
    // second time in a row the same parameters come up and replayed from then on.
    hipGraphExec_t epoch_exec = nullptr;
    std::vector<uint64_t> epoch_key;
    bool graphs = true;   // SIP_SERVER_GRAPHS=0 launches every epoch eagerly
    // device-side scratch for launches
    Ctl *ctl = nullptr;                      // MAX_SLOTS control blocks
    Ctl *h_ctl = nullptr;                    // pinned mirror
    // per launch group: factor storage or sweep arithmetic; NARITH + arith for pairs
    Job *d_jobs[2 * NARITH] = {};
    int2 *d_order[2 * NARITH][2] = {};
    int order_cap[2 * NARITH] = {};
    int jobs_cap[2 * NARITH] = {};
    Ctl *pctl = nullptr, *h_pctl = nullptr;   // 3 * MAX_PAIRS control blocks of pairs (device, pinned mirror)
    std::vector<int> free_pairs;
    std::vector<Pair *> pairs;                // live pairs
    bool pairing = false;                     // SIP_SERVER_PAIRS=1 turns pairing on
    LaunchCtl *lc = nullptr;
    unsigned *d_bad = nullptr, *h_bad = nullptr;   // symmetry check counter (device, pinned mirror)
    // persistent launches (k_persist): per launch group the jobs' tile orders,
    // their offsets and the task queue; one queue control block; two coherent
    // pinned flags (pause requests from the host, stop reports from the device)
    // persistent launches while no request arrives (a batch then runs every
    // block at its own pace); per-iteration epochs while requests keep
    // arriving (admission at every epoch boundary costs no drain).
    // SIP_SERVER_PERSISTENT=1 / 0 forces one of the two.
    int persistent = -1;                      // -1 adaptive, 1 always, 0 never
    int *d_torder[2 * NARITH] = {};
    int *d_off[2 * NARITH] = {};
    Task *d_tasks[2 * NARITH] = {};
    uint32_t *d_dep[2 * NARITH] = {};         // dataflow counters, 2 per tile
    int torder_cap[2 * NARITH] = {}, off_cap[2 * NARITH] = {}, tasks_cap[2 * NARITH] = {}, dep_cap[2 * NARITH] = {};
    // persistent launches publish each sweep tile by tile as upstream tiles are
    // taken (SIP_SERVER_DATAFLOW=0: whole sweeps in topological order)
    bool dataflow = true;
    PersistCtl *d_pc = nullptr, *h_pc = nullptr;
    uint32_t *h_pause = nullptr, *h_stopped = nullptr;   // coherent host memory, read / written by the device
    uint32_t *d_pause = nullptr, *d_stopped = nullptr;   // their device addresses
    // forward then backward tile order of a block of nti x ntj tiles (the
    // default order depends on nothing else)
    std::map<std::pair<int, int>, std::vector<int>> tile_orders;
    SweepPlan plan{};
    bool plan_forced = false;   // SIP_SWEEP_PHASES set: no tuned plans

    // race testing: a different random ticket order for every launch group
    uint32_t order_seed(int grp) const
    {
        return torture ? (torture + 7919u * (uint32_t)steps + 104729u * (uint32_t)grp) | 1u : 0u;
    }

    sip_status init(sip_server_config &c);
    ~GpuBackend() override;

    double now() override
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void thread_start() override { (void)hipSetDevice(device); }
    sip_status check_problem(const sip_problem &p) override
    {
        // kernels address every array with 32-bit byte offsets
        if (make_geom(p.ni, p.nj, p.nk).elems >= MAX_ELEMS) return set_error(SIP_EINVAL, "block too large");
        return SIP_OK;
    }
    size_t system_bytes(const sip_problem &p) override
    {
        return resident_bytes(make_geom(p.ni, p.nj, p.nk), p.precision != SIP_FP64);
    }
    size_t request_bytes(const sip_problem &p, const Resident *res) override
    {
        if (res) return slot_bytes(static_cast<const GpuResident *>(res)->g, static_cast<const GpuResident *>(res)->fp32);
        return slot_bytes(make_geom(p.ni, p.nj, p.nk), p.precision != SIP_FP64);
    }
    sip_status new_request(const sip_request &r, std::unique_ptr<Req> *out) override;
    sip_status new_system(const Req &q, std::unique_ptr<Resident> *out) override;
    void free_system(Resident *s) override
    {
        auto *gs = static_cast<GpuResident *>(s);
        dev_free(gs->A, stream);
        dev_free(gs->LU, stream);
        gs->A = nullptr;
        gs->LU = nullptr;
    }
    sip_status alloc_request(Req *q) override;
    size_t release_request(Req *q) override;
    void wait_for_callers(const std::vector<Req *> &admitted) override
    {
        // the coefficients, b and x0 were produced on the caller's stream:
        // everything after this that reads them runs after that stream's work
        for (Req *q : admitted)
            if (hipEvent_t e = static_cast<GpuReq *>(q)->ready) (void)hipStreamWaitEvent(stream, e, 0);
    }
    void factor(const std::vector<Resident *> &sys, const std::vector<Req *> &owners,
                std::vector<sip_status> &result) override;
    void stage(std::vector<Req *> &ready) override;
    sip_status step(std::vector<Req *> &act) override;
    Outcome outcome(const Req *q, sip_status st) override;
    void retire(const std::vector<Req *> &fin, sip_status st) override;
    void drain() override { (void)hipStreamSynchronize(stream); }

private:
    sip_status run_factor(const std::vector<GpuResident *> &sys, const std::vector<GpuReq *> &owners,
                          std::vector<sip_status> &result);
    sip_status run_persist(int grp, const std::vector<Job> &jobs, const std::vector<Geom> &gs, const SweepPlan &gp,
                           bool others_waiting);
    bool want_pause(double since_launch, bool others_waiting);
    // The bound of every device-side wait: 2 s, or SIP_WAIT_LIMIT_MS (read at
    // every factorisation and step; a test hook, see sip_solve).
    void refresh_wait_limit() { timeout_ticks = timeout_ticks_for(device, wait_limit_seconds()); }
    void form_pairs(std::vector<GpuReq *> &ready);
    void free_pair(Pair *p);
    sip_status ensure_launch_buffers(int grp, int njobs, int ntiles);
};

sip_status GpuBackend::new_request(const sip_request &r, std::unique_ptr<Req> *out)
{
    // orders the server's reads of the request's arrays after the caller's
    // work on its stream (the event is destroyed with the request object)
    auto q = std::make_unique<GpuReq>();
    if (hipEventCreateWithFlags(&q->ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(q->ready, (hipStream_t)r.stream) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(SIP_EDEVICE, "could not record the ordering event on the caller's stream");
    }
    *out = std::move(q);
    return SIP_OK;
}

sip_status GpuBackend::new_system(const Req &q, std::unique_ptr<Resident> *out)
{
    const sip_problem &pb = q.r.problem;
    auto rs = std::make_unique<GpuResident>();
    rs->g = make_geom(pb.ni, pb.nj, pb.nk);
    rs->arith = pb.precision;
    rs->fp32 = pb.precision != SIP_FP64;
    rs->alpha = pb.alpha;
    rs->sym = pb.storage == SIP_STORAGE_SYMMETRIC;
    if (dev_alloc((void **)&rs->A, 7 * (size_t)rs->g.elems * 8, stream) != SIP_OK ||
        dev_alloc(&rs->LU, 7 * (size_t)rs->g.elems * (rs->fp32 ? 4 : 8), stream) != SIP_OK) {
        free_system(rs.get());
        return SIP_ENOMEM;
    }
    *out = std::move(rs);
    return SIP_OK;
}

sip_status GpuBackend::alloc_request(Req *rq)
{
    auto *q = static_cast<GpuReq *>(rq);
    const Geom &g = gsys(q)->g;
    const size_t E = (size_t)g.elems;
    const size_t fbytes = (size_t)g.ntiles * g.steps * FACE_WORDS * 8;
    if (dev_alloc((void **)&q->bx, 2 * E * 8, stream) != SIP_OK ||
        dev_alloc(&q->y, E * (gsys(q)->fp32 ? 4 : 8), stream) != SIP_OK ||
        dev_alloc((void **)&q->face, fbytes, stream) != SIP_OK ||
        dev_alloc((void **)&q->part, (size_t)g.ntiles * 16, stream) != SIP_OK)
        return SIP_ENOMEM;   // release_request frees what was allocated
    (void)hipMemsetAsync(q->face, 0, fbytes, stream);
    return SIP_OK;
}

size_t GpuBackend::release_request(Req *rq)
{
    auto *q = static_cast<GpuReq *>(rq);
    dev_free(q->bx, stream);
    dev_free(q->y, stream);
    dev_free(q->face, stream);
    dev_free(q->part, stream);
    q->bx = nullptr;
    q->y = nullptr;
    q->face = nullptr;
    q->part = nullptr;
    if (q->ready) {   // the server stream's wait on it, if any, is already enqueued
        (void)hipEventDestroy(q->ready);
        q->ready = nullptr;
    }
    size_t give = q->bytes;
    if (Pair *p = q->pair) {
        // the pair's buffers stand for both members' budget bytes: they are
        // released when the second member is done
        p->done[q->pm] = true;
        p->held += q->bytes;
        give = 0;
        q->pair = nullptr;
        if (p->done[0] && p->done[1]) {
            give = p->held;
            free_pair(p);
        }
    }
    return give;
}

void GpuBackend::free_pair(Pair *p)
{
    dev_free(p->bx, stream);
    dev_free(p->y, stream);
    dev_free(p->face, stream);
    dev_free(p->part, stream);
    free_pairs.push_back(p->idx);
    pairs.erase(std::find(pairs.begin(), pairs.end(), p));
    delete p;
}

// Pairs freshly admitted requests of one resident system (FP32 factors, the
// same rtol and max_iter, start vectors both given or both zero): they share
// one pass of the sweeps over A and the factors.  The pair's buffers replace
// the members' own, inside the budget the members were admitted with.
void GpuBackend::form_pairs(std::vector<GpuReq *> &ready)
{
    if (!pairing) return;
    std::vector<GpuReq *> open;
    for (GpuReq *q : ready) {
        const GpuResident *rs = gsys(q);
        if (rs->arith != ARITH_MIXED && rs->arith != ARITH_F32) continue;
        GpuReq *mate = nullptr;
        for (GpuReq *o : open)
            if (o->sys == rs && o->r.rtol == q->r.rtol && o->r.max_iter == q->r.max_iter &&
                (o->r.x0 == nullptr) == (q->r.x0 == nullptr)) {
                mate = o;
                break;
            }
        if (!mate) {
            open.push_back(q);
            continue;
        }
        open.erase(std::find(open.begin(), open.end(), mate));
        if (free_pairs.empty()) continue;
        const Geom &g = rs->g;
        const size_t E = (size_t)g.elems;
        const size_t fbytes = (size_t)g.ntiles * g.steps * FACE_WORDS * 8;
        Pair *p = new Pair();
        p->sys = gsys(q);
        if (dev_alloc((void **)&p->bx, 4 * E * 8, stream) != SIP_OK || dev_alloc(&p->y, 2 * E * 4, stream) != SIP_OK ||
            dev_alloc((void **)&p->face, fbytes, stream) != SIP_OK ||
            dev_alloc((void **)&p->part, (size_t)g.ntiles * 32, stream) != SIP_OK) {
            dev_free(p->bx, stream);
            dev_free(p->y, stream);
            dev_free(p->face, stream);
            dev_free(p->part, stream);
            delete p;
            continue;   // both stay single
        }
        p->idx = free_pairs.back();
        free_pairs.pop_back();
        p->r[0] = mate;
        p->r[1] = q;
        const bool f32 = rs->arith == ARITH_F32;
        const int sh = f32 ? SHEAR_PAIR_F32 : SHEAR_PAIR_F64;
        const double *bs[2] = {mate->r.b, q->r.b};
        (void)hipMemsetAsync(p->face, 0, fbytes, stream);   // fresh tags: the pair's epochs start at 1
        (void)launch_to_sheared(g, 2, bs, p->bx, g.elems, sh, stream);
        if (q->r.x0) {
            const double *xs[2] = {mate->r.x0, q->r.x0};
            (void)launch_to_sheared(g, 2, xs, pair_x(p), g.elems, sh, stream);
        } else {
            (void)hipMemsetAsync(pair_x(p), 0, 2 * E * (f32 ? 4 : 8), stream);
        }
        (void)launch_init_ctl(pctl + 3 * p->idx, 3, (uint32_t)q->r.max_iter, q->r.rtol, 1, stream);
        for (int m = 0; m < 2; m++) {
            GpuReq *r = p->r[m];
            dev_free(r->bx, stream);
            dev_free(r->y, stream);
            dev_free(r->face, stream);
            dev_free(r->part, stream);
            r->bx = nullptr;
            r->y = nullptr;
            r->face = nullptr;
            r->part = nullptr;
            r->pair = p;
            r->pm = m;
        }
        pairs.push_back(p);
        host->count(STAT_PAIRS, 1);
    }
}

sip_status GpuBackend::ensure_launch_buffers(int grp, int njobs, int ntiles)
{
    if (njobs > jobs_cap[grp]) {
        dev_free(d_jobs[grp], stream);
        const int cap = std::max(njobs, 64);
        if (dev_alloc((void **)&d_jobs[grp], (size_t)cap * sizeof(Job), stream) != SIP_OK) return SIP_ENOMEM;
        jobs_cap[grp] = cap;
    }
    if (ntiles > order_cap[grp]) {
        dev_free(d_order[grp][0], stream);
        dev_free(d_order[grp][1], stream);
        const int cap = std::max(ntiles, 4096);
        if (dev_alloc((void **)&d_order[grp][0], (size_t)cap * sizeof(int2), stream) != SIP_OK ||
            dev_alloc((void **)&d_order[grp][1], (size_t)cap * sizeof(int2), stream) != SIP_OK)
            return SIP_ENOMEM;
        order_cap[grp] = cap;
    }
    return SIP_OK;
}

void GpuBackend::factor(const std::vector<Resident *> &sys, const std::vector<Req *> &owners,
                        std::vector<sip_status> &result)
{
    std::vector<GpuResident *> gs;
    std::vector<GpuReq *> go;
    for (size_t k = 0; k < sys.size(); k++) {
        gs.push_back(static_cast<GpuResident *>(sys[k]));
        go.push_back(static_cast<GpuReq *>(owners[k]));
    }
    refresh_wait_limit();
    if (const sip_status e = run_factor(gs, go, result); e != SIP_OK)
        for (sip_status &r : result)
            if (r == SIP_OK) r = e;
}

// Factorise newly resident systems, all of them in one batched launch per
// precision; each uses the face words of the request that brought it in.
// A symmetric-storage request whose A is not symmetric fails with SIP_EINVAL,
// a factorisation that breaks down with SIP_EBREAKDOWN.
sip_status GpuBackend::run_factor(const std::vector<GpuResident *> &sys, const std::vector<GpuReq *> &owners,
                                  std::vector<sip_status> &result)
{
    const Range range("server factorisations");
    for (int grp = 0; grp < 2; grp++) {
        std::vector<Job> jobs;
        std::vector<Geom> gs;
        for (size_t k = 0; k < sys.size(); k++) {
            if (sys[k]->fp32 != grp) continue;
            const sip_problem &pb = owners[k]->r.problem;
            if (sys[k]->sym) {   // the symmetric storage is only valid for a symmetric A
                if (hipMemsetAsync(d_bad, 0, sizeof(unsigned), stream) != hipSuccess ||
                    launch_check_symmetric(pb.ni, pb.nj, pb.nk, pb.a, d_bad, stream) != hipSuccess ||
                    hipMemcpyAsync(h_bad, d_bad, sizeof(unsigned), hipMemcpyDeviceToHost, stream) != hipSuccess ||
                    hipStreamSynchronize(stream) != hipSuccess)
                    return set_error(SIP_EDEVICE, "symmetry check failed");
                if (*h_bad) {
                    result[k] = SIP_EINVAL;
                    continue;
                }
            }
            if (launch_to_sheared(sys[k]->g, 7, pb.a, sys[k]->A, sys[k]->g.elems, SHEAR_COEF, stream) != hipSuccess)
                return set_error(SIP_EDEVICE, "reorder failed");
            // tags stay monotonic per slot (never reset): face words of the
            // factorisation can never be mistaken for a later sweep's
            if (launch_init_ctl(ctl + owners[k]->slot, 1, 0, 0.0, 0, stream) != hipSuccess)
                return set_error(SIP_EDEVICE, "init failed");
            jobs.push_back(job_of(sys[k], owners[k], ctl, FACE_WORDS));
            gs.push_back(sys[k]->g);
        }
        if (jobs.empty()) continue;
        const std::vector<int2> of = topo_order(gs, false, order_seed(grp));
        if (ensure_launch_buffers(grp, (int)jobs.size(), (int)of.size()) != SIP_OK) return SIP_ENOMEM;
        if (hipMemcpyAsync(d_jobs[grp], jobs.data(), jobs.size() * sizeof(Job), hipMemcpyHostToDevice, stream) !=
                hipSuccess ||
            hipMemcpyAsync(d_order[grp][0], of.data(), of.size() * sizeof(int2), hipMemcpyHostToDevice, stream) !=
                hipSuccess)
            return set_error(SIP_EDEVICE, "upload failed");
        const LaunchArgs la{d_jobs[grp], d_order[grp][0], lc, (int)of.size(), timeout_ticks, torture};
        if (launch_factor(la, grp, stream) != hipSuccess) return set_error(SIP_EDEVICE, "factor launch failed");
        // the sweeps of symmetric systems read the symmetric storage, those of
        // the all-FP32 arithmetic FP32 coefficients; either overwrites the full
        // FP64 storage once the factorisation is done
        for (size_t k = 0; k < sys.size(); k++) {
            if (sys[k]->fp32 != grp || result[k] != SIP_OK) continue;
            const int sc = sys[k]->sym ? SHEAR_SYM : sys[k]->arith == ARITH_F32 ? SHEAR_COEF32 : SHEAR_COEF;
            if (sc != SHEAR_COEF &&
                launch_to_sheared(sys[k]->g, 7, owners[k]->r.problem.a, sys[k]->A, sys[k]->g.elems, sc, stream) !=
                    hipSuccess)
                return set_error(SIP_EDEVICE, "reorder failed");
        }
        // the host copies of jobs/orders must live until the copies ran
        if (hipStreamSynchronize(stream) != hipSuccess) return set_error(SIP_EDEVICE, "factorisation failed");
        host->count(STAT_LAUNCHES, 1);
    }
    if (hipMemcpyAsync(h_ctl, ctl, sizeof(Ctl) * MAX_SLOTS, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return set_error(SIP_EDEVICE, "factorisation status copy failed");
    for (size_t k = 0; k < sys.size(); k++) {
        const uint32_t fs = h_ctl[owners[k]->slot].stop;
        if (result[k] == SIP_OK && fs != RUN) result[k] = fs == TIMEOUT ? SIP_EDEVICE : SIP_EBREAKDOWN;
    }
    return SIP_OK;
}

// Stages b and x0 of newly admitted requests (pairs with their partner).
void GpuBackend::stage(std::vector<Req *> &ready_reqs)
{
    std::vector<GpuReq *> ready;
    for (Req *q : ready_reqs) ready.push_back(static_cast<GpuReq *>(q));
    form_pairs(ready);
    for (GpuReq *q : ready) {
        if (q->pair) continue;   // staged with its partner
        const GpuResident *rs = gsys(q);
        const Geom &g = rs->g;
        const double *src[2] = {q->r.b, q->r.x0 ? q->r.x0 : nullptr};
        const bool f32 = rs->arith == ARITH_F32;   // the relaxation starts from FP32 copies
        const int sh = f32 ? SHEAR_F32 : SHEAR_F64;
        if (q->r.x0) {
            (void)launch_to_sheared(g, 2, src, q->bx, g.elems, sh, stream);
        } else {
            (void)launch_to_sheared(g, 1, src, q->bx, g.elems, sh, stream);
            (void)hipMemsetAsync(x_of(rs, q), 0, (size_t)g.elems * (f32 ? 4 : 8), stream);
        }
        (void)launch_init_ctl(ctl + q->slot, 1, (uint32_t)q->r.max_iter, q->r.rtol, 0, stream);
    }
}

// One step: epoch_iters (forward, backward) pairs over every running request,
// or one persistent launch.
sip_status GpuBackend::step(std::vector<Req *> &act)
{
    const Range range("server epoch");
    steps++;
    refresh_wait_limit();
    // groups 0..NARITH-1: single requests by arithmetic; NARITH + arith: pairs
    constexpr int NG = 2 * NARITH;
    std::vector<Job> jobs[NG];
    std::vector<Geom> gs[NG];
    for (Req *rq : act) {
        const auto *q = static_cast<const GpuReq *>(rq);
        if (q->pair) continue;
        const int grp = gsys(q)->arith;
        jobs[grp].push_back(job_of(gsys(q), q, ctl, FACE_WORDS_SWEEP));
        gs[grp].push_back(gsys(q)->g);
    }
    for (Pair *p : pairs) {
        const GpuResident *rs = p->sys;
        Job J{};
        J.g = rs->g;
        J.A = rs->A;
        J.LU = rs->LU;
        J.b = p->bx;
        J.x = pair_x(p);
        J.y = p->y;
        J.face = p->face;
        J.part = p->part;
        J.hist = nullptr;
        J.ctl = pctl + 3 * p->idx;
        J.alpha = rs->alpha;
        J.fw = FACE_WORDS_SWEEP;
        J.sym = rs->sym;
        J.m = 2;
        jobs[NARITH + rs->arith].push_back(J);
        gs[NARITH + rs->arith].push_back(rs->g);
    }
    std::vector<int2> of[NG], ob[NG];
    LaunchArgs fa[NG], ba[NG];
    for (int grp = 0; grp < NG; grp++) {
        if (jobs[grp].empty()) continue;
        of[grp] = topo_order(gs[grp], false, order_seed(grp));
        ob[grp] = topo_order(gs[grp], true, order_seed(grp));
        if (ensure_launch_buffers(grp, (int)jobs[grp].size(), (int)of[grp].size()) != SIP_OK) return SIP_ENOMEM;
        if (hipMemcpyAsync(d_jobs[grp], jobs[grp].data(), jobs[grp].size() * sizeof(Job), hipMemcpyHostToDevice,
                           stream) != hipSuccess ||
            hipMemcpyAsync(d_order[grp][0], of[grp].data(), of[grp].size() * sizeof(int2), hipMemcpyHostToDevice,
                           stream) != hipSuccess ||
            hipMemcpyAsync(d_order[grp][1], ob[grp].data(), ob[grp].size() * sizeof(int2), hipMemcpyHostToDevice,
                           stream) != hipSuccess)
            return set_error(SIP_EDEVICE, "upload failed");
        fa[grp] = LaunchArgs{d_jobs[grp], d_order[grp][0], lc, (int)of[grp].size(), timeout_ticks, torture};
        ba[grp] = LaunchArgs{d_jobs[grp], d_order[grp][1], lc, (int)ob[grp].size(), timeout_ticks, torture};
    }
    // launch shape of each group: the tuned plan of its largest block
    // (sip_tune); without one, the split three-phase turns while the group has
    // no more tiles than compute units (latency-bound, like a single system),
    // else two phases (two workgroups per compute unit hide more latency)
    SweepPlan gplan[NG];
    for (int grp = 0; grp < NG; grp++) {
        gplan[grp] = plan;
        if (plan_forced || jobs[grp].empty()) continue;
        if ((int)of[grp].size() <= num_cu) gplan[grp].phases = SINGLE_SYSTEM_PHASES;
        const Job *big = &jobs[grp][0];
        for (const Job &J : jobs[grp])
            if (J.g.elems > big->g.elems) big = &J;
        (void)tuned_plan(big->g, grp % NARITH, big->sym, &gplan[grp]);
    }
    // persistent while nothing was submitted since the last step
    const bool use_persistent = persistent < 0 ? !host->arrivals_since_last_step() : persistent == 1;
    if (use_persistent) {
        int groups = 0;
        for (int grp = 0; grp < NG; grp++) groups += !jobs[grp].empty();
        for (int grp = 0; grp < NG; grp++) {
            if (jobs[grp].empty()) continue;
            const sip_status st = run_persist(grp, jobs[grp], gs[grp], gplan[grp], groups > 1);
            if (st != SIP_OK) return st;
        }
        if (hipMemcpyAsync(h_ctl, ctl, sizeof(Ctl) * MAX_SLOTS, hipMemcpyDeviceToHost, stream) != hipSuccess ||
            (!pairs.empty() &&
             hipMemcpyAsync(h_pctl, pctl, sizeof(Ctl) * 3 * MAX_PAIRS, hipMemcpyDeviceToHost, stream) != hipSuccess) ||
            hipStreamSynchronize(stream) != hipSuccess)
            return set_error(SIP_EDEVICE, "launch failed: %s", hipGetErrorString(hipGetLastError()));
        host->count(STAT_EPOCHS, 1);
        return SIP_OK;
    }
    auto launch_all = [&]() -> bool {
        for (int it = 0; it < cfg.epoch_iters; it++) {
            for (int grp = 0; grp < NG; grp++) {
                if (jobs[grp].empty()) continue;
                const int arith = grp % NARITH, nrhs = grp < NARITH ? 1 : 2;
                if (launch_forward(fa[grp], arith, gplan[grp], stream, nrhs) != hipSuccess ||
                    launch_backward(ba[grp], arith, gplan[grp], stream, nrhs) != hipSuccess)
                    return false;
            }
        }
        return true;
    };
    std::vector<uint64_t> key{(uint64_t)cfg.epoch_iters};
    for (int grp = 0; grp < NG; grp++) {
        if (jobs[grp].empty()) {
            key.push_back(0);
            continue;
        }
        key.insert(key.end(), {1, (uint64_t)gplan[grp].phases, (uint64_t)gplan[grp].poll,
                               (uint64_t)(uintptr_t)fa[grp].jobs, (uint64_t)(uintptr_t)fa[grp].order,
                               (uint64_t)(uintptr_t)ba[grp].order, (uint64_t)(uintptr_t)fa[grp].lc,
                               (uint64_t)fa[grp].total, (uint64_t)ba[grp].total, fa[grp].timeout_ticks,
                               (uint64_t)fa[grp].jitter});
        host->count(STAT_LAUNCHES, 2 * (uint64_t)cfg.epoch_iters);
    }
    const bool same = key == epoch_key;
    epoch_key = key;
    if (!same && epoch_exec) {
        (void)hipGraphExecDestroy(epoch_exec);
        epoch_exec = nullptr;
    }
    if (same && !epoch_exec && graphs) {
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            const bool ok = launch_all();
            if (hipStreamEndCapture(stream, &graph) == hipSuccess && ok && graph &&
                hipGraphInstantiate(&epoch_exec, graph, nullptr, nullptr, 0) != hipSuccess)
                epoch_exec = nullptr;
            if (graph) (void)hipGraphDestroy(graph);
        }
        (void)hipGetLastError();   // a failed capture leaves the eager launches below
    }
    if (epoch_exec) {
        if (hipGraphLaunch(epoch_exec, stream) != hipSuccess) return set_error(SIP_EDEVICE, "epoch graph launch failed");
        host->count(STAT_GRAPH_EPOCHS, 1);
    } else if (!launch_all()) {
        return set_error(SIP_EDEVICE, "sweep launch failed");
    }
    if (hipMemcpyAsync(h_ctl, ctl, sizeof(Ctl) * MAX_SLOTS, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        (!pairs.empty() &&
         hipMemcpyAsync(h_pctl, pctl, sizeof(Ctl) * 3 * MAX_PAIRS, hipMemcpyDeviceToHost, stream) != hipSuccess) ||
        hipStreamSynchronize(stream) != hipSuccess)
        return set_error(SIP_EDEVICE, "epoch failed: %s", hipGetErrorString(hipGetLastError()));
    host->count(STAT_EPOCHS, 1);
    return SIP_OK;
}

// Whether the running persistent launch should let its requests pause: new
// requests wait for admission (after a short minimum run, so that a queue that
// cannot be admitted yet does not restart the launch over and over), a request
// has stopped and waits to be retired, another launch group waits for its
// turn, or the server is shutting down.
bool GpuBackend::want_pause(double since_launch, bool others_waiting)
{
    // a pause drains the launch (every request finishes its iteration), so it
    // is asked for no more often than these intervals
    constexpr double ADMIT = 10e-3, RETIRE = 20e-3, SLICE = 20e-3;
    if (since_launch >= RETIRE && __atomic_load_n(h_stopped, __ATOMIC_ACQUIRE)) return true;
    if (others_waiting && since_launch >= SLICE) return true;
    if (host->quitting()) return true;
    return since_launch >= ADMIT && host->admission_waiting();
}

// One persistent launch for the jobs of launch group grp: every job starts at
// its next forward sweep (an iteration boundary) and runs until it stops or
// the host asks for a pause.
sip_status GpuBackend::run_persist(int grp, const std::vector<Job> &jobs, const std::vector<Geom> &gs,
                                   const SweepPlan &gp, bool others_waiting)
{
    const int arith = grp % NARITH, nrhs = grp < NARITH ? 1 : 2;
    const int nj = (int)jobs.size();
    std::vector<int> off(nj + 1, 0), tord;
    for (int j = 0; j < nj; j++) off[j + 1] = off[j] + gs[j].ntiles;
    const int total = off[nj];
    tord.reserve(2 * (size_t)total);
    for (int j = 0; j < nj; j++) {
        if (order_seed(grp)) {   // race testing: a random order per job and launch
            for (int b = 0; b < 2; b++)
                for (const int2 &o : topo_order({gs[j]}, b != 0, order_seed(grp) + 31u * j)) tord.push_back(o.y);
            continue;
        }
        std::vector<int> &c = tile_orders[{gs[j].nti, gs[j].ntj}];
        if (c.empty())
            for (int b = 0; b < 2; b++)
                for (const int2 &o : topo_order({gs[j]}, b != 0, 0u)) c.push_back(o.y);
        tord.insert(tord.end(), c.begin(), c.end());
    }
    // the first forward sweeps: every job's first tile (dataflow), or all
    // tiles merged over the jobs (topological per job)
    std::vector<int2> first;
    if (dataflow)
        for (int j = 0; j < nj; j++) first.push_back(make_int2(j, 0));
    else
        first = topo_order(gs, false, order_seed(grp));
    const uint32_t cap = (uint32_t)total + 64u;   // more than the tiles of all jobs
    if (nj > (1 << TASK_JOB_BITS) || total > (1 << TASK_TILE_BITS))
        return set_error(SIP_EINVAL, "persistent launch of %d jobs / %d tiles exceeds the task encoding", nj, total);
    std::vector<Task> tasks(cap, (Task)0);
    for (size_t t = 0; t < first.size(); t++) tasks[t] = make_task((uint32_t)t, first[t].x, 0, first[t].y);
    auto grow = [&](void **p, int &have, int need, size_t elem) -> bool {
        if (need <= have) return true;
        dev_free(*p, stream);
        const int c = std::max(need, 4096);
        if (dev_alloc(p, (size_t)c * elem, stream) != SIP_OK) return false;
        have = c;
        return true;
    };
    if (ensure_launch_buffers(grp, nj, (int)first.size()) != SIP_OK ||
        !grow((void **)&d_torder[grp], torder_cap[grp], 2 * total, sizeof(int)) ||
        !grow((void **)&d_off[grp], off_cap[grp], nj + 1, sizeof(int)) ||
        !grow((void **)&d_tasks[grp], tasks_cap[grp], (int)cap, sizeof(Task)) ||
        (dataflow && !grow((void **)&d_dep[grp], dep_cap[grp], 2 * total, sizeof(uint32_t))))
        return SIP_ENOMEM;
    *h_pc = PersistCtl{0u, (uint32_t)first.size(), (uint32_t)nj, 0u};
    __atomic_store_n(h_pause, 0u, __ATOMIC_RELEASE);
    __atomic_store_n(h_stopped, 0u, __ATOMIC_RELEASE);
    if (hipMemcpyAsync(d_jobs[grp], jobs.data(), jobs.size() * sizeof(Job), hipMemcpyHostToDevice, stream) !=
            hipSuccess ||
        hipMemcpyAsync(d_torder[grp], tord.data(), tord.size() * sizeof(int), hipMemcpyHostToDevice, stream) !=
            hipSuccess ||
        hipMemcpyAsync(d_off[grp], off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice, stream) !=
            hipSuccess ||
        hipMemcpyAsync(d_tasks[grp], tasks.data(), tasks.size() * sizeof(Task), hipMemcpyHostToDevice, stream) !=
            hipSuccess ||
        hipMemcpyAsync(d_pc, h_pc, sizeof(PersistCtl), hipMemcpyHostToDevice, stream) != hipSuccess ||
        (dataflow && hipMemsetAsync(d_dep[grp], 0, 2 * (size_t)total * sizeof(uint32_t), stream) != hipSuccess))
        return set_error(SIP_EDEVICE, "upload failed");
    const PersistArgs pa{d_jobs[grp], d_torder[grp], d_off[grp], d_tasks[grp], cap, d_pc, d_pause, d_stopped,
                         timeout_ticks, torture, dataflow ? d_dep[grp] : nullptr};
    // persistent workgroups: one per compute unit (the kernel holds both
    // sweeps and needs about 120 VGPRs, so a unit fits one workgroup of either
    // phase count; three phases shorten the step), never more than the tiles
    // that can be in flight.  SIP_SWEEP_PHASES=2 still selects two phases.
    SweepPlan pp = gp;
    pp.phases = plan_forced ? std::max(2, std::min(3, gp.phases)) : 3;
    const int wgs = std::max(1, std::min(total, num_cu));
    const auto tl = std::chrono::steady_clock::now();
    if (launch_persist(pa, arith, pp, wgs, stream, nrhs) != hipSuccess)
        return set_error(SIP_EDEVICE, "persistent launch failed");
    if (hipMemcpyAsync(h_pc, d_pc, sizeof(PersistCtl), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return set_error(SIP_EDEVICE, "status copy failed");
    host->count(STAT_LAUNCHES, 1);
    // while it runs: pause requests (the host vectors above stay alive until
    // the launch is over, so the copies from them have run)
    bool paused = false;
    for (;;) {
        const hipError_t q = hipStreamQuery(stream);
        if (q == hipSuccess) break;
        if (q != hipErrorNotReady) return set_error(SIP_EDEVICE, "persistent launch failed: %s", hipGetErrorString(q));
        if (!paused &&
            want_pause(std::chrono::duration<double>(std::chrono::steady_clock::now() - tl).count(), others_waiting)) {
            __atomic_store_n(h_pause, 1u, __ATOMIC_RELEASE);
            paused = true;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(paused ? 20 : 100));
    }
    if (h_pc->err) return set_error(SIP_EDEVICE, "a device-side queue wait timed out");
    return SIP_OK;
}

// Where a request stands after the step: its control block (a pair member's
// own, with the pair's sweep failures) as copied back at the step's end.
Outcome GpuBackend::outcome(const Req *rq, sip_status st)
{
    const auto *q = static_cast<const GpuReq *>(rq);
    Outcome o;
    Ctl c = h_ctl[q->slot];
    if (const Pair *p = q->pair) {
        c = h_pctl[3 * p->idx + 1 + q->pm];
        const uint32_t js = h_pctl[3 * p->idx].stop;
        if (js == BREAKDOWN || js == TIMEOUT) c.stop = js;
        if (c.stop == ZERO_RHS) c.rho = 0.0;
    }
    o.done = st != SIP_OK || c.stop != RUN;
    if (!o.done) return o;
    o.iters = (int)c.iter;
    o.rho = c.rho;
    if (st != SIP_OK) o.status = st;
    else if (c.stop == MAXITER) o.status = SIP_ENOTCONV;
    else if (c.stop == BREAKDOWN || c.stop == DIVERGED) o.status = SIP_EBREAKDOWN;
    else if (c.stop == BAD_INPUT) o.status = SIP_EINVAL;   // non-finite b, x0 or A x0
    else if (c.stop == TIMEOUT) o.status = SIP_EDEVICE;
    return o;
}

// Copies x of the stopped requests out (after a failed step, nothing).
void GpuBackend::retire(const std::vector<Req *> &fin, sip_status st)
{
    if (st == SIP_OK)
        for (Req *rq : fin) {
            const auto *q = static_cast<const GpuReq *>(rq);
            const GpuResident *rs = gsys(q);
            if (const Pair *p = q->pair)
                (void)launch_from_sheared(rs->g, pair_x(p), rs->arith == ARITH_F32, q->r.x,
                                          pctl + 3 * p->idx + 1 + q->pm, stream, 2, q->pm);
            else
                (void)launch_from_sheared(rs->g, x_of(rs, q), rs->arith == ARITH_F32, q->r.x, ctl + q->slot, stream);
        }
    (void)hipStreamSynchronize(stream);
}

sip_status GpuBackend::init(sip_server_config &c)
{
    cfg = c;
    if (const hipError_t e = hipGetDevice(&device); e != hipSuccess)
        return set_error(SIP_EDEVICE, "no HIP device: hipGetDevice: %s", hipGetErrorString(e));
    if (c.hbm_budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = (size_t)8 << 30;
        c.hbm_budget_bytes = fr / 4 * 3;
    }
    if (const char *e = getenv("SIP_SWEEP_PHASES")) {
        const int nl = atoi(e);
        if (nl >= 1 && nl <= sipk::MAX_PHASES) {
            plan.phases = nl;
            plan_forced = true;
        }
    }
    if (const char *e = getenv("SIP_POLL_DISTANCE")) {
        const int pd = atoi(e);
        if (pd >= 1 && pd <= sipk::MAX_POLL) {
            plan.poll = pd;
            plan_forced = true;
        }
    }
    if (const char *e = getenv("SIP_SERVER_PAIRS")) pairing = atoi(e) != 0;
    if (const char *e = getenv("SIP_SERVER_GRAPHS")) graphs = atoi(e) != 0;
    if (const char *e = getenv("SIP_SERVER_PERSISTENT")) persistent = atoi(e) != 0 ? 1 : 0;
    if (const char *e = getenv("SIP_SERVER_DATAFLOW")) dataflow = atoi(e) != 0;
    timeout_ticks = timeout_ticks_for(device, 2.0);
    torture = schedule_seed();
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
            num_cu = ncu;
    }
    t0 = std::chrono::steady_clock::now();
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc((void **)&ctl, sizeof(Ctl) * MAX_SLOTS) != hipSuccess ||
        hipHostMalloc((void **)&h_ctl, sizeof(Ctl) * MAX_SLOTS, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&lc, sizeof(LaunchCtl)) != hipSuccess ||
        hipMalloc((void **)&pctl, sizeof(Ctl) * 3 * MAX_PAIRS) != hipSuccess ||
        hipHostMalloc((void **)&h_pctl, sizeof(Ctl) * 3 * MAX_PAIRS, hipHostMallocDefault) != hipSuccess ||
        hipMemsetAsync(pctl, 0, sizeof(Ctl) * 3 * MAX_PAIRS, stream) != hipSuccess ||
        launch_init_ctl(pctl, 3 * MAX_PAIRS, 0, 0.0, 1, stream) != hipSuccess ||
        hipMalloc((void **)&d_bad, sizeof(unsigned)) != hipSuccess ||
        hipHostMalloc((void **)&h_bad, sizeof(unsigned), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&d_pc, sizeof(PersistCtl)) != hipSuccess ||
        hipHostMalloc((void **)&h_pc, sizeof(PersistCtl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&h_pause, sizeof(uint32_t), hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc((void **)&h_stopped, sizeof(uint32_t), hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer((void **)&d_pause, h_pause, 0) != hipSuccess ||
        hipHostGetDevicePointer((void **)&d_stopped, h_stopped, 0) != hipSuccess ||
        // on the server's own stream, in order: the stream does not synchronise
        // with the legacy default stream, so a plain hipMemset could land after
        // the initialisation and reset the epochs to 0, which the zeroed face
        // words of a fresh request would then match
        hipMemsetAsync(ctl, 0, sizeof(Ctl) * MAX_SLOTS, stream) != hipSuccess ||
        hipMemsetAsync(lc, 0, sizeof(LaunchCtl), stream) != hipSuccess ||
        launch_init_ctl(ctl, MAX_SLOTS, 0, 0.0, 1, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(SIP_ENOMEM, "server buffers");
    }
    for (int k = MAX_PAIRS - 1; k >= 0; k--) free_pairs.push_back(k);
    return SIP_OK;
}

GpuBackend::~GpuBackend()
{
    if (!stream) return;
    for (Pair *p : std::vector<Pair *>(pairs)) free_pair(p);
    for (int grp = 0; grp < 2 * NARITH; grp++) {
        dev_free(d_jobs[grp], stream);
        dev_free(d_order[grp][0], stream);
        dev_free(d_order[grp][1], stream);
        dev_free(d_torder[grp], stream);
        dev_free(d_off[grp], stream);
        dev_free(d_tasks[grp], stream);
        dev_free(d_dep[grp], stream);
    }
    (void)hipStreamSynchronize(stream);
    if (epoch_exec) (void)hipGraphExecDestroy(epoch_exec);
    (void)hipFree(ctl);
    (void)hipFree(lc);
    (void)hipFree(pctl);
    (void)hipHostFree(h_pctl);
    (void)hipHostFree(h_ctl);
    (void)hipFree(d_bad);
    (void)hipHostFree(h_bad);
    (void)hipFree(d_pc);
    (void)hipHostFree(h_pc);
    (void)hipHostFree(h_pause);
    (void)hipHostFree(h_stopped);
    (void)hipStreamDestroy(stream);
}

}  // namespace

sip_status sipk::make_backend(sip_server_config &cfg, std::unique_ptr<Backend> *out)
{
    auto be = std::make_unique<GpuBackend>();
    if (const sip_status e = be->init(cfg); e != SIP_OK) return e;
    *out = std::move(be);
    return SIP_OK;
}
