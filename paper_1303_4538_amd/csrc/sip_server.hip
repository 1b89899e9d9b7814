// Batched and served SIP solves (sip_server_* / sip_batch_* in include/sip.h).
//
// The paper's redesigned solver owns its coefficients and reuses one
// factorisation "for all iterations and time steps" (Sec. 4.1); a server
// generalises that to many blocks and many right-hand sides on one GPU:
//   - a request names a system by id; the first request of an id copies and
//     factorises the coefficients, later requests reuse the resident factors;
//   - admission is by an HBM budget (resident systems + per-request state);
//     when space is needed, resident systems that no running or queued
//     request names are evicted, least-recently-used first (a system stays
//     resident after its last request only if a request asked to retain it);
//   - a request's arrays (coefficients, b, x0) are read on the server's
//     stream only after an event recorded on the caller's stream at submit;
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
//     SIP_SERVER_PERSISTENT=1 / 0 forces one mode;
//   - between launches converged requests retire (x copied to the caller's
//     array) and queued requests are admitted (continuous batching).
// Every request's arithmetic depends only on its own data and tile order, so
// a result is the same alone and in any mix.
#include "sip_internal.h"
#include "sip_runtime.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace sipk;

namespace {

constexpr int MAX_SLOTS = 4096;
constexpr int MAX_PAIRS = 1024;   // pairs of requests swept together

struct Resident {
    uint64_t id = 0;
    Geom g{};
    int fp32 = 0;          // factors stored in FP32
    int arith = 0;         // sweep arithmetic (sip_precision)
    double alpha = 0.92;
    double *A = nullptr;
    void *LU = nullptr;
    size_t bytes = 0;
    int refs = 0;
    bool factored = false;
    bool retain = false;
    bool broken = false;
    int sym = 0;           // sweeps read the symmetric coefficient storage
    bool asym = false;     // symmetric storage requested for a non-symmetric A
    uint64_t last_use = 0;
};

struct Req;

// Two requests of one resident system swept together (FP32 factors): b and x
// of both interleaved, their own face words and three control blocks (the
// sweep's, one per request).  Each request stops at its own tolerance; the
// pair's buffers go when both have.
struct Pair {
    Req *r[2] = {nullptr, nullptr};
    Resident *sys = nullptr;
    int idx = -1;             // control blocks pctl[3 idx .. 3 idx + 2]
    double *bx = nullptr;     // b pairs, then x pairs
    void *y = nullptr;
    uint64_t *face = nullptr;
    double *part = nullptr;
    bool done[2] = {false, false};
    size_t held = 0;          // budget bytes of a finished member, released with the pair
};

struct Req {
    uint64_t ticket = 0;
    sip_request r{};
    double t_submit = 0, t_admit = 0, t_done = 0;
    int state = 0;   // 0 queued, 1 running, 2 done
    sip_result res{};
    // running state
    Resident *sys = nullptr;
    int slot = -1;
    double *bx = nullptr;
    void *y = nullptr;
    uint64_t *face = nullptr;
    double *part = nullptr;
    double *hist = nullptr;
    size_t bytes = 0;
    bool fresh = true;       // b / x0 not staged yet
    int factorised = 0;
    Pair *pair = nullptr;    // swept together with another request
    int pm = 0;              // which of the pair
    hipEvent_t ready = nullptr;   // recorded on the caller's stream at submit
};

size_t slot_bytes(const Geom &g, int fp32, int max_iter)
{
    const size_t E = (size_t)g.elems;
    (void)max_iter;   // served requests keep no residual history
    return E * (2 * 8 + (fp32 ? 4 : 8)) + (size_t)g.ntiles * g.steps * FACE_WORDS * 8 + (size_t)g.ntiles * 16;
}

size_t resident_bytes(const Geom &g, int fp32) { return (size_t)g.elems * (7 * 8 + 7 * (fp32 ? 4 : 8)); }

}  // namespace

struct sip_server_s {
    sip_server_config cfg{};
    int device = 0;
    int num_cu = 256;   // compute units of the device
    hipStream_t stream = nullptr;
    uint64_t timeout_ticks = 0;
    uint32_t torture = 0;   // schedule_seed() at creation: a new random order every launch group
    std::chrono::steady_clock::time_point t0;
    std::thread thread;
    std::once_flag stop_once;   // sip_server_shutdown / sip_server_destroy stop the thread once
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool quit = false;
    uint64_t next_ticket = 1;
    std::deque<Req *> queue;
    std::vector<Req *> running;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    std::unordered_map<uint64_t, std::unique_ptr<Resident>> systems;
    std::unordered_map<uint64_t, int> queued_ids;   // system id -> queued requests naming it
    size_t used = 0, peak = 0;
    uint64_t clock = 0;
    // factorisations, evictions, epochs, resident, peak, completed, admitted, launches, pairs formed,
    // epochs replayed from a graph
    uint64_t stats[SIP_SERVER_NSTATS] = {0};
    // The sweeps of an epoch as a captured graph.  Its kernels read the job
    // list and ticket orders from device buffers uploaded before every epoch,
    // so the graph stays valid while the launch parameters (buffer addresses,
    // tile counts, plans, epoch length) stay the same; it is captured the
    // second time in a row the same parameters come up and replayed from then on.
    hipGraphExec_t epoch_exec = nullptr;
    std::vector<uint64_t> epoch_key;
    bool graphs = true;   // SIP_SERVER_GRAPHS=0 launches every epoch eagerly
    // race testing: a different random ticket order for every launch group
    uint32_t order_seed(int grp) const
    {
        return torture ? (torture + 7919u * (uint32_t)stats[2] + 104729u * (uint32_t)grp) | 1u : 0u;
    }
    // device-side scratch for launches
    Ctl *ctl = nullptr;                      // MAX_SLOTS control blocks
    Ctl *h_ctl = nullptr;                    // pinned mirror
    std::vector<int> free_slots;
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
    uint64_t tickets_at_launch = 0;           // next_ticket when the last launch was decided
    int *d_torder[2 * NARITH] = {};
    int *d_off[2 * NARITH] = {};
    Task *d_tasks[2 * NARITH] = {};
    int torder_cap[2 * NARITH] = {}, off_cap[2 * NARITH] = {}, tasks_cap[2 * NARITH] = {};
    PersistCtl *d_pc = nullptr, *h_pc = nullptr;
    uint32_t *h_pause = nullptr, *h_stopped = nullptr;   // coherent host memory, read / written by the device
    uint32_t *d_pause = nullptr, *d_stopped = nullptr;   // their device addresses
    // forward then backward tile order of a block of nti x ntj tiles (the
    // default order depends on nothing else)
    std::map<std::pair<int, int>, std::vector<int>> tile_orders;
    SweepPlan plan{};
    bool plan_forced = false;   // SIP_SWEEP_PHASES set: no tuned plans

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
    void loop();
    bool admit_locked(std::vector<Req *> &admitted, std::vector<Resident *> &to_factor);
    bool make_room_locked(size_t need);
    void dequeue_locked(Req *q);
    void free_resident_locked(Resident *s);
    void finish_locked(Req *q, sip_status st, int iters, double rho);
    sip_status run_factor(const std::vector<Resident *> &sys, const std::vector<Req *> &owners);
    sip_status run_epoch(std::vector<Req *> &act);
    sip_status run_persist(int grp, const std::vector<Job> &jobs, const std::vector<Geom> &gs, const SweepPlan &gp,
                           bool others_waiting);
    bool want_pause(double since_launch, bool others_waiting);
    void form_pairs(std::vector<Req *> &ready);
    void free_pair(Pair *p);
    sip_status ensure_launch_buffers(int grp, int njobs, int ntiles);
};

namespace {

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

}  // namespace

void sip_server_s::free_resident_locked(Resident *s)
{
    dev_free(s->A, stream);
    dev_free(s->LU, stream);
    used -= s->bytes;
    systems.erase(s->id);
}

void sip_server_s::dequeue_locked(Req *q)
{
    auto f = queued_ids.find(q->r.system_id);
    if (f != queued_ids.end() && --f->second == 0) queued_ids.erase(f);
}

// Evicts unreferenced systems, least-recently-used first, until `need` more
// bytes fit.  A system that a queued request names is kept: that request may
// carry no coefficients and could not be served once its factors are gone.
bool sip_server_s::make_room_locked(size_t need)
{
    while (used + need > cfg.hbm_budget_bytes) {
        Resident *victim = nullptr;
        for (auto &kv : systems) {
            Resident *s = kv.second.get();
            if (s->refs != 0 || queued_ids.count(s->id)) continue;
            if (!victim || s->last_use < victim->last_use) victim = s;
        }
        if (!victim) return false;
        free_resident_locked(victim);
        stats[1]++;
    }
    return true;
}

bool sip_server_s::admit_locked(std::vector<Req *> &admitted, std::vector<Resident *> &to_factor)
{
    bool any = false;
    for (auto it = queue.begin(); it != queue.end();) {
        Req *q = *it;
        if ((int)running.size() + (int)admitted.size() >= cfg.max_slots || free_slots.empty()) break;
        const sip_problem &pb = q->r.problem;
        Resident *s = nullptr;
        auto f = systems.find(q->r.system_id);
        if (f != systems.end()) s = f->second.get();
        const Geom g = s ? s->g : make_geom(pb.ni, pb.nj, pb.nk);
        const int arith = s ? s->arith : pb.precision;
        const int fp32 = arith != SIP_FP64;
        const size_t need_slot = slot_bytes(g, fp32, q->r.max_iter);
        const size_t need_sys = s ? 0 : resident_bytes(g, fp32);
        if (s) s->refs++;   // pin while making room
        const bool fits = make_room_locked(need_slot + need_sys);
        if (s) s->refs--;
        if (!fits) {
            ++it;           // first fit: a smaller request behind may still fit
            continue;
        }
        if (!s) {
            bool ok = pb.ni == g.ni && pb.alpha >= 0.0 && pb.alpha <= 1.0;
            for (int d = 0; d < 7; d++) ok = ok && pb.a[d] != nullptr;
            if (!ok) {   // a request that must factorise needs its coefficients
                finish_locked(q, SIP_EINVAL, 0, 0.0);
                dequeue_locked(q);
            it = queue.erase(it);
                continue;
            }
            auto rs = std::make_unique<Resident>();
            rs->id = q->r.system_id;
            rs->g = g;
            rs->fp32 = fp32;
            rs->arith = arith;
            rs->alpha = pb.alpha;
            rs->sym = pb.storage == SIP_STORAGE_SYMMETRIC;
            rs->bytes = need_sys;
            if (dev_alloc((void **)&rs->A, 7 * (size_t)g.elems * 8, stream) != SIP_OK ||
                dev_alloc(&rs->LU, 7 * (size_t)g.elems * (fp32 ? 4 : 8), stream) != SIP_OK) {
                dev_free(rs->A, stream);
                dev_free(rs->LU, stream);
                finish_locked(q, SIP_ENOMEM, 0, 0.0);
                dequeue_locked(q);
            it = queue.erase(it);
                continue;
            }
            used += need_sys;
            s = rs.get();
            systems[rs->id] = std::move(rs);
            to_factor.push_back(s);
            q->factorised = 1;
        }
        q->sys = s;
        s->refs++;
        s->retain = s->retain || q->r.retain;
        s->last_use = ++clock;
        q->bytes = need_slot;
        const size_t E = (size_t)g.elems;
        if (dev_alloc((void **)&q->bx, 2 * E * 8, stream) != SIP_OK ||
            dev_alloc(&q->y, E * (fp32 ? 4 : 8), stream) != SIP_OK ||
            dev_alloc((void **)&q->face, (size_t)g.ntiles * g.steps * FACE_WORDS * 8, stream) != SIP_OK ||
            dev_alloc((void **)&q->part, (size_t)g.ntiles * 16, stream) != SIP_OK) {
            dev_free(q->bx, stream);
            dev_free(q->y, stream);
            dev_free(q->face, stream);
            dev_free(q->part, stream);
            dev_free(q->hist, stream);
            q->bx = nullptr;
            q->y = nullptr;
            q->face = nullptr;
            q->part = nullptr;
            q->hist = nullptr;
            s->refs--;
            finish_locked(q, SIP_ENOMEM, 0, 0.0);
            dequeue_locked(q);
            it = queue.erase(it);
            continue;
        }
        (void)hipMemsetAsync(q->face, 0, (size_t)g.ntiles * g.steps * FACE_WORDS * 8, stream);
        used += need_slot;
        peak = std::max(peak, used);
        q->slot = free_slots.back();
        free_slots.pop_back();
        q->state = 1;
        q->t_admit = now();
        admitted.push_back(q);
        stats[6]++;
        dequeue_locked(q);
        it = queue.erase(it);
        any = true;
    }
    return any;
}

void sip_server_s::finish_locked(Req *q, sip_status st, int iters, double rho)
{
    q->state = 2;
    q->t_done = now();
    q->res.status = st;
    q->res.info.iters = iters;
    q->res.info.rel_res = rho;
    q->res.info.seconds = q->t_done - q->t_submit;
    q->res.t_submit = q->t_submit;
    q->res.t_admit = q->t_admit;
    q->res.t_done = q->t_done;
    q->res.factorised = q->factorised;
    dev_free(q->bx, stream);
    dev_free(q->y, stream);
    dev_free(q->face, stream);
    dev_free(q->part, stream);
    dev_free(q->hist, stream);
    q->bx = nullptr;
    q->y = nullptr;
    q->face = nullptr;
    q->part = nullptr;
    q->hist = nullptr;
    if (q->ready) {   // the server stream's wait on it, if any, is already enqueued
        (void)hipEventDestroy(q->ready);
        q->ready = nullptr;
    }
    if (Pair *p = q->pair) {
        // the pair's buffers stand for both members' budget bytes: they are
        // released when the second member is done
        p->done[q->pm] = true;
        p->held += q->bytes;
        q->bytes = 0;
        q->pair = nullptr;
        if (p->done[0] && p->done[1]) {
            used -= p->held;
            free_pair(p);
        }
    }
    if (q->slot >= 0) {
        free_slots.push_back(q->slot);
        q->slot = -1;
        used -= q->bytes;
    }
    if (q->sys) {
        Resident *s = q->sys;
        q->sys = nullptr;
        s->refs--;
        s->last_use = ++clock;
        if (s->refs == 0 && (!s->retain || s->broken)) free_resident_locked(s);
    }
    stats[5]++;
    cv_done.notify_all();
}

void sip_server_s::free_pair(Pair *p)
{
    dev_free(p->bx, stream);
    dev_free(p->y, stream);
    dev_free(p->face, stream);
    dev_free(p->part, stream);
    free_pairs.push_back(p->idx);
    pairs.erase(std::find(pairs.begin(), pairs.end(), p));
    delete p;
}

// x pairs behind the b pairs, in the precision of the sweeps
static void *pair_x(const Pair *p)
{
    const size_t E = (size_t)p->sys->g.elems;
    return p->sys->arith == ARITH_F32 ? (void *)((float *)p->bx + 2 * E) : (void *)(p->bx + 2 * E);
}

// Pairs freshly admitted requests of one resident system (FP32 factors, the
// same rtol and max_iter, start vectors both given or both zero): they share
// one pass of the sweeps over A and the factors.  The pair's buffers replace
// the members' own, inside the budget the members were admitted with.
void sip_server_s::form_pairs(std::vector<Req *> &ready)
{
    if (!pairing) return;
    std::vector<Req *> open;
    for (Req *q : ready) {
        const Resident *rs = q->sys;
        if (rs->arith != ARITH_MIXED && rs->arith != ARITH_F32) continue;
        Req *mate = nullptr;
        for (Req *o : open)
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
        p->sys = q->sys;
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
            Req *r = p->r[m];
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
        stats[8]++;
    }
}

sip_status sip_server_s::ensure_launch_buffers(int grp, int njobs, int ntiles)
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

// x behind b in the request's buffer, in the precision of the sweeps
static void *x_of(const Resident *s, const Req *q)
{
    return s->arith == ARITH_F32 ? (void *)((float *)q->bx + s->g.elems) : (void *)(q->bx + s->g.elems);
}

static Job job_of(const Resident *s, const Req *q, Ctl *ctl, int fw)
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
    J.hist = q->hist;
    J.ctl = ctl + q->slot;
    J.alpha = s->alpha;
    J.fw = fw;
    J.sym = fw == FACE_WORDS ? 0 : s->sym;   // the factorisation reads the full coefficients
    return J;
}

// Factorise newly resident systems, all of them in one batched launch per
// precision; each uses the face words of the request that brought it in.
sip_status sip_server_s::run_factor(const std::vector<Resident *> &sys, const std::vector<Req *> &owners)
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
                    sys[k]->asym = true;
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
            if (sys[k]->fp32 != grp || sys[k]->asym) continue;
            const int sc = sys[k]->sym ? SHEAR_SYM : sys[k]->arith == ARITH_F32 ? SHEAR_COEF32 : SHEAR_COEF;
            if (sc != SHEAR_COEF &&
                launch_to_sheared(sys[k]->g, 7, owners[k]->r.problem.a, sys[k]->A, sys[k]->g.elems, sc, stream) !=
                    hipSuccess)
                return set_error(SIP_EDEVICE, "reorder failed");
        }
        // the host copies of jobs/orders must live until the copies ran
        if (hipStreamSynchronize(stream) != hipSuccess) return set_error(SIP_EDEVICE, "factorisation failed");
        stats[7]++;
    }
    stats[0] += sys.size();
    return SIP_OK;
}

// One epoch: epoch_iters (forward, backward) pairs over every running request.
sip_status sip_server_s::run_epoch(std::vector<Req *> &act)
{
    const Range range("server epoch");
    // groups 0..NARITH-1: single requests by arithmetic; NARITH + arith: pairs
    constexpr int NG = 2 * NARITH;
    std::vector<Job> jobs[NG];
    std::vector<Geom> gs[NG];
    for (Req *q : act) {
        if (q->pair) continue;
        const int grp = q->sys->arith;
        jobs[grp].push_back(job_of(q->sys, q, ctl, FACE_WORDS_SWEEP));
        gs[grp].push_back(q->sys->g);
    }
    for (Pair *p : pairs) {
        const Resident *rs = p->sys;
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
    bool use_persistent = persistent == 1;
    if (persistent < 0) {
        std::lock_guard<std::mutex> lk(mu);
        use_persistent = next_ticket == tickets_at_launch;   // nothing submitted since the last launch
        tickets_at_launch = next_ticket;
    }
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
        stats[2]++;
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
        key.insert(key.end(), {1, (uint64_t)gplan[grp].phases, (uint64_t)(uintptr_t)fa[grp].jobs,
                               (uint64_t)(uintptr_t)fa[grp].order, (uint64_t)(uintptr_t)ba[grp].order,
                               (uint64_t)(uintptr_t)fa[grp].lc, (uint64_t)fa[grp].total, (uint64_t)ba[grp].total,
                               fa[grp].timeout_ticks, (uint64_t)fa[grp].jitter});
        stats[7] += 2 * (uint64_t)cfg.epoch_iters;
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
        stats[9]++;
    } else if (!launch_all()) {
        return set_error(SIP_EDEVICE, "sweep launch failed");
    }
    if (hipMemcpyAsync(h_ctl, ctl, sizeof(Ctl) * MAX_SLOTS, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        (!pairs.empty() &&
         hipMemcpyAsync(h_pctl, pctl, sizeof(Ctl) * 3 * MAX_PAIRS, hipMemcpyDeviceToHost, stream) != hipSuccess) ||
        hipStreamSynchronize(stream) != hipSuccess)
        return set_error(SIP_EDEVICE, "epoch failed: %s", hipGetErrorString(hipGetLastError()));
    stats[2]++;
    return SIP_OK;
}

// Whether the running persistent launch should let its requests pause: new
// requests wait for admission (after a short minimum run, so that a queue that
// cannot be admitted yet does not restart the launch over and over), a request
// has stopped and waits to be retired, another launch group waits for its
// turn, or the server is shutting down.
bool sip_server_s::want_pause(double since_launch, bool others_waiting)
{
    // a pause drains the launch (every request finishes its iteration), so it
    // is asked for no more often than these intervals
    constexpr double ADMIT = 10e-3, RETIRE = 20e-3, SLICE = 20e-3;
    if (since_launch >= RETIRE && __atomic_load_n(h_stopped, __ATOMIC_ACQUIRE)) return true;
    if (others_waiting && since_launch >= SLICE) return true;
    std::lock_guard<std::mutex> lk(mu);
    if (quit) return true;
    return since_launch >= ADMIT && !queue.empty() && (int)running.size() < cfg.max_slots;
}

// One persistent launch for the jobs of launch group grp: every job starts at
// its next forward sweep (an iteration boundary) and runs until it stops or
// the host asks for a pause.
sip_status sip_server_s::run_persist(int grp, const std::vector<Job> &jobs, const std::vector<Geom> &gs,
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
    // the first forward sweeps, merged over the jobs (topological per job)
    const std::vector<int2> first = topo_order(gs, false, order_seed(grp));
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
        !grow((void **)&d_tasks[grp], tasks_cap[grp], (int)cap, sizeof(Task)))
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
        hipMemcpyAsync(d_pc, h_pc, sizeof(PersistCtl), hipMemcpyHostToDevice, stream) != hipSuccess)
        return set_error(SIP_EDEVICE, "upload failed");
    const PersistArgs pa{d_jobs[grp], d_torder[grp], d_off[grp], d_tasks[grp], cap, d_pc, d_pause, d_stopped,
                         timeout_ticks, torture};
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
    stats[7]++;
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

void sip_server_s::loop()
{
    (void)hipSetDevice(device);
    for (;;) {
        std::vector<Req *> admitted;
        std::vector<Resident *> to_factor;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return quit || !queue.empty() || !running.empty(); });
            if (quit) break;
            admit_locked(admitted, to_factor);
        }
        // the coefficients, b and x0 were produced on the caller's stream:
        // everything below that reads them runs after that stream's work
        for (Req *q : admitted)
            if (q->ready) (void)hipStreamWaitEvent(stream, q->ready, 0);
        // factorise new systems (owners = the admitted request that brought each in)
        if (!to_factor.empty()) {
            std::vector<Req *> owners;
            for (Resident *s : to_factor)
                for (Req *q : admitted)
                    if (q->sys == s) {
                        owners.push_back(q);
                        break;
                    }
            const sip_status st = run_factor(to_factor, owners);
            (void)hipMemcpyAsync(h_ctl, ctl, sizeof(Ctl) * MAX_SLOTS, hipMemcpyDeviceToHost, stream);
            (void)hipStreamSynchronize(stream);
            std::lock_guard<std::mutex> lk(mu);
            for (size_t k = 0; k < to_factor.size(); k++) {
                const uint32_t stop = st == SIP_OK ? h_ctl[owners[k]->slot].stop : TIMEOUT;
                if (stop == RUN && !to_factor[k]->asym) {
                    to_factor[k]->factored = true;
                } else {
                    to_factor[k]->broken = true;
                }
            }
        }
        // stage b and x0 of newly admitted requests; fail those whose system broke down
        std::vector<Req *> ready;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (Req *q : admitted) {
                if (q->sys->broken) {
                    finish_locked(q, q->sys->asym ? SIP_EINVAL : SIP_EBREAKDOWN, 0, 0.0);
                    continue;
                }
                ready.push_back(q);
            }
        }
        form_pairs(ready);
        for (Req *q : ready) {
            if (q->pair) continue;   // staged with its partner
            const Geom &g = q->sys->g;
            const double *src[2] = {q->r.b, q->r.x0 ? q->r.x0 : nullptr};
            const bool f32 = q->sys->arith == ARITH_F32;   // the relaxation starts from FP32 copies
            const int sh = f32 ? SHEAR_F32 : SHEAR_F64;
            if (q->r.x0) {
                (void)launch_to_sheared(g, 2, src, q->bx, g.elems, sh, stream);
            } else {
                (void)launch_to_sheared(g, 1, src, q->bx, g.elems, sh, stream);
                (void)hipMemsetAsync(x_of(q->sys, q), 0, (size_t)g.elems * (f32 ? 4 : 8), stream);
            }
            (void)launch_init_ctl(ctl + q->slot, 1, (uint32_t)q->r.max_iter, q->r.rtol, 0, stream);
        }
        std::vector<Req *> act;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (Req *q : ready) running.push_back(q);
            act = running;
        }
        if (act.empty()) continue;
        const sip_status st = run_epoch(act);
        // retire finished requests: copy x out, then report them done
        std::vector<Req *> fin;
        for (Req *q : act) {
            if (Pair *p = q->pair) {
                const Ctl &c = h_pctl[3 * p->idx + 1 + q->pm];
                const uint32_t js = h_pctl[3 * p->idx].stop;
                if (st != SIP_OK || c.stop != RUN || js == BREAKDOWN || js == TIMEOUT) {
                    if (st == SIP_OK)
                        (void)launch_from_sheared(q->sys->g, pair_x(p), q->sys->arith == ARITH_F32, q->r.x,
                                                  pctl + 3 * p->idx + 1 + q->pm, stream, 2, q->pm);
                    fin.push_back(q);
                }
                continue;
            }
            const Ctl &c = h_ctl[q->slot];
            if (st != SIP_OK || c.stop != RUN) {
                if (st == SIP_OK)
                    (void)launch_from_sheared(q->sys->g, x_of(q->sys, q), q->sys->arith == ARITH_F32, q->r.x,
                                              ctl + q->slot, stream);
                fin.push_back(q);
            }
        }
        if (!fin.empty()) (void)hipStreamSynchronize(stream);
        std::lock_guard<std::mutex> lk(mu);
        for (Req *q : fin) {
            Ctl c = h_ctl[q->slot];
            if (const Pair *p = q->pair) {
                c = h_pctl[3 * p->idx + 1 + q->pm];
                const uint32_t js = h_pctl[3 * p->idx].stop;
                if (js == BREAKDOWN || js == TIMEOUT) c.stop = js;
                if (c.stop == ZERO_RHS) c.rho = 0.0;
            }
            sip_status rs = SIP_OK;
            if (st != SIP_OK) rs = st;
            else if (c.stop == MAXITER) rs = SIP_ENOTCONV;
            else if (c.stop == BREAKDOWN || c.stop == DIVERGED) rs = SIP_EBREAKDOWN;
            else if (c.stop == BAD_INPUT) rs = SIP_EINVAL;   // non-finite b, x0 or A x0
            else if (c.stop == TIMEOUT) rs = SIP_EDEVICE;
            finish_locked(q, rs, (int)c.iter, c.rho);
            running.erase(std::find(running.begin(), running.end(), q));
        }
    }
    // cancel everything still queued or running
    std::lock_guard<std::mutex> lk(mu);
    for (Req *q : queue) finish_locked(q, SIP_ECANCELLED, 0, 0.0);
    queue.clear();
    queued_ids.clear();
    for (Req *q : running) finish_locked(q, SIP_ECANCELLED, 0, 0.0);
    running.clear();
}

extern "C" {

sip_status sip_server_create(const sip_server_config *c, sip_server *out)
{
    if (!c || !out) return set_error(SIP_EINVAL, "NULL argument");
    if (c->max_slots < 1 || c->max_slots > MAX_SLOTS || c->epoch_iters < 1 || c->max_queue < 1)
        return set_error(SIP_EINVAL, "bad server configuration");
    auto *s = new sip_server_s();
    s->cfg = *c;
    if (const hipError_t e = hipGetDevice(&s->device); e != hipSuccess) {
        delete s;
        return set_error(SIP_EDEVICE, "no HIP device: hipGetDevice: %s", hipGetErrorString(e));
    }
    if (s->cfg.hbm_budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = (size_t)8 << 30;
        s->cfg.hbm_budget_bytes = fr / 4 * 3;
    }
    if (const char *e = getenv("SIP_SWEEP_PHASES")) {
        const int nl = atoi(e);
        if (nl >= 1 && nl <= sipk::MAX_PHASES) {
            s->plan.phases = nl;
            s->plan_forced = true;
        }
    }
    if (const char *e = getenv("SIP_POLL_DISTANCE")) {
        const int pd = atoi(e);
        if (pd >= 1 && pd <= sipk::MAX_POLL) {
            s->plan.poll = pd;
            s->plan_forced = true;
        }
    }
    if (const char *e = getenv("SIP_SERVER_PAIRS")) s->pairing = atoi(e) != 0;
    if (const char *e = getenv("SIP_SERVER_GRAPHS")) s->graphs = atoi(e) != 0;
    if (const char *e = getenv("SIP_SERVER_PERSISTENT")) s->persistent = atoi(e) != 0 ? 1 : 0;
    s->timeout_ticks = timeout_ticks_for(s->device, 2.0);
    s->torture = schedule_seed();
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, s->device) == hipSuccess && ncu > 0)
            s->num_cu = ncu;
    }
    s->t0 = std::chrono::steady_clock::now();
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc((void **)&s->ctl, sizeof(Ctl) * MAX_SLOTS) != hipSuccess ||
        hipHostMalloc((void **)&s->h_ctl, sizeof(Ctl) * MAX_SLOTS, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&s->lc, sizeof(LaunchCtl)) != hipSuccess ||
        hipMalloc((void **)&s->pctl, sizeof(Ctl) * 3 * MAX_PAIRS) != hipSuccess ||
        hipHostMalloc((void **)&s->h_pctl, sizeof(Ctl) * 3 * MAX_PAIRS, hipHostMallocDefault) != hipSuccess ||
        hipMemsetAsync(s->pctl, 0, sizeof(Ctl) * 3 * MAX_PAIRS, s->stream) != hipSuccess ||
        launch_init_ctl(s->pctl, 3 * MAX_PAIRS, 0, 0.0, 1, s->stream) != hipSuccess ||
        hipMalloc((void **)&s->d_bad, sizeof(unsigned)) != hipSuccess ||
        hipHostMalloc((void **)&s->h_bad, sizeof(unsigned), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&s->d_pc, sizeof(PersistCtl)) != hipSuccess ||
        hipHostMalloc((void **)&s->h_pc, sizeof(PersistCtl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&s->h_pause, sizeof(uint32_t), hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc((void **)&s->h_stopped, sizeof(uint32_t), hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer((void **)&s->d_pause, s->h_pause, 0) != hipSuccess ||
        hipHostGetDevicePointer((void **)&s->d_stopped, s->h_stopped, 0) != hipSuccess ||
        // on the server's own stream, in order: the stream does not synchronise
        // with the legacy default stream, so a plain hipMemset could land after
        // the initialisation and reset the epochs to 0, which the zeroed face
        // words of a fresh request would then match
        hipMemsetAsync(s->ctl, 0, sizeof(Ctl) * MAX_SLOTS, s->stream) != hipSuccess ||
        hipMemsetAsync(s->lc, 0, sizeof(LaunchCtl), s->stream) != hipSuccess ||
        launch_init_ctl(s->ctl, MAX_SLOTS, 0, 0.0, 1, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return set_error(SIP_ENOMEM, "server buffers");
    }
    for (int k = MAX_SLOTS - 1; k >= 0; k--) s->free_slots.push_back(k);
    for (int k = MAX_PAIRS - 1; k >= 0; k--) s->free_pairs.push_back(k);
    s->thread = std::thread([s] { s->loop(); });
    *out = s;
    return SIP_OK;
}

sip_status sip_batch_submit(sip_server s, const sip_request *r, uint64_t *ticket)
{
    if (!s || !r || !ticket) return set_error(SIP_EINVAL, "NULL argument");
    if (!r->b || !r->x) return set_error(SIP_EINVAL, "b and x are required");
    if (!(r->rtol > 0.0) || r->max_iter < 0) return set_error(SIP_EINVAL, "need rtol > 0 and max_iter >= 0");
    const sip_problem &p = r->problem;
    // orders the server's reads of the request's arrays after the caller's
    // work on its stream (the event is destroyed when the request finishes)
    hipEvent_t ready = nullptr;
    if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(ready, (hipStream_t)r->stream) != hipSuccess) {
        if (ready) (void)hipEventDestroy(ready);
        (void)hipGetLastError();
        return set_error(SIP_EDEVICE, "could not record the ordering event on the caller's stream");
    }
    struct EventGuard {   // destroys the event unless the request takes it
        hipEvent_t e;
        ~EventGuard() { if (e) (void)hipEventDestroy(e); }
    } guard{ready};
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->quit) return set_error(SIP_ECANCELLED, "the server is shut down");
    auto f = s->systems.find(r->system_id);
    const bool resident = f != s->systems.end();
    bool queued_same = false;
    for (Req *q : s->queue) queued_same = queued_same || q->r.system_id == r->system_id;
    if (!resident && !queued_same) {
        if (p.ni < 1 || p.nj < 1 || p.nk < 1) return set_error(SIP_EINVAL, "dims must be >= 1");
        if (!(p.alpha >= 0.0 && p.alpha <= 1.0)) return set_error(SIP_EINVAL, "alpha must be in [0, 1]");
        if (p.precision != SIP_FP64 && p.precision != SIP_MIXED && p.precision != SIP_FP32)
            return set_error(SIP_EINVAL, "unknown precision");
        if (p.storage != SIP_STORAGE_FULL && p.storage != SIP_STORAGE_SYMMETRIC)
            return set_error(SIP_EINVAL, "unknown storage");
        if (p.storage == SIP_STORAGE_SYMMETRIC && p.precision == SIP_FP32)
            return set_error(SIP_EINVAL, "the symmetric storage is available with SIP_FP64 and SIP_MIXED only");
        for (int d = 0; d < 7; d++)
            if (!p.a[d]) return set_error(SIP_EINVAL, "coefficient pointer %d is NULL", d);
    }
    const Geom g = resident ? f->second->g : make_geom(p.ni, p.nj, p.nk);
    if (g.elems >= sipk::MAX_ELEMS) return set_error(SIP_EINVAL, "block too large");
    if (resident && (p.ni != g.ni || p.nj != g.nj || p.nk != g.nk))
        return set_error(SIP_EINVAL, "dims differ from the resident system");
    const int fp32 = resident ? f->second->fp32 : p.precision != SIP_FP64;
    const size_t need = slot_bytes(g, fp32, r->max_iter) + (resident ? 0 : resident_bytes(g, fp32));
    if (need > s->cfg.hbm_budget_bytes) return set_error(SIP_ENOMEM, "request needs %zu bytes, budget %zu", need, s->cfg.hbm_budget_bytes);
    if ((int)s->queue.size() >= s->cfg.max_queue) return set_error(SIP_EBUSY, "queue full");
    auto q = std::make_unique<Req>();
    q->ticket = s->next_ticket++;
    q->r = *r;
    q->t_submit = s->now();
    q->ready = ready;
    guard.e = nullptr;
    *ticket = q->ticket;
    s->queued_ids[r->system_id]++;
    s->queue.push_back(q.get());
    s->reqs[q->ticket] = std::move(q);
    s->cv_work.notify_one();
    return SIP_OK;
}

sip_status sip_batch_poll(sip_server s, uint64_t ticket, int32_t wait_ms, sip_result *out)
{
    if (!s || !out) return set_error(SIP_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(SIP_EINVAL, "unknown ticket");
    Req *q = it->second.get();
    auto done = [&] { return q->state == 2; };
    if (!done()) {
        if (wait_ms < 0) s->cv_done.wait(lk, done);
        else if (wait_ms > 0) s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), done);
    }
    if (!done()) return SIP_PENDING;
    *out = q->res;
    s->reqs.erase(it);
    return SIP_OK;
}

sip_status sip_server_release(sip_server s, uint64_t system_id)
{
    if (!s) return set_error(SIP_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto f = s->systems.find(system_id);
    if (f == s->systems.end()) return SIP_OK;
    f->second->retain = false;
    if (f->second->refs == 0) s->free_resident_locked(f->second.get());
    return SIP_OK;
}

sip_status sip_server_stats(sip_server s, uint64_t out[SIP_SERVER_NSTATS])
{
    if (!s || !out) return set_error(SIP_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    s->stats[3] = s->used;
    s->stats[4] = s->peak;
    std::memcpy(out, s->stats, sizeof s->stats);
    return SIP_OK;
}

// Ends the scheduler thread after its current step; it cancels what is not
// done.  Afterwards no kernel of the server touches a request's arrays.
static void stop_server(sip_server s)
{
    std::call_once(s->stop_once, [s] {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->quit = true;
        }
        s->cv_work.notify_all();
        if (s->thread.joinable()) s->thread.join();
        (void)hipStreamSynchronize(s->stream);
    });
}

sip_status sip_server_shutdown(sip_server s)
{
    if (!s) return set_error(SIP_EINVAL, "NULL argument");
    stop_server(s);
    return SIP_OK;
}

sip_status sip_server_destroy(sip_server s)
{
    if (!s) return set_error(SIP_EINVAL, "NULL argument");
    stop_server(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        std::vector<Resident *> all;
        for (auto &kv : s->systems) all.push_back(kv.second.get());
        for (Resident *r : all) s->free_resident_locked(r);
    }
    for (int grp = 0; grp < 2 * NARITH; grp++) {
        dev_free(s->d_jobs[grp], s->stream);
        dev_free(s->d_order[grp][0], s->stream);
        dev_free(s->d_order[grp][1], s->stream);
        dev_free(s->d_torder[grp], s->stream);
        dev_free(s->d_off[grp], s->stream);
        dev_free(s->d_tasks[grp], s->stream);
    }
    (void)hipStreamSynchronize(s->stream);
    if (s->epoch_exec) (void)hipGraphExecDestroy(s->epoch_exec);
    (void)hipFree(s->ctl);
    (void)hipFree(s->lc);
    (void)hipFree(s->pctl);
    (void)hipHostFree(s->h_pctl);
    (void)hipHostFree(s->h_ctl);
    (void)hipFree(s->d_bad);
    (void)hipHostFree(s->h_bad);
    (void)hipFree(s->d_pc);
    (void)hipHostFree(s->h_pc);
    (void)hipHostFree(s->h_pause);
    (void)hipHostFree(s->h_stopped);
    (void)hipStreamDestroy(s->stream);
    delete s;
    return SIP_OK;
}

}  // extern "C"
