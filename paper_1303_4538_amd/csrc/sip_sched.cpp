// Request scheduler of the SIP server and the server half of the C ABI
// (sip_server_* / sip_batch_* in include/sip.h).
//
//   - a request names a system by id; the first request of an id brings the
//     system in (the backend copies and factorises the coefficients), later
//     requests reuse the resident factors (Sec. 4.1: the factorisation is
//     computed once, in advance, and reused);
//   - admission is by a device-memory budget (resident systems + running
//     requests), first fit in submission order; when space is needed,
//     resident systems that no running or queued request names are evicted,
//     least-recently-used first (a system stays resident after its last
//     request only if a request asked to retain it);
//   - between steps, stopped requests retire (x written to the caller's
//     array) and queued requests are admitted (continuous batching);
//   - shutdown ends the scheduler thread after its current step and cancels
//     what is queued or running.
// The device work of a step is the backend's (sip_sched.h).
#include "sip_host.h"
#include "sip_sched.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

using namespace sipk;

struct sip_server_s final : Host {
    sip_server_config cfg{};
    std::unique_ptr<Backend> be;
    std::thread thread;
    std::once_flag stop_once;   // sip_server_shutdown / sip_server_destroy stop the thread once
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool quit = false;
    uint64_t next_ticket = 1;
    uint64_t tickets_at_step = 0;   // next_ticket at the last arrivals_since_last_step
    std::deque<Req *> queue;
    std::vector<Req *> running;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    std::unordered_map<uint64_t, std::unique_ptr<Resident>> systems;
    std::unordered_map<uint64_t, int> queued_ids;   // system id -> queued requests naming it
    std::vector<int> free_slots;
    size_t used = 0, peak = 0;
    uint64_t clock = 0;
    std::atomic<uint64_t> stats[SIP_SERVER_NSTATS] = {};

    // Host
    bool arrivals_since_last_step() override
    {
        std::lock_guard<std::mutex> lk(mu);
        const bool any = next_ticket != tickets_at_step;
        tickets_at_step = next_ticket;
        return any;
    }
    bool admission_waiting() override
    {
        std::lock_guard<std::mutex> lk(mu);
        return !queue.empty() && (int)running.size() < cfg.max_slots;
    }
    bool quitting() override
    {
        std::lock_guard<std::mutex> lk(mu);
        return quit;
    }
    void count(ServerStat st, uint64_t n) override { stats[st].fetch_add(n, std::memory_order_relaxed); }

    void loop();
    bool admit_locked(std::vector<Req *> &admitted, std::vector<Resident *> &to_factor);
    bool make_room_locked(size_t need);
    void dequeue_locked(Req *q);
    void free_resident_locked(Resident *s);
    void finish_locked(Req *q, sip_status st, int iters, double rho);
    sip_status submit(const sip_request *r, uint64_t *ticket);
    void stop();
};

void sip_server_s::free_resident_locked(Resident *s)
{
    be->free_system(s);
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
        count(STAT_EVICTIONS, 1);
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
        const size_t need_slot = be->request_bytes(pb, s);
        const size_t need_sys = s ? 0 : be->system_bytes(pb);
        if (s) s->refs++;   // pin while making room
        const bool fits = make_room_locked(need_slot + need_sys);
        if (s) s->refs--;
        if (!fits) {
            ++it;           // first fit: a smaller request behind may still fit
            continue;
        }
        sip_status fail = SIP_OK;
        if (!s) {
            bool ok = pb.alpha >= 0.0 && pb.alpha <= 1.0;
            for (int d = 0; d < 7; d++) ok = ok && pb.a[d] != nullptr;
            std::unique_ptr<Resident> rs;
            if (!ok) {   // a request that must factorise needs its coefficients
                fail = SIP_EINVAL;
            } else if (be->new_system(*q, &rs) != SIP_OK) {
                fail = SIP_ENOMEM;
            } else {
                rs->id = q->r.system_id;
                rs->ni = pb.ni;
                rs->nj = pb.nj;
                rs->nk = pb.nk;
                rs->bytes = need_sys;
                used += need_sys;
                s = rs.get();
                systems[rs->id] = std::move(rs);
                to_factor.push_back(s);
                q->factorised = 1;
            }
        }
        if (fail == SIP_OK) {
            q->sys = s;
            s->refs++;
            s->retain = s->retain || q->r.retain;
            s->last_use = ++clock;
            if (be->alloc_request(q) != SIP_OK) {   // finish_locked drops the reference
                fail = SIP_ENOMEM;
                if (q->factorised) {   // the system it brought in goes with it
                    to_factor.pop_back();
                    s->broken = SIP_ENOMEM;
                    q->factorised = 0;
                }
            }
        }
        if (fail != SIP_OK) {
            finish_locked(q, fail, 0, 0.0);
            dequeue_locked(q);
            it = queue.erase(it);
            continue;
        }
        q->bytes = need_slot;
        used += need_slot;
        peak = std::max(peak, used);
        q->slot = free_slots.back();
        free_slots.pop_back();
        q->state = 1;
        q->t_admit = be->now();
        admitted.push_back(q);
        count(STAT_ADMITTED, 1);
        dequeue_locked(q);
        it = queue.erase(it);
        any = true;
    }
    return any;
}

void sip_server_s::finish_locked(Req *q, sip_status st, int iters, double rho)
{
    q->state = 2;
    q->t_done = be->now();
    q->res.status = st;
    q->res.info.iters = iters;
    q->res.info.rel_res = rho;
    q->res.info.seconds = q->t_done - q->t_submit;
    q->res.t_submit = q->t_submit;
    q->res.t_admit = q->t_admit;
    q->res.t_done = q->t_done;
    q->res.factorised = q->factorised;
    used -= be->release_request(q);
    q->bytes = 0;
    if (q->slot >= 0) {
        free_slots.push_back(q->slot);
        q->slot = -1;
    }
    if (q->sys) {
        Resident *s = q->sys;
        q->sys = nullptr;
        s->refs--;
        s->last_use = ++clock;
        if (s->refs == 0 && (!s->retain || s->broken != SIP_OK)) free_resident_locked(s);
    }
    count(STAT_COMPLETED, 1);
    cv_done.notify_all();
}

void sip_server_s::loop()
{
    be->thread_start();
    for (;;) {
        std::vector<Req *> admitted;
        std::vector<Resident *> to_factor;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return quit || !queue.empty() || !running.empty(); });
            if (quit) break;
            admit_locked(admitted, to_factor);
        }
        be->wait_for_callers(admitted);
        // factorise new systems (owners = the admitted request that brought each in)
        if (!to_factor.empty()) {
            std::vector<Req *> owners;
            for (Resident *s : to_factor)
                for (Req *q : admitted)
                    if (q->sys == s) {
                        owners.push_back(q);
                        break;
                    }
            std::vector<sip_status> result(to_factor.size(), SIP_OK);
            be->factor(to_factor, owners, result);
            count(STAT_FACTORISATIONS, to_factor.size());
            std::lock_guard<std::mutex> lk(mu);
            for (size_t k = 0; k < to_factor.size(); k++) {
                to_factor[k]->factored = result[k] == SIP_OK;
                to_factor[k]->broken = result[k];
            }
        }
        // stage b and x0 of newly admitted requests; fail those whose system broke down
        std::vector<Req *> ready;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (Req *q : admitted) {
                if (q->sys->broken != SIP_OK) {
                    finish_locked(q, q->sys->broken, 0, 0.0);
                    continue;
                }
                ready.push_back(q);
            }
        }
        be->stage(ready);
        std::vector<Req *> act;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (Req *q : ready) running.push_back(q);
            act = running;
        }
        if (act.empty()) continue;
        const sip_status st = be->step(act);
        // retire stopped requests: x written out, then reported done
        std::vector<Req *> fin;
        std::vector<Outcome> outs;
        for (Req *q : act) {
            const Outcome o = be->outcome(q, st);
            if (!o.done) continue;
            fin.push_back(q);
            outs.push_back(o);
        }
        if (!fin.empty()) be->retire(fin, st);
        std::lock_guard<std::mutex> lk(mu);
        for (size_t k = 0; k < fin.size(); k++) {
            finish_locked(fin[k], outs[k].status, outs[k].iters, outs[k].rho);
            running.erase(std::find(running.begin(), running.end(), fin[k]));
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

sip_status sip_server_s::submit(const sip_request *r, uint64_t *ticket)
{
    if (!r->b || !r->x) return set_error(SIP_EINVAL, "b and x are required");
    if (!(r->rtol > 0.0) || r->max_iter < 0) return set_error(SIP_EINVAL, "need rtol > 0 and max_iter >= 0");
    const sip_problem &p = r->problem;
    // ordering after the caller's work on its stream, taken before the lock
    // (the request object is destroyed with it if the request is refused)
    std::unique_ptr<Req> q;
    if (const sip_status e = be->new_request(*r, &q); e != SIP_OK) return e;
    std::lock_guard<std::mutex> lk(mu);
    if (quit) return set_error(SIP_ECANCELLED, "the server is shut down");
    auto f = systems.find(r->system_id);
    const Resident *res = f != systems.end() ? f->second.get() : nullptr;
    if (!res && !queued_ids.count(r->system_id)) {   // this request may have to bring the system in
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
    if (res && (p.ni != res->ni || p.nj != res->nj || p.nk != res->nk))
        return set_error(SIP_EINVAL, "dims differ from the resident system");
    if (!res)
        if (const sip_status e = be->check_problem(p); e != SIP_OK) return e;
    const size_t need = be->request_bytes(p, res) + (res ? 0 : be->system_bytes(p));
    if (need > cfg.hbm_budget_bytes)
        return set_error(SIP_ENOMEM, "request needs %zu bytes, budget %zu", need, (size_t)cfg.hbm_budget_bytes);
    if ((int)queue.size() >= cfg.max_queue) return set_error(SIP_EBUSY, "queue full");
    q->ticket = next_ticket++;
    q->r = *r;
    q->t_submit = be->now();
    *ticket = q->ticket;
    queued_ids[r->system_id]++;
    queue.push_back(q.get());
    reqs[q->ticket] = std::move(q);
    cv_work.notify_one();
    return SIP_OK;
}

// Ends the scheduler thread after its current step; it cancels what is not
// done.  Afterwards the backend touches no request's arrays.
void sip_server_s::stop()
{
    std::call_once(stop_once, [this] {
        {
            std::lock_guard<std::mutex> lk(mu);
            quit = true;
        }
        cv_work.notify_all();
        if (thread.joinable()) thread.join();
        be->drain();
    });
}

extern "C" {

sip_status sip_server_create(const sip_server_config *c, sip_server *out)
{
    if (!c || !out) return set_error(SIP_EINVAL, "NULL argument");
    if (c->max_slots < 1 || c->max_slots > SERVER_MAX_SLOTS || c->epoch_iters < 1 || c->max_queue < 1)
        return set_error(SIP_EINVAL, "bad server configuration");
    auto s = std::make_unique<sip_server_s>();
    s->cfg = *c;
    if (const sip_status e = make_backend(s->cfg, &s->be); e != SIP_OK) return e;
    s->be->host = s.get();
    for (int k = s->cfg.max_slots - 1; k >= 0; k--) s->free_slots.push_back(k);
    sip_server_s *p = s.release();
    p->thread = std::thread([p] { p->loop(); });
    *out = p;
    return SIP_OK;
}

sip_status sip_batch_submit(sip_server s, const sip_request *r, uint64_t *ticket)
{
    if (!s || !r || !ticket) return set_error(SIP_EINVAL, "NULL argument");
    return s->submit(r, ticket);
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
    for (int k = 0; k < SIP_SERVER_NSTATS; k++) out[k] = s->stats[k].load(std::memory_order_relaxed);
    out[STAT_RESIDENT_BYTES] = s->used;
    out[STAT_PEAK_BYTES] = s->peak;
    return SIP_OK;
}

sip_status sip_server_shutdown(sip_server s)
{
    if (!s) return set_error(SIP_EINVAL, "NULL argument");
    s->stop();
    return SIP_OK;
}

sip_status sip_server_destroy(sip_server s)
{
    if (!s) return set_error(SIP_EINVAL, "NULL argument");
    s->stop();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        std::vector<Resident *> all;
        for (auto &kv : s->systems) all.push_back(kv.second.get());
        for (Resident *r : all) s->free_resident_locked(r);
    }
    s->be.reset();
    delete s;
    return SIP_OK;
}

}  // extern "C"
