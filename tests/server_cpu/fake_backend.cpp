// CPU backend of the SIP server, for host-side tests of the scheduler
// (admission, budget, eviction, retirement, cancellation, shutdown) under
// ThreadSanitizer and AddressSanitizer.
//
// TEST INFRASTRUCTURE ONLY: it stands in for the GPU backend of the library
// (paper_1303_4538_amd/csrc/sip_server.hip) and runs every step with the
// oracle (oracle/sip_oracle.c) on the host.  A request's arrays (b, x, x0,
// the coefficients) are host arrays here.  Each request iterates from its own
// b and x alone: a step of epoch_iters iterations is one call of oracle_solve
// with that many iterations left, resumed from the x the previous step left,
// which is the same sequence of iterates as one call over the whole solve.
// Budget bytes follow the device layout's sizes (coefficients and factors per
// system; b, x and the sweep result per request).
#include "fake_backend.h"

#include "../../paper_1303_4538_amd/csrc/sip_host.h"
#include "../../paper_1303_4538_amd/csrc/sip_sched.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <vector>

extern "C" {
int oracle_factor(int ni, int nj, int nk, const double *A, double alpha, double *LU);
long oracle_solve(int ni, int nj, int nk, const double *A, const double *LU, const double *b, double *x,
                  double rtol, long max_iter, int mode, double *hist, double *rel_res);
}

namespace {

std::atomic<uint64_t> g_ticks{0}, g_steps{0}, g_psteps{0};
std::atomic<int64_t> g_live{0};
std::atomic<int> g_fail_sys{0}, g_fail_req{0};
std::atomic<bool> g_fail_step{false};
std::mutex g_gate_mu;
std::condition_variable g_gate_cv;
bool g_gate_closed = false, g_at_gate = false, g_until_quit = false;

bool take(std::atomic<int> &n)
{
    int v = n.load();
    while (v > 0)
        if (n.compare_exchange_weak(v, v - 1)) return true;
    return false;
}

struct FakeSystem final : sipk::Resident {
    int mode = 0;    // oracle mode: 0 FP64, 1 mixed, 2 all-FP32
    int fp32 = 0;
    int sym = 0;
    double alpha = 0.0;
    std::vector<double> A, LU;
    size_t held = 0;
    ~FakeSystem() override { g_live -= (int64_t)held; }
};

struct FakeReq final : sipk::Req {
    std::vector<double> b, x;
    long iters = 0;
    double rho = 0.0;
    bool stopped = false;
    sip_status st = SIP_OK;
    size_t held = 0;
    ~FakeReq() override { g_live -= (int64_t)held; }
};

FakeSystem *fsys(const sipk::Req *q) { return static_cast<FakeSystem *>(q->sys); }
size_t cells(const sip_problem &p) { return (size_t)p.ni * p.nj * p.nk; }

class FakeBackend final : public sipk::Backend {
public:
    explicit FakeBackend(const sip_server_config &c) : cfg(c) {}
    sip_server_config cfg;

    double now() override { return (double)g_ticks.load() * 1e-3; }
    sip_status check_problem(const sip_problem &p) override
    {
        if (cells(p) > ((size_t)1 << 24)) return sipk::set_error(SIP_EINVAL, "block too large");
        return SIP_OK;
    }
    size_t system_bytes(const sip_problem &p) override
    {
        return cells(p) * (7 * 8 + 7 * (p.precision != SIP_FP64 ? 4 : 8));
    }
    size_t request_bytes(const sip_problem &p, const sipk::Resident *res) override
    {
        const size_t n = res ? (size_t)res->ni * res->nj * res->nk : cells(p);
        const int fp32 = res ? static_cast<const FakeSystem *>(res)->fp32 : p.precision != SIP_FP64;
        return n * (2 * 8 + (fp32 ? 4 : 8));
    }
    sip_status new_request(const sip_request &, std::unique_ptr<sipk::Req> *out) override
    {
        *out = std::make_unique<FakeReq>();
        return SIP_OK;
    }
    sip_status new_system(const sipk::Req &q, std::unique_ptr<sipk::Resident> *out) override
    {
        if (take(g_fail_sys)) return sipk::set_error(SIP_ENOMEM, "injected system allocation failure");
        const sip_problem &p = q.r.problem;
        auto s = std::make_unique<FakeSystem>();
        s->mode = p.precision == SIP_FP64 ? 0 : p.precision == SIP_MIXED ? 1 : 2;
        s->fp32 = p.precision != SIP_FP64;
        s->sym = p.storage == SIP_STORAGE_SYMMETRIC;
        s->alpha = p.alpha;
        s->A.assign(7 * cells(p), 0.0);
        s->LU.assign(7 * cells(p), 0.0);
        s->held = system_bytes(p);
        g_live += (int64_t)s->held;
        *out = std::move(s);
        return SIP_OK;
    }
    void free_system(sipk::Resident *rs) override
    {
        auto *s = static_cast<FakeSystem *>(rs);
        s->A.clear();
        s->LU.clear();
    }
    sip_status alloc_request(sipk::Req *rq) override
    {
        if (take(g_fail_req)) return sipk::set_error(SIP_ENOMEM, "injected request allocation failure");
        auto *q = static_cast<FakeReq *>(rq);
        const size_t n = (size_t)q->sys->ni * q->sys->nj * q->sys->nk;
        q->b.assign(n, 0.0);
        q->x.assign(n, 0.0);
        q->held = request_bytes(q->r.problem, q->sys);
        g_live += (int64_t)q->held;
        return SIP_OK;
    }
    size_t release_request(sipk::Req *rq) override
    {
        auto *q = static_cast<FakeReq *>(rq);
        q->b.clear();
        q->x.clear();
        g_live -= (int64_t)q->held;
        q->held = 0;
        return q->bytes;
    }
    void wait_for_callers(const std::vector<sipk::Req *> &) override {}
    // copies the coefficients in and factorises; the symmetric storage needs
    // a symmetric A (each coupling equal to its mirror at the neighbour)
    void factor(const std::vector<sipk::Resident *> &sys, const std::vector<sipk::Req *> &owners,
                std::vector<sip_status> &result) override
    {
        for (size_t k = 0; k < sys.size(); k++) {
            auto *s = static_cast<FakeSystem *>(sys[k]);
            const sip_problem &p = owners[k]->r.problem;
            const size_t n = cells(p);
            for (int d = 0; d < 7; d++) std::memcpy(s->A.data() + d * n, p.a[d], n * sizeof(double));
            if (s->sym && !symmetric(p)) {
                result[k] = SIP_EINVAL;
                continue;
            }
            result[k] = oracle_factor(p.ni, p.nj, p.nk, s->A.data(), s->alpha, s->LU.data()) == 0 ? SIP_OK
                                                                                                  : SIP_EBREAKDOWN;
        }
    }
    void stage(std::vector<sipk::Req *> &ready) override
    {
        for (sipk::Req *rq : ready) {
            auto *q = static_cast<FakeReq *>(rq);
            std::memcpy(q->b.data(), q->r.b, q->b.size() * sizeof(double));
            if (q->r.x0) std::memcpy(q->x.data(), q->r.x0, q->x.size() * sizeof(double));
        }
    }
    sip_status step(std::vector<sipk::Req *> &act) override
    {
        {
            std::unique_lock<std::mutex> lk(g_gate_mu);
            if (g_gate_closed) {
                g_at_gate = true;
                g_gate_cv.notify_all();
                // the gate opens, or (gate_until_quit) the server shuts down
                while (g_gate_closed && !(g_until_quit && host->quitting()))
                    g_gate_cv.wait_for(lk, std::chrono::milliseconds(1));
                g_at_gate = false;
            }
        }
        g_steps++;
        host->count(sipk::STAT_EPOCHS, 1);
        if (g_fail_step.exchange(false)) return sipk::set_error(SIP_EDEVICE, "injected step failure");
        // persistent while nothing arrived since the last step: run until every
        // request stops or the scheduler has requests to admit (or quits)
        const bool persistent = !host->arrivals_since_last_step();
        g_psteps += persistent;
        for (int round = 0; round < (persistent ? 8 : 1); round++) {
            bool any = false;
            for (sipk::Req *rq : act) {
                auto *q = static_cast<FakeReq *>(rq);
                if (q->stopped) continue;
                advance(q);
                any = any || !q->stopped;
            }
            if (!any || host->admission_waiting() || host->quitting()) break;
        }
        return SIP_OK;
    }
    sipk::Outcome outcome(const sipk::Req *rq, sip_status st) override
    {
        const auto *q = static_cast<const FakeReq *>(rq);
        sipk::Outcome o;
        o.done = st != SIP_OK || q->stopped;
        o.status = st != SIP_OK ? st : q->st;
        o.iters = (int)q->iters;
        o.rho = q->rho;
        return o;
    }
    void retire(const std::vector<sipk::Req *> &fin, sip_status st) override
    {
        if (st != SIP_OK) return;
        for (sipk::Req *rq : fin) {
            auto *q = static_cast<FakeReq *>(rq);
            std::memcpy(q->r.x, q->x.data(), q->x.size() * sizeof(double));
        }
    }
    void drain() override {}

private:
    static bool symmetric(const sip_problem &p)
    {
        const int ni = p.ni, nj = p.nj, nk = p.nk;
        for (int k = 0; k < nk; k++)
            for (int j = 0; j < nj; j++)
                for (int i = 0; i < ni; i++) {
                    const size_t c = (size_t)i + (size_t)ni * ((size_t)j + (size_t)nj * k);
                    if (i + 1 < ni && p.a[2][c] != p.a[1][c + 1]) return false;
                    if (j + 1 < nj && p.a[4][c] != p.a[3][c + ni]) return false;
                    if (k + 1 < nk && p.a[6][c] != p.a[5][c + (size_t)ni * nj]) return false;
                }
        return true;
    }
    // epoch_iters iterations of q (fewer if its limit comes first)
    void advance(FakeReq *q)
    {
        const FakeSystem *s = fsys(q);
        const long left = std::max<long>(0, (long)q->r.max_iter - q->iters);
        const long chunk = std::min<long>(cfg.epoch_iters, left);
        double rho = 0.0;
        const long it = oracle_solve(s->ni, s->nj, s->nk, s->A.data(), s->LU.data(), q->b.data(), q->x.data(),
                                     q->r.rtol, chunk, s->mode, nullptr, &rho);
        if (it < 0) {
            q->stopped = true;
            q->st = SIP_ENOMEM;
            return;
        }
        q->iters += it;
        q->rho = rho;
        g_ticks += (uint64_t)std::max<long>(it, 1);
        if (rho <= q->r.rtol) {
            q->stopped = true;
            q->st = SIP_OK;
        } else if (q->iters >= q->r.max_iter) {
            q->stopped = true;
            q->st = SIP_ENOTCONV;
        }
    }
};

}  // namespace

sip_status sipk::make_backend(sip_server_config &cfg, std::unique_ptr<Backend> *out)
{
    if (cfg.hbm_budget_bytes == 0) cfg.hbm_budget_bytes = (size_t)1 << 30;
    *out = std::make_unique<FakeBackend>(cfg);
    return SIP_OK;
}

namespace fake {

uint64_t ticks() { return g_ticks.load(); }
void close_gate(bool until_quit)
{
    std::lock_guard<std::mutex> lk(g_gate_mu);
    g_gate_closed = true;
    g_until_quit = until_quit;
}
void open_gate()
{
    std::lock_guard<std::mutex> lk(g_gate_mu);
    g_gate_closed = false;
    g_until_quit = false;
    g_gate_cv.notify_all();
}
void wait_at_gate()
{
    std::unique_lock<std::mutex> lk(g_gate_mu);
    g_gate_cv.wait(lk, [] { return g_at_gate; });
}
void fail_system_allocs(int n) { g_fail_sys = n; }
void fail_request_allocs(int n) { g_fail_req = n; }
void fail_next_step() { g_fail_step = true; }
uint64_t steps() { return g_steps.load(); }
uint64_t persistent_steps() { return g_psteps.load(); }
int64_t live_bytes() { return g_live.load(); }

}  // namespace fake
