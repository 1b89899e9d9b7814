// Host-side scenarios of the SIP server's scheduler, run through the C ABI
// (include/sip.h) over the CPU test backend (fake_backend.cpp), built with
// ThreadSanitizer or AddressSanitizer by tests/test_server_cpu.py.
//
// Every solved request is compared with its own oracle solve (oracle_factor,
// then oracle_solve from its x0 with its rtol and max_iter): x bitwise, the
// iteration count and the relative residual exactly, the status SIP_OK when
// the residual reached rtol and SIP_ENOTCONV otherwise.  The scenarios cover
// admission under the budget (first fit), least-recently-used eviction, the
// protection of systems that queued requests name, the queue limit, argument
// errors, factorisation failures, allocation failures, a failed step,
// cancellation at shutdown, and many threads submitting, polling, releasing
// and reading the counters at once.
//
// usage: server_driver [scenario ...]   (no argument: all)
#include "fake_backend.h"

#include "../../include/sip.h"

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

extern "C" {
int oracle_factor(int ni, int nj, int nk, const double *A, double alpha, double *LU);
long oracle_solve(int ni, int nj, int nk, const double *A, const double *LU, const double *b, double *x,
                  double rtol, long max_iter, int mode, double *hist, double *rel_res);
}

namespace {

#define CHECK(cond)                                                                                     \
    do {                                                                                                \
        if (!(cond)) {                                                                                  \
            std::fprintf(stderr, "CHECK failed %s:%d: %s (last error: %s)\n", __FILE__, __LINE__, #cond, \
                         sip_last_error());                                                             \
            std::fflush(stderr);                                                                        \
            std::exit(1);                                                                               \
        }                                                                                               \
    } while (0)

// A block with a 7-point operator: diffusion with random positive
// conductances (symmetric) plus, unless symmetric, a random upwind
// convection term; A_P is the sum of the couplings' magnitudes plus a shift.
struct Sys {
    uint64_t id = 0;
    int ni = 0, nj = 0, nk = 0;
    int precision = SIP_FP64;
    int storage = SIP_STORAGE_FULL;
    double alpha = 0.92;
    std::vector<double> A;
    size_t n() const { return (size_t)ni * nj * nk; }
    sip_problem problem(bool with_coefficients) const
    {
        sip_problem p{};
        p.ni = ni;
        p.nj = nj;
        p.nk = nk;
        for (int d = 0; d < 7; d++) p.a[d] = with_coefficients ? A.data() + d * n() : nullptr;
        p.alpha = alpha;
        p.precision = precision;
        p.storage = storage;
        return p;
    }
};

Sys make_sys(uint64_t id, int ni, int nj, int nk, int precision, bool symmetric, uint64_t seed)
{
    Sys s;
    s.id = id;
    s.ni = ni;
    s.nj = nj;
    s.nk = nk;
    s.precision = precision;
    s.storage = symmetric ? SIP_STORAGE_SYMMETRIC : SIP_STORAGE_FULL;
    const size_t n = s.n();
    s.A.assign(7 * n, 0.0);
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> u(0.5, 1.5), c(-0.3, 0.3);
    auto at = [&](int i, int j, int k) { return (size_t)i + (size_t)ni * ((size_t)j + (size_t)nj * k); };
    // conductance of the face between a cell and its E / N / T neighbour
    std::vector<double> gx(n), gy(n), gz(n);
    for (size_t p = 0; p < n; p++) {
        gx[p] = u(rng);
        gy[p] = u(rng);
        gz[p] = u(rng);
    }
    for (int k = 0; k < nk; k++)
        for (int j = 0; j < nj; j++)
            for (int i = 0; i < ni; i++) {
                const size_t p = at(i, j, k);
                const double vx = symmetric ? 0.0 : c(rng), vy = symmetric ? 0.0 : c(rng), vz = symmetric ? 0.0 : c(rng);
                double *a = s.A.data();
                if (i > 0) a[1 * n + p] = -gx[at(i - 1, j, k)] - std::max(vx, 0.0);
                if (i + 1 < ni) a[2 * n + p] = -gx[p] + std::min(vx, 0.0);
                if (j > 0) a[3 * n + p] = -gy[at(i, j - 1, k)] - std::max(vy, 0.0);
                if (j + 1 < nj) a[4 * n + p] = -gy[p] + std::min(vy, 0.0);
                if (k > 0) a[5 * n + p] = -gz[at(i, j, k - 1)] - std::max(vz, 0.0);
                if (k + 1 < nk) a[6 * n + p] = -gz[p] + std::min(vz, 0.0);
                double diag = 0.1;
                for (int d = 1; d < 7; d++) diag += std::fabs(a[d * n + p]);
                a[p] = diag;
            }
    return s;
}

std::vector<double> random_vec(size_t n, uint64_t seed)
{
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    std::vector<double> v(n);
    for (double &x : v) x = u(rng);
    return v;
}

// One request with its own arrays, and what the oracle says it must return.
struct Job {
    const Sys *sys = nullptr;
    std::vector<double> b, x0, x;
    bool has_x0 = false, coefficients = true;
    bool refused = false;
    double rtol = 1e-8;
    int max_iter = 200;
    int retain = 0;
    uint64_t ticket = 0;
    sip_result res{};
    // the oracle's answer
    sip_status want = SIP_OK;
    long want_iters = 0;
    double want_rho = 0.0;
    std::vector<double> want_x;

    sip_request request()
    {
        sip_request r{};
        r.system_id = sys->id;
        r.problem = sys->problem(coefficients);
        r.b = b.data();
        r.x = x.data();
        r.x0 = has_x0 ? x0.data() : nullptr;
        r.rtol = rtol;
        r.max_iter = max_iter;
        r.retain = retain;
        r.stream = nullptr;
        return r;
    }
};

int oracle_mode(int precision) { return precision == SIP_FP64 ? 0 : precision == SIP_MIXED ? 1 : 2; }

void expect(Job &j)
{
    const Sys &s = *j.sys;
    std::vector<double> LU(7 * s.n());
    if (oracle_factor(s.ni, s.nj, s.nk, s.A.data(), s.alpha, LU.data()) != 0) {
        j.want = SIP_EBREAKDOWN;
        return;
    }
    j.want_x = j.has_x0 ? j.x0 : std::vector<double>(s.n(), 0.0);
    double rho = 0.0;
    j.want_iters = oracle_solve(s.ni, s.nj, s.nk, s.A.data(), LU.data(), j.b.data(), j.want_x.data(), j.rtol,
                                j.max_iter, oracle_mode(s.precision), nullptr, &rho);
    j.want_rho = rho;
    j.want = rho <= j.rtol ? SIP_OK : SIP_ENOTCONV;
}

Job make_job(const Sys &s, uint64_t seed, double rtol, int max_iter, bool x0, int retain = 0)
{
    Job j;
    j.sys = &s;
    j.b = random_vec(s.n(), seed);
    j.has_x0 = x0;
    if (x0) j.x0 = random_vec(s.n(), seed + 1);
    j.x.assign(s.n(), 7.0);   // sentinel: written only when the request is done
    j.rtol = rtol;
    j.max_iter = max_iter;
    j.retain = retain;
    expect(j);
    return j;
}

void check_solved(const Job &j)
{
    if (j.res.status != j.want || j.res.info.iters != j.want_iters || j.res.info.rel_res != j.want_rho ||
        j.x != j.want_x) {
        std::fprintf(stderr, "request on system %llu: status %s (want %s), iters %d (want %ld), rho %.17g (want %.17g), x %s\n",
                     (unsigned long long)j.sys->id, sip_status_str(j.res.status), sip_status_str(j.want),
                     j.res.info.iters, j.want_iters, j.res.info.rel_res, j.want_rho,
                     j.x == j.want_x ? "equal" : "differs");
        std::exit(1);
    }
    CHECK(j.res.t_submit <= j.res.t_admit && j.res.t_admit <= j.res.t_done);
}

void check_untouched(const Job &j)
{
    for (double v : j.x) CHECK(v == 7.0);
}

sip_server make_server(size_t budget, int max_slots = 64, int epoch_iters = 8, int max_queue = 1024)
{
    sip_server_config c{};
    c.hbm_budget_bytes = budget;
    c.max_slots = max_slots;
    c.epoch_iters = epoch_iters;
    c.max_queue = max_queue;
    sip_server s = nullptr;
    CHECK(sip_server_create(&c, &s) == SIP_OK && s);
    return s;
}

void submit(sip_server s, Job &j)
{
    const sip_request r = j.request();
    CHECK(sip_batch_submit(s, &r, &j.ticket) == SIP_OK);
}

void wait(sip_server s, Job &j) { CHECK(sip_batch_poll(s, j.ticket, -1, &j.res) == SIP_OK); }

void run(sip_server s, Job &j)
{
    submit(s, j);
    wait(s, j);
}

std::vector<uint64_t> stats(sip_server s)
{
    std::vector<uint64_t> v(SIP_SERVER_NSTATS);
    CHECK(sip_server_stats(s, v.data()) == SIP_OK);
    return v;
}
enum { FACT = 0, EVICT = 1, RESIDENT = 3, PEAK = 4, DONE = 5, ADMITTED = 6 };

size_t sys_bytes(const Sys &s) { return s.n() * (56 + (s.precision != SIP_FP64 ? 28 : 56)); }
size_t req_bytes(const Sys &s) { return s.n() * (16 + (s.precision != SIP_FP64 ? 4 : 8)); }

void destroy(sip_server s)
{
    CHECK(sip_server_destroy(s) == SIP_OK);
    CHECK(fake::live_bytes() == 0);
}

// ------------------------------------------------------------------ scenarios

// Requests on six systems (every arithmetic, both storages) from four threads
// at once; every result is the oracle's.
void results_concurrent()
{
    std::vector<Sys> sys;
    const int prec[3] = {SIP_FP64, SIP_MIXED, SIP_FP32};
    for (int k = 0; k < 6; k++)
        sys.push_back(make_sys(100 + k, 5 + k, 4 + (k % 3), 3 + (k % 2), prec[k % 3], k == 3 || k == 4, 11 + k));
    sip_server s = make_server(0, 5, 4);
    std::vector<std::vector<Job>> jobs(4);
    for (int t = 0; t < 4; t++)
        for (int m = 0; m < 12; m++) {
            const Sys &y = sys[(t * 5 + m) % 6];
            const double rtol = y.precision == SIP_FP32 ? 1e-4 : (m % 3 == 0 ? 1e-6 : 1e-9);
            jobs[t].push_back(make_job(y, 1000 * t + m, rtol, m % 4 == 0 ? 6 : 300, m % 2 == 1, m % 3 == 1));
        }
    std::atomic<bool> done{false};
    std::thread watcher([&] {   // the budget holds at every moment the counters are read
        while (!done) {
            const auto v = stats(s);
            CHECK(v[PEAK] >= v[RESIDENT]);
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
    });
    std::vector<std::thread> th;
    for (int t = 0; t < 4; t++)
        th.emplace_back([&, t] {
            for (Job &j : jobs[t]) submit(s, j);
            for (Job &j : jobs[t]) {
                if (t % 2) {   // poll without waiting, then wait
                    sip_status st;
                    while ((st = sip_batch_poll(s, j.ticket, 0, &j.res)) == SIP_PENDING) std::this_thread::yield();
                    CHECK(st == SIP_OK);
                } else {
                    wait(s, j);
                }
            }
        });
    for (auto &t : th) t.join();
    done = true;
    watcher.join();
    for (auto &v : jobs)
        for (Job &j : v) check_solved(j);
    const auto v = stats(s);
    CHECK(v[DONE] == 48 && v[ADMITTED] == 48);
    CHECK(v[FACT] >= 6);
    destroy(s);
}

// Budget for two systems and one request: the least recently used
// unreferenced system goes first; an evicted system needs its coefficients
// again, a resident one does not.
void lru_eviction()
{
    const Sys a = make_sys(1, 7, 6, 5, SIP_FP64, false, 1), b = make_sys(2, 7, 6, 5, SIP_FP64, false, 2),
              c = make_sys(3, 7, 6, 5, SIP_FP64, false, 3);
    const size_t budget = 2 * sys_bytes(a) + req_bytes(a) + 64;
    sip_server s = make_server(budget);
    Job j1 = make_job(a, 1, 1e-8, 300, false, 1), j2 = make_job(b, 2, 1e-8, 300, false, 1);
    run(s, j1);
    run(s, j2);
    check_solved(j1);
    check_solved(j2);
    CHECK(j1.res.factorised == 1 && j2.res.factorised == 1);
    CHECK(stats(s)[RESIDENT] == 2 * sys_bytes(a));
    Job j3 = make_job(a, 3, 1e-8, 300, true);
    j3.coefficients = false;   // a is resident
    run(s, j3);
    check_solved(j3);
    CHECK(j3.res.factorised == 0);
    Job j4 = make_job(c, 4, 1e-8, 300, false, 1);   // needs room: b is the least recently used
    run(s, j4);
    check_solved(j4);
    CHECK(stats(s)[EVICT] == 1);
    Job j5 = make_job(b, 5, 1e-8, 300, false);
    j5.coefficients = false;   // b was evicted: refused at submit
    const sip_request r5 = j5.request();
    CHECK(sip_batch_submit(s, &r5, &j5.ticket) == SIP_EINVAL);
    Job j6 = make_job(a, 6, 1e-8, 300, false);
    j6.coefficients = false;   // a stayed
    run(s, j6);
    check_solved(j6);
    CHECK(j6.res.factorised == 0);
    CHECK(sip_server_release(s, 1) == SIP_OK);
    CHECK(stats(s)[RESIDENT] == sys_bytes(c));
    CHECK(stats(s)[PEAK] <= budget);
    destroy(s);
}

// A resident system that a queued request names is not evicted for another
// request queued before it: that one waits, first fit admits the later one.
void queued_protection()
{
    const Sys a = make_sys(1, 8, 6, 4, SIP_MIXED, false, 4), b = make_sys(2, 8, 6, 4, SIP_MIXED, false, 5);
    const size_t budget = sys_bytes(a) + req_bytes(a) + 64;
    sip_server s = make_server(budget);
    Job j0 = make_job(a, 1, 1e-8, 300, false, 1);
    run(s, j0);
    check_solved(j0);
    fake::close_gate();
    Job l = make_job(a, 2, 1e-8, 3, false);   // stops at its limit in one step
    l.coefficients = false;
    submit(s, l);
    fake::wait_at_gate();
    Job jb = make_job(b, 3, 1e-8, 300, false), ja = make_job(a, 4, 1e-8, 300, true);
    ja.coefficients = false;
    submit(s, jb);
    submit(s, ja);
    fake::open_gate();
    wait(s, l);
    wait(s, jb);
    wait(s, ja);
    check_solved(l);
    check_solved(ja);
    check_solved(jb);
    CHECK(ja.res.factorised == 0 && jb.res.factorised == 1);
    CHECK(ja.res.t_admit <= jb.res.t_admit);
    CHECK(stats(s)[EVICT] == 1);
    CHECK(stats(s)[PEAK] <= budget);
    destroy(s);
}

// First fit: a large request that does not fit waits while a small one
// behind it is admitted and finishes.
void first_fit()
{
    const Sys big1 = make_sys(1, 10, 9, 8, SIP_FP64, false, 6), big2 = make_sys(2, 10, 9, 8, SIP_FP64, false, 7),
              small = make_sys(3, 4, 3, 3, SIP_FP64, false, 8);
    const size_t budget = sys_bytes(big1) + req_bytes(big1) + sys_bytes(small) + req_bytes(small) + 64;
    sip_server s = make_server(budget, 64, 2);
    Job l = make_job(big1, 1, 1e-13, 40, false);
    fake::close_gate();
    submit(s, l);
    fake::wait_at_gate();
    Job jb = make_job(big2, 2, 1e-8, 300, false), js = make_job(small, 3, 1e-8, 300, false);
    submit(s, jb);
    submit(s, js);
    fake::open_gate();
    wait(s, l);
    wait(s, jb);
    wait(s, js);
    check_solved(l);
    check_solved(jb);
    check_solved(js);
    CHECK(js.res.t_admit < jb.res.t_admit);
    CHECK(l.res.t_done <= jb.res.t_admit);
    CHECK(stats(s)[PEAK] <= budget);
    destroy(s);
}

// The queue limit, then every queued request still completes.
void queue_full()
{
    const Sys a = make_sys(1, 6, 5, 4, SIP_FP64, false, 9);
    sip_server s = make_server(0, 1, 8, 3);
    fake::close_gate();
    Job l = make_job(a, 1, 1e-8, 300, false, 1);
    submit(s, l);
    fake::wait_at_gate();
    std::vector<Job> q;
    for (int k = 0; k < 4; k++) q.push_back(make_job(a, 10 + k, 1e-8, 300, k % 2 == 0));
    for (int k = 0; k < 3; k++) submit(s, q[k]);
    sip_request r = q[3].request();
    uint64_t t = 0;
    CHECK(sip_batch_submit(s, &r, &t) == SIP_EBUSY);
    fake::open_gate();
    wait(s, l);
    check_solved(l);
    for (int k = 0; k < 3; k++) {
        wait(s, q[k]);
        check_solved(q[k]);
    }
    destroy(s);
}

// Argument and configuration errors.
void invalid_arguments()
{
    sip_server_config c{};
    c.max_slots = 0;
    c.epoch_iters = 8;
    c.max_queue = 8;
    sip_server s = nullptr;
    CHECK(sip_server_create(&c, &s) == SIP_EINVAL);
    c.max_slots = 4097;
    CHECK(sip_server_create(&c, &s) == SIP_EINVAL);
    c.max_slots = 4;
    c.epoch_iters = 0;
    CHECK(sip_server_create(&c, &s) == SIP_EINVAL);
    c.epoch_iters = 8;
    c.max_queue = 0;
    CHECK(sip_server_create(&c, &s) == SIP_EINVAL);
    CHECK(sip_server_create(nullptr, &s) == SIP_EINVAL);
    const Sys a = make_sys(1, 6, 5, 4, SIP_FP64, false, 10);
    const size_t budget = sys_bytes(a) + req_bytes(a);
    s = make_server(budget);
    Job j = make_job(a, 1, 1e-8, 300, false, 1);
    uint64_t t = 0;
    auto refused = [&](std::function<void(sip_request &)> edit, sip_status want) {
        sip_request r = j.request();
        edit(r);
        CHECK(sip_batch_submit(s, &r, &t) == want);
    };
    refused([](sip_request &r) { r.problem.ni = 0; }, SIP_EINVAL);
    refused([](sip_request &r) { r.problem.alpha = 1.5; }, SIP_EINVAL);
    refused([](sip_request &r) { r.problem.precision = 7; }, SIP_EINVAL);
    refused([](sip_request &r) { r.problem.storage = 5; }, SIP_EINVAL);
    refused([](sip_request &r) {
        r.problem.storage = SIP_STORAGE_SYMMETRIC;
        r.problem.precision = SIP_FP32;
    }, SIP_EINVAL);
    refused([](sip_request &r) { r.b = nullptr; }, SIP_EINVAL);
    refused([](sip_request &r) { r.x = nullptr; }, SIP_EINVAL);
    refused([](sip_request &r) { r.rtol = 0.0; }, SIP_EINVAL);
    refused([](sip_request &r) { r.max_iter = -1; }, SIP_EINVAL);
    refused([](sip_request &r) { r.problem.a[4] = nullptr; }, SIP_EINVAL);
    refused([](sip_request &r) { r.problem.ni = 9; }, SIP_ENOMEM);   // more than the budget
    refused([](sip_request &r) {
        r.problem.ni = 1 << 12;
        r.problem.nj = 1 << 12;
        r.problem.nk = 2;
    }, SIP_EINVAL);   // beyond the backend's block limit
    CHECK(sip_batch_submit(nullptr, nullptr, &t) == SIP_EINVAL);
    run(s, j);
    check_solved(j);
    refused([](sip_request &r) { r.problem.nk = 3; }, SIP_EINVAL);   // differs from the resident system
    sip_result res{};
    CHECK(sip_batch_poll(s, j.ticket, 0, &res) == SIP_EINVAL);   // collected already
    CHECK(sip_batch_poll(s, 12345, 0, &res) == SIP_EINVAL);
    CHECK(sip_server_release(s, 999) == SIP_OK);
    CHECK(sip_server_stats(s, nullptr) == SIP_EINVAL);
    destroy(s);
}

// A factorisation that breaks down, and a symmetric-storage request whose A
// is not symmetric: their requests fail, the systems are not kept even when
// retained, and a second request queued on the broken system fails too.
void factorisation_failures()
{
    Sys bad = make_sys(1, 5, 4, 3, SIP_FP64, false, 11);
    bad.A[0] = 0.0;   // zero pivot at the first cell
    for (int d = 1; d < 7; d++) bad.A[d * bad.n()] = 0.0;
    Sys asym = make_sys(2, 5, 4, 3, SIP_MIXED, false, 12);
    asym.storage = SIP_STORAGE_SYMMETRIC;
    const Sys good = make_sys(3, 5, 4, 3, SIP_MIXED, true, 13);
    sip_server s = make_server(0);
    fake::close_gate();
    Job l = make_job(good, 1, 1e-8, 300, false, 1);
    submit(s, l);
    fake::wait_at_gate();
    Job jb1 = make_job(bad, 2, 1e-8, 300, false, 1), jb2 = make_job(bad, 3, 1e-8, 300, true, 1);
    Job ja = make_job(asym, 4, 1e-8, 300, false, 1);
    submit(s, jb1);
    submit(s, jb2);
    submit(s, ja);
    fake::open_gate();
    for (Job *j : {&l, &jb1, &jb2, &ja}) wait(s, *j);
    check_solved(l);
    CHECK(jb1.want == SIP_EBREAKDOWN);
    CHECK(jb1.res.status == SIP_EBREAKDOWN && jb2.res.status == SIP_EBREAKDOWN);
    CHECK(ja.res.status == SIP_EINVAL);
    for (Job *j : {&jb1, &jb2, &ja}) check_untouched(*j);
    CHECK(stats(s)[RESIDENT] == sys_bytes(good));   // only the good system stays
    destroy(s);
}

// Injected allocation failures: the request fails with SIP_ENOMEM, a system
// it brought in does not stay resident, and the reference counts stay right
// (a released system goes at once).
void allocation_failures()
{
    const Sys a = make_sys(1, 6, 5, 4, SIP_FP64, false, 14), b = make_sys(2, 6, 5, 4, SIP_FP64, false, 15);
    sip_server s = make_server(0);
    fake::fail_system_allocs(1);
    Job j1 = make_job(a, 1, 1e-8, 300, false, 1);
    run(s, j1);
    CHECK(j1.res.status == SIP_ENOMEM && j1.res.factorised == 0);
    check_untouched(j1);
    CHECK(stats(s)[RESIDENT] == 0);
    fake::fail_request_allocs(1);
    Job j2 = make_job(a, 2, 1e-8, 300, false, 1);   // brings a in; its own state fails
    run(s, j2);
    CHECK(j2.res.status == SIP_ENOMEM && j2.res.factorised == 0);
    CHECK(stats(s)[RESIDENT] == 0);   // a went with it
    Job j3 = make_job(a, 3, 1e-8, 300, false, 1);
    j3.coefficients = false;   // a is not resident: refused at submit
    const sip_request r3 = j3.request();
    CHECK(sip_batch_submit(s, &r3, &j3.ticket) == SIP_EINVAL);
    Job j4 = make_job(a, 4, 1e-8, 300, false, 1);
    run(s, j4);
    check_solved(j4);
    CHECK(j4.res.factorised == 1);
    fake::fail_request_allocs(1);
    Job j5 = make_job(a, 5, 1e-8, 300, false);   // a resident: the failed request drops its reference once
    j5.coefficients = false;
    run(s, j5);
    CHECK(j5.res.status == SIP_ENOMEM);
    CHECK(sip_server_release(s, 1) == SIP_OK);
    CHECK(stats(s)[RESIDENT] == 0);
    Job j6 = make_job(b, 6, 1e-8, 300, true);
    run(s, j6);
    check_solved(j6);
    destroy(s);
}

// A failed step ends every running request with its status and writes no x;
// the server goes on serving.
void step_failure()
{
    const Sys a = make_sys(1, 6, 5, 4, SIP_MIXED, false, 16);
    sip_server s = make_server(0);
    fake::close_gate();
    Job j1 = make_job(a, 1, 1e-8, 300, false, 1), j2 = make_job(a, 2, 1e-8, 300, true);
    submit(s, j1);
    fake::wait_at_gate();
    submit(s, j2);
    fake::fail_next_step();
    fake::open_gate();
    wait(s, j1);
    CHECK(j1.res.status == SIP_EDEVICE);
    check_untouched(j1);
    wait(s, j2);
    check_solved(j2);
    Job j3 = make_job(a, 3, 1e-8, 300, false);
    j3.coefficients = false;
    run(s, j3);
    check_solved(j3);
    destroy(s);
}

// Shutdown while a request runs and others are queued: the running one ends
// after its step, every request not done is cancelled (no x written), a
// waiting poll returns, later submits are refused.
void shutdown_cancels()
{
    const Sys a = make_sys(1, 9, 8, 6, SIP_FP64, false, 17), b = make_sys(2, 5, 5, 5, SIP_FP32, false, 18);
    sip_server s = make_server(0, 1);
    fake::close_gate(true);
    Job l = make_job(a, 1, 1e-14, 100000, false);
    submit(s, l);
    fake::wait_at_gate();
    std::vector<Job> q;
    for (int k = 0; k < 5; k++) q.push_back(make_job(k % 2 ? a : b, 10 + k, 1e-8, 300, false));
    for (Job &j : q) submit(s, j);
    std::thread waiter([&] { wait(s, q[4]); });
    CHECK(sip_server_shutdown(s) == SIP_OK);
    waiter.join();
    fake::open_gate();
    wait(s, l);
    CHECK(l.res.status == SIP_ECANCELLED);
    check_untouched(l);
    for (int k = 0; k < 4; k++) wait(s, q[k]);
    for (Job &j : q) {
        CHECK(j.res.status == SIP_ECANCELLED);
        check_untouched(j);
    }
    Job late = make_job(b, 99, 1e-8, 300, false);
    const sip_request r = late.request();
    uint64_t t = 0;
    CHECK(sip_batch_submit(s, &r, &t) == SIP_ECANCELLED);
    CHECK(sip_server_shutdown(s) == SIP_OK);   // a second shutdown is harmless
    destroy(s);
}

// Six threads submit random requests over ten systems with a small budget
// and few slots (eviction and queueing all the time), poll with random waits,
// while another releases systems and reads the counters; the server is shut
// down with requests still queued.  Every ticket resolves exactly once; a
// solved request has the oracle's result, a request without coefficients may
// find its system evicted (SIP_EINVAL), the rest are cancelled.
void stress()
{
    std::vector<Sys> sys;
    const int prec[3] = {SIP_FP64, SIP_MIXED, SIP_FP32};
    for (int k = 0; k < 10; k++)
        sys.push_back(make_sys(200 + k, 4 + k % 4, 4 + k % 3, 3 + k % 2, prec[k % 3], false, 40 + k));
    size_t budget = 0;
    for (int k = 0; k < 3; k++) budget += sys_bytes(sys[k]) + req_bytes(sys[k]);
    sip_server s = make_server(budget, 3, 2);
    constexpr int T = 6, M = 20;
    std::vector<std::vector<Job>> jobs(T);
    for (int t = 0; t < T; t++)
        for (int m = 0; m < M; m++) {
            const Sys &y = sys[(7 * t + 3 * m) % 10];
            Job j = make_job(y, 5000 + 100 * t + m, y.precision == SIP_FP32 ? 1e-4 : 1e-8, m % 5 == 0 ? 4 : 200,
                             m % 3 == 0, m % 2);
            j.coefficients = m % 4 != 3;
            jobs[t].push_back(std::move(j));
        }
    std::atomic<int> finished{0};
    std::thread side([&] {
        std::mt19937 rng(1);
        while (finished < T) {
            CHECK(sip_server_release(s, 200 + rng() % 10) == SIP_OK);
            const auto v = stats(s);
            CHECK(v[RESIDENT] <= budget && v[PEAK] <= budget);
            std::this_thread::sleep_for(std::chrono::microseconds(300));
        }
    });
    std::vector<std::thread> th;
    for (int t = 0; t < T; t++)
        th.emplace_back([&, t] {
            std::mt19937 rng(t);
            for (Job &j : jobs[t]) {
                const sip_request r = j.request();
                const sip_status st0 = sip_batch_submit(s, &r, &j.ticket);
                if (!j.coefficients && st0 == SIP_EINVAL) {   // the system was not resident
                    j.refused = true;
                    j.ticket = 0;
                    continue;
                }
                CHECK(st0 == SIP_OK);
                if (rng() % 3 == 0) {
                    sip_status st;
                    while ((st = sip_batch_poll(s, j.ticket, (int)(rng() % 3), &j.res)) == SIP_PENDING) {
                    }
                    CHECK(st == SIP_OK);
                    j.ticket = 0;
                }
            }
            for (Job &j : jobs[t])
                if (j.ticket) wait(s, j);
            finished++;
        });
    for (auto &t : th) t.join();
    side.join();
    for (auto &v : jobs)
        for (Job &j : v) {
            if (j.refused) continue;
            if (!j.coefficients && j.res.status == SIP_EINVAL) {   // evicted or released before admission
                check_untouched(j);
                continue;
            }
            check_solved(j);
        }
    // a last wave, cut off by shutdown
    std::vector<Job> tail;
    for (int m = 0; m < 12; m++) tail.push_back(make_job(sys[m % 10], 9000 + m, 1e-12, 100000, false));
    for (Job &j : tail) submit(s, j);
    CHECK(sip_server_shutdown(s) == SIP_OK);
    for (Job &j : tail) {
        wait(s, j);
        CHECK(j.res.status == SIP_ECANCELLED || j.res.status == SIP_OK || j.res.status == SIP_ENOTCONV);
        if (j.res.status == SIP_ECANCELLED) check_untouched(j);
        sip_result again{};
        CHECK(sip_batch_poll(s, j.ticket, 0, &again) == SIP_EINVAL);
    }
    destroy(s);
}

// With no arrivals between steps the backend runs its persistent mode (the
// scheduler reports that no request was submitted since the last step).
void persistent_mode()
{
    const Sys a = make_sys(1, 6, 6, 6, SIP_MIXED, false, 19);
    sip_server s = make_server(0, 4, 2);
    const uint64_t p0 = fake::persistent_steps();
    Job j = make_job(a, 1, 1e-10, 300, false);
    run(s, j);
    check_solved(j);
    CHECK(fake::persistent_steps() > p0);
    destroy(s);
}

struct Scenario {
    const char *name;
    void (*fn)();
};
const Scenario SCENARIOS[] = {
    {"results_concurrent", results_concurrent}, {"lru_eviction", lru_eviction},
    {"queued_protection", queued_protection},   {"first_fit", first_fit},
    {"queue_full", queue_full},                 {"invalid_arguments", invalid_arguments},
    {"factorisation_failures", factorisation_failures}, {"allocation_failures", allocation_failures},
    {"step_failure", step_failure},             {"shutdown_cancels", shutdown_cancels},
    {"stress", stress},                         {"persistent_mode", persistent_mode},
};

}  // namespace

int main(int argc, char **argv)
{
    int ran = 0;
    for (const Scenario &sc : SCENARIOS) {
        bool want = argc == 1;
        for (int k = 1; k < argc; k++) want = want || std::strcmp(argv[k], sc.name) == 0;
        if (!want) continue;
        std::printf("scenario %s\n", sc.name);
        std::fflush(stdout);
        sc.fn();
        std::printf("ok %s\n", sc.name);
        std::fflush(stdout);
        ran++;
    }
    std::printf("%d scenarios passed\n", ran);
    return ran > 0 ? 0 : 1;
}
