// Host runtime and C ABI of the SIP library (include/sip.h).
//
// A sip_system owns, in device memory and in the tile-sheared layout of
// sip_internal.h: the coefficients (FP64; FP32 for the sweeps of the all-FP32
// arithmetic), the factors (FP64 or FP32), b, x (FP64, or FP32 in the all-FP32
// arithmetic), the forward-sweep result y, the tagged face words, per-tile
// partial sums, the residual history and a control block.  A solve is a
// stream-ordered sequence of launches: reorder b and x in, (forward sweep,
// backward sweep) per iteration, reorder x out.  The stop test runs on the
// device; the host replays graph-captured chunks of iterations and reads the
// control block back one chunk behind, so the GPU never waits for the host.
#include "sip_internal.h"
#include "sip_runtime.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <random>
#include <string>
#include <tuple>
#include <vector>

using namespace sipk;

namespace sipk {

uint64_t timeout_ticks_for(int device, double seconds)
{
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || rate_khz <= 0)
        rate_khz = 100000;
    return (uint64_t)(seconds * rate_khz * 1000.0);
}

double wait_limit_seconds()
{
    const char *e = getenv("SIP_WAIT_LIMIT_MS");
    char *end = nullptr;
    const double ms = e ? strtod(e, &end) : 0.0;
    if (!e || end == e || !(ms >= 0.0) || ms > 1e9) return 2.0;   // unset or not a time: the default
    return ms * 1e-3;
}

// The bound of every device-side wait of a handle's sweeps, read at every
// call (SIP_WAIT_LIMIT_MS exercises the error paths without a stalled device).
static void refresh_wait_limit(sip_system_s *h) { h->timeout_ticks = timeout_ticks_for(h->device, wait_limit_seconds()); }

uint32_t schedule_seed()
{
    const char *e = getenv("SIP_SCHEDULE_SEED");
    return e ? (uint32_t)strtoul(e, nullptr, 10) : 0u;
}

// Random topological order: repeatedly take a random tile whose upstream
// neighbours have all been listed.
static std::vector<int2> random_topo_order(const std::vector<Geom> &gs, bool backward, uint32_t seed)
{
    std::vector<std::vector<int>> wait(gs.size());
    std::vector<int2> ready, out;
    const int step = backward ? -1 : 1;
    for (size_t jb = 0; jb < gs.size(); jb++) {
        const Geom &g = gs[jb];
        wait[jb].resize(g.ntiles);
        for (int t = 0; t < g.ntiles; t++) {
            const int ti = t % g.nti, tj = t / g.nti;
            const int up = backward ? (ti < g.nti - 1) + (tj < g.ntj - 1) : (ti > 0) + (tj > 0);
            wait[jb][t] = up;
            if (up == 0) ready.push_back(make_int2((int)jb, t));
        }
    }
    std::mt19937 rng(seed * 2654435761u + (backward ? 1u : 0u));
    while (!ready.empty()) {
        const size_t q = rng() % ready.size();
        const int2 it = ready[q];
        ready[q] = ready.back();
        ready.pop_back();
        out.push_back(it);
        const Geom &g = gs[it.x];
        const int ti = it.y % g.nti, tj = it.y / g.nti;
        const int down[2][2] = {{ti + step, tj}, {ti, tj + step}};
        for (const auto &d : down)
            if (d[0] >= 0 && d[0] < g.nti && d[1] >= 0 && d[1] < g.ntj) {
                const int t = d[1] * g.nti + d[0];
                if (--wait[it.x][t] == 0) ready.push_back(make_int2(it.x, t));
            }
    }
    return out;
}

std::vector<int2> topo_order(const std::vector<Geom> &gs, bool backward, uint32_t seed)
{
    if (seed) return random_topo_order(gs, backward, seed);
    struct Item {
        long long key;
        int job, tile;
    };
    std::vector<Item> items;
    for (size_t jb = 0; jb < gs.size(); jb++) {
        const Geom &g = gs[jb];
        const int dmax = g.nti + g.ntj - 2;
        for (int t = 0; t < g.ntiles; t++) {
            const int ti = t % g.nti, tj = t / g.nti;
            const int d = backward ? dmax - (ti + tj) : ti + tj;
            const int tjk = backward ? g.ntj - 1 - tj : tj;
            items.push_back({((long long)d << 40) | ((long long)jb << 20) | tjk, (int)jb, t});
        }
    }
    std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &b) { return a.key < b.key; });
    std::vector<int2> out(items.size());
    for (size_t q = 0; q < items.size(); q++) out[q] = make_int2(items[q].job, items[q].tile);
    return out;
}

size_t system_bytes(const Geom &g, int fp32)
{
    const size_t E = (size_t)g.elems, fs = fp32 ? 4 : 8;
    return E * (7 * 8 + 7 * fs + 2 * 8 + fs) + (size_t)g.ntiles * g.steps * FACE_WORDS * 8 +
           (size_t)g.ntiles * 2 * 8 + sizeof(Ctl) + 2 * (size_t)g.ntiles * sizeof(int2);
}

// ---------------------------------------------------------------- System

static void free_system(sip_system_s *h)
{
    if (!h) return;
    if (h->chunk_exec) (void)hipGraphExecDestroy(h->chunk_exec);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (void *p : {(void *)h->A, h->LU, (void *)h->bx, h->y, (void *)h->face, (void *)h->part, (void *)h->ctl,
                    (void *)h->hist, (void *)h->d_job, (void *)h->d_job_factor, (void *)h->order_f, (void *)h->order_b,
                    (void *)h->lc, (void *)h->mbx, h->my, (void *)h->mface, (void *)h->mpart, (void *)h->mctl,
                    (void *)h->mhist, (void *)h->d_mjob, (void *)h->p_tord, (void *)h->p_off, (void *)h->p_tasks,
                    (void *)h->p_pc, (void *)h->p_flags})
        if (p) (void)hipFree(p);
    if (h->h_ctl) (void)hipHostFree(h->h_ctl);
    if (h->h_mctl) (void)hipHostFree(h->h_mctl);
    if (h->h_hist) (void)hipHostFree(h->h_hist);
    for (hipEvent_t e : h->p_ev)
        if (e) (void)hipEventDestroy(e);
    delete h;
}

static sip_status alloc_dev(void **p, size_t n, const char *what)
{
    hipError_t e = hipMalloc(p, n ? n : 1);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return set_error(SIP_ENOMEM, "hipMalloc(%zu) for %s failed: %s", n, what, hipGetErrorString(e));
    }
    return SIP_OK;
}

#define TRY(x)                                  \
    do {                                        \
        sip_status st_ = (x);                   \
        if (st_ != SIP_OK) return st_;          \
    } while (0)
#define HIPTRY(x)                                                                                 \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess) return set_error(SIP_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

sip_status system_alloc(sip_system_s *h, hipStream_t s)
{
    const Geom &g = h->g;
    const size_t E = (size_t)g.elems, fs = h->fp32 ? 4 : 8;
    TRY(alloc_dev((void **)&h->A, 7 * E * 8, "coefficients"));
    TRY(alloc_dev(&h->LU, 7 * E * fs, "factors"));
    TRY(alloc_dev((void **)&h->bx, 2 * E * 8, "b and x"));
    TRY(alloc_dev(&h->y, E * fs, "y"));
    const size_t fbytes = (size_t)g.ntiles * g.steps * FACE_WORDS * 8;
    TRY(alloc_dev((void **)&h->face, fbytes, "face words"));
    TRY(alloc_dev((void **)&h->part, (size_t)g.ntiles * 2 * 8, "partials"));
    TRY(alloc_dev((void **)&h->ctl, sizeof(Ctl), "control"));
    TRY(alloc_dev((void **)&h->d_job, sizeof(Job), "job"));
    TRY(alloc_dev((void **)&h->d_job_factor, sizeof(Job), "job"));
    TRY(alloc_dev((void **)&h->order_f, g.ntiles * sizeof(int2), "order"));
    TRY(alloc_dev((void **)&h->order_b, g.ntiles * sizeof(int2), "order"));
    TRY(alloc_dev((void **)&h->lc, sizeof(LaunchCtl), "launch control"));
    HIPTRY(hipHostMalloc((void **)&h->h_ctl, 4 * sizeof(Ctl), hipHostMallocDefault));
    HIPTRY(hipMemsetAsync(h->LU, 0, 7 * E * fs, s));
    HIPTRY(hipMemsetAsync(h->y, 0, E * fs, s));
    HIPTRY(hipMemsetAsync(h->face, 0, fbytes, s));
    HIPTRY(hipMemsetAsync(h->lc, 0, sizeof(LaunchCtl), s));
    h->bytes = system_bytes(g, h->fp32);
    return SIP_OK;
}

sip_status ensure_hist(sip_system_s *h, int n, hipStream_t s)
{
    if (n <= h->hist_cap) return SIP_OK;
    HIPTRY(hipStreamSynchronize(s));
    if (h->hist) (void)hipFree(h->hist);
    if (h->h_hist) (void)hipHostFree(h->h_hist);
    h->hist = nullptr;
    h->h_hist = nullptr;
    h->hist_cap = 0;
    const int cap = std::max(n, 64);
    TRY(alloc_dev((void **)&h->hist, (size_t)cap * 8, "history"));
    HIPTRY(hipHostMalloc((void **)&h->h_hist, (size_t)cap * 8, hipHostMallocDefault));
    h->hist_cap = cap;
    // the job descriptor holds the history pointer
    h->job.hist = h->hist;
    HIPTRY(hipMemcpyAsync(h->d_job, &h->job, sizeof(Job), hipMemcpyHostToDevice, s));
    HIPTRY(hipStreamSynchronize(s));
    if (h->chunk_exec) {
        (void)hipGraphExecDestroy(h->chunk_exec);
        h->chunk_exec = nullptr;
    }
    return SIP_OK;
}

// x in the library's layout: behind b, in the arithmetic's precision
static void *x_of(const sip_system_s *h)
{
    return h->precision == ARITH_F32 ? (void *)((float *)h->bx + h->g.elems) : (void *)(h->bx + h->g.elems);
}

// Copies b and x into the library's layout (rounded to FP32 in the all-FP32
// arithmetic, where the relaxation starts from single-precision copies).
static hipError_t stage_in(const sip_system_s *h, const double *b, const double *x, hipStream_t s)
{
    const double *src[2] = {b, x};
    return launch_to_sheared(h->g, 2, src, h->bx, h->g.elems, h->precision == ARITH_F32 ? SHEAR_F32 : SHEAR_F64, s);
}

// Natural-order FP64 x (widened from FP32 in the all-FP32 arithmetic).
static hipError_t stage_out(const sip_system_s *h, double *x, hipStream_t s)
{
    return launch_from_sheared(h->g, x_of(h), h->precision == ARITH_F32, x, h->ctl, s);
}

// Tuned sweep plans by block shape and arithmetic (filled by sip_tune,
// consulted by sip_factor and the server).
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int, int, int>, SweepPlan> g_tuned;

bool tuned_plan(const Geom &g, int arith, int sym, SweepPlan *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto f = g_tuned.find(std::make_tuple(g.ni, g.nj, g.nk, arith, sym));
    if (f == g_tuned.end()) return false;
    out->phases = f->second.phases;   // the caller keeps its own stream choice
    out->poll = f->second.poll;
    return true;
}

LaunchArgs fwd_args(const sip_system_s *h)
{
    return LaunchArgs{h->d_job, h->order_f, h->lc, h->g.ntiles, h->timeout_ticks, h->torture};
}
LaunchArgs bwd_args(const sip_system_s *h)
{
    return LaunchArgs{h->d_job, h->order_b, h->lc, h->g.ntiles, h->timeout_ticks, h->torture};
}

static sip_status launch_iterations(sip_system_s *h, int n, hipStream_t s)
{
    const LaunchArgs fa = fwd_args(h), ba = bwd_args(h);
    for (int q = 0; q < n; q++) {
        HIPTRY(launch_forward(fa, h->precision, h->plan, s));
        HIPTRY(launch_backward(ba, h->precision, h->plan, s));
    }
    return SIP_OK;
}

// Replays CHUNK iterations as one captured graph.
static sip_status launch_chunk(sip_system_s *h, hipStream_t s)
{
    if (h->chunk_exec && h->chunk_ticks != h->timeout_ticks) {   // the graph holds the wait bound
        (void)hipGraphExecDestroy(h->chunk_exec);
        h->chunk_exec = nullptr;
    }
    if (!h->chunk_exec) {
        h->chunk_ticks = h->timeout_ticks;
        if (!h->cap_stream) HIPTRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        HIPTRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
        sip_status st = launch_iterations(h, CHUNK, h->cap_stream);
        hipError_t e = hipStreamEndCapture(h->cap_stream, &graph);
        if (st != SIP_OK) return st;
        if (e != hipSuccess) return set_error(SIP_EDEVICE, "graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&h->chunk_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return set_error(SIP_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
    }
    HIPTRY(hipGraphLaunch(h->chunk_exec, s));
    return SIP_OK;
}

// A solve that stopped on a non-finite norm has no residual from that
// iteration on: the history reads NaN there.
static void nan_from(double *hist, uint32_t from, size_t n)
{
    for (size_t q = from; q < n; q++) hist[q] = std::numeric_limits<double>::quiet_NaN();
}

static bool non_finite(uint32_t stop) { return stop == BAD_INPUT || stop == DIVERGED; }

static sip_status stop_status(uint32_t stop)
{
    switch (stop) {
    case RUN:
    case CONVERGED:
    case ZERO_RHS:
        return SIP_OK;
    case MAXITER:
        return SIP_ENOTCONV;
    case BREAKDOWN:
        return set_error(SIP_EBREAKDOWN, "SIP factorisation breakdown (zero or non-finite pivot)");
    case BAD_INPUT:
        return set_error(SIP_EINVAL, "non-finite input: ||b|| or the residual of the start vector is not finite");
    case DIVERGED:
        return set_error(SIP_EBREAKDOWN, "the iteration diverged (non-finite residual)");
    case TIMEOUT:
    default:
        return set_error(SIP_EDEVICE, "a device-side wait timed out");
    }
}

// ------------------------------------------------ two right-hand sides

// Buffers of the two-right-hand-side sweeps, allocated on first use, and a
// residual history of at least hist_n entries per right-hand side.
static sip_status ensure_multi(sip_system_s *h, int hist_n, hipStream_t s)
{
    const Geom &g = h->g;
    const size_t E = (size_t)g.elems;
    bool upload = false;
    if (!h->mbx) {
        const size_t fbytes = (size_t)g.ntiles * g.steps * FACE_WORDS_SWEEP * 8 + (size_t)g.ntiles * SINK_WORDS * 8;
        TRY(alloc_dev((void **)&h->mbx, 4 * E * 8, "b and x pairs"));
        TRY(alloc_dev(&h->my, 2 * E * 4, "y pairs"));
        TRY(alloc_dev((void **)&h->mface, fbytes, "face words"));
        TRY(alloc_dev((void **)&h->mpart, (size_t)g.ntiles * 4 * 8, "partials"));
        TRY(alloc_dev((void **)&h->mctl, 3 * sizeof(Ctl), "control"));
        TRY(alloc_dev((void **)&h->d_mjob, sizeof(Job), "job"));
        HIPTRY(hipHostMalloc((void **)&h->h_mctl, 9 * sizeof(Ctl), hipHostMallocDefault));
        HIPTRY(hipMemsetAsync(h->my, 0, 2 * E * 4, s));
        HIPTRY(hipMemsetAsync(h->mface, 0, fbytes, s));   // tags start at 1: no stale word matches
        HIPTRY(launch_init_ctl(h->mctl, 3, 0, 0.0, 1, s));
        h->bytes += 4 * E * 8 + 2 * E * 4 + fbytes + (size_t)g.ntiles * 32 + 3 * sizeof(Ctl);
        upload = true;
    }
    if (hist_n > h->mhist_cap) {
        HIPTRY(hipStreamSynchronize(s));
        if (h->mhist) (void)hipFree(h->mhist);
        h->mhist = nullptr;
        h->mhist_cap = 0;
        const int cap = std::max(hist_n, 64);
        TRY(alloc_dev((void **)&h->mhist, (size_t)2 * cap * 8, "history"));
        h->mhist_cap = cap;
        upload = true;
    }
    if (upload) {
        Job &J = h->mjob;
        J = h->job;
        const bool f32 = h->precision == ARITH_F32;
        J.b = h->mbx;
        J.x = f32 ? (void *)((float *)h->mbx + 2 * E) : (void *)(h->mbx + 2 * E);
        J.y = h->my;
        J.face = h->mface;
        J.part = h->mpart;
        J.ctl = h->mctl;
        J.hist = h->mhist;
        J.hstride = h->mhist_cap;
        J.m = 2;
        J.fw = FACE_WORDS_SWEEP;
        HIPTRY(hipMemcpyAsync(h->d_mjob, &J, sizeof(Job), hipMemcpyHostToDevice, s));
        HIPTRY(hipStreamSynchronize(s));
    }
    return SIP_OK;
}

// The pair job's split flag (Job::coupled for m > 1): a solve stops the pair
// sweeps once one right-hand side has stopped and continues the other alone;
// a fixed number of iterations keeps both in the pair sweeps throughout.
static sip_status set_split(sip_system_s *h, int on, hipStream_t s)
{
    if (h->mjob.coupled == on) return SIP_OK;
    h->mjob.coupled = on;
    HIPTRY(hipMemcpyAsync(h->d_mjob, &h->mjob, sizeof(Job), hipMemcpyHostToDevice, s));
    HIPTRY(hipStreamSynchronize(s));
    return SIP_OK;
}

static LaunchArgs multi_args(const sip_system_s *h, bool backward)
{
    return LaunchArgs{h->d_mjob, backward ? h->order_b : h->order_f, h->lc, h->g.ntiles, h->timeout_ticks,
                      h->torture};
}

static sip_status multi_iterations(sip_system_s *h, int n, hipStream_t s)
{
    const LaunchArgs fa = multi_args(h, false), ba = multi_args(h, true);
    for (int q = 0; q < n; q++) {
        HIPTRY(launch_forward(fa, h->precision, h->plan, s, 2));
        HIPTRY(launch_backward(ba, h->precision, h->plan, s, 2));
    }
    return SIP_OK;
}

static hipError_t multi_stage_in(const sip_system_s *h, const double *b0, const double *b1, const double *x0,
                                 const double *x1, hipStream_t s)
{
    const Geom &g = h->g;
    const bool f32 = h->precision == ARITH_F32;
    const int sh = f32 ? SHEAR_PAIR_F32 : SHEAR_PAIR_F64;
    const double *bs[2] = {b0, b1}, *xs[2] = {x0, x1};
    hipError_t e = launch_to_sheared(g, 2, bs, h->mbx, g.elems, sh, s);
    if (e != hipSuccess) return e;
    return launch_to_sheared(g, 2, xs, h->mjob.x, g.elems, sh, s);
}

static hipError_t multi_stage_out(const sip_system_s *h, double *x0, double *x1, hipStream_t s)
{
    const bool f32 = h->precision == ARITH_F32;
    hipError_t e = launch_from_sheared(h->g, h->mjob.x, f32, x0, h->mctl + 1, s, 2, 0);
    if (e != hipSuccess) return e;
    return launch_from_sheared(h->g, h->mjob.x, f32, x1, h->mctl + 2, s, 2, 1);
}

// ------------------------------------------------ persistent solve
// sip_solve runs the whole solve as one persistent launch (k_persist with a
// single job): the finalisers publish the sweeps one after the other and
// decide the stop on the device, so no launch gap separates two sweeps and
// the host only waits.  The chunked graph replay remains for plans the
// persistent kernel is not compiled for (one loader phase, poll distances
// other than 2) and with SIP_SOLVE_PERSISTENT=0.
static bool solve_persistent(const sip_system_s *h)
{
    const char *e = getenv("SIP_SOLVE_PERSISTENT");
    return (!e || atoi(e) != 0) && h->plan.phases >= 2 && h->plan.poll == DEFAULT_POLL;
}

static sip_status ensure_persist(sip_system_s *h, hipStream_t s)
{
    if (h->p_tasks) return SIP_OK;
    const Geom &g = h->g;
    h->p_cap = (uint32_t)g.ntiles + 64u;
    if (h->num_cu <= 0) {
        int ncu = 0;
        h->num_cu = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess &&
                            ncu > 0
                        ? ncu
                        : 256;
    }
    TRY(alloc_dev((void **)&h->p_tord, 2 * (size_t)g.ntiles * sizeof(int), "tile orders"));
    TRY(alloc_dev((void **)&h->p_off, 2 * sizeof(int), "tile order offsets"));
    TRY(alloc_dev((void **)&h->p_tasks, (size_t)h->p_cap * sizeof(Task), "task queue"));
    TRY(alloc_dev((void **)&h->p_pc, sizeof(PersistCtl), "queue control"));
    TRY(alloc_dev((void **)&h->p_flags, 2 * sizeof(uint32_t), "queue flags"));
    for (hipEvent_t &e : h->p_ev) HIPTRY(hipEventCreate(&e));
    std::vector<int> tord;
    for (int b = 0; b < 2; b++)
        for (const int2 &o : topo_order({g}, b != 0, h->torture ? h->torture + 17u * b : 0u)) tord.push_back(o.y);
    const int off[2] = {0, g.ntiles};
    h->p_host_tasks.assign(h->p_cap, (Task)0);
    for (int k = 0; k < g.ntiles; k++) h->p_host_tasks[k] = make_task((uint32_t)k, 0, 0, tord[k]);
    HIPTRY(hipMemcpyAsync(h->p_tord, tord.data(), tord.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIPTRY(hipMemcpyAsync(h->p_off, off, sizeof off, hipMemcpyHostToDevice, s));
    HIPTRY(hipStreamSynchronize(s));   // the host copies above are locals
    return SIP_OK;
}

// Enqueues one persistent launch that runs the job (the handle's own, or
// its pair job with nrhs = 2) until its stop decision.
static sip_status launch_solve_persistent(sip_system_s *h, hipStream_t s, const Job *job = nullptr, int nrhs = 1)
{
    TRY(ensure_persist(h, s));
    const Geom &g = h->g;
    h->p_host_pc = PersistCtl{0u, (uint32_t)g.ntiles, 1u, 0u};
    HIPTRY(hipMemcpyAsync(h->p_tasks, h->p_host_tasks.data(), h->p_host_tasks.size() * sizeof(Task),
                          hipMemcpyHostToDevice, s));
    HIPTRY(hipMemcpyAsync(h->p_pc, &h->p_host_pc, sizeof(PersistCtl), hipMemcpyHostToDevice, s));
    HIPTRY(launch_init_flags(h->p_flags, s));
    const PersistArgs pa{job ? job : h->d_job, h->p_tord, h->p_off, h->p_tasks, h->p_cap, h->p_pc, h->p_flags,
                         h->p_flags + 1, h->timeout_ticks, h->torture, nullptr};
    const int wgs = std::max(1, std::min(g.ntiles, h->num_cu * (h->plan.phases >= 3 ? 1 : 2)));
    HIPTRY(hipEventRecord(h->p_ev[0], s));
    HIPTRY(launch_persist(pa, h->precision, h->plan, wgs, s, nrhs));
    HIPTRY(hipEventRecord(h->p_ev[1], s));
    return SIP_OK;
}

// After a persistent launch whose task queue timed out: the sweep then in
// progress may not have reached its finaliser, so face records tagged with
// the control block's current epoch can remain; the next sweep on the handle
// must use a newer tag.  hc: the block as copied back after the launch.
static sip_status skip_epoch(Ctl *dctl, Ctl *hc, hipStream_t s)
{
    hc->epoch += 1u;
    HIPTRY(hipMemcpyAsync(dctl, hc, sizeof(Ctl), hipMemcpyHostToDevice, s));
    HIPTRY(hipStreamSynchronize(s));
    return SIP_OK;
}

// After the stream has synchronised: adds the launch's device time to the
// solve call's sum.
static sip_status count_solve_launch(sip_system_s *h)
{
    float t = 0.0f;
    HIPTRY(hipEventElapsedTime(&t, h->p_ev[0], h->p_ev[1]));
    h->p_ms += t;
    h->p_timed = true;
    return SIP_OK;
}

// ------------------------------------------------ no-allocation iterate
// sip_iterate_noalloc keeps the per-call state of its sweeps -- the job
// descriptor, the control block, the launch counters, the per-tile partial
// norms and the residual history -- in this file-scope array instead of the
// buffers sip_iterate uses, so that a call allocates nothing.  Each GPU holds
// its own copy for the life of the process; in host code the name is only a
// stand-in, and every use goes through the device address that
// hipGetSymbolAddress returns for the current device (noalloc_scratch).
static __device__ __align__(256) unsigned char scratch[SIP_NOALLOC_SCRATCH_BYTES];

constexpr size_t NA_OFF_JOB = 0, NA_OFF_CTL = 256, NA_OFF_LC = 512, NA_OFF_PART = 1024;
static_assert(sizeof(Job) <= NA_OFF_CTL - NA_OFF_JOB, "job descriptor slot");
static_assert(sizeof(Ctl) <= NA_OFF_LC - NA_OFF_CTL, "control block slot");
static_assert(sizeof(LaunchCtl) <= NA_OFF_PART - NA_OFF_LC, "launch counter slot");

static std::mutex g_scratch_mu;
static std::map<int, unsigned char *> g_scratch_addr;   // device -> its scratch

// Device address of `scratch` on `device` (which must be current), looked up
// once per device.
static sip_status noalloc_scratch(int device, unsigned char **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto f = g_scratch_addr.find(device);
    if (f != g_scratch_addr.end()) {
        *out = f->second;
        return SIP_OK;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return set_error(SIP_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                         hipGetErrorString(e));
    g_scratch_addr[device] = (unsigned char *)ptr;
    *out = (unsigned char *)ptr;
    return SIP_OK;
}

// Start of a call: the job descriptor (passed by value), zeroed launch
// counters, and a control block for n_iter iterations that continues the
// system's sweep tags (the tags in the system's face words must never repeat).
__global__ void k_noalloc_begin(Job j, Job *job, LaunchCtl *lc, Ctl *ctl, const Ctl *sys, uint32_t max_iter)
{
    if (threadIdx.x != 0) return;
    *job = j;
    lc->ticket = 0u;
    lc->done = 0u;
    Ctl c{};
    c.epoch = sys->epoch;
    c.max_iter = max_iter;
    c.stop = RUN;
    *ctl = c;
}

// End of a call: the system's control block takes the final state, so later
// calls on the system go on with fresh tags.
__global__ void k_noalloc_end(Ctl *sys, const Ctl *ctl)
{
    if (threadIdx.x == 0) *sys = *ctl;
}

}  // namespace sipk

// ================================================================= C ABI

extern "C" {

int32_t sip_abi_version(void) { return 1; }

sip_status sip_factor(const sip_problem *p, void *stream, sip_system *out)
{
    const Range range("sip_factor");
    if (!p || !out) return set_error(SIP_EINVAL, "NULL argument");
    if (p->ni < 1 || p->nj < 1 || p->nk < 1) return set_error(SIP_EINVAL, "dims must be >= 1");
    if ((long long)p->ni * p->nj * p->nk > (1ll << 34)) return set_error(SIP_EINVAL, "block too large");
    if (!(p->alpha >= 0.0 && p->alpha <= 1.0)) return set_error(SIP_EINVAL, "alpha must be in [0, 1]");
    if (p->precision != SIP_FP64 && p->precision != SIP_MIXED && p->precision != SIP_FP32)
        return set_error(SIP_EINVAL, "unknown precision");
    if (p->storage != SIP_STORAGE_FULL && p->storage != SIP_STORAGE_SYMMETRIC)
        return set_error(SIP_EINVAL, "unknown storage");
    if (p->storage == SIP_STORAGE_SYMMETRIC && p->precision == SIP_FP32)
        return set_error(SIP_EINVAL, "the symmetric storage is available with SIP_FP64 and SIP_MIXED only");
    for (int d = 0; d < 7; d++)
        if (!p->a[d]) return set_error(SIP_EINVAL, "coefficient pointer %d is NULL", d);
    hipStream_t s = (hipStream_t)stream;
    sip_system_s *h = new sip_system_s();
    h->g = make_geom(p->ni, p->nj, p->nk);
    if (h->g.elems >= MAX_ELEMS) {   // kernels address every array with 32-bit byte offsets
        delete h;
        return set_error(SIP_EINVAL, "block too large: more than 2^28 cells in the sheared layout");
    }
    h->fp32 = p->precision != SIP_FP64;
    h->precision = p->precision;
    h->alpha = p->alpha;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return set_error(SIP_EDEVICE, "no HIP device");
    }
    h->timeout_ticks = timeout_ticks_for(h->device, wait_limit_seconds());
    h->torture = schedule_seed();
    // one system per launch: three loader phases (split turns) shorten the
    // step; a solve server with many blocks per launch keeps two (more
    // workgroups per compute unit)
    h->plan.phases = SINGLE_SYSTEM_PHASES;
    const char *env_ph = getenv("SIP_SWEEP_PHASES"), *env_pd = getenv("SIP_POLL_DISTANCE");
    if (env_ph || env_pd) {   // tuning overrides
        const int nl = env_ph ? atoi(env_ph) : 0, pd = env_pd ? atoi(env_pd) : 0;
        if (nl >= 1 && nl <= sipk::MAX_PHASES) h->plan.phases = nl;
        if (pd >= 1 && pd <= sipk::MAX_POLL) h->plan.poll = pd;
    } else {
        (void)tuned_plan(h->g, p->precision, p->storage == SIP_STORAGE_SYMMETRIC, &h->plan);
    }
    // non-temporal streams for systems far beyond the caches;
    // SIP_STREAM_LOADS=0 / 1 forces the choice (the results are the same)
    const char *env_st = getenv("SIP_STREAM_LOADS");
    h->plan.stream = env_st ? (atoi(env_st) != 0) : ((long long)p->ni * p->nj * p->nk >= STREAM_HINT_CELLS);
    sip_status st = system_alloc(h, s);
    if (st != SIP_OK) {
        free_system(h);
        return st;
    }
    auto bail = [&](sip_status e) {
        (void)hipStreamSynchronize(s);
        free_system(h);
        return e;
    };
    const Geom &g = h->g;
    h->sym = p->storage == SIP_STORAGE_SYMMETRIC;
    if (h->sym) {   // the symmetric storage is only valid for a symmetric A
        unsigned bad = 0;
        if (hipMemsetAsync(h->part, 0, sizeof(unsigned), s) != hipSuccess ||
            launch_check_symmetric(p->ni, p->nj, p->nk, p->a, (unsigned *)h->part, s) != hipSuccess ||
            hipMemcpyAsync(&bad, h->part, sizeof(unsigned), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return bail(set_error(SIP_EDEVICE, "symmetry check failed"));
        if (bad) return bail(set_error(SIP_EINVAL, "symmetric storage requested but %u couplings differ", bad));
    }
    if (launch_to_sheared(g, 7, p->a, h->A, g.elems, SHEAR_COEF, s) != hipSuccess)
        return bail(set_error(SIP_EDEVICE, "reorder launch failed"));
    if (launch_init_ctl(h->ctl, 1, 0, 0.0, 1, s) != hipSuccess) return bail(set_error(SIP_EDEVICE, "init failed"));
    st = ensure_hist(h, 64, s);
    if (st != SIP_OK) return bail(st);
    Job &J = h->job;
    J.g = g;
    J.A = h->A;
    J.b = h->bx;
    J.x = x_of(h);
    J.LU = h->LU;
    J.y = h->y;
    J.face = h->face;
    J.part = h->part;
    J.hist = h->hist;
    J.ctl = h->ctl;
    J.alpha = h->alpha;
    J.fw = FACE_WORDS_SWEEP;
    J.sym = h->sym;
    const std::vector<Geom> gs{g};
    const std::vector<int2> of = topo_order(gs, false, h->torture), ob = topo_order(gs, true, h->torture);
    if (hipMemcpyAsync(h->d_job, &J, sizeof(Job), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->order_f, of.data(), of.size() * sizeof(int2), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->order_b, ob.data(), ob.size() * sizeof(int2), hipMemcpyHostToDevice, s) != hipSuccess)
        return bail(set_error(SIP_EDEVICE, "upload failed"));
    // the factorisation exchanges U triples (FACE_WORDS per step); the sweeps one value
    h->job_factor = J;
    h->job_factor.fw = FACE_WORDS;
    h->job_factor.sym = 0;   // the factorisation reads the full coefficients
    J.fw = FACE_WORDS_SWEEP;
    if (hipMemcpyAsync(h->d_job_factor, &h->job_factor, sizeof(Job), hipMemcpyHostToDevice, s) != hipSuccess)
        return bail(set_error(SIP_EDEVICE, "upload failed"));
    LaunchArgs fa = fwd_args(h);
    fa.jobs = h->d_job_factor;
    if (launch_factor(fa, h->fp32, s) != hipSuccess) return bail(set_error(SIP_EDEVICE, "factor launch failed"));
    if (hipMemcpyAsync(h->h_ctl, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return bail(set_error(SIP_EDEVICE, "factorisation failed: %s", hipGetErrorString(hipGetLastError())));
    if (h->h_ctl->stop != RUN) return bail(stop_status(h->h_ctl->stop));
    // the sweeps read the symmetric or the FP32 storage; it overwrites the full
    // FP64 one, which only the factorisation needed
    const int sweep_coef = h->sym ? SHEAR_SYM : h->precision == SIP_FP32 ? SHEAR_COEF32 : SHEAR_COEF;
    if (sweep_coef != SHEAR_COEF && (launch_to_sheared(g, 7, p->a, h->A, g.elems, sweep_coef, s) != hipSuccess ||
                                     hipStreamSynchronize(s) != hipSuccess))
        return bail(set_error(SIP_EDEVICE, "reorder launch failed"));
    *out = h;
    return SIP_OK;
}

sip_status sip_iterate(sip_system h, const double *b, double *x, int32_t n_iter, double *rel_res_hist, void *stream)
{
    const Range range("sip_iterate");
    if (!h || !b || !x) return set_error(SIP_EINVAL, "NULL argument");
    refresh_wait_limit(h);
    if (n_iter < 0) return set_error(SIP_EINVAL, "n_iter must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    TRY(ensure_hist(h, n_iter + 1, s));
    HIPTRY(stage_in(h, b, x, s));
    HIPTRY(launch_init_ctl(h->ctl, 1, (uint32_t)n_iter, 0.0, 0, s));
    int left = n_iter;
    while (left >= CHUNK) {
        TRY(launch_chunk(h, s));
        left -= CHUNK;
    }
    TRY(launch_iterations(h, left, s));
    HIPTRY(launch_forward(fwd_args(h), h->precision, h->plan, s));   // residual of the final iterate
    HIPTRY(stage_out(h, x, s));
    if (!rel_res_hist) return SIP_OK;
    HIPTRY(hipMemcpyAsync(h->h_hist, h->hist, (size_t)(n_iter + 1) * 8, hipMemcpyDeviceToHost, s));
    HIPTRY(hipMemcpyAsync(h->h_ctl, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    std::memcpy(rel_res_hist, h->h_hist, (size_t)(n_iter + 1) * 8);
    const uint32_t stop = h->h_ctl->stop;
    if (stop == ZERO_RHS) {
        for (int q = 0; q <= n_iter; q++) rel_res_hist[q] = 0.0;
        return SIP_OK;
    }
    if (non_finite(stop)) nan_from(rel_res_hist, h->h_ctl->iter, (size_t)n_iter + 1);
    if (stop == MAXITER || stop == RUN) return SIP_OK;
    return stop_status(stop);
}

sip_status sip_iterate_noalloc(sip_system h, const double *b, double *x, int32_t n_iter, double *rel_res_hist,
                               void *stream)
{
    if (!h || !b || !x) return set_error(SIP_EINVAL, "NULL argument");
    refresh_wait_limit(h);
    if (n_iter < 0) return set_error(SIP_EINVAL, "n_iter must be >= 0");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != h->device)
        return set_error(SIP_EINVAL, "the system lives on device %d, the current device is %d", h->device, cur);
    const Geom &g = h->g;
    const size_t part = (size_t)2 * g.ntiles * sizeof(double);
    const size_t off_hist = NA_OFF_PART + ((part + 255) & ~(size_t)255);
    const size_t need = off_hist + (rel_res_hist ? (size_t)(n_iter + 1) * sizeof(double) : 0);
    if (need > SIP_NOALLOC_SCRATCH_BYTES)
        return set_error(SIP_EINVAL,
                         "sip_iterate_noalloc: %d tiles and %s need %zu bytes of scratch, more than the %d available",
                         g.ntiles, rel_res_hist ? "the history" : "no history", need, SIP_NOALLOC_SCRATCH_BYTES);
    unsigned char *base = nullptr;
    TRY(noalloc_scratch(h->device, &base));
    hipStream_t s = (hipStream_t)stream;
    Job J = h->job;
    J.part = (double *)(base + NA_OFF_PART);
    J.ctl = (Ctl *)(base + NA_OFF_CTL);
    J.hist = rel_res_hist ? (double *)(base + off_hist) : nullptr;
    Job *dj = (Job *)(base + NA_OFF_JOB);
    LaunchCtl *lc = (LaunchCtl *)(base + NA_OFF_LC);
    hipLaunchKernelGGL(k_noalloc_begin, dim3(1), dim3(64), 0, s, J, dj, lc, J.ctl, h->ctl, (uint32_t)n_iter);
    HIPTRY(hipGetLastError());
    HIPTRY(stage_in(h, b, x, s));
    const LaunchArgs fa{dj, h->order_f, lc, g.ntiles, h->timeout_ticks, h->torture};
    const LaunchArgs ba{dj, h->order_b, lc, g.ntiles, h->timeout_ticks, h->torture};
    for (int q = 0; q < n_iter; q++) {
        HIPTRY(launch_forward(fa, h->precision, h->plan, s));
        HIPTRY(launch_backward(ba, h->precision, h->plan, s));
    }
    HIPTRY(launch_forward(fa, h->precision, h->plan, s));   // residual of the final iterate
    HIPTRY(launch_from_sheared(g, x_of(h), h->precision == ARITH_F32, x, J.ctl, s));
    hipLaunchKernelGGL(k_noalloc_end, dim3(1), dim3(64), 0, s, h->ctl, (const Ctl *)J.ctl);
    HIPTRY(hipGetLastError());
    if (!rel_res_hist) return SIP_OK;
    HIPTRY(hipMemcpyAsync(rel_res_hist, base + off_hist, (size_t)(n_iter + 1) * sizeof(double),
                          hipMemcpyDeviceToHost, s));
    HIPTRY(hipMemcpyAsync(h->h_ctl, J.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    const uint32_t stop = h->h_ctl->stop;
    if (stop == ZERO_RHS) {
        for (int q = 0; q <= n_iter; q++) rel_res_hist[q] = 0.0;
        return SIP_OK;
    }
    if (non_finite(stop)) nan_from(rel_res_hist, h->h_ctl->iter, (size_t)n_iter + 1);
    if (stop == MAXITER || stop == RUN) return SIP_OK;
    return stop_status(stop);
}

// sip_solve without resetting the call's launch time (sip_solve_multi runs
// it for the continuations of pairs and for an odd last right-hand side).
static sip_status solve_one(sip_system h, const double *b, double *x, double rtol, int32_t max_iter,
                            sip_info *info, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    TRY(ensure_hist(h, max_iter + 1, s));
    HIPTRY(stage_in(h, b, x, s));
    HIPTRY(launch_init_ctl(h->ctl, 1, (uint32_t)max_iter, rtol, 0, s));
    if (solve_persistent(h)) {
        TRY(launch_solve_persistent(h, s));
        HIPTRY(stage_out(h, x, s));
        HIPTRY(hipMemcpyAsync(&h->h_ctl[2], h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        HIPTRY(hipMemcpyAsync(&h->p_host_pc, h->p_pc, sizeof(PersistCtl), hipMemcpyDeviceToHost, s));
        HIPTRY(hipStreamSynchronize(s));
        TRY(count_solve_launch(h));
        const Ctl &c = h->h_ctl[2];
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (info) {
            info->iters = (int32_t)c.iter;
            info->rel_res = non_finite(c.stop) ? std::numeric_limits<double>::quiet_NaN() : c.rho;
            info->seconds = secs;
        }
        if (h->p_host_pc.err) {
            TRY(skip_epoch(h->ctl, &h->h_ctl[2], s));
            return set_error(SIP_EDEVICE, "a device-side queue wait timed out");
        }
        if (c.stop == RUN) return set_error(SIP_EDEVICE, "solve ended without a stop decision");
        return stop_status(c.stop);
    }
    hipEvent_t ev[2];
    HIPTRY(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    HIPTRY(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    long long fwd_launched = 0;
    sip_status st = SIP_OK;
    for (int c = 0;; c++) {
        st = launch_chunk(h, s);
        if (st != SIP_OK) break;
        fwd_launched += CHUNK;
        if (hipMemcpyAsync(&h->h_ctl[c & 1], h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipEventRecord(ev[c & 1], s) != hipSuccess) {
            st = set_error(SIP_EDEVICE, "status copy failed");
            break;
        }
        if (fwd_launched > max_iter) break;
        if (c > 0) {
            if (hipEventSynchronize(ev[(c - 1) & 1]) != hipSuccess) {
                st = set_error(SIP_EDEVICE, "event wait failed");
                break;
            }
            if (h->h_ctl[(c - 1) & 1].stop != RUN) break;
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (st != SIP_OK) {
        (void)hipStreamSynchronize(s);
        return st;
    }
    HIPTRY(stage_out(h, x, s));
    HIPTRY(hipMemcpyAsync(&h->h_ctl[2], h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    const Ctl &c = h->h_ctl[2];
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) {
        info->iters = (int32_t)c.iter;
        info->rel_res = non_finite(c.stop) ? std::numeric_limits<double>::quiet_NaN() : c.rho;
        info->seconds = secs;
    }
    if (c.stop == RUN) return set_error(SIP_EDEVICE, "solve ended without a stop decision");
    return stop_status(c.stop);
}

sip_status sip_solve(sip_system h, const double *b, double *x, double rtol, int32_t max_iter, sip_info *info,
                     void *stream)
{
    const Range range("sip_solve");
    if (!h || !b || !x) return set_error(SIP_EINVAL, "NULL argument");
    if (!(rtol > 0.0) || max_iter < 0) return set_error(SIP_EINVAL, "need rtol > 0 and max_iter >= 0");
    refresh_wait_limit(h);
    h->p_timed = false;
    h->p_ms = 0.0;
    return solve_one(h, b, x, rtol, max_iter, info, stream);
}

sip_status sip_export_factors(sip_system h, double *const out[7], void *stream)
{
    if (!h || !out) return set_error(SIP_EINVAL, "NULL argument");
    for (int d = 0; d < 7; d++)
        if (!out[d]) return set_error(SIP_EINVAL, "output pointer %d is NULL", d);
    HIPTRY(launch_export_factors(h->g, h->LU, h->fp32, out, (hipStream_t)stream));
    return SIP_OK;
}

sip_status sip_profile_sweeps(sip_system h, const double *b, double *x, int32_t n_iter, double ms[2], void *stream)
{
    if (!h || !b || !x || !ms) return set_error(SIP_EINVAL, "NULL argument");
    refresh_wait_limit(h);
    if (n_iter < 1) return set_error(SIP_EINVAL, "n_iter must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    TRY(ensure_hist(h, n_iter + 1, s));
    HIPTRY(stage_in(h, b, x, s));
    HIPTRY(launch_init_ctl(h->ctl, 1, (uint32_t)n_iter, 0.0, 0, s));
    std::vector<hipEvent_t> ev(2 * n_iter + 1);
    for (auto &e : ev) HIPTRY(hipEventCreate(&e));
    const LaunchArgs fa = fwd_args(h), ba = bwd_args(h);
    sip_status st = SIP_OK;
    if (hipEventRecord(ev[0], s) != hipSuccess) st = set_error(SIP_EDEVICE, "event record failed");
    for (int q = 0; q < n_iter && st == SIP_OK; q++) {
        if (launch_forward(fa, h->precision, h->plan, s) != hipSuccess ||
            hipEventRecord(ev[2 * q + 1], s) != hipSuccess ||
            launch_backward(ba, h->precision, h->plan, s) != hipSuccess ||
            hipEventRecord(ev[2 * q + 2], s) != hipSuccess)
            st = set_error(SIP_EDEVICE, "launch failed");
    }
    if (st == SIP_OK && stage_out(h, x, s) != hipSuccess)
        st = set_error(SIP_EDEVICE, "reorder failed");
    if (st == SIP_OK && hipStreamSynchronize(s) != hipSuccess) st = set_error(SIP_EDEVICE, "synchronise failed");
    double f = 0.0, bk = 0.0;
    for (int q = 0; q < n_iter && st == SIP_OK; q++) {
        float a = 0.f, c = 0.f;
        if (hipEventElapsedTime(&a, ev[2 * q], ev[2 * q + 1]) != hipSuccess ||
            hipEventElapsedTime(&c, ev[2 * q + 1], ev[2 * q + 2]) != hipSuccess)
            st = set_error(SIP_EDEVICE, "event timing failed");
        f += a;
        bk += c;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (st != SIP_OK) return st;
    ms[0] = f / n_iter;
    ms[1] = bk / n_iter;
    return SIP_OK;
}

// Right-hand sides without a partner (FP64 factors, or the last of an odd
// count) run through the one-right-hand-side path.
static bool pairs_ok(const sip_system_s *h) { return h->precision == SIP_MIXED || h->precision == SIP_FP32; }

sip_status sip_iterate_multi(sip_system h, int32_t nrhs, const double *const *b, double *const *x, int32_t n_iter,
                             double *rel_res_hist, void *stream)
{
    const Range range("sip_iterate_multi");
    if (!h || !b || !x) return set_error(SIP_EINVAL, "NULL argument");
    if (nrhs < 1 || n_iter < 0) return set_error(SIP_EINVAL, "need nrhs >= 1 and n_iter >= 0");
    for (int r = 0; r < nrhs; r++)
        if (!b[r] || !x[r]) return set_error(SIP_EINVAL, "right-hand side %d: NULL b or x", r);
    refresh_wait_limit(h);
    hipStream_t s = (hipStream_t)stream;
    const int npair = pairs_ok(h) ? nrhs / 2 : 0;
    const size_t hn = (size_t)n_iter + 1;
    sip_status bad = SIP_OK;   // first right-hand side with a non-finite norm; the others still run
    int bad_r = -1;
    if (npair > 0) {
        TRY(ensure_multi(h, n_iter + 1, s));
        TRY(set_split(h, 0, s));
    }
    for (int pr = 0; pr < npair; pr++) {
        const int r0 = 2 * pr, r1 = r0 + 1;
        HIPTRY(multi_stage_in(h, b[r0], b[r1], x[r0], x[r1], s));
        HIPTRY(launch_init_ctl(h->mctl, 3, (uint32_t)n_iter, 0.0, 0, s));
        TRY(multi_iterations(h, n_iter, s));
        HIPTRY(launch_forward(multi_args(h, false), h->precision, h->plan, s, 2));   // residual of the final iterates
        HIPTRY(multi_stage_out(h, x[r0], x[r1], s));
        if (!rel_res_hist) continue;
        std::vector<double> hb(2 * (size_t)h->mhist_cap);
        HIPTRY(hipMemcpyAsync(hb.data(), h->mhist, hb.size() * 8, hipMemcpyDeviceToHost, s));
        HIPTRY(hipMemcpyAsync(h->h_mctl, h->mctl, 3 * sizeof(Ctl), hipMemcpyDeviceToHost, s));
        HIPTRY(hipStreamSynchronize(s));
        for (int m = 0; m < 2; m++) {
            double *dst = rel_res_hist + (size_t)(r0 + m) * hn;
            std::memcpy(dst, hb.data() + (size_t)m * h->mhist_cap, hn * 8);
            const uint32_t sm = h->h_mctl[1 + m].stop;
            if (sm == ZERO_RHS)
                for (size_t q = 0; q < hn; q++) dst[q] = 0.0;
            if (non_finite(sm)) {
                nan_from(dst, h->h_mctl[1 + m].iter, hn);
                if (bad == SIP_OK) bad = stop_status(sm), bad_r = r0 + m;
            }
        }
        const uint32_t stop = h->h_mctl[0].stop;
        if (stop == BREAKDOWN || stop == TIMEOUT) return stop_status(stop);
    }
    for (int r = 2 * npair; r < nrhs; r++) {
        const sip_status st = sip_iterate(h, b[r], x[r], n_iter, rel_res_hist ? rel_res_hist + (size_t)r * hn : nullptr,
                                          stream);
        if (st == SIP_OK) continue;
        if ((st != SIP_EINVAL && st != SIP_EBREAKDOWN) || !non_finite(h->h_ctl->stop)) return st;
        if (bad == SIP_OK) bad = st, bad_r = r;
    }
    if (bad != SIP_OK) return set_error(bad, "right-hand side %d: non-finite %s", bad_r,
                                        bad == SIP_EINVAL ? "input" : "residual (diverged)");
    return SIP_OK;
}

sip_status sip_solve_multi(sip_system h, int32_t nrhs, const double *const *b, double *const *x, double rtol,
                           int32_t max_iter, sip_info *info, void *stream)
{
    const Range range("sip_solve_multi");
    if (!h || !b || !x) return set_error(SIP_EINVAL, "NULL argument");
    if (nrhs < 1) return set_error(SIP_EINVAL, "need nrhs >= 1");
    if (!(rtol > 0.0) || max_iter < 0) return set_error(SIP_EINVAL, "need rtol > 0 and max_iter >= 0");
    for (int r = 0; r < nrhs; r++)
        if (!b[r] || !x[r]) return set_error(SIP_EINVAL, "right-hand side %d: NULL b or x", r);
    hipStream_t s = (hipStream_t)stream;
    const int npair = pairs_ok(h) ? nrhs / 2 : 0;
    sip_status worst = SIP_OK;
    sip_status bad = SIP_OK;   // first right-hand side with a non-finite norm; the others are still solved
    int bad_r = -1;
    refresh_wait_limit(h);
    h->p_timed = false;
    h->p_ms = 0.0;
    // the finaliser records rho_n for n <= max_iter
    if (npair > 0) {
        TRY(ensure_multi(h, max_iter + 1, s));
        TRY(set_split(h, 1, s));
    }
    for (int pr = 0; pr < npair; pr++) {
        const auto t0 = std::chrono::steady_clock::now();
        const int r0 = 2 * pr, r1 = r0 + 1;
        HIPTRY(multi_stage_in(h, b[r0], b[r1], x[r0], x[r1], s));
        HIPTRY(launch_init_ctl(h->mctl, 3, (uint32_t)max_iter, rtol, 0, s));
        sip_status st = SIP_OK;
        long long launched = 0;
        bool split = false;   // one right-hand side stopped: its partner goes on alone
        hipEvent_t ev[2];
        HIPTRY(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
        HIPTRY(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
        // one persistent launch runs the pair until it stops (both right-hand
        // sides, or one of them: PARTNER); otherwise chunks of iterations
        const bool persist = solve_persistent(h);
        if (persist) st = launch_solve_persistent(h, s, h->d_mjob, 2);
        for (int c = 0; !persist; c++) {
            st = multi_iterations(h, CHUNK, s);
            if (st != SIP_OK) break;
            launched += CHUNK;
            if (hipMemcpyAsync(&h->h_mctl[3 * (c & 1)], h->mctl, 3 * sizeof(Ctl), hipMemcpyDeviceToHost, s) !=
                    hipSuccess ||
                hipEventRecord(ev[c & 1], s) != hipSuccess) {
                st = set_error(SIP_EDEVICE, "status copy failed");
                break;
            }
            if (launched > max_iter) break;
            if (c > 0) {
                if (hipEventSynchronize(ev[(c - 1) & 1]) != hipSuccess) {
                    st = set_error(SIP_EDEVICE, "event wait failed");
                    break;
                }
                const Ctl *hc = &h->h_mctl[3 * ((c - 1) & 1)];
                if (hc[0].stop != RUN) break;
                if (hc[1].stop != RUN || hc[2].stop != RUN) {
                    split = true;
                    break;
                }
            }
        }
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
        if (st != SIP_OK) {
            (void)hipStreamSynchronize(s);
            return st;
        }
        HIPTRY(multi_stage_out(h, x[r0], x[r1], s));
        HIPTRY(hipMemcpyAsync(&h->h_mctl[6], h->mctl, 3 * sizeof(Ctl), hipMemcpyDeviceToHost, s));
        if (persist) HIPTRY(hipMemcpyAsync(&h->p_host_pc, h->p_pc, sizeof(PersistCtl), hipMemcpyDeviceToHost, s));
        HIPTRY(hipStreamSynchronize(s));
        if (persist) TRY(count_solve_launch(h));
        if (persist && h->p_host_pc.err) {
            TRY(skip_epoch(h->mctl, &h->h_mctl[6], s));
            return set_error(SIP_EDEVICE, "a device-side queue wait timed out");
        }
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        const Ctl *c = &h->h_mctl[6];
        if (c[0].stop == RUN && !split) return set_error(SIP_EDEVICE, "solve ended without a stop decision");
        if (c[0].stop == BREAKDOWN || c[0].stop == TIMEOUT) return stop_status(c[0].stop);
        for (int m = 0; m < 2; m++) {
            sip_info one{(int32_t)c[1 + m].iter, c[1 + m].stop == ZERO_RHS ? 0.0 : c[1 + m].rho, secs};
            if (non_finite(c[1 + m].stop)) {
                one.rel_res = std::numeric_limits<double>::quiet_NaN();
                if (bad == SIP_OK) bad = stop_status(c[1 + m].stop), bad_r = r0 + m;
            } else if (c[1 + m].stop == RUN) {
                // The partner has stopped: this one continues from its iterate
                // x_N through the one-right-hand-side sweeps, which compute the
                // same iterates and residuals as the pair sweeps.
                const int32_t done = (int32_t)c[0].iter;
                sip_info more{};
                const sip_status s1 = solve_one(h, b[r0 + m], x[r0 + m], rtol, max_iter - done, &more, stream);
                const bool nf = (s1 == SIP_EINVAL || s1 == SIP_EBREAKDOWN) && non_finite(h->h_ctl[2].stop);
                if (s1 != SIP_OK && s1 != SIP_ENOTCONV && !nf) return s1;
                one = sip_info{done + more.iters, more.rel_res, secs + more.seconds};
                if (s1 == SIP_ENOTCONV) worst = SIP_ENOTCONV;
                if (nf && bad == SIP_OK) bad = s1, bad_r = r0 + m;
            } else if (c[1 + m].stop == MAXITER) {
                worst = SIP_ENOTCONV;
            }
            if (info) info[r0 + m] = one;
        }
    }
    for (int r = 2 * npair; r < nrhs; r++) {
        const sip_status st = solve_one(h, b[r], x[r], rtol, max_iter, info ? info + r : nullptr, stream);
        if (st == SIP_ENOTCONV) worst = SIP_ENOTCONV;
        else if ((st == SIP_EINVAL || st == SIP_EBREAKDOWN) && non_finite(h->h_ctl[2].stop)) {
            if (bad == SIP_OK) bad = st, bad_r = r;
        } else if (st != SIP_OK) return st;
    }
    if (bad != SIP_OK) return set_error(bad, "right-hand side %d: non-finite %s", bad_r,
                                        bad == SIP_EINVAL ? "input" : "residual (diverged)");
    if (worst == SIP_ENOTCONV) return set_error(SIP_ENOTCONV, "a right-hand side reached max_iter");
    return SIP_OK;
}

sip_status sip_profile_sweeps_multi(sip_system h, const double *const *b, double *const *x, int32_t n_iter,
                                    double ms[2], void *stream)
{
    if (!h || !b || !x || !b[0] || !b[1] || !x[0] || !x[1] || !ms) return set_error(SIP_EINVAL, "NULL argument");
    refresh_wait_limit(h);
    if (n_iter < 1) return set_error(SIP_EINVAL, "n_iter must be >= 1");
    if (!pairs_ok(h)) return set_error(SIP_EINVAL, "pairs of right-hand sides need FP32 factors");
    hipStream_t s = (hipStream_t)stream;
    TRY(ensure_multi(h, n_iter + 1, s));
    HIPTRY(multi_stage_in(h, b[0], b[1], x[0], x[1], s));
    HIPTRY(launch_init_ctl(h->mctl, 3, (uint32_t)n_iter, 0.0, 0, s));
    std::vector<hipEvent_t> ev(2 * n_iter + 1);
    for (auto &e : ev) HIPTRY(hipEventCreate(&e));
    const LaunchArgs fa = multi_args(h, false), ba = multi_args(h, true);
    sip_status st = SIP_OK;
    if (hipEventRecord(ev[0], s) != hipSuccess) st = set_error(SIP_EDEVICE, "event record failed");
    for (int q = 0; q < n_iter && st == SIP_OK; q++) {
        if (launch_forward(fa, h->precision, h->plan, s, 2) != hipSuccess ||
            hipEventRecord(ev[2 * q + 1], s) != hipSuccess ||
            launch_backward(ba, h->precision, h->plan, s, 2) != hipSuccess ||
            hipEventRecord(ev[2 * q + 2], s) != hipSuccess)
            st = set_error(SIP_EDEVICE, "launch failed");
    }
    if (st == SIP_OK && multi_stage_out(h, x[0], x[1], s) != hipSuccess) st = set_error(SIP_EDEVICE, "reorder failed");
    if (st == SIP_OK && hipStreamSynchronize(s) != hipSuccess) st = set_error(SIP_EDEVICE, "synchronise failed");
    double f = 0.0, bk = 0.0;
    for (int q = 0; q < n_iter && st == SIP_OK; q++) {
        float a = 0.f, c = 0.f;
        if (hipEventElapsedTime(&a, ev[2 * q], ev[2 * q + 1]) != hipSuccess ||
            hipEventElapsedTime(&c, ev[2 * q + 1], ev[2 * q + 2]) != hipSuccess)
            st = set_error(SIP_EDEVICE, "event timing failed");
        f += a;
        bk += c;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (st != SIP_OK) return st;
    ms[0] = f / n_iter;
    ms[1] = bk / n_iter;
    return SIP_OK;
}

sip_status sip_tune(sip_system h, const double *b, int32_t n_iter, int32_t *phases, void *stream)
{
    const Range range("sip_tune");
    if (!h || !b) return set_error(SIP_EINVAL, "NULL argument");
    refresh_wait_limit(h);
    if (n_iter < 1) return set_error(SIP_EINVAL, "n_iter must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    TRY(ensure_hist(h, n_iter + 1, s));
    const Geom &g = h->g;
    const LaunchArgs fa = fwd_args(h), ba = bwd_args(h);
    hipEvent_t e0, e1;
    HIPTRY(hipEventCreate(&e0));
    HIPTRY(hipEventCreate(&e1));
    // candidates: every phase count with the default poll distance, and the
    // other distances with two and three phases (compiled for one
    // right-hand side)
    std::vector<SweepPlan> cand;
    for (int np = 1; np <= MAX_PHASES; np++)
        for (int pd = 1; pd <= MAX_POLL; pd++)
            if (pd == DEFAULT_POLL || np >= 2) cand.push_back(SweepPlan{np, pd, h->plan.stream});
    SweepPlan best = h->plan;
    float best_ms = 0.f;
    sip_status st = SIP_OK;
    for (size_t ci = 0; ci < cand.size() && st == SIP_OK; ci++) {
        const SweepPlan pl = cand[ci];
        // the same iterations from x = 0 for every candidate
        const double *src[1] = {b};
        if (launch_to_sheared(g, 1, src, h->bx, g.elems, h->precision == ARITH_F32 ? SHEAR_F32 : SHEAR_F64, s) !=
                hipSuccess ||
            hipMemsetAsync(x_of(h), 0, (size_t)g.elems * (h->precision == ARITH_F32 ? 4 : 8), s) != hipSuccess ||
            launch_init_ctl(h->ctl, 1, (uint32_t)n_iter, 0.0, 0, s) != hipSuccess ||
            hipEventRecord(e0, s) != hipSuccess) {
            st = set_error(SIP_EDEVICE, "tuning launch failed");
            break;
        }
        for (int q = 0; q < n_iter && st == SIP_OK; q++)
            if (launch_forward(fa, h->precision, pl, s) != hipSuccess ||
                launch_backward(ba, h->precision, pl, s) != hipSuccess)
                st = set_error(SIP_EDEVICE, "tuning launch failed");
        float ms = 0.f;
        if (st == SIP_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = set_error(SIP_EDEVICE, "tuning timing failed");
        if (st == SIP_OK && (ci == 0 || ms < best_ms)) {
            best = pl;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SIP_OK) return st;
    if ((h->plan.phases != best.phases || h->plan.poll != best.poll) && h->chunk_exec) {
        HIPTRY(hipStreamSynchronize(s));   // the captured chunk holds the old kernels
        (void)hipGraphExecDestroy(h->chunk_exec);
        h->chunk_exec = nullptr;
    }
    h->plan = best;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[std::make_tuple(g.ni, g.nj, g.nk, h->precision, h->sym)] = h->plan;
    }
    if (phases) *phases = best.phases;
    return SIP_OK;
}

sip_status sip_system_plan(sip_system h, int32_t *phases, int32_t *poll)
{
    if (!h) return set_error(SIP_EINVAL, "NULL argument");
    if (phases) *phases = h->plan.phases;
    if (poll) *poll = h->plan.poll;
    return SIP_OK;
}

sip_status sip_system_solve_ms(sip_system h, double *ms)
{
    if (!h || !ms) return set_error(SIP_EINVAL, "NULL argument");
    if (!h->p_timed) return set_error(SIP_EINVAL, "the handle's last solve call ran no persistent launch");
    *ms = h->p_ms;
    return SIP_OK;
}

// The tuning table as text: one JSON object per line, keys in a fixed order.
sip_status sip_tune_save(const char *path)
{
    if (!path) return set_error(SIP_EINVAL, "NULL argument");
    std::string out;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const auto &kv : g_tuned) {
            char line[160];
            snprintf(line, sizeof line,
                     "{\"ni\": %d, \"nj\": %d, \"nk\": %d, \"precision\": %d, \"symmetric\": %d, \"phases\": %d, "
                     "\"poll\": %d}\n",
                     std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first),
                     std::get<4>(kv.first), kv.second.phases, kv.second.poll);
            out += line;
        }
    }
    FILE *f = fopen(path, "w");
    if (!f) return set_error(SIP_EINVAL, "cannot open %s for writing", path);
    const bool ok = fwrite(out.data(), 1, out.size(), f) == out.size();
    if (fclose(f) != 0 || !ok) return set_error(SIP_EINVAL, "cannot write %s", path);
    return SIP_OK;
}

// Value of "key": <integer> in a line; false if absent or not an integer.
static bool json_int(const char *line, const char *key, long *v)
{
    char pat[32];
    snprintf(pat, sizeof pat, "\"%s\"", key);
    const char *p = strstr(line, pat);
    if (!p) return false;
    p += strlen(pat);
    while (*p == ' ' || *p == '\t') p++;
    if (*p++ != ':') return false;
    char *end = nullptr;
    *v = strtol(p, &end, 10);
    return end != p;
}

sip_status sip_tune_load(const char *path)
{
    if (!path) return set_error(SIP_EINVAL, "NULL argument");
    FILE *f = fopen(path, "r");
    if (!f) return set_error(SIP_EINVAL, "cannot open %s", path);
    std::vector<std::pair<std::tuple<int, int, int, int, int>, SweepPlan>> got;
    char line[512];
    int lineno = 0;
    sip_status st = SIP_OK;
    while (st == SIP_OK && fgets(line, sizeof line, f)) {
        lineno++;
        const char *q = line;
        while (*q == ' ' || *q == '\t' || *q == '\r' || *q == '\n') q++;
        if (!*q) continue;   // blank line
        long ni, nj, nk, prec, sym, ph;
        if (!json_int(line, "ni", &ni) || !json_int(line, "nj", &nj) || !json_int(line, "nk", &nk) ||
            !json_int(line, "precision", &prec) || !json_int(line, "symmetric", &sym) ||
            !json_int(line, "phases", &ph) || ni < 1 || nj < 1 || nk < 1 || ni > INT32_MAX || nj > INT32_MAX ||
            nk > INT32_MAX || prec < SIP_FP64 || prec > SIP_FP32 || sym < 0 || sym > 1 || ph < 1 ||
            ph > MAX_PHASES) {
            st = set_error(SIP_EINVAL, "%s:%d: not a tuning entry", path, lineno);
            break;
        }
        long pd = DEFAULT_POLL;   // entries written before the poll distance was tuned have none
        if (strstr(line, "\"poll\"") && (!json_int(line, "poll", &pd) || pd < 1 || pd > MAX_POLL)) {
            st = set_error(SIP_EINVAL, "%s:%d: not a tuning entry", path, lineno);
            break;
        }
        SweepPlan pl;
        pl.phases = (int)ph;
        pl.poll = (int)pd;
        got.push_back({std::make_tuple((int)ni, (int)nj, (int)nk, (int)prec, (int)sym), pl});
    }
    fclose(f);
    if (st != SIP_OK) return st;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &e : got) g_tuned[e.first] = e.second;
    return SIP_OK;
}

sip_status sip_system_info(sip_system h, int32_t dims[3], int32_t *precision, size_t *device_bytes)
{
    if (!h) return set_error(SIP_EINVAL, "NULL handle");
    if (dims) {
        dims[0] = h->g.ni;
        dims[1] = h->g.nj;
        dims[2] = h->g.nk;
    }
    if (precision) *precision = h->precision;
    if (device_bytes) *device_bytes = h->bytes;
    return SIP_OK;
}

sip_status sip_system_destroy(sip_system h)
{
    if (!h) return set_error(SIP_EINVAL, "NULL handle");
    free_system(h);
    return SIP_OK;
}

}  // extern "C"
