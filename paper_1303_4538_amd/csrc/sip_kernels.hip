// gfx950 kernels of Stone's SIP: layout reorder, factorisation, fused
// residual + forward sweep, backward sweep + update.
//
// Every recurrence kernel is a pipeline over tile columns (see the layout in
// sip_internal.h).  One workgroup = one tile = two waves:
//   wave 0, "recurrence": walks the tile's local hyperplanes s = 0..steps-1;
//     lane (i', j') handles cell (i', j', k = s - i' - j').  Its W/S (or E/N)
//     neighbours inside the tile are the neighbouring lanes one step earlier
//     (exchanged through LDS); across the tile edge the value comes from the
//     neighbour tile's face words.  It touches global memory only to read
//     those face words.
//   wave 1, "loader": streams the coefficient / factor / vector planes from
//     HBM a few steps ahead (register pipeline of depth LP), does all work
//     that does not depend on the recurrence (the FP64 residual, the FP64
//     update of x), stages operands in an LDS ring for wave 0 and writes wave
//     0's results and face words back to HBM.
// The two waves meet at one workgroup barrier per step; the barrier waits on
// LDS traffic only, so the loader's loads stay in flight across it.
//
// Face words: a value crossing a tile edge is written as 64-bit words
// (sweep tag << 32 | 32 payload bits) with agent-scope relaxed atomic stores;
// the consumer polls the words with agent-scope atomic loads until the tag
// equals the current sweep's tag.  Each word is self-validating, so no fence
// is needed on the hot path.  Waits are bounded by a wall-clock limit that
// raises a sticky error instead of hanging.
//
// Workgroups take tiles from a ticket counter in a topological order (W and S
// tiles before a tile in forward order, the reverse for the backward sweep),
// so a tile only ever waits for tiles owned by workgroups that started
// earlier; no co-residency is assumed.
#include "sip_internal.h"

#include <cmath>

namespace sipk {

Geom make_geom(int ni, int nj, int nk)
{
    Geom g;
    g.ni = ni;
    g.nj = nj;
    g.nk = nk;
    g.nti = (ni + TI - 1) / TI;
    g.ntj = (nj + TJ - 1) / TJ;
    g.ntiles = g.nti * g.ntj;
    g.steps = nk + TI + TJ - 2;
    g.planes = g.steps + 2;
    g.tile_elems = (long long)g.planes * TT;
    g.elems = (long long)g.ntiles * g.tile_elems;
    return g;
}

namespace {

// Pointers read from a job descriptor are generic to the compiler, which then
// emits flat loads; flat loads count against the LDS counter, so every LDS
// wait (e.g. before a barrier) would also wait for all outstanding prefetches.
// Qualifying them as global memory keeps HBM traffic on the vector counter only.
#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL T *gp(T *p)
{
    return (GLOBAL T *)p;
}

// The job descriptors do not change while a kernel runs.  Reading them
// through the constant address space with a uniform index gives scalar loads,
// so the descriptor's pointers and sizes live in scalar registers; a plain
// load (the kernel has already written memory through its ticket counter)
// would put every uniform pointer in vector registers.
#define CONSTANT __attribute__((address_space(4)))
__device__ __forceinline__ Job load_job(const LaunchArgs &a, int job)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const CONSTANT Job *)a.jobs)[job];
#else
    return a.jobs[job];   // host pass of a device function: never executed
#endif
}

constexpr int WAVE = 64;
constexpr int BLOCK = 2 * WAVE;
constexpr int LP = 4;   // loader register-pipeline depth (steps of look-ahead)
constexpr int PD = 2;   // face-word prefetch distance of the recurrence wave

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ uint64_t ll_load(const GLOBAL uint64_t *p)
{
    return __hip_atomic_load(const_cast<GLOBAL uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void ll_store(GLOBAL uint64_t *p, uint32_t tag, uint32_t payload)
{
    __hip_atomic_store(p, ((uint64_t)tag << 32) | payload, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void wg_barrier()
{
    // Orders LDS traffic only (s_waitcnt lgkmcnt); global loads stay in flight.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <typename F> struct NW;
template <> struct NW<float> { static constexpr int n = 1; };
template <> struct NW<double> { static constexpr int n = 2; };

__device__ __forceinline__ void to_words(float v, uint32_t *w) { w[0] = __float_as_uint(v); }
__device__ __forceinline__ void to_words(double v, uint32_t *w)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    w[0] = (uint32_t)b;
    w[1] = (uint32_t)(b >> 32);
}
__device__ __forceinline__ void from_words(const uint64_t *w, float &v) { v = __uint_as_float((uint32_t)w[0]); }
__device__ __forceinline__ void from_words(const uint64_t *w, double &v)
{
    v = __longlong_as_double((long long)(((uint64_t)(uint32_t)w[1] << 32) | (uint32_t)w[0]));
}

// Materialises a value in every lane: keeps the compiler from sinking an LDS
// read into a divergent branch (exec-masked branches cost more than the read).
__device__ __forceinline__ void keep(float &x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void keep(double &x) { asm volatile("" : "+v"(x)); }

__device__ __forceinline__ double wave_sum(double v)
{
    // fixed butterfly order: the result does not depend on timing
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Halo words polled by the recurrence wave: NWORDS per side.
template <int NWORDS>
struct Halo {
    uint64_t a[NWORDS];
    uint64_t b[NWORDS];
};

// Every lane loads its words unconditionally: lanes that need no halo point
// at a dummy word.  Keeping the poll loads free of control flow lets the
// compiler count them exactly (s_waitcnt vmcnt(N)) instead of draining all
// prefetched polls at every step.
template <int NWORDS>
__device__ __forceinline__ void halo_issue(Halo<NWORDS> &h, const GLOBAL uint64_t *pa, const GLOBAL uint64_t *pb)
{
#pragma unroll
    for (int w = 0; w < NWORDS; w++) {
        h.a[w] = ll_load(pa + w);
        h.b[w] = ll_load(pb + w);
    }
}

template <int NWORDS>
__device__ __forceinline__ bool halo_ok(const Halo<NWORDS> &h, bool na, bool nb, uint32_t tag)
{
    bool ok = true;
#pragma unroll
    for (int w = 0; w < NWORDS; w++) {
        if (na && (uint32_t)(h.a[w] >> 32) != tag) ok = false;
        if (nb && (uint32_t)(h.b[w] >> 32) != tag) ok = false;
    }
    return ok;
}

// Re-poll until every lane's needed words carry `tag`.  Returns false if the
// wait timed out or another workgroup raised the error flag.
template <int NWORDS>
__device__ __forceinline__ bool halo_wait(Halo<NWORDS> &h, bool na, const GLOBAL uint64_t *pa, bool nb, const GLOBAL uint64_t *pb,
                          uint32_t tag, GLOBAL Ctl *ctl, uint64_t timeout)
{
    if (!__any(!halo_ok(h, na, nb, tag))) return true;
    const uint64_t t0 = wall_clock64();
    for (;;) {
        halo_issue(h, pa, pb);
        if (!__any(!halo_ok(h, na, nb, tag))) return true;
        if (__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1u) return false;
        if (wall_clock64() - t0 > timeout) {
            __hip_atomic_fetch_or(&ctl->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Per-lane view of the tile a workgroup owns.
struct TileView {
    int t, ti, tj, ip, jp, gi, gj;
    bool in_ij;                 // (i, j) inside the block
    long long base;             // sheared index of (plane 0, this lane) in this tile
    __device__ bool active(int s, int nk) const
    {
        const int k = s - ip - jp;
        return in_ij && (unsigned)k < (unsigned)nk;
    }
};

__device__ __forceinline__ TileView make_view(const Geom &g, int t, int lane)
{
    TileView v;
    v.t = t;
    v.ti = t % g.nti;
    v.tj = t / g.nti;
    v.ip = lane % TI;
    v.jp = lane / TI;
    v.gi = v.ti * TI + v.ip;
    v.gj = v.tj * TJ + v.jp;
    v.in_ij = v.gi < g.ni && v.gj < g.nj;
    v.base = (long long)t * g.tile_elems + TT + lane;
    return v;
}

// Workgroup prologue: take a ticket.  Returns the job index (or -1 if the
// job is already stopped) and the tile in *tile.
struct Assign {
    int job, tile;
};

__device__ Assign take_ticket(const LaunchArgs &a, int *s_buf)
{
    if (threadIdx.x == 0) {
        const uint32_t tk = atomicAdd(&a.lc->ticket, 1u);
        const int2 o = a.order[tk];
        s_buf[0] = o.x;
        s_buf[1] = o.y;
    }
    __syncthreads();
    Assign r;
    r.job = __builtin_amdgcn_readfirstlane(s_buf[0]);
    r.tile = __builtin_amdgcn_readfirstlane(s_buf[1]);
    return r;
}

// Launch epilogue: the last workgroup of the launch resets the counters.
__device__ void launch_done(const LaunchArgs &a)
{
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(&a.lc->done, 1u);
        if (prev == (uint32_t)a.total - 1u) {
            a.lc->ticket = 0u;
            a.lc->done = 0u;
        }
    }
}

// Job epilogue: returns true (uniformly) in the workgroup that finished last.
__device__ bool job_last(const Job &J, int *s_buf)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(&J.ctl->done, 1u);
        s_buf[2] = (prev == (uint32_t)J.g.ntiles - 1u) ? 1 : 0;
    }
    __syncthreads();
    const bool last = __builtin_amdgcn_readfirstlane(s_buf[2]) != 0;
    if (last) __threadfence();
    return last;
}

__device__ __forceinline__ int padded_intervals(int steps)
{
    // intervals: fill f = u, recurrence s = u - 1, post p = u - 2
    const int u = steps + 2;
    return (u + LP - 1) / LP * LP;
}

// ------------------------------------------------------ sweeps
// Workgroup = one recurrence wave (wave 0) + NL loader waves.  Loader wave l
// owns the steps f with f % NL == l: at its turn (interval f) it consumes the
// loads it issued NL intervals earlier, stages the operands of step f in the
// LDS ring and issues the loads of step f + NL.  Its own vector-memory wait at
// a turn therefore only covers loads that had NL intervals to arrive.
// Interval u: loaders fill step u, the recurrence wave processes step u - 1
// and publishes its face words (and, forward, y) at once, so the neighbour
// tiles see them without waiting for a loader turn; one workgroup barrier
// ends every interval.  Backward, the owning loader applies x += d of step
// u - 2.

// Face records.  At every step a tile publishes the 16 face entries its
// downstream neighbours read (entry e < TJ: row e of the column facing the i
// neighbour; entry TJ + c: column c of the row facing the j neighbour), NV
// words each.  The recurrence wave writes the whole record with one store in
// which every lane writes a word (the 64 lanes cover the 16 NV words 64 / (16
// NV) times over, with identical data), taking the value from the LDS copy
// of the step it has just written.  With no store behind a branch the
// compiler's vector-memory counts stay exact, and the wait for a prefetched
// poll never waits for a later store.  Steps past the last one write the
// tile's sink words.
struct Post {
    uint32_t rec;    // word index of this lane's word in the tile's record at step 0
    uint32_t sink;   // word index of this lane's word in the tile's sink
    int src;         // lane whose value this lane's word carries
    int half;        // which 32-bit half of that value (FP64)
};

template <int NV>
__device__ __forceinline__ Post make_post(const Geom &g, const TileView &v, long long fstride, int lane, int col_i, int row_j)
{
    Post p;
    const int word = lane & (16 * NV - 1);
    const int e = word / NV;
    p.half = word % NV;
    p.src = e < TJ ? e * TI + col_i : row_j * TI + (e - TJ);
    p.rec = (uint32_t)v.t * (uint32_t)fstride + (uint32_t)word;
    p.sink = (uint32_t)g.ntiles * (uint32_t)fstride + (uint32_t)v.t * SINK_WORDS + (uint32_t)word;
    return p;
}

template <int NV, typename F>
__device__ __forceinline__ void post_record(GLOBAL uint64_t *fbase, const Post &p, int s, int steps, int fw, uint32_t tag, F val)
{
    uint32_t wd[NV];
    to_words(val, wd);
    uint32_t w = wd[0];
#pragma unroll
    for (int q = 1; q < NV; q++) w = p.half == q ? wd[q] : w;
    ll_store(fbase + (s < steps ? p.rec + (uint32_t)s * (uint32_t)fw : p.sink), tag, w);
}

__device__ __forceinline__ int sweep_intervals(int steps, int pd)
{
    // interval 0 (fill only) plus the recurrence steps 0..steps (step `steps`
    // only lets the last backward x update happen), padded to the poll unroll
    return 1 + (steps + 1 + pd - 1) / pd * pd;
}

// Forward: residual r = b - A x (FP64, fused), forward substitution
// y = (r - Lb y_B - Lw y_W - Ls y_S) / Lp in precision F, per-tile partial
// sums of r^2 (and of b^2, used at iteration 0).

template <typename F>
struct FwdLoad {
    double a[7];
    double b;
    double xt;     // x on plane f + 1 (this lane's T neighbour), staged into the LDS plane ring
    double hx;     // x across the W or E tile edge (edge lanes only)
    double hy;     // x across the S or N tile edge (edge lanes only)
    F l[4];        // Lb, Lw, Ls, 1/Lp
};

// Load through a uniform base pointer and a 32-bit element index (the host
// guarantees every array stays below 4 GiB), which maps onto the
// saddr + voffset form of global_load.
template <typename T>
__device__ __forceinline__ T ldg(const GLOBAL T *base, uint32_t idx)
{
    return *(const GLOBAL T *)((const GLOBAL char *)base + (size_t)(idx * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void stg(GLOBAL T *base, uint32_t idx, T v)
{
    *(GLOBAL T *)((GLOBAL char *)base + (size_t)(idx * (uint32_t)sizeof(T))) = v;
}

// Uniform base pointers and per-lane index deltas of the forward loader.
template <typename F>
struct FwdSrc {
    const GLOBAL double *A[7];
    const GLOBAL double *b, *x;
    const GLOBAL F *L[4];
    uint32_t e0;          // sheared index of (plane 0, this lane)
    int32_t hx, hy;       // index deltas of the x halo this lane reads across a tile edge (0: none)
};

template <typename F>
__device__ __forceinline__ FwdSrc<F> fwd_src(const Job &J, const TileView &v)
{
    const Geom &g = J.g;
    FwdSrc<F> q;
#pragma unroll
    for (int d = 0; d < 7; d++) q.A[d] = gp(J.A) + d * g.elems;
    q.b = gp(J.b);
    q.x = gp((const double *)J.x);
#pragma unroll
    for (int d = 0; d < 4; d++) q.L[d] = gp((const F *)J.LU) + d * g.elems;
    q.e0 = (uint32_t)v.base;
    const int te = (int)g.tile_elems;
    // Across a tile edge the neighbour is the neighbour tile's edge column/row
    // on that tile's own local plane: W at plane f+TI-1, E at f-TI+1, S at
    // f+TJ-1, N at f-TJ+1.  A lane sits on at most one of the W/E edges and
    // one of the S/N edges, so two loads cover every halo; in-tile
    // neighbours come from the LDS plane ring.
    q.hx = (v.ip == 0 && v.ti > 0) ? -te + (TI - 1) * TT + (TI - 1)
         : (v.ip == TI - 1 && v.ti < g.nti - 1) ? te - (TI - 1) * TT - (TI - 1) : 0;
    q.hy = (v.jp == 0 && v.tj > 0) ? -g.nti * te + (TJ - 1) * TT + (TJ - 1) * TI
         : (v.jp == TJ - 1 && v.tj < g.ntj - 1) ? g.nti * te - (TJ - 1) * TT - (TJ - 1) * TI : 0;
    return q;
}

// Branch-free: inactive lanes read their own zero-padded slot (every index
// stays inside the tile's planes -1..steps for f in [0, steps)).
template <typename F>
__device__ __forceinline__ void fwd_issue(FwdLoad<F> &c, const FwdSrc<F> &q, const TileView &v, int f, int nk)
{
    const bool act = v.active(f, nk);
    const uint32_t e = q.e0 + (uint32_t)f * TT;
#pragma unroll
    for (int d = 0; d < 7; d++) c.a[d] = ldg(q.A[d], e);
    c.b = ldg(q.b, e);
#pragma unroll
    for (int d = 0; d < 4; d++) c.l[d] = ldg(q.L[d], e);
    c.xt = ldg(q.x, e + TT);
    c.hx = ldg(q.x, e + (act ? q.hx : 0));
    c.hy = ldg(q.x, e + (act ? q.hy : 0));
}

template <typename F, int NL, int PD>
__global__ __launch_bounds__(WAVE *(1 + NL)) void k_forward(LaunchArgs a)
{
    constexpr int NV = NW<F>::n;
    __shared__ F ring[2][5][TT];     // r, Lb, Lw, Ls, 1/Lp of two steps
    __shared__ F ybuf[2][TT];
    __shared__ double xring[4][TT];  // x on planes f-1, f, f+1 (slot = plane & 3)
    __shared__ int s_buf[4];
    __shared__ double s_part[NL][2];

    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    if (threadIdx.x == 0) s_buf[3] = 0;
    const Assign as = take_ticket(a, s_buf);
    const Job J = load_job(a, as.job);
    const uint32_t stop = J.ctl->stop;
    if (stop != RUN) {
        launch_done(a);
        return;
    }
    const uint32_t tag = J.ctl->epoch;
    const uint32_t iter = J.ctl->iter;
    const Geom g = J.g;
    const TileView v = make_view(g, as.tile, lane);
    const int U = sweep_intervals(g.steps, PD);
    const int FW = J.fw;
    const long long fstride = (long long)g.steps * FW;
    GLOBAL Ctl *ctl = gp(J.ctl);

    ybuf[0][lane] = F(0);
    ybuf[1][lane] = F(0);
    __syncthreads();

    if (wave == 0) {
        // ---------------- recurrence wave
        // Poll addresses are word indices from one uniform base, chosen with
        // selects: lanes without a halo read their own tile's first word.
        // Everything in the step stays free of divergent branches.
        GLOBAL uint64_t *fbase = gp(J.face);
        const uint32_t own = (uint32_t)v.t * (uint32_t)fstride;
        const uint32_t baseW = (uint32_t)(v.t - 1) * (uint32_t)fstride + (uint32_t)((TI - 1) * FW + v.jp * NV);
        const uint32_t baseS = (uint32_t)(v.t - g.nti) * (uint32_t)fstride + (uint32_t)((TJ - 1) * FW + (TJ + v.ip) * NV);
        const bool edgeW = v.ip == 0 && v.ti > 0, edgeS = v.jp == 0 && v.tj > 0;
        GLOBAL F *yout = gp((F *)J.y);
        const uint32_t e0 = (uint32_t)v.base;
        const Post post = make_post<NV>(g, v, fstride, lane, TI - 1, TJ - 1);   // E column, N row
        Halo<NV> pv[PD];
        bool needW[PD], needS[PD];
        const GLOBAL uint64_t *pW[PD], *pS[PD];
        auto plan = [&](int q, int s2) {
            const bool act = v.active(s2, g.nk);
            needW[q] = act && edgeW;
            needS[q] = act && edgeS;
            pW[q] = fbase + (needW[q] ? baseW + (uint32_t)s2 * FW : own);
            pS[q] = fbase + (needS[q] ? baseS + (uint32_t)s2 * FW : own);
            halo_issue(pv[q], pW[q], pS[q]);
        };
        // The prologue repeats a step's store pattern (zero margin, sink) ahead
        // of each poll, so the loop is entered with the same counts as it
        // loops back with.
#pragma unroll
        for (int q = 0; q < PD; q++) {
            stg(yout, e0 + (uint32_t)g.steps * TT, F(0));
            post_record<NV>(fbase, post, g.steps, g.steps, FW, tag, F(0));
            plan(q, q);
        }
        F yB = F(0);
        bool aborted = false;
        wg_barrier();   // interval 0: the loaders stage step 0
        for (int s0 = 0; s0 + 1 < U; s0 += PD) {
#pragma unroll
            for (int q = 0; q < PD; q++) {
                const int s = s0 + q;
                const int slot = s & 1;
                const F r = ring[slot][0][lane];
                const F lb = ring[slot][1][lane];
                const F lw = ring[slot][2][lane];
                const F ls = ring[slot][3][lane];
                const F ilp = ring[slot][4][lane];
                if (!aborted && !halo_wait(pv[q], needW[q], pW[q], needS[q], pS[q], tag, ctl, a.timeout_ticks))
                    aborted = true;
                F hw, hs;
                from_words(pv[q].a, hw);
                from_words(pv[q].b, hs);
                const int pr = (s - 1) & 1;
                F nW = ybuf[pr][lane - (v.ip > 0 ? 1 : 0)];
                F nS = ybuf[pr][lane - (v.jp > 0 ? TI : 0)];
                keep(nW);
                keep(nS);
                const F yW = v.ip > 0 ? nW : (needW[q] ? hw : F(0));
                const F yS = v.jp > 0 ? nS : (needS[q] ? hs : F(0));
                const bool act = v.active(s, g.nk);
                F t = r - lb * yB;
                t = t - lw * yW;
                t = t - ls * yS;
                const F y = act ? t * ilp : F(0);
                yB = y;
                ybuf[s & 1][lane] = y;
                // publish at once (the neighbour tiles' next steps wait on
                // these words); past the last step y lands in the zero margin
                stg(yout, e0 + (uint32_t)min(s, g.steps) * TT, y);   // inactive lanes rewrite their zero padding
                post_record<NV>(fbase, post, s, g.steps, FW, tag, ybuf[s & 1][post.src]);
                plan(q, s + PD);
                if (q == PD - 1 && aborted) s_buf[3] = 1;   // read by every wave after this barrier
                wg_barrier();
            }
            if (s_buf[3]) break;
        }
    } else {
        // ---------------- loader waves
        const int lw = wave - 1;
        const FwdSrc<F> src = fwd_src<F>(J, v);
        FwdLoad<F> c;
        if (lw == 0) {   // planes -1 (zero margin) and 0 of the x ring
            xring[3][lane] = 0.0;
            xring[0][lane] = ldg(src.x, src.e0);
        }
        if (lw < g.steps) fwd_issue(c, src, v, lw, g.nk);
        double rr = 0.0, bb = 0.0;
        auto turn = [&](int u) {
            const int f = u;
            if (f < g.steps) {
                // planes f-1 and f were staged by the two previous turns
                xring[(f + 1) & 3][lane] = c.xt;
                const double xP = xring[f & 3][lane];
                const double xB = xring[(f - 1) & 3][lane];
                const double xW = v.ip > 0 ? xring[(f - 1) & 3][lane - (v.ip > 0 ? 1 : 0)] : c.hx;
                const double xE = v.ip < TI - 1 ? xring[(f + 1) & 3][lane + (v.ip < TI - 1 ? 1 : 0)] : c.hx;
                const double xS = v.jp > 0 ? xring[(f - 1) & 3][lane - (v.jp > 0 ? TI : 0)] : c.hy;
                const double xN = v.jp < TJ - 1 ? xring[(f + 1) & 3][lane + (v.jp < TJ - 1 ? TI : 0)] : c.hy;
                const double ax = c.a[0] * xP + c.a[1] * xW + c.a[2] * xE + c.a[3] * xS + c.a[4] * xN +
                                  c.a[5] * xB + c.a[6] * c.xt;
                const double r = c.b - ax;
                rr += r * r;
                bb += c.b * c.b;
                const int slot = f & 1;
                ring[slot][0][lane] = (F)r;
                ring[slot][1][lane] = c.l[0];
                ring[slot][2][lane] = c.l[1];
                ring[slot][3][lane] = c.l[2];
                ring[slot][4][lane] = c.l[3];
            }
            if (u + NL < g.steps) fwd_issue(c, src, v, u + NL, g.nk);
        };
        if (lw == 0) turn(0);
        wg_barrier();
        for (int s0 = 0; s0 + 1 < U; s0 += PD) {
            for (int q = 0; q < PD; q++) {
                const int u = s0 + q + 1;
                if (u % NL == lw) turn(u);
                wg_barrier();
            }
            if (s_buf[3]) break;
        }
        rr = wave_sum(rr);
        bb = wave_sum(bb);
        if (lane == 0) {
            s_part[lw][0] = rr;
            s_part[lw][1] = bb;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sr = 0.0, sb = 0.0;
        for (int l = 0; l < NL; l++) {
            sr += s_part[l][0];
            sb += s_part[l][1];
        }
        gp(J.part)[2 * v.t] = sr;
        gp(J.part)[2 * v.t + 1] = sb;
    }

    if (job_last(J, s_buf) && wave == 0) {
        double sr = 0.0, sb = 0.0;
        for (int t = lane; t < g.ntiles; t += WAVE) {
            sr += J.part[2 * t];
            sb += J.part[2 * t + 1];
        }
        sr = wave_sum(sr);
        sb = wave_sum(sb);
        if (lane == 0) {
            Ctl *c = J.ctl;
            if (iter == 0) c->bnorm2 = sb;
            const double nb2 = iter == 0 ? sb : c->bnorm2;
            uint32_t st = RUN;
            const uint32_t err = c->err;
            if (err) {
                st = (err & 2u) ? BREAKDOWN : TIMEOUT;
            } else if (nb2 == 0.0) {
                st = ZERO_RHS;
                c->rho = 0.0;
                if (J.hist) J.hist[iter] = 0.0;
            } else {
                const double rho = sqrt(sr) / sqrt(nb2);
                c->rho = rho;
                if (J.hist) J.hist[iter] = rho;
                if (c->rtol > 0.0 && rho <= c->rtol) st = CONVERGED;
                else if (iter >= c->max_iter) st = MAXITER;
            }
            c->stop = st;
            c->epoch = tag + 1u;
            c->done = 0u;
        }
    }
    launch_done(a);
}

// Backward: d = y - Un d_N - Ue d_E - Ut d_T in reverse local-hyperplane
// order (step s visits plane steps - 1 - s), then x += d in FP64.

template <typename F>
struct BwdLoad {
    F y, u[3];   // y, Un, Ue, Ut
    double x;
};

template <typename F>
struct BwdSrc {
    const GLOBAL F *y;
    const GLOBAL F *U[3];
    GLOBAL double *x;
    uint32_t e0;
};

template <typename F>
__device__ __forceinline__ void bwd_issue(BwdLoad<F> &c, const BwdSrc<F> &q, int steps, int step)
{
    const uint32_t e = q.e0 + (uint32_t)(steps - 1 - step) * TT;
    c.y = ldg(q.y, e);
#pragma unroll
    for (int d = 0; d < 3; d++) c.u[d] = ldg(q.U[d], e);
    c.x = ldg((const GLOBAL double *)q.x, e);
}

template <typename F, int NL, int PD>
__global__ __launch_bounds__(WAVE *(1 + NL)) void k_backward(LaunchArgs a)
{
    constexpr int NV = NW<F>::n;
    __shared__ F ring[2][4][TT];     // y, Un, Ue, Ut
    __shared__ double xring[4][TT];
    __shared__ F dbuf[2][TT];
    __shared__ int s_buf[4];

    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    if (threadIdx.x == 0) s_buf[3] = 0;
    const Assign as = take_ticket(a, s_buf);
    const Job J = load_job(a, as.job);
    const uint32_t stop = J.ctl->stop;
    if (stop != RUN) {
        launch_done(a);
        return;
    }
    const uint32_t tag = J.ctl->epoch;
    const Geom g = J.g;
    const TileView v = make_view(g, as.tile, lane);
    const int U = sweep_intervals(g.steps, PD);
    const int FW = J.fw;
    const long long fstride = (long long)g.steps * FW;
    GLOBAL Ctl *ctl = gp(J.ctl);

    dbuf[0][lane] = F(0);
    dbuf[1][lane] = F(0);
    __syncthreads();

    if (wave == 0) {
        GLOBAL uint64_t *fbase = gp(J.face);
        const uint32_t own = (uint32_t)v.t * (uint32_t)fstride;
        const uint32_t baseE = (uint32_t)(v.t + 1) * (uint32_t)fstride + (uint32_t)((TI - 1) * FW + v.jp * NV);
        const uint32_t baseN = (uint32_t)(v.t + g.nti) * (uint32_t)fstride + (uint32_t)((TJ - 1) * FW + (TJ + v.ip) * NV);
        const bool edgeE = v.ip == TI - 1 && v.ti < g.nti - 1, edgeN = v.jp == TJ - 1 && v.tj < g.ntj - 1;
        const Post post = make_post<NV>(g, v, fstride, lane, 0, 0);   // W column, S row
        Halo<NV> pv[PD];
        bool needE[PD], needN[PD];
        const GLOBAL uint64_t *pE[PD], *pN[PD];
        auto plan = [&](int q, int s2) {   // s2: backward step
            const bool act = s2 < g.steps && v.active(g.steps - 1 - s2, g.nk);
            needE[q] = act && edgeE;
            needN[q] = act && edgeN;
            pE[q] = fbase + (needE[q] ? baseE + (uint32_t)s2 * FW : own);
            pN[q] = fbase + (needN[q] ? baseN + (uint32_t)s2 * FW : own);
            halo_issue(pv[q], pE[q], pN[q]);
        };
#pragma unroll
        for (int q = 0; q < PD; q++) {   // same store pattern as a step (sink only)
            post_record<NV>(fbase, post, g.steps, g.steps, FW, tag, F(0));
            plan(q, q);
        }
        F dT = F(0);
        bool aborted = false;
        wg_barrier();
        for (int s0 = 0; s0 + 1 < U; s0 += PD) {
#pragma unroll
            for (int q = 0; q < PD; q++) {
                const int s = s0 + q;
                const int slot = s & 1;
                const F yv = ring[slot][0][lane];
                const F un = ring[slot][1][lane];
                const F ue = ring[slot][2][lane];
                const F ut = ring[slot][3][lane];
                if (!aborted && !halo_wait(pv[q], needE[q], pE[q], needN[q], pN[q], tag, ctl, a.timeout_ticks))
                    aborted = true;
                F he, hn;
                from_words(pv[q].a, he);
                from_words(pv[q].b, hn);
                const int pr = (s - 1) & 1;
                F nE = dbuf[pr][lane + (v.ip < TI - 1 ? 1 : 0)];
                F nN = dbuf[pr][lane + (v.jp < TJ - 1 ? TI : 0)];
                keep(nE);
                keep(nN);
                const F dE = v.ip < TI - 1 ? nE : (needE[q] ? he : F(0));
                const F dN = v.jp < TJ - 1 ? nN : (needN[q] ? hn : F(0));
                const bool act = s < g.steps && v.active(g.steps - 1 - s, g.nk);
                F t = yv - un * dN;
                t = t - ue * dE;
                t = t - ut * dT;
                const F d = act ? t : F(0);
                dT = d;
                dbuf[s & 1][lane] = d;
                post_record<NV>(fbase, post, s, g.steps, FW, tag, dbuf[s & 1][post.src]);
                plan(q, s + PD);
                if (q == PD - 1 && aborted) s_buf[3] = 1;
                wg_barrier();
            }
            if (s_buf[3]) break;
        }
    } else {
        const int lw = wave - 1;
        BwdSrc<F> src;
        src.y = gp((const F *)J.y);
#pragma unroll
        for (int d = 0; d < 3; d++) src.U[d] = gp((const F *)J.LU) + (4 + d) * g.elems;
        src.x = gp(J.x);
        src.e0 = (uint32_t)v.base;
        BwdLoad<F> c;
        if (lw < g.steps) bwd_issue(c, src, g.steps, lw);
        auto turn = [&](int u) {
            const int f = u;
            if (f < g.steps) {
                const int slot = f & 1;
                ring[slot][0][lane] = c.y;
                ring[slot][1][lane] = c.u[0];
                ring[slot][2][lane] = c.u[1];
                ring[slot][3][lane] = c.u[2];
                xring[f & 3][lane] = c.x;
            }
            // Issue the next loads before the x store: a load of x behind a
            // store to x would wait for the store to complete.
            if (u + NL < g.steps) bwd_issue(c, src, g.steps, u + NL);
            const int p = u - 2;
            if (p >= 0 && p < g.steps) {
                const int sp = g.steps - 1 - p;
                const F d = dbuf[p & 1][lane];
                const double xv = xring[p & 3][lane];
                stg(src.x, src.e0 + (uint32_t)sp * TT, xv + (double)d);   // padding: 0 + 0
            }
        };
        if (lw == 0) turn(0);
        wg_barrier();
        for (int s0 = 0; s0 + 1 < U; s0 += PD) {
            for (int q = 0; q < PD; q++) {
                const int u = s0 + q + 1;
                if (u % NL == lw) turn(u);
                wg_barrier();
            }
            if (s_buf[3]) break;
        }
    }

    if (job_last(J, s_buf) && wave == 0 && lane == 0) {
        Ctl *c = J.ctl;
        if (c->err) c->stop = (c->err & 2u) ? BREAKDOWN : TIMEOUT;
        c->iter = c->iter + 1u;
        c->epoch = tag + 1u;
        c->done = 0u;
    }
    launch_done(a);
}

// ------------------------------------------------------ factorisation
// Stone's factorisation in local-hyperplane order.  Per cell, with X_B the
// value at the B neighbour:
//   Lb = A_B / (1 + a (Un_B + Ue_B)),  Lw = A_W / (1 + a (Un_W + Ut_W)),
//   Ls = A_S / (1 + a (Ue_S + Ut_S)),
//   P1 = a (Lb Un_B + Lw Un_W), P2 = a (Ls Ue_S + Lb Ue_B), P3 = a (Ls Ut_S + Lw Ut_W),
//   Lp = A_P + P1 + P2 + P3 - Lb Ut_B - Lw Ue_W - Ls Un_S,
//   Un = (A_N - P1) / Lp, Ue = (A_E - P2) / Lp, Ut = (A_T - P3) / Lp.
// Computed in FP64; stored as F (the mixed form rounds the FP64 factors).

template <typename F>
__global__ __launch_bounds__(BLOCK) void k_factor(LaunchArgs a)
{
    constexpr int NV = 6;   // 3 FP64 values per face entry
    __shared__ double ring[2][7][TT];
    __shared__ double ubuf[2][3][TT];
    __shared__ double obuf[2][4][TT];
    __shared__ int s_buf[4];

    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    if (threadIdx.x == 0) s_buf[3] = 0;
    const Assign as = take_ticket(a, s_buf);
    const Job J = load_job(a, as.job);
    const uint32_t stop = J.ctl->stop;
    if (stop != RUN) {
        launch_done(a);
        return;
    }
    const uint32_t tag = J.ctl->epoch;
    const Geom g = J.g;
    const double alpha = J.alpha;
    const TileView v = make_view(g, as.tile, lane);
    const int U = padded_intervals(g.steps);
    const int FW = J.fw;
    const long long fstride = (long long)g.steps * FW;
    GLOBAL uint64_t *face_t = gp(J.face) + (long long)v.t * fstride;
    GLOBAL Ctl *ctl = gp(J.ctl);

#pragma unroll
    for (int d = 0; d < 3; d++) {
        ubuf[0][d][lane] = 0.0;
        ubuf[1][d][lane] = 0.0;
    }
    __syncthreads();

    if (wave == 0) {
        const GLOBAL uint64_t *faceW = v.ti > 0 ? gp(J.face) + (long long)(v.t - 1) * fstride : face_t;
        const GLOBAL uint64_t *faceS = v.tj > 0 ? gp(J.face) + (long long)(v.t - g.nti) * fstride : face_t;
        double unB = 0.0, ueB = 0.0, utB = 0.0;
        bool aborted = false, broke = false;
        for (int u0 = 0; u0 < U; u0 += LP) {
#pragma unroll
            for (int w = 0; w < LP; w++) {
                const int u = u0 + w;
                const int s = u - 1;
                if (s >= 0 && s < g.steps && !aborted) {
                    const bool act = v.active(s, g.nk);
                    const bool nW = act && v.ip == 0 && v.ti > 0;
                    const bool nS = act && v.jp == 0 && v.tj > 0;
                    const GLOBAL uint64_t *pW = nW ? faceW + (long long)(s + TI - 1) * FW + v.jp * NV : face_t;
                    const GLOBAL uint64_t *pS = nS ? faceS + (long long)(s + TJ - 1) * FW + (TJ + v.ip) * NV : face_t;
                    Halo<NV> h;
                    halo_issue(h, pW, pS);
                    if (!halo_wait(h, nW, pW, nS, pS, tag, ctl, a.timeout_ticks)) {
                        aborted = true;
                    }
                    double hw[3], hs[3];
#pragma unroll
                    for (int d = 0; d < 3; d++) {
                        from_words(&h.a[2 * d], hw[d]);
                        from_words(&h.b[2 * d], hs[d]);
                        if (!nW) hw[d] = 0.0;
                        if (!nS) hs[d] = 0.0;
                    }
                    const int pr = (s - 1) & 1;
                    const int lw_ = lane - (v.ip > 0 ? 1 : 0);
                    const int ls_ = lane - (v.jp > 0 ? TI : 0);
                    const double unW = v.ip > 0 ? ubuf[pr][0][lw_] : hw[0];
                    const double ueW = v.ip > 0 ? ubuf[pr][1][lw_] : hw[1];
                    const double utW = v.ip > 0 ? ubuf[pr][2][lw_] : hw[2];
                    const double unS = v.jp > 0 ? ubuf[pr][0][ls_] : hs[0];
                    const double ueS = v.jp > 0 ? ubuf[pr][1][ls_] : hs[1];
                    const double utS = v.jp > 0 ? ubuf[pr][2][ls_] : hs[2];
                    const int slot = s & 1;
                    const double aP = ring[slot][0][lane], aW = ring[slot][1][lane], aE = ring[slot][2][lane];
                    const double aS = ring[slot][3][lane], aN = ring[slot][4][lane], aB = ring[slot][5][lane];
                    const double aT = ring[slot][6][lane];
                    double lb = 0, lw = 0, ls = 0, ilp = 0, un = 0, ue = 0, ut = 0;
                    if (act) {
                        const double denB = 1.0 + alpha * (unB + ueB);
                        const double denW = 1.0 + alpha * (unW + utW);
                        const double denS = 1.0 + alpha * (ueS + utS);
                        lb = aB / denB;
                        lw = aW / denW;
                        ls = aS / denS;
                        const double p1 = alpha * (lb * unB + lw * unW);
                        const double p2 = alpha * (ls * ueS + lb * ueB);
                        const double p3 = alpha * (ls * utS + lw * utW);
                        const double lp = aP + p1 + p2 + p3 - lb * utB - lw * ueW - ls * unS;
                        if (denB == 0.0 || denW == 0.0 || denS == 0.0 || lp == 0.0 || !isfinite(lp)) broke = true;
                        ilp = 1.0 / lp;
                        un = (aN - p1) / lp;
                        ue = (aE - p2) / lp;
                        ut = (aT - p3) / lp;
                    }
                    unB = un;
                    ueB = ue;
                    utB = ut;
                    ubuf[s & 1][0][lane] = un;
                    ubuf[s & 1][1][lane] = ue;
                    ubuf[s & 1][2][lane] = ut;
                    obuf[s & 1][0][lane] = lb;
                    obuf[s & 1][1][lane] = lw;
                    obuf[s & 1][2][lane] = ls;
                    obuf[s & 1][3][lane] = ilp;
                }
                if (w == LP - 1 && aborted) s_buf[3] = 1;   // read by both waves after this barrier
                wg_barrier();
            }
            if (s_buf[3]) break;
        }
        if (__any(broke) && lane == 0)
            __hip_atomic_fetch_or(&ctl->err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        double pipe[LP][7];
        auto issue = [&](double *c, int f) {
            const bool act = f < g.steps && v.active(f, g.nk);
            const long long e = v.base + (long long)f * TT;
#pragma unroll
            for (int d = 0; d < 7; d++) c[d] = act ? gp(J.A)[d * g.elems + e] : 0.0;
        };
#pragma unroll
        for (int q = 0; q < LP; q++) issue(pipe[q], q);
        GLOBAL F *LU = gp((F *)J.LU);
        for (int u0 = 0; u0 < U; u0 += LP) {
#pragma unroll
            for (int w = 0; w < LP; w++) {
                const int u = u0 + w;
                const int p = u - 2;
                if (p >= 0 && p < g.steps) {
                    const long long e = v.base + (long long)p * TT;
                    const int sl = p & 1;
                    if (v.active(p, g.nk)) {
#pragma unroll
                        for (int d = 0; d < 4; d++) LU[d * g.elems + e] = (F)obuf[sl][d][lane];
#pragma unroll
                        for (int d = 0; d < 3; d++) LU[(4 + d) * g.elems + e] = (F)ubuf[sl][d][lane];
                    }
                    uint32_t wd[6];
#pragma unroll
                    for (int d = 0; d < 3; d++) to_words(ubuf[sl][d][lane], &wd[2 * d]);
                    if (v.ip == TI - 1) {
#pragma unroll
                        for (int q = 0; q < 6; q++) ll_store(face_t + (long long)p * FW + v.jp * NV + q, tag, wd[q]);
                    }
                    if (v.jp == TJ - 1) {
#pragma unroll
                        for (int q = 0; q < 6; q++)
                            ll_store(face_t + (long long)p * FW + (TJ + v.ip) * NV + q, tag, wd[q]);
                    }
                }
                const int f = u;
                if (f < g.steps) {
                    const int slot = f & 1;
#pragma unroll
                    for (int d = 0; d < 7; d++) ring[slot][d][lane] = pipe[w][d];
                    issue(pipe[w], f + LP);
                }
                wg_barrier();
            }
            if (s_buf[3]) break;
        }
    }

    if (job_last(J, s_buf) && wave == 0 && lane == 0) {
        Ctl *c = J.ctl;
        if (c->err) c->stop = (c->err & 2u) ? BREAKDOWN : TIMEOUT;
        c->epoch = tag + 1u;
        c->done = 0u;
    }
    launch_done(a);
}

// ------------------------------------------------------ layout kernels

struct SrcPtrs {
    const double *p[9];
};
struct DstPtrs {
    double *p[7];
};

__device__ __forceinline__ bool decode_sheared(const Geom &g, long long e, int &i, int &j, int &k)
{
    const int t = (int)(e / g.tile_elems);
    const long long rem = e - (long long)t * g.tile_elems;
    const int pl = (int)(rem / TT) - 1;
    const int ln = (int)(rem % TT);
    const int ip = ln % TI, jp = ln / TI;
    i = (t % g.nti) * TI + ip;
    j = (t / g.nti) * TJ + jp;
    k = pl - ip - jp;
    return pl >= 0 && pl < g.steps && i < g.ni && j < g.nj && k >= 0 && k < g.nk;
}

__device__ __forceinline__ long long sheared_index(const Geom &g, int i, int j, int k)
{
    const int ti = i / TI, tj = j / TJ, ip = i % TI, jp = j % TJ;
    const int t = tj * g.nti + ti;
    return (long long)t * g.tile_elems + (long long)(k + ip + jp + 1) * TT + jp * TI + ip;
}

__global__ void k_to_sheared(Geom g, int narr, SrcPtrs src, double *dst, long long dst_stride, int mask)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < g.elems; e += stride) {
        int i, j, k;
        const bool ok = decode_sheared(g, e, i, j, k);
        const long long n = ok ? ((long long)k * g.nj + j) * g.ni + i : 0;
        for (int a = 0; a < narr; a++) {
            double v = ok ? src.p[a][n] : 0.0;
            if (mask && ok) {
                // couplings that point out of the block are ignored
                if ((a == 1 && i == 0) || (a == 2 && i == g.ni - 1) || (a == 3 && j == 0) ||
                    (a == 4 && j == g.nj - 1) || (a == 5 && k == 0) || (a == 6 && k == g.nk - 1))
                    v = 0.0;
            }
            dst[a * dst_stride + e] = v;
        }
    }
}

__global__ void k_from_sheared(Geom g, const double *src, double *dst, const Ctl *ctl)
{
    const long long n = (long long)g.ni * g.nj * g.nk;
    const bool zero = ctl != nullptr && ctl->stop == ZERO_RHS;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n; c += stride) {
        const int i = (int)(c % g.ni);
        const int j = (int)((c / g.ni) % g.nj);
        const int k = (int)(c / ((long long)g.ni * g.nj));
        dst[c] = zero ? 0.0 : src[sheared_index(g, i, j, k)];
    }
}

template <typename F>
__global__ void k_export_factors(Geom g, const F *LU, DstPtrs out)
{
    const long long n = (long long)g.ni * g.nj * g.nk;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n; c += stride) {
        const int i = (int)(c % g.ni);
        const int j = (int)((c / g.ni) % g.nj);
        const int k = (int)(c / ((long long)g.ni * g.nj));
        const long long e = sheared_index(g, i, j, k);
#pragma unroll
        for (int d = 0; d < 7; d++) {
            const double v = (double)LU[d * g.elems + e];
            out.p[d][c] = (d == 3) ? 1.0 / v : v;
        }
    }
}

__global__ void k_init_ctl(Ctl *ctl, int n, uint32_t max_iter, double rtol, int reset_epoch)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    Ctl &c = ctl[q];
    c.done = 0u;
    if (reset_epoch) c.epoch = 1u;
    c.iter = 0u;
    c.max_iter = max_iter;
    c.stop = RUN;
    c.err = 0u;
    c.rtol = rtol;
    c.bnorm2 = 0.0;
    c.rho = 0.0;
}

int grid_for(long long n)
{
    long long b = (n + 255) / 256;
    if (b > 256 * 64) b = 256 * 64;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

hipError_t launch_init_ctl(Ctl *ctl, int n, uint32_t max_iter, double rtol, int reset_epoch, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_ctl, dim3((n + 63) / 64), dim3(64), 0, s, ctl, n, max_iter, rtol, reset_epoch);
    return hipGetLastError();
}

hipError_t launch_to_sheared(const Geom &g, int narr, const double *const *src, double *dst, long long dst_stride,
                             int mask_couplings, hipStream_t s)
{
    SrcPtrs sp{};
    for (int a = 0; a < narr && a < 9; a++) sp.p[a] = src[a];
    hipLaunchKernelGGL(k_to_sheared, dim3(grid_for(g.elems)), dim3(256), 0, s, g, narr, sp, dst, dst_stride,
                       mask_couplings);
    return hipGetLastError();
}

hipError_t launch_from_sheared_f64(const Geom &g, const double *src, double *dst, const Ctl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k_from_sheared, dim3(grid_for((long long)g.ni * g.nj * g.nk)), dim3(256), 0, s, g, src, dst,
                       ctl);
    return hipGetLastError();
}

hipError_t launch_export_factors(const Geom &g, const void *LU, int fp32, double *const *dst, hipStream_t s)
{
    DstPtrs dp{};
    for (int d = 0; d < 7; d++) dp.p[d] = dst[d];
    const dim3 grid(grid_for((long long)g.ni * g.nj * g.nk));
    if (fp32)
        hipLaunchKernelGGL(k_export_factors<float>, grid, dim3(256), 0, s, g, (const float *)LU, dp);
    else
        hipLaunchKernelGGL(k_export_factors<double>, grid, dim3(256), 0, s, g, (const double *)LU, dp);
    return hipGetLastError();
}

hipError_t launch_factor(const LaunchArgs &a, int fp32, hipStream_t s)
{
    if (fp32)
        hipLaunchKernelGGL(k_factor<float>, dim3(a.total), dim3(BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL(k_factor<double>, dim3(a.total), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <int NL, int PD>
static hipError_t launch_sweep_nl(const LaunchArgs &a, int fp32, int backward, hipStream_t s)
{
    const dim3 block(WAVE * (1 + NL));
    if (backward) {
        if (fp32)
            hipLaunchKernelGGL((k_backward<float, NL, PD>), dim3(a.total), block, 0, s, a);
        else
            hipLaunchKernelGGL((k_backward<double, NL, PD>), dim3(a.total), block, 0, s, a);
    } else {
        if (fp32)
            hipLaunchKernelGGL((k_forward<float, NL, PD>), dim3(a.total), block, 0, s, a);
        else
            hipLaunchKernelGGL((k_forward<double, NL, PD>), dim3(a.total), block, 0, s, a);
    }
    return hipGetLastError();
}

static hipError_t launch_sweep(const LaunchArgs &a, int fp32, int backward, const SweepPlan &p, hipStream_t s)
{
    switch (p.loaders) {
    case 2: return launch_sweep_nl<2, 4>(a, fp32, backward, s);
    case 4: return launch_sweep_nl<4, 4>(a, fp32, backward, s);
    case 6: return launch_sweep_nl<6, 4>(a, fp32, backward, s);
    case 8: return launch_sweep_nl<8, 4>(a, fp32, backward, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_forward(const LaunchArgs &a, int fp32, const SweepPlan &p, hipStream_t s)
{
    return launch_sweep(a, fp32, 0, p, s);
}

hipError_t launch_backward(const LaunchArgs &a, int fp32, const SweepPlan &p, hipStream_t s)
{
    return launch_sweep(a, fp32, 1, p, s);
}

}  // namespace sipk
