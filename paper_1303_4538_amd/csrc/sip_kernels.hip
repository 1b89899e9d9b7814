// gfx950 kernels of Stone's SIP: layout reorder, factorisation, fused
// residual + forward sweep, backward sweep + update.
//
// Every recurrence kernel is a pipeline over tile columns (see the layout in
// sip_internal.h).  One workgroup works one tile.  A "recurrence" wave walks
// the tile's local hyperplanes s = 0..steps-1; lane (i', j') handles its four
// cells (2 i' + a, 2 j' + b, k = s - i' - j') in dependency order.  Values of
// the neighbouring lanes from the previous step come through LDS; across the
// tile edge they come from the neighbour tile's face record in global memory.
// In the sweeps, "loader" waves stream coefficient / factor / vector planes
// from HBM a few steps ahead, do all work that does not depend on the
// recurrence (the residual, the update of x; FP64 except in the all-FP32
// arithmetic) and stage operands in an LDS ring.  Recurrence and loader
// waves meet at one workgroup barrier per step; the barrier waits on LDS
// traffic only, so loads stay in flight.
//
// The forward sweep's last workgroup of a job reduces the per-tile partial
// norms in tile order and takes the stop decision on the device (converged,
// iteration limit, zero right-hand side, non-finite input or residual).
//
// Face records: a value crossing a tile edge is written as 64-bit words
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
#include <type_traits>

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
    g.steps = nk + LI + LJ - 2;
    g.planes = g.steps + 2;
    g.tile_elems = (long long)g.planes * PLANE;
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
// The face-record prefetch distance of the recurrence wave (steps), PD, is a
// template parameter of the sweeps (SweepPlan::poll).

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
__device__ __forceinline__ bool halo_wait(Halo<NWORDS> &h, bool na, const GLOBAL uint64_t *pa, bool nb,
                                          const GLOBAL uint64_t *pb, uint32_t tag, GLOBAL Ctl *ctl, uint64_t timeout)
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
    int t, ti, tj, ip, jp;
    uint32_t inq;               // bit q: quadrant q's cell lies inside the block in (i, j)
    long long base;             // sheared index of (plane 0, quadrant 0, this lane)
    __device__ bool kin(int s, int nk) const { return (unsigned)(s - ip - jp) < (unsigned)nk; }
    __device__ bool active(int s, int nk, int q) const { return ((inq >> q) & 1u) && kin(s, nk); }
};

__device__ __forceinline__ TileView make_view(const Geom &g, int t, int lane)
{
    TileView v;
    v.t = t;
    v.ti = t % g.nti;
    v.tj = t / g.nti;
    v.ip = lane % LI;
    v.jp = lane / LI;
    const int i0 = v.ti * TI + 2 * v.ip, j0 = v.tj * TJ + 2 * v.jp;
    v.inq = 0u;
#pragma unroll
    for (int q = 0; q < NQ; q++)
        if (i0 + (q & 1) < g.ni && j0 + (q >> 1) < g.nj) v.inq |= 1u << q;
    v.base = (long long)t * g.tile_elems + PLANE + lane;
    return v;
}

// Workgroup prologue: take a ticket.  Returns the job index and the tile.
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

// Race testing (LaunchArgs::jitter != 0): at about one step in four a wave
// pauses for up to 15 x 1024 clocks, chosen by a hash of the seed, the job,
// the tile, the step and the wave (all wave-uniform).  Only the timing of the
// waves changes, never what they compute.
__device__ __forceinline__ void jitter_pause(uint32_t seed, int job, int tile, int step, int wave)
{
    if (seed == 0u) return;
    uint32_t h = seed ^ ((uint32_t)tile * 0x9e3779b9u) ^ ((uint32_t)step * 0x85ebca6bu) ^
                 ((uint32_t)(job * 16 + wave) * 0xc2b2ae35u);
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    if ((h & 3u) != 0u) return;
    const int n = (int)((h >> 2) & 15u);
    for (int q = 0; q < n; q++) __builtin_amdgcn_s_sleep(16);
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

// Load through a uniform base pointer and a 32-bit element index (the host
// guarantees every array stays below 4 GiB), which maps onto the
// saddr + voffset form of global_load.
template <typename T>
__device__ __forceinline__ T ldg(const GLOBAL T *base, uint32_t idx)
{
    return *(const GLOBAL T *)((const GLOBAL char *)base + (size_t)(idx * (uint32_t)sizeof(T)));
}
// The same with the non-temporal hint, for streams that no other load of the
// sweep reads again (coefficients, factors, b) in systems much larger than the
// caches: they then do not displace the x planes, which the halo loads of the
// neighbour tiles and the tile's own slot loads read again shortly after.
// (Smaller systems, whose data the caches can hold from one iteration to the
// next, load them as usual: ST = false.)
template <typename T>
__device__ __forceinline__ T ldg_stream(const GLOBAL T *base, uint32_t idx)
{
    return __builtin_nontemporal_load((const GLOBAL T *)((const GLOBAL char *)base + (size_t)(idx * (uint32_t)sizeof(T))));
}
template <bool ST, typename T>
__device__ __forceinline__ T ldg_st(const GLOBAL T *base, uint32_t idx)
{
    if constexpr (ST) return ldg_stream(base, idx);
    else return ldg(base, idx);
}
template <typename T>
__device__ __forceinline__ void stg(GLOBAL T *base, uint32_t idx, T v)
{
    *(GLOBAL T *)((GLOBAL char *)base + (size_t)(idx * (uint32_t)sizeof(T))) = v;
}

// 16-byte groups of the coefficient and factor storage (sip_internal.h).
typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef float flt3 __attribute__((ext_vector_type(3)));   // 16-byte slot, 12 bytes loaded
typedef float flt2 __attribute__((ext_vector_type(2)));

// The values of M right-hand sides at one cell, stored together: T for
// M = 1, a two-lane vector for M = 2 (b, x, y, d and the face records of the
// right-hand sides of one multi-RHS sweep travel together).
template <typename T, int M> struct PackOf;
template <> struct PackOf<double, 1> { typedef double T; };
template <> struct PackOf<float, 1> { typedef float T; };
template <> struct PackOf<double, 2> { typedef dbl2 T; };
template <> struct PackOf<float, 2> { typedef flt2 T; };
template <typename T, int M> using Pk = typename PackOf<T, M>::T;
__device__ __forceinline__ double el(double v, int) { return v; }
__device__ __forceinline__ float el(float v, int) { return v; }
__device__ __forceinline__ double el(const dbl2 &v, int m) { return m ? v.y : v.x; }
__device__ __forceinline__ float el(const flt2 &v, int m) { return m ? v.y : v.x; }
__device__ __forceinline__ void set_el(double &v, int, double x) { v = x; }
__device__ __forceinline__ void set_el(float &v, int, float x) { v = x; }
__device__ __forceinline__ void set_el(dbl2 &v, int m, double x)
{
    if (m) v.y = x;
    else v.x = x;
}
__device__ __forceinline__ void set_el(flt2 &v, int m, float x)
{
    if (m) v.y = x;
    else v.x = x;
}
// a pair of FP32 values travels in the face records as two words, like FP64
template <> struct NW<flt2> { static constexpr int n = 2; };
__device__ __forceinline__ void to_words(const flt2 &v, uint32_t *w)
{
    w[0] = __float_as_uint(v.x);
    w[1] = __float_as_uint(v.y);
}
__device__ __forceinline__ void from_words(const uint64_t *w, flt2 &v)
{
    v.x = __uint_as_float((uint32_t)w[0]);
    v.y = __uint_as_float((uint32_t)w[1]);
}
__device__ __forceinline__ void keep(flt2 &x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void keep(dbl2 &x) { asm volatile("" : "+v"(x)); }
template <typename F> struct Grp;
template <> struct Grp<float> {
    typedef flt4 V;
    static constexpr int W = 4, N = 1;   // factors per group, groups per cell
};
template <> struct Grp<double> {
    typedef dbl2 V;
    static constexpr int W = 2, N = 2;
};
__device__ __forceinline__ float lane_of(const flt4 &v, int k) { return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w; }
__device__ __forceinline__ double lane_of(const dbl2 &v, int k) { return k == 0 ? v.x : v.y; }

// ------------------------------------------------------ face records
// Entry e < TJ: cell row j = e of the tile column facing the i neighbour
// (lane column ci, quadrant column ca); entry TJ + i: cell column i of the
// tile row facing the j neighbour (lane row cj, quadrant row cb).  Downstream
// in the forward direction the faces are the E column / N row (ci = LI - 1,
// ca = 1, cj = LJ - 1, cb = 1), in the backward direction the W column / S row.
__device__ __forceinline__ void entry_owner(int e, int ci, int ca, int cj, int cb, int &lane, int &q)
{
    if (e < TJ) {
        lane = (e >> 1) * LI + ci;
        q = (e & 1) * 2 + ca;
    } else {
        const int c = e - TJ;
        lane = cj * LI + (c >> 1);
        q = cb * 2 + (c & 1);
    }
}

// The recurrence wave writes a step's whole record with one store in which
// every lane writes a word (64 lanes cover the FACE_ENTRIES * NV words
// 64 / (FACE_ENTRIES * NV) times over, with identical data), taking the value
// from the LDS copy of the step it has just written.  With no store behind a
// branch the compiler's vector-memory counts stay exact, and the wait for a
// prefetched poll never waits for a later store.  Steps past the last one
// write the tile's sink words.
struct Post {
    uint32_t rec;    // word index of this lane's word in the tile's record at step 0
    uint32_t sink;   // word index of this lane's word in the tile's sink
    int src, q;      // lane and quadrant whose value this lane's word carries
    int half;        // which 32-bit half of that value (FP64)
};

template <int NV>
__device__ __forceinline__ Post make_post(const Geom &g, const TileView &v, long long fstride, int lane, int ci, int ca,
                                          int cj, int cb)
{
    static_assert(FACE_ENTRIES * NV <= WAVE, "one store per record");
    Post p;
    const int word = lane & (FACE_ENTRIES * NV - 1);
    p.half = word % NV;
    entry_owner(word / NV, ci, ca, cj, cb, p.src, p.q);
    p.rec = (uint32_t)v.t * (uint32_t)fstride + (uint32_t)word;
    p.sink = (uint32_t)g.ntiles * (uint32_t)fstride + (uint32_t)v.t * SINK_WORDS + (uint32_t)word;
    return p;
}

template <int NV, typename F>
__device__ __forceinline__ void post_record(GLOBAL uint64_t *fbase, const Post &p, int s, int steps, int fw, uint32_t tag,
                                            F val)
{
    uint32_t wd[NV];
    to_words(val, wd);
    uint32_t w = wd[0];
#pragma unroll
    for (int q = 1; q < NV; q++) w = p.half == q ? wd[q] : w;
    ll_store(fbase + (s < steps ? p.rec + (uint32_t)s * (uint32_t)fw : p.sink), tag, w);
}

// Poll plan of a recurrence wave.  A lane on the upstream i edge reads the
// two entries of its cell rows (2 j', 2 j' + 1) from the i neighbour's record
// LI - 1 steps ahead (the neighbour's edge lanes reach the same k that many
// steps later); a lane on the j edge reads entries TJ + 2 i', TJ + 2 i' + 1
// from the j neighbour.  NV words per entry.  Word indices come from one
// uniform base with selects; lanes without a halo read their own tile's first
// word.
struct PollPlan {
    uint32_t own, base_i, base_j;
    bool edge_i, edge_j;
};

template <int NV>
__device__ __forceinline__ PollPlan make_polls(const Geom &g, const TileView &v, long long fstride, int fw, bool backward)
{
    PollPlan p;
    const int ti_up = backward ? v.t + 1 : v.t - 1;
    const int tj_up = backward ? v.t + g.nti : v.t - g.nti;
    p.own = (uint32_t)v.t * (uint32_t)fstride;
    p.edge_i = backward ? (v.ip == LI - 1 && v.ti < g.nti - 1) : (v.ip == 0 && v.ti > 0);
    p.edge_j = backward ? (v.jp == LJ - 1 && v.tj < g.ntj - 1) : (v.jp == 0 && v.tj > 0);
    p.base_i = (uint32_t)(p.edge_i ? ti_up : v.t) * (uint32_t)fstride + (uint32_t)((LI - 1) * fw + 2 * v.jp * NV);
    p.base_j = (uint32_t)(p.edge_j ? tj_up : v.t) * (uint32_t)fstride + (uint32_t)((LJ - 1) * fw + (TJ + 2 * v.ip) * NV);
    return p;
}

// ------------------------------------------------------ sweeps
// Workgroup = one recurrence wave (wave 0) + NL = NQ * NP loader waves.
// Loader wave l works quadrant q = l % NQ of the steps f with f % NP = l / NQ.
// Its turn for step f comes in interval f - 1: it consumes the loads it
// issued NP turns earlier, stages the operands of step f in the LDS ring and
// issues the loads of step f + NP, so its own vector-memory wait only covers
// loads that had NP intervals to arrive.  In interval s + 1 the recurrence
// wave processes step s with operands already in registers, publishes its
// face record at once, and then reads the operands of step s + 1 (staged in
// interval s) before the barrier, so no LDS round trip follows a barrier.
// One workgroup barrier ends every interval.  Results of step f - 3 (forward
// y, backward x += d) are written back by step f's loaders.

__device__ __forceinline__ int sweep_steps(int steps, int pd)
{
    // recurrence steps 0..steps (step `steps` only lets the last write-back
    // happen), padded to the poll unroll
    return (steps + 1 + pd - 1) / pd * pd;
}

// Forward: residual r = b - A x (fused, in the precision R of b and x: FP64,
// or FP32 in the all-FP32 arithmetic), forward substitution
// y = (r - Lb y_B - Lw y_W - Ls y_S) / Lp in precision F, per-tile partial
// sums of r^2 (and of b^2, used at iteration 0), summed in FP64.

// Full storage: a[] = A_P..A_T of plane f.  Symmetric storage (FP64 only):
// a[0] = A_P of plane f, a[2], a[4], a[6] = A_E, A_N, A_T of plane f + 1
// (staged into the coefficient ring), a[1], a[3] = A_E of the W neighbour /
// A_N of the S neighbour across a tile edge.
template <typename F, typename R, int M>
struct FwdLoad {
    R a[7];
    Pk<R, M> b;
    Pk<R, M> x2;   // x on plane f + 2, staged into the LDS plane ring for the next steps
    Pk<R, M> hx;   // x across the W or E tile edge (edge slots only)
    Pk<R, M> hy;   // x across the S or N tile edge (edge slots only)
    typename Grp<F>::V lv[Grp<F>::N];   // Lb, Lw, Ls, 1/Lp as stored (16-byte groups)
};

// Uniform base pointers and per-lane index deltas of a forward loader.
template <typename F, typename R, int M>
struct FwdSrc {
    const GLOBAL dbl2 *AP[3];   // FP64: (A_P, A_W), (A_E, A_S), (A_N, A_B)
    const GLOBAL double *AT;
    const GLOBAL flt4 *A4;      // FP32: (A_P, A_W, A_E, A_S)
    const GLOBAL flt3 *A3;      // FP32: (A_N, A_B, A_T) of the (A_N, A_B, A_T, 0) group
    const GLOBAL Pk<R, M> *b, *x;
    const GLOBAL typename Grp<F>::V *L[Grp<F>::N];   // Lb, Lw, Ls, 1/Lp
    const GLOBAL double *SP, *ST, *SEN;                // symmetric storage: A_P, A_T, (A_E, A_N) pairs
    uint32_t e0;          // sheared index of (plane 0, this quadrant, this lane)
    int32_t hx, hy;       // index deltas of the x halo this slot reads across a tile edge (0: none)
};

template <typename F, typename R, int M>
__device__ __forceinline__ FwdSrc<F, R, M> fwd_src(const Job &J, const TileView &v, int q)
{
    const Geom &g = J.g;
    FwdSrc<F, R, M> s;
#pragma unroll
    for (int p = 0; p < 3; p++) s.AP[p] = (const GLOBAL dbl2 *)(gp(J.A) + 2 * p * g.elems);
    s.AT = gp(J.A) + 6 * g.elems;
    s.A4 = (const GLOBAL flt4 *)gp((const float *)J.A);
    s.A3 = (const GLOBAL flt3 *)(gp((const float *)J.A) + 4 * g.elems);
    s.SP = gp(J.A);
    s.SEN = gp(J.A) + g.elems;
    s.ST = gp(J.A) + 3 * g.elems;
    s.b = gp((const Pk<R, M> *)J.b);
    s.x = gp((const Pk<R, M> *)J.x);
#pragma unroll
    for (int k = 0; k < Grp<F>::N; k++)
        s.L[k] = (const GLOBAL typename Grp<F>::V *)(gp((const F *)J.LU) + k * Grp<F>::W * g.elems);
    s.e0 = (uint32_t)v.base + (uint32_t)(q * TT);
    const int te = (int)g.tile_elems;
    const int a = q & 1, b = q >> 1;
    const int dqi = ((q ^ 1) - q) * TT, dqj = ((q ^ 2) - q) * TT;
    // Across a tile edge the neighbour cell sits on the neighbour tile's own
    // local plane: W at f + LI - 1, E at f - LI + 1, S at f + LJ - 1, N at
    // f - LJ + 1, in the other quadrant column (row).  A slot lies on at most
    // one of the W/E edges and one of the S/N edges; in-tile neighbours come
    // from the LDS plane ring.
    s.hx = (a == 0) ? ((v.ip == 0 && v.ti > 0) ? -te + (LI - 1) * PLANE + dqi + (LI - 1) : 0)
                    : ((v.ip == LI - 1 && v.ti < g.nti - 1) ? te - (LI - 1) * PLANE + dqi - (LI - 1) : 0);
    s.hy = (b == 0) ? ((v.jp == 0 && v.tj > 0) ? -g.nti * te + (LJ - 1) * PLANE + dqj + (LJ - 1) * LI : 0)
                    : ((v.jp == LJ - 1 && v.tj < g.ntj - 1) ? g.nti * te - (LJ - 1) * PLANE + dqj - (LJ - 1) * LI : 0);
    return s;
}

// Branch-free: inactive slots read their own zero-padded slot (every index
// stays inside the tile's planes -1..steps for f in [0, steps)).
template <typename F, typename R, int M, bool ST>
__device__ __forceinline__ void fwd_issue(FwdLoad<F, R, M> &c, const FwdSrc<F, R, M> &s, const TileView &v, int q,
                                          int f, int steps, int nk, bool sym)
{
    const bool act = v.active(f, nk, q);
    const uint32_t e = s.e0 + (uint32_t)f * PLANE;
    if constexpr (std::is_same<R, float>::value) {
        // the pad of the second group is not loaded: a dead lane of a load in
        // flight would be reused as soon as the load completes, which makes
        // the compiler wait for every outstanding load
        const flt4 c0 = ldg_st<ST>(s.A4, e);
        const flt3 c1 = ldg_st<ST>(s.A3, e);
        c.a[0] = c0.x;
        c.a[1] = c0.y;
        c.a[2] = c0.z;
        c.a[3] = c0.w;
        c.a[4] = c1.x;
        c.a[5] = c1.y;
        c.a[6] = c1.z;
    } else if (sym) {
        const uint32_t e1 = s.e0 + (uint32_t)min(f + 1, steps) * PLANE;   // plane `steps` is the zero margin
        c.a[0] = ldg(s.SP, e);
        const dbl2 en = ldg((const GLOBAL dbl2 *)s.SEN, e1);
        c.a[2] = en.x;
        c.a[4] = en.y;
        c.a[6] = ldg(s.ST, e1);
        // W / S couplings across a tile edge: the neighbour cell's A_E / A_N
        // (edge slots of quadrant column / row 0; the other lanes share one word)
        c.a[1] = ldg(s.SEN, 2u * (e + (act && !(q & 1) ? s.hx : 0)));
        c.a[3] = ldg(s.SEN, 2u * (e + (act && !(q & 2) ? s.hy : 0)) + 1u);
    } else {
#pragma unroll
        for (int p = 0; p < 3; p++) {
            const dbl2 v2 = ldg_st<ST>(s.AP[p], e);
            c.a[2 * p] = v2.x;
            c.a[2 * p + 1] = v2.y;
        }
        c.a[6] = ldg_st<ST>(s.AT, e);
    }
    c.b = ldg_st<ST>(s.b, e);
#pragma unroll
    for (int k = 0; k < Grp<F>::N; k++) c.lv[k] = ldg_st<ST>(s.L[k], e);
    c.x2 = ldg(s.x, s.e0 + (uint32_t)min(f + 2, steps) * PLANE);   // plane `steps` is the zero margin
    // x across a tile edge, loaded without control flow (a branch would cost
    // the loader exact wait counts): the edge slots of a quadrant read the
    // neighbour tile, the other lanes their own slot (unused, or zero padding
    // for inactive slots, which keeps their residual zero)
    c.hx = ldg(s.x, e + (act ? s.hx : 0));
    c.hy = ldg(s.x, e + (act ? s.hy : 0));
}

// Finaliser of a forward sweep with several right-hand sides: per
// right-hand side r, Ctl ctl[1 + r] holds its own stop state, residual and
// iteration count; ctl[0] keeps the launch sequence (epoch, iteration) and
// stops once every right-hand side has stopped.  A right-hand side that has
// stopped keeps its x (the backward sweep skips its update), so its result is
// the iterate at which it stopped, as in a solve of its own.
// Finite and not NaN (non-finite inputs or a diverging iteration stop the solve).
__device__ __forceinline__ bool finite_val(double v) { return v <= 1.7976931348623157e308 && v >= -1.7976931348623157e308; }

template <int M>
__device__ void finalise_multi(const Job &J, const double *sr, const double *sb, uint32_t iter, uint32_t tag)
{
    Ctl *c0 = J.ctl;
    const uint32_t err = c0->err;
    bool running = false, capped = false, stopped = false;
#pragma unroll
    for (int m = 0; m < M; m++) {
        Ctl *cr = J.ctl + 1 + m;
        if (iter == 0) cr->bnorm2 = sb[m];
        const double nb2 = iter == 0 ? sb[m] : cr->bnorm2;
        double rho = 0.0;
        if (nb2 != 0.0) rho = sqrt(sr[m]) / sqrt(nb2);
        if (!finite_val(nb2)) rho = __builtin_nan("");
        if (J.hist) J.hist[m * J.hstride + iter] = rho;
        if (cr->stop != RUN) {
            stopped = true;
            continue;
        }
        uint32_t st = RUN;
        if (!finite_val(nb2) || !finite_val(rho)) st = (iter == 0 || !finite_val(nb2)) ? BAD_INPUT : DIVERGED;
        else if (nb2 == 0.0) st = ZERO_RHS;
        else if (c0->rtol > 0.0 && rho <= c0->rtol) st = CONVERGED;
        else if (iter >= c0->max_iter) st = MAXITER;
        cr->rho = rho;
        cr->iter = iter;
        cr->stop = st;
        running = running || st == RUN;
        stopped = stopped || st != RUN;
        capped = capped || st == MAXITER;
    }
    uint32_t st = running ? RUN : capped ? MAXITER : CONVERGED;
    if (J.coupled && running && stopped) st = PARTNER;   // the one still running goes on alone
    if (err) st = (err & 2u) ? BREAKDOWN : TIMEOUT;
    c0->stop = st;
    c0->epoch = tag + 1u;
    c0->done = 0u;
}

// LDS of one forward-sweep workgroup.
template <typename F, typename R, int M>
struct FwdLds {
    static constexpr bool R64 = std::is_same<R, double>::value;
    F ring[2][M][NQ][TT];                 // r of each right-hand side; two steps
    typename Grp<F>::V lring[2][Grp<F>::N][NQ][TT];   // (Lb, Lw, Ls, 1/Lp) in the stored 16-byte groups
    Pk<F, M> ybuf[2][NQ][TT];
    Pk<R, M> xring[4][NQ][TT];            // x on planes f-1..f+2 (slot = plane & 3)
    double cring[R64 ? 4 : 1][3][NQ][TT]; // symmetric storage: A_E, A_N, A_T on planes f-1..f+1
    // sums of r^2 and b^2 per right-hand side, quadrant and lane, added plane
    // by plane in plane order (whichever loader phase owns the plane), so the
    // tile's norms do not depend on the number of loader phases
    double acc[2 * M][NQ][TT];
};

// One tile of a forward sweep: the whole workgroup works tile as.tile of job
// J.  Returns (uniformly) true in the workgroup that finished the job's
// sweep last, after it has run the job's finaliser (norm and stop decision).
template <typename F, typename R, int NP, int M, int PD, bool ST>
__device__ bool fwd_tile(const LaunchArgs &a, const Assign &as, const Job &J, FwdLds<F, R, M> &L, int *s_buf)
{
    static_assert(M == 1 || std::is_same<F, float>::value, "several right-hand sides need FP32 factors");
    typedef Pk<F, M> FV;   // y of the M right-hand sides
    typedef Pk<R, M> RV;   // b, x of the M right-hand sides
    constexpr int NV = NW<FV>::n;
    // With three loader phases a loader owns three intervals per turn, and the
    // turn is split over two of them: staging (and the residual) of plane f in
    // one, the loads of plane f + NP and the write-back in the next, so that no
    // interval has to hold a whole turn (the loads keep their two intervals of
    // lead).
    constexpr bool SPLIT = NP >= 3;
    constexpr bool R64 = std::is_same<R, double>::value;   // the symmetric storage exists in FP64 only
    auto &ring = L.ring;
    auto &lring = L.lring;
    auto &ybuf = L.ybuf;
    auto &xring = L.xring;
    auto &cring = L.cring;
    auto &acc = L.acc;

    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const uint32_t tag = J.ctl->epoch;
    const uint32_t iter = J.ctl->iter;
    const Geom g = J.g;
    const bool sym = R64 && J.sym != 0;
    const TileView v = make_view(g, as.tile, lane);
    const int U = sweep_steps(g.steps, PD);
    const int FW = J.fw;
    const long long fstride = (long long)g.steps * FW;
    GLOBAL Ctl *ctl = gp(J.ctl);

    for (int x = threadIdx.x; x < 2 * NQ * TT; x += blockDim.x) (&ybuf[0][0][0])[x] = FV(0);
    for (int x = threadIdx.x; x < 2 * M * NQ * TT; x += blockDim.x) (&acc[0][0][0])[x] = 0.0;
    if (threadIdx.x == 0) s_buf[3] = 0;
    if (wave >= 1 && wave <= NQ) {   // phase-0 loaders: planes -1 (zero margin), 0 and 1 of the x ring
        const int q = wave - 1;
        const uint32_t e0 = (uint32_t)v.base + (uint32_t)(q * TT);
        const GLOBAL RV *xg = gp((const RV *)J.x);
        xring[3][q][lane] = RV(0);
        xring[0][q][lane] = ldg(xg, e0);
        xring[1][q][lane] = ldg(xg, e0 + (uint32_t)min(1, g.steps) * PLANE);
        if constexpr (R64) if (sym) {   // A_E, A_N, A_T of planes -1 (zero margin) and 0
            const GLOBAL double *ag = gp(J.A);
#pragma unroll
            for (int d = 0; d < 3; d++) cring[3][d][q][lane] = 0.0;
            cring[0][0][q][lane] = ldg(ag, (uint32_t)g.elems + 2u * e0);
            cring[0][1][q][lane] = ldg(ag, (uint32_t)g.elems + 2u * e0 + 1u);
            cring[0][2][q][lane] = ldg(ag, 3u * (uint32_t)g.elems + e0);
        }
    }
    __syncthreads();   // the x ring prologue is read across quadrants by the first turn

    if (wave == 0) {
        // ---------------- recurrence wave
        GLOBAL uint64_t *fbase = gp(J.face);
        const PollPlan pp = make_polls<NV>(g, v, fstride, FW, false);
        const Post post = make_post<NV>(g, v, fstride, lane, LI - 1, 1, LJ - 1, 1);   // E column, N row
        Halo<2 * NV> pv[PD];
        bool needW[PD], needS[PD];
        uint32_t oW[PD], oS[PD];
        auto plan = [&](int q, int s2) {
            const bool act = v.inq != 0u && v.kin(s2, g.nk);
            needW[q] = act && pp.edge_i;
            needS[q] = act && pp.edge_j;
            oW[q] = needW[q] ? pp.base_i + (uint32_t)s2 * FW : pp.own;
            oS[q] = needS[q] ? pp.base_j + (uint32_t)s2 * FW : pp.own;
            halo_issue(pv[q], fbase + oW[q], fbase + oS[q]);
        };
        // The prologue repeats a step's store pattern (the sink) ahead of each
        // poll, so the loop is entered with the same counts as it loops back with.
#pragma unroll
        for (int q = 0; q < PD; q++) {
            post_record<NV>(fbase, post, g.steps, g.steps, FW, tag, FV(0));
            plan(q, q);
        }
        FV yB[NQ] = {FV(0), FV(0), FV(0), FV(0)};
        bool aborted = false;
        const int dW = v.ip > 0 ? 1 : 0, dS = v.jp > 0 ? LI : 0;
        F r[M][NQ], lb[NQ], lw[NQ], ls[NQ], il[NQ];
        FV nW1, nW3, nS2, nS3;
        auto prefetch = [&](int s) {   // operands of step s: ring slot, in-tile neighbours of step s - 1
            const int slot = s & 1, pr = (s - 1) & 1;
#pragma unroll
            for (int c = 0; c < NQ; c++) {
#pragma unroll
                for (int m = 0; m < M; m++) r[m][c] = ring[slot][m][c][lane];
                F lf[4];
#pragma unroll
                for (int k = 0; k < Grp<F>::N; k++) {
                    const typename Grp<F>::V gv = lring[slot][k][c][lane];   // one 16-byte read
#pragma unroll
                    for (int w = 0; w < Grp<F>::W; w++) lf[k * Grp<F>::W + w] = lane_of(gv, w);
                }
                lb[c] = lf[0];
                lw[c] = lf[1];
                ls[c] = lf[2];
                il[c] = lf[3];
            }
            nW1 = ybuf[pr][1][lane - dW];
            nW3 = ybuf[pr][3][lane - dW];
            nS2 = ybuf[pr][2][lane - dS];
            nS3 = ybuf[pr][3][lane - dS];
        };
        wg_barrier();   // interval -1: the loaders stage step 0
        prefetch(0);
        wg_barrier();   // interval 0: the loaders stage step 1
        for (int s0 = 0; s0 < U; s0 += PD) {
#pragma unroll
            for (int q = 0; q < PD; q++) {
                const int s = s0 + q;
                jitter_pause(a.jitter, as.job, as.tile, s, 0);
                if (!aborted && !halo_wait(pv[q], needW[q], fbase + oW[q], needS[q], fbase + oS[q], tag, ctl,
                                           a.timeout_ticks))
                    aborted = true;
                FV hw0, hw1, hs0, hs1;
                from_words(&pv[q].a[0], hw0);
                from_words(&pv[q].a[NV], hw1);
                from_words(&pv[q].b[0], hs0);
                from_words(&pv[q].b[NV], hs1);
                // pinned here, after the barrier that completed the reads: the
                // selects below must not pull them into divergent branches
                keep(nW1);
                keep(nW3);
                keep(nS2);
                keep(nS3);
                const FV zero = FV(0);
                const FV W0 = dW ? nW1 : (needW[q] ? hw0 : zero);   // W of quadrant (0,0)
                const FV W2 = dW ? nW3 : (needW[q] ? hw1 : zero);   // W of quadrant (0,1)
                const FV S0 = dS ? nS2 : (needS[q] ? hs0 : zero);   // S of quadrant (0,0)
                const FV S1 = dS ? nS3 : (needS[q] ? hs1 : zero);   // S of quadrant (1,0)
                const bool kin = v.kin(s, g.nk);
                FV y[NQ];
#pragma unroll
                for (int m = 0; m < M; m++) {
                    F y0, y1, y2, y3;
                    {
                        F t = r[m][0] - lb[0] * el(yB[0], m);
                        t = t - lw[0] * el(W0, m);
                        t = t - ls[0] * el(S0, m);
                        y0 = (kin && (v.inq & 1u)) ? t * il[0] : F(0);
                    }
                    {
                        F t = r[m][1] - lb[1] * el(yB[1], m);
                        t = t - lw[1] * y0;
                        t = t - ls[1] * el(S1, m);
                        y1 = (kin && (v.inq & 2u)) ? t * il[1] : F(0);
                    }
                    {
                        F t = r[m][2] - lb[2] * el(yB[2], m);
                        t = t - lw[2] * el(W2, m);
                        t = t - ls[2] * y0;
                        y2 = (kin && (v.inq & 4u)) ? t * il[2] : F(0);
                    }
                    {
                        F t = r[m][3] - lb[3] * el(yB[3], m);
                        t = t - lw[3] * y2;
                        t = t - ls[3] * y1;
                        y3 = (kin && (v.inq & 8u)) ? t * il[3] : F(0);
                    }
                    set_el(y[0], m, y0);
                    set_el(y[1], m, y1);
                    set_el(y[2], m, y2);
                    set_el(y[3], m, y3);
                }
#pragma unroll
                for (int c = 0; c < NQ; c++) {
                    yB[c] = y[c];
                    ybuf[s & 1][c][lane] = y[c];
                }
                // publish at once: the neighbour tiles' next steps wait on this record
                const FV rec = ybuf[s & 1][post.q][post.src];
                prefetch(s + 1);   // issued before the record store waits for its value
                post_record<NV>(fbase, post, s, g.steps, FW, tag, rec);
                plan(q, s + PD);
                if (q == PD - 1 && aborted) s_buf[3] = 1;   // read by every wave after this barrier
                wg_barrier();
            }
            if (s_buf[3]) break;
        }
    } else {
        // ---------------- loader waves
        const int lw = wave - 1;
        const int q = lw % NQ, ph = lw / NQ;
        const int qa = q & 1, qb = q >> 1;
        const FwdSrc<F, R, M> src = fwd_src<F, R, M>(J, v, q);
        FwdLoad<F, R, M> c;
        if (ph < g.steps) fwd_issue<F, R, M, ST>(c, src, v, q, ph, g.steps, g.nk, sym);
        GLOBAL FV *yout = gp((FV *)J.y);
        // In-ring neighbours: the other quadrant column (row) of the same
        // lane on the same plane, or of the neighbouring lane one plane down
        // (W, S) / up (E, N).
        const int dW = qa ? 0 : (v.ip > 0 ? 1 : 0), dE = qa ? (v.ip < LI - 1 ? 1 : 0) : 0;
        const int dS = qb ? 0 : (v.jp > 0 ? LI : 0), dN = qb ? (v.jp < LJ - 1 ? LI : 0) : 0;
        const bool inW = qa || v.ip > 0, inE = !qa || v.ip < LI - 1;
        const bool inS = qb || v.jp > 0, inN = !qb || v.jp < LJ - 1;
        const bool wall_w = !inW && v.ti == 0, wall_s = !inS && v.tj == 0;   // block boundary: no coupling
        auto turn = [&](int f) {
            if (f < g.steps) {
                // planes f-1..f+1 were staged by earlier turns
                xring[(f + 2) & 3][q][lane] = c.x2;
                const RV xP = xring[f & 3][q][lane];
                const RV xB = xring[(f - 1) & 3][q][lane];
                const RV xT = xring[(f + 1) & 3][q][lane];
                // every lane reads the ring (an edge lane its own slot: dW .. dN are
                // 0 there) and then selects: read only where needed, the reads
                // became exec-masked branches around the LDS accesses
                RV rW = xring[(f - 1 + qa) & 3][q ^ 1][lane - dW], rE = xring[(f + qa) & 3][q ^ 1][lane + dE];
                RV rS = xring[(f - 1 + qb) & 3][q ^ 2][lane - dS], rN = xring[(f + qb) & 3][q ^ 2][lane + dN];
                keep(rW);
                keep(rE);
                keep(rS);
                keep(rN);
                const RV xW = inW ? rW : c.hx;
                const RV xE = inE ? rE : c.hx;
                const RV xS = inS ? rS : c.hy;
                const RV xN = inN ? rN : c.hy;
                R aP = c.a[0], aW = c.a[1], aE = c.a[2], aS = c.a[3], aN = c.a[4], aB = c.a[5], aT = c.a[6];
                if constexpr (R64) if (sym) {
                    // A_W = A_E of the W cell, A_S = A_N of the S cell, A_B = A_T of the B
                    // cell, found where the x ring finds x_W, x_S, x_B; plane f + 1 is
                    // staged for the next turns
                    cring[(f + 1) & 3][0][q][lane] = c.a[2];
                    cring[(f + 1) & 3][1][q][lane] = c.a[4];
                    cring[(f + 1) & 3][2][q][lane] = c.a[6];
                    aE = cring[f & 3][0][q][lane];
                    aN = cring[f & 3][1][q][lane];
                    aT = cring[f & 3][2][q][lane];
                    aB = cring[(f - 1) & 3][2][q][lane];
                    double cW = cring[(f - 1 + qa) & 3][0][q ^ 1][lane - dW];
                    double cS = cring[(f - 1 + qb) & 3][1][q ^ 2][lane - dS];
                    keep(cW);
                    keep(cS);
                    aW = inW ? cW : (wall_w ? 0.0 : c.a[1]);
                    aS = inS ? cS : (wall_s ? 0.0 : c.a[3]);
                }
                const int slot = f & 1;
#pragma unroll
                for (int m = 0; m < M; m++) {
                    const R ax = aP * el(xP, m) + aW * el(xW, m) + aE * el(xE, m) + aS * el(xS, m) +
                                 aN * el(xN, m) + aB * el(xB, m) + aT * el(xT, m);
                    const R bm = el(c.b, m);
                    const R r = bm - ax;
                    // plane f of quadrant q is this wave's alone in this interval
                    acc[2 * m][q][lane] += (double)r * (double)r;
                    acc[2 * m + 1][q][lane] += (double)bm * (double)bm;
                    ring[slot][m][q][lane] = (F)r;
                }
#pragma unroll
                for (int k = 0; k < Grp<F>::N; k++) lring[slot][k][q][lane] = c.lv[k];
            }
            if constexpr (!SPLIT) {
                if (f + NP < g.steps) fwd_issue<F, R, M, ST>(c, src, v, q, f + NP, g.steps, g.nk, sym);
                const int p = f - 3;
                if (p >= 0 && p < g.steps)   // inactive slots rewrite their zero padding
                    stg(yout, src.e0 + (uint32_t)p * PLANE, ybuf[p & 1][q][lane]);
            }
        };
        // Second half of a split turn, one interval later: the loads of plane
        // f + NP and the write-back of plane f - 2 (written by the recurrence
        // in the interval before, rewritten two intervals later).
        auto turn_b = [&](int f) {
            if (f + NP < g.steps) fwd_issue<F, R, M, ST>(c, src, v, q, f + NP, g.steps, g.nk, sym);
            const int p = f - 2;
            if (p >= 0 && p < g.steps) stg(yout, src.e0 + (uint32_t)p * PLANE, ybuf[p & 1][q][lane]);
        };
        if (ph == 0) turn(0);
        wg_barrier();   // interval -1
        if (1 % NP == ph) turn(1);
        if constexpr (SPLIT) if (ph == 0) turn_b(0);
        wg_barrier();   // interval 0
        for (int s0 = 0; s0 < U; s0 += PD) {
            for (int k = 0; k < PD; k++) {
                const int f = s0 + k + 2;
                if (f % NP == ph) {
                    jitter_pause(a.jitter, as.job, as.tile, f, wave);
                    turn(f);
                }
                if constexpr (SPLIT) if ((f - 1) % NP == ph) turn_b(f - 1);
                wg_barrier();
            }
            if (s_buf[3]) break;
        }
    }
    __syncthreads();
    if (wave == 0) {   // per-tile partials: quadrants in order, lanes by a fixed butterfly
#pragma unroll
        for (int k = 0; k < 2 * M; k++) {
            double sum = 0.0;
#pragma unroll
            for (int c = 0; c < NQ; c++) sum += wave_sum(acc[k][c][lane]);
            if (lane == 0) gp(J.part)[2 * M * v.t + k] = sum;
        }
    }

    const bool last = job_last(J, s_buf);
    if (last && wave == 0) {
        double sr[M], sb[M];
#pragma unroll
        for (int m = 0; m < M; m++) {
            double a0 = 0.0, a1 = 0.0;
            for (int t = lane; t < g.ntiles; t += WAVE) {
                a0 += J.part[2 * M * t + 2 * m];
                a1 += J.part[2 * M * t + 2 * m + 1];
            }
            sr[m] = wave_sum(a0);
            sb[m] = wave_sum(a1);
        }
        if (lane == 0) {
            if constexpr (M > 1) {
                finalise_multi<M>(J, sr, sb, iter, tag);
            } else if (J.coupled) {   // the domain's control kernel decides
                Ctl *cc = J.ctl;
                cc->rho = sr[0];
                if (iter == 0) cc->bnorm2 = sb[0];
                cc->epoch = tag + 1u;
                cc->done = 0u;
            } else {
                Ctl *cc = J.ctl;
                if (iter == 0) cc->bnorm2 = sb[0];
                const double nb2 = iter == 0 ? sb[0] : cc->bnorm2;
                uint32_t st = RUN;
                const uint32_t err = cc->err;
                if (err) {
                    st = (err & 2u) ? BREAKDOWN : TIMEOUT;
                } else if (!finite_val(nb2)) {
                    st = BAD_INPUT;
                    cc->rho = __builtin_nan("");
                    if (J.hist) J.hist[iter] = cc->rho;
                } else if (nb2 == 0.0) {
                    st = ZERO_RHS;
                    cc->rho = 0.0;
                    if (J.hist) J.hist[iter] = 0.0;
                } else {
                    const double rho = sqrt(sr[0]) / sqrt(nb2);
                    cc->rho = rho;
                    if (J.hist) J.hist[iter] = rho;
                    if (!finite_val(rho)) st = iter == 0 ? BAD_INPUT : DIVERGED;
                    else if (cc->rtol > 0.0 && rho <= cc->rtol) st = CONVERGED;
                    else if (iter >= cc->max_iter) st = MAXITER;
                }
                cc->stop = st;
                cc->epoch = tag + 1u;
                cc->done = 0u;
            }
        }
    }
    return last;
}

template <typename F, typename R, int NP, int M, int PD, bool ST>
__global__ __launch_bounds__(WAVE *(1 + NQ * NP)) void k_forward(LaunchArgs a)
{
    __shared__ FwdLds<F, R, M> L;
    __shared__ int s_buf[8];
    const Assign as = take_ticket(a, s_buf);
    const Job J = load_job(a, as.job);
    if (J.ctl->stop == RUN) (void)fwd_tile<F, R, NP, M, PD, ST>(a, as, J, L, s_buf);
    launch_done(a);
}

// Backward: d = y - Un d_N - Ue d_E - Ut d_T in reverse local-hyperplane
// order (step s visits plane steps - 1 - s; inside a lane quadrant (1,1)
// first, (0,0) last), then x += d in the precision R of x.

template <typename F, typename R, int M>
struct BwdLoad {
    Pk<F, M> y;
    F u[3];      // Un, Ue, Ut
    Pk<R, M> x;
};

template <typename F, typename R, int M>
struct BwdSrc {
    const GLOBAL Pk<F, M> *y;
    const GLOBAL F *U[3];
    GLOBAL Pk<R, M> *x;
    uint32_t e0;
};

template <typename F, typename R, int M>
__device__ __forceinline__ void bwd_issue(BwdLoad<F, R, M> &c, const BwdSrc<F, R, M> &s, int steps, int step)
{
    const uint32_t e = s.e0 + (uint32_t)(steps - 1 - step) * PLANE;
    c.y = ldg(s.y, e);
#pragma unroll
    for (int d = 0; d < 3; d++) c.u[d] = ldg(s.U[d], e);
    c.x = ldg((const GLOBAL Pk<R, M> *)s.x, e);
}

// LDS of one backward-sweep workgroup.
template <typename F, typename R, int M>
struct BwdLds {
    Pk<F, M> yring[2][NQ][TT];
    F ring[2][3][NQ][TT];     // Un, Ue, Ut
    Pk<R, M> xring[4][NQ][TT];
    Pk<F, M> dbuf[2][NQ][TT];
};

// One tile of a backward sweep (as fwd_tile).
template <typename F, typename R, int NP, int M, int PD>
__device__ bool bwd_tile(const LaunchArgs &a, const Assign &as, const Job &J, BwdLds<F, R, M> &L, int *s_buf)
{
    typedef Pk<F, M> FV;
    typedef Pk<R, M> RV;
    constexpr int NV = NW<FV>::n;
    // With three loader phases a loader owns three intervals per turn, and the
    // turn is split over two of them: staging (and the residual) of plane f in
    // one, the loads of plane f + NP and the write-back in the next, so that no
    // interval has to hold a whole turn (the loads keep their two intervals of
    // lead).
    constexpr bool SPLIT = NP >= 3;
    auto &yring = L.yring;
    auto &ring = L.ring;
    auto &xring = L.xring;
    auto &dbuf = L.dbuf;

    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const uint32_t tag = J.ctl->epoch;
    const Geom g = J.g;
    const TileView v = make_view(g, as.tile, lane);
    const int U = sweep_steps(g.steps, PD);
    const int FW = J.fw;
    const long long fstride = (long long)g.steps * FW;
    GLOBAL Ctl *ctl = gp(J.ctl);

    for (int x = threadIdx.x; x < 2 * NQ * TT; x += blockDim.x) (&dbuf[0][0][0])[x] = FV(0);
    if (threadIdx.x == 0) s_buf[3] = 0;
    __syncthreads();

    if (wave == 0) {
        GLOBAL uint64_t *fbase = gp(J.face);
        const PollPlan pp = make_polls<NV>(g, v, fstride, FW, true);
        const Post post = make_post<NV>(g, v, fstride, lane, 0, 0, 0, 0);   // W column, S row
        Halo<2 * NV> pv[PD];
        bool needE[PD], needN[PD];
        uint32_t oE[PD], oN[PD];
        auto plan = [&](int q, int s2) {   // s2: backward step
            const bool act = s2 < g.steps && v.inq != 0u && v.kin(g.steps - 1 - s2, g.nk);
            needE[q] = act && pp.edge_i;
            needN[q] = act && pp.edge_j;
            oE[q] = needE[q] ? pp.base_i + (uint32_t)s2 * FW : pp.own;
            oN[q] = needN[q] ? pp.base_j + (uint32_t)s2 * FW : pp.own;
            halo_issue(pv[q], fbase + oE[q], fbase + oN[q]);
        };
#pragma unroll
        for (int q = 0; q < PD; q++) {   // same store pattern as a step (sink only)
            post_record<NV>(fbase, post, g.steps, g.steps, FW, tag, FV(0));
            plan(q, q);
        }
        FV dT[NQ] = {FV(0), FV(0), FV(0), FV(0)};
        bool aborted = false;
        const int dE = v.ip < LI - 1 ? 1 : 0, dN = v.jp < LJ - 1 ? LI : 0;
        FV yv[NQ];
        F un[NQ], ue[NQ], ut[NQ];
        FV nE0, nE2, nN0, nN1;
        auto prefetch = [&](int s) {   // operands of step s: ring slot, in-tile neighbours of step s - 1
            const int slot = s & 1, pr = (s - 1) & 1;
#pragma unroll
            for (int c = 0; c < NQ; c++) {
                yv[c] = yring[slot][c][lane];
                un[c] = ring[slot][0][c][lane];
                ue[c] = ring[slot][1][c][lane];
                ut[c] = ring[slot][2][c][lane];
            }
            nE0 = dbuf[pr][0][lane + dE];
            nE2 = dbuf[pr][2][lane + dE];
            nN0 = dbuf[pr][0][lane + dN];
            nN1 = dbuf[pr][1][lane + dN];
        };
        wg_barrier();   // interval -1
        prefetch(0);
        wg_barrier();   // interval 0
        for (int s0 = 0; s0 < U; s0 += PD) {
#pragma unroll
            for (int q = 0; q < PD; q++) {
                const int s = s0 + q;
                jitter_pause(a.jitter, as.job, as.tile, s, 0);
                if (!aborted && !halo_wait(pv[q], needE[q], fbase + oE[q], needN[q], fbase + oN[q], tag, ctl,
                                           a.timeout_ticks))
                    aborted = true;
                FV he0, he1, hn0, hn1;
                from_words(&pv[q].a[0], he0);
                from_words(&pv[q].a[NV], he1);
                from_words(&pv[q].b[0], hn0);
                from_words(&pv[q].b[NV], hn1);
                keep(nE0);   // after the barrier that completed the reads
                keep(nE2);
                keep(nN0);
                keep(nN1);
                const FV zero = FV(0);
                const FV E1 = dE ? nE0 : (needE[q] ? he0 : zero);   // E of quadrant (1,0)
                const FV E3 = dE ? nE2 : (needE[q] ? he1 : zero);   // E of quadrant (1,1)
                const FV N2 = dN ? nN0 : (needN[q] ? hn0 : zero);   // N of quadrant (0,1)
                const FV N3 = dN ? nN1 : (needN[q] ? hn1 : zero);   // N of quadrant (1,1)
                const bool kin = s < g.steps && v.kin(g.steps - 1 - s, g.nk);
                FV d[NQ];
#pragma unroll
                for (int m = 0; m < M; m++) {
                    F d0, d1, d2, d3;
                    {
                        F t = el(yv[3], m) - un[3] * el(N3, m);
                        t = t - ue[3] * el(E3, m);
                        t = t - ut[3] * el(dT[3], m);
                        d3 = (kin && (v.inq & 8u)) ? t : F(0);
                    }
                    {
                        F t = el(yv[2], m) - un[2] * el(N2, m);
                        t = t - ue[2] * d3;
                        t = t - ut[2] * el(dT[2], m);
                        d2 = (kin && (v.inq & 4u)) ? t : F(0);
                    }
                    {
                        F t = el(yv[1], m) - un[1] * d3;
                        t = t - ue[1] * el(E1, m);
                        t = t - ut[1] * el(dT[1], m);
                        d1 = (kin && (v.inq & 2u)) ? t : F(0);
                    }
                    {
                        F t = el(yv[0], m) - un[0] * d2;
                        t = t - ue[0] * d1;
                        t = t - ut[0] * el(dT[0], m);
                        d0 = (kin && (v.inq & 1u)) ? t : F(0);
                    }
                    set_el(d[0], m, d0);
                    set_el(d[1], m, d1);
                    set_el(d[2], m, d2);
                    set_el(d[3], m, d3);
                }
#pragma unroll
                for (int c = 0; c < NQ; c++) {
                    dT[c] = d[c];
                    dbuf[s & 1][c][lane] = d[c];
                }
                const FV rec = dbuf[s & 1][post.q][post.src];
                prefetch(s + 1);   // issued before the record store waits for its value
                post_record<NV>(fbase, post, s, g.steps, FW, tag, rec);
                plan(q, s + PD);
                if (q == PD - 1 && aborted) s_buf[3] = 1;
                wg_barrier();
            }
            if (s_buf[3]) break;
        }
    } else {
        const int lw = wave - 1;
        const int q = lw % NQ, ph = lw / NQ;
        BwdSrc<F, R, M> src;
        src.y = gp((const FV *)J.y);
#pragma unroll
        for (int d = 0; d < 3; d++) src.U[d] = gp((const F *)J.LU) + (4 + d) * g.elems;
        src.x = gp((RV *)J.x);
        src.e0 = (uint32_t)v.base + (uint32_t)(q * TT);
        // several right-hand sides: one that has stopped keeps its x
        bool frozen[M];
#pragma unroll
        for (int m = 0; m < M; m++) frozen[m] = M > 1 && J.ctl[1 + m].stop != RUN;
        BwdLoad<F, R, M> c;
        if (ph < g.steps) bwd_issue(c, src, g.steps, ph);
        auto update = [&](int p) {   // x += d of plane p (padding slots: 0 + 0)
            if (p >= 0 && p < g.steps) {
                const int sp = g.steps - 1 - p;
                const FV dv = dbuf[p & 1][q][lane];
                RV xv = xring[p & 3][q][lane];
#pragma unroll
                for (int m = 0; m < M; m++)
                    if (!frozen[m]) set_el(xv, m, el(xv, m) + (R)el(dv, m));
                stg(src.x, src.e0 + (uint32_t)sp * PLANE, xv);
            }
        };
        auto turn = [&](int f) {
            if (f < g.steps) {
                const int slot = f & 1;
                yring[slot][q][lane] = c.y;
                ring[slot][0][q][lane] = c.u[0];
                ring[slot][1][q][lane] = c.u[1];
                ring[slot][2][q][lane] = c.u[2];
                xring[f & 3][q][lane] = c.x;
            }
            if constexpr (!SPLIT) {
                // Issue the next loads before the x store: a load of x behind a
                // store to x would wait for the store to complete.
                if (f + NP < g.steps) bwd_issue(c, src, g.steps, f + NP);
                update(f - 3);
            }
        };
        auto turn_b = [&](int f) {   // second half of a split turn: loads of f + NP, x of plane f - 2
            if (f + NP < g.steps) bwd_issue(c, src, g.steps, f + NP);
            update(f - 2);
        };
        if (ph == 0) turn(0);
        wg_barrier();   // interval -1
        if (1 % NP == ph) turn(1);
        if constexpr (SPLIT) if (ph == 0) turn_b(0);
        wg_barrier();   // interval 0
        for (int s0 = 0; s0 < U; s0 += PD) {
            for (int k = 0; k < PD; k++) {
                const int f = s0 + k + 2;
                if (f % NP == ph) {
                    jitter_pause(a.jitter, as.job, as.tile, f, wave);
                    turn(f);
                }
                if constexpr (SPLIT) if ((f - 1) % NP == ph) turn_b(f - 1);
                wg_barrier();
            }
            if (s_buf[3]) break;
        }
    }

    const bool last = job_last(J, s_buf);
    if (last && wave == 0 && lane == 0) {
        Ctl *cc = J.ctl;
        if (cc->err) cc->stop = (cc->err & 2u) ? BREAKDOWN : TIMEOUT;
        cc->iter = cc->iter + 1u;
        cc->epoch = tag + 1u;
        cc->done = 0u;
    }
    return last;
}

template <typename F, typename R, int NP, int M, int PD>
__global__ __launch_bounds__(WAVE *(1 + NQ * NP)) void k_backward(LaunchArgs a)
{
    __shared__ BwdLds<F, R, M> L;
    __shared__ int s_buf[8];
    const Assign as = take_ticket(a, s_buf);
    const Job J = load_job(a, as.job);
    if (J.ctl->stop == RUN) (void)bwd_tile<F, R, NP, M, PD>(a, as, J, L, s_buf);
    launch_done(a);
}

// ------------------------------------------------------ persistent sweeps
// k_persist: the sweeps of many jobs in one launch, each job at its own pace
// (the queue protocol is described with Task in sip_internal.h).  A job's
// forward finaliser decides its stop as in a single solve; when it runs on,
// the workgroup publishes the job's backward sweep; the backward finaliser
// publishes the next forward sweep unless the job stopped (a wait timed out)
// or the host asked for a pause.  A job that publishes nothing leaves the
// launch; the launch ends when no job is left and every workgroup finds the
// queue empty.

template <typename F, typename R, int M>
union PersistLds {
    FwdLds<F, R, M> f;
    BwdLds<F, R, M> b;
};

// Takes the next ticket and waits until its task is published (thread 0;
// s_buf[4..6] = job, tile, kind; job -1 when no task will come).  The polls
// are relaxed (an acquire would invalidate the caches at every poll); one
// acquire fence follows a task, before the workgroup reads the job's data.
__device__ void release_downstream(const PersistArgs &e, int job, int kind, int tile);

template <bool DF>
__device__ void take_task(const PersistArgs &e, int *s_buf)
{
    int job = -1, tile = 0, kind = 0;
    const uint32_t t = atomicAdd(&e.pc->head, 1u);
    Task *slot = e.tasks + (t % e.cap);
    const uint64_t t0 = wall_clock64();
    for (;;) {
        const Task w = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(w >> 32) == t + 1u) {
            tile = (int)(w & ((1u << TASK_TILE_BITS) - 1u));
            kind = (int)((w >> TASK_TILE_BITS) & 1u);
            job = (int)((w >> (TASK_TILE_BITS + 1)) & ((1u << TASK_JOB_BITS) - 1u));
            __hip_atomic_store(slot, (Task)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);   // the slot is free
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if constexpr (DF) release_downstream(e, job, kind, tile);
            break;
        }
        // with no job left nothing is published any more: a ticket beyond the
        // reserved ones will never hold a task
        if (__hip_atomic_load(&e.pc->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u &&
            t >= __hip_atomic_load(&e.pc->alloc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            break;
        if (__hip_atomic_load(&e.pc->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        if (wall_clock64() - t0 > e.timeout_ticks) {
            __hip_atomic_fetch_or(&e.pc->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(4);
    }
    s_buf[4] = job;
    s_buf[5] = tile;
    s_buf[6] = kind;
}

// One task, published alone (thread 0 of a workgroup): reserve a ticket,
// wait until its slot is free (the capacity argument says it is; the wait is
// bounded all the same), store the task.
__device__ void publish_task(const PersistArgs &e, int job, int kind, int tile)
{
    const uint32_t t = atomicAdd(&e.pc->alloc, 1u);
    Task *slot = e.tasks + (t % e.cap);
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != (Task)0) {
        if (wall_clock64() - t0 > e.timeout_ticks) {
            __hip_atomic_fetch_or(&e.pc->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    __hip_atomic_store(slot, make_task(t, job, kind, tile), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Dataflow publication (thread 0, when the workgroup has taken tile `tile` of
// job `job`'s sweep `kind`): count this tile as taken for each downstream
// neighbour (E and N in a forward sweep, W and S backward) and publish a
// neighbour's task once all of its upstream tiles are taken.  The neighbour
// then waits at most about one tile hop in its polls, instead of holding a
// compute unit while the sweep's wavefront reaches it.  A tile's own counter
// is cleared here: every increment of this sweep came before its task was
// published, and the job's next sweep of this kind starts after this one ends.
__device__ void release_downstream(const PersistArgs &e, int job, int kind, int tile)
{
    const int nti = e.jobs[job].g.nti, ntj = e.jobs[job].g.ntj;
    uint32_t *cnt = e.dep + 2 * e.off[job] + kind * nti * ntj;
    __hip_atomic_store(cnt + tile, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int ti = tile % nti, tj = tile / nti;
    const int step = kind == 0 ? 1 : -1;
#pragma unroll
    for (int axis = 0; axis < 2; axis++) {
        const int di = ti + (axis == 0 ? step : 0), dj = tj + (axis == 1 ? step : 0);
        if (di < 0 || di >= nti || dj < 0 || dj >= ntj) continue;
        // upstream tiles of (di, dj) in this sweep's direction
        const uint32_t nup = kind == 0 ? (uint32_t)(di > 0) + (uint32_t)(dj > 0)
                                       : (uint32_t)(di < nti - 1) + (uint32_t)(dj < ntj - 1);
        const int d = dj * nti + di;
        if (__hip_atomic_fetch_add(cnt + d, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u == nup) {
            // what this workgroup acquired with its task (the previous sweep's
            // results) is released to the neighbour's workgroup
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            publish_task(e, job, kind, d);
        }
    }
}

// After the finaliser of job `job`'s sweep of kind `kind` (whole workgroup):
// publish the job's next sweep, or let the job leave the launch.
template <bool DF>
__device__ void publish_next(const PersistArgs &e, const Job &J, int job, int kind, int *s_buf)
{
    if (threadIdx.x == 0) {
        const uint32_t stop = J.ctl->stop;   // written by this thread in the finaliser
        int next = -1;
        if (stop == RUN) {
            if (kind == 0) next = 1;
            else if (__hip_atomic_load(e.pause, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) == 0u) next = 0;
        }
        if (next < 0) {
            if (stop != RUN) __hip_atomic_store(e.stopped, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_fetch_sub(&e.pc->active, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else if constexpr (DF) {
            // dataflow: the next sweep's first tile; the others follow as their
            // upstream tiles are taken.  The sweep's results are released first.
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            publish_task(e, job, next, next == 0 ? 0 : J.g.ntiles - 1);
        } else {
            s_buf[7] = (int)atomicAdd(&e.pc->alloc, (uint32_t)J.g.ntiles);
        }
        s_buf[6] = next;
    }
    __syncthreads();
    const int next = s_buf[6];
    if (next < 0 || DF) return;
    // the sweep's results (every tile's, gathered by this workgroup's
    // finaliser) are released before any task of the next sweep is visible
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t base = (uint32_t)s_buf[7];
    const int nt = J.g.ntiles;
    const int *ord = e.tile_order + 2 * e.off[job] + (next ? nt : 0);
    for (int k = threadIdx.x; k < nt; k += blockDim.x) {
        const uint32_t t = base + (uint32_t)k;
        Task *slot = e.tasks + (t % e.cap);
        // free by the capacity argument; waited for all the same (bounded)
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != (Task)0) {
            if (wall_clock64() - t0 > e.timeout_ticks) {
                __hip_atomic_fetch_or(&e.pc->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __hip_atomic_store(slot, make_task(t, job, next, ord[k]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Both sweeps are inlined into one loop and register-allocated together
// (mixed form: about 120 VGPRs against 82 for the forward sweep alone), so a
// compute unit holds one workgroup of either phase count; the server runs it
// with three phases, which hold one per unit anyway.
template <typename F, typename R, int NP, int M, bool DF, bool ST>
__global__ __launch_bounds__(WAVE *(1 + NQ * NP)) void k_persist(PersistArgs e)
{
    __shared__ PersistLds<F, R, M> L;
    __shared__ int s_buf[8];
    const LaunchArgs a{e.jobs, nullptr, nullptr, 0, e.timeout_ticks, e.jitter};
    for (;;) {
        if (threadIdx.x == 0) take_task<DF>(e, s_buf);
        __syncthreads();
        const int job = __builtin_amdgcn_readfirstlane(s_buf[4]);
        const int tile = __builtin_amdgcn_readfirstlane(s_buf[5]);
        const int kind = __builtin_amdgcn_readfirstlane(s_buf[6]);
        if (job < 0) break;
        const Assign as{job, tile};
        const Job J = load_job(a, job);
        const bool last = kind == 0 ? fwd_tile<F, R, NP, M, 2, ST>(a, as, J, L.f, s_buf)
                                    : bwd_tile<F, R, NP, M, 2>(a, as, J, L.b, s_buf);
        if (last) publish_next<DF>(e, J, job, kind, s_buf);
        __syncthreads();   // LDS and s_buf are reused by the next task
    }
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
// It runs once per system, so one wave per tile does everything: it loads
// the coefficients one step ahead, polls the neighbour records, computes the
// four cells of each lane in dependency order and writes the factors.

struct U3 {
    double n, e, t;
};

struct Fac {
    double lb, lw, ls, ilp;
    U3 u;
};

__device__ __forceinline__ Fac stone(const double *A, const U3 &B, const U3 &W, const U3 &S, double alpha, bool act,
                                     bool &broke)
{
    Fac f{0.0, 0.0, 0.0, 0.0, {0.0, 0.0, 0.0}};
    if (act) {
        const double denB = 1.0 + alpha * (B.n + B.e);
        const double denW = 1.0 + alpha * (W.n + W.t);
        const double denS = 1.0 + alpha * (S.e + S.t);
        f.lb = A[5] / denB;
        f.lw = A[1] / denW;
        f.ls = A[3] / denS;
        const double p1 = alpha * (f.lb * B.n + f.lw * W.n);
        const double p2 = alpha * (f.ls * S.e + f.lb * B.e);
        const double p3 = alpha * (f.ls * S.t + f.lw * W.t);
        const double lp = A[0] + p1 + p2 + p3 - f.lb * B.t - f.lw * W.e - f.ls * S.n;
        if (denB == 0.0 || denW == 0.0 || denS == 0.0 || lp == 0.0 || !isfinite(lp)) broke = true;
        f.ilp = 1.0 / lp;
        f.u.n = (A[4] - p1) / lp;
        f.u.e = (A[2] - p2) / lp;
        f.u.t = (A[6] - p3) / lp;
    }
    return f;
}

template <typename F>
__global__ __launch_bounds__(WAVE) void k_factor(LaunchArgs a)
{
    constexpr int NV = 6;   // 3 FP64 values per face entry
    __shared__ double ubuf[2][3][NQ][TT];
    __shared__ int s_buf[4];

    const int lane = threadIdx.x;
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
    const int FW = J.fw;
    const long long fstride = (long long)g.steps * FW;
    GLOBAL Ctl *ctl = gp(J.ctl);
    GLOBAL uint64_t *fbase = gp(J.face);
    const PollPlan pp = make_polls<NV>(g, v, fstride, FW, false);

    for (int x = lane; x < 2 * 3 * NQ * TT; x += WAVE) (&ubuf[0][0][0][0])[x] = 0.0;

    // this lane's three record words: word w = lane + 64 m of entry w / 6
    int rsrc[3], rq[3], rd[3], rh[3];
#pragma unroll
    for (int m = 0; m < 3; m++) {
        const int w = lane + WAVE * m;
        entry_owner(w / NV, LI - 1, 1, LJ - 1, 1, rsrc[m], rq[m]);
        rd[m] = (w % NV) / 2;
        rh[m] = w & 1;
    }

    const uint32_t base = (uint32_t)v.base;
    const GLOBAL dbl2 *AP[3];
#pragma unroll
    for (int p = 0; p < 3; p++) AP[p] = (const GLOBAL dbl2 *)(gp(J.A) + 2 * p * g.elems);
    const GLOBAL double *AT = gp(J.A) + 6 * g.elems;
    typedef typename Grp<F>::V LV;
    GLOBAL LV *LG[Grp<F>::N];
#pragma unroll
    for (int k = 0; k < Grp<F>::N; k++) LG[k] = (GLOBAL LV *)(gp((F *)J.LU) + k * Grp<F>::W * g.elems);
    GLOBAL F *UG[3];
#pragma unroll
    for (int d = 0; d < 3; d++) UG[d] = gp((F *)J.LU) + (4 + d) * g.elems;
    auto load_step = [&](double (*A)[7], int s) {   // plane `steps` is the zero margin
        const uint32_t e = base + (uint32_t)min(s, g.steps) * PLANE;
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            const uint32_t eq = e + (uint32_t)(q * TT);
#pragma unroll
            for (int p = 0; p < 3; p++) {
                const dbl2 v2 = ldg(AP[p], eq);
                A[q][2 * p] = v2.x;
                A[q][2 * p + 1] = v2.y;
            }
            A[q][6] = ldg(AT, eq);
        }
    };
    double Ac[NQ][7], An[NQ][7];
    load_step(Ac, 0);
    U3 uB[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) uB[q] = U3{0.0, 0.0, 0.0};
    bool aborted = false, broke = false;
    const int dW = v.ip > 0 ? 1 : 0, dS = v.jp > 0 ? LI : 0;
    for (int s = 0; s < g.steps && !aborted; s++) {
        jitter_pause(a.jitter, as.job, as.tile, s, 0);
        load_step(An, s + 1);
        const bool act = v.inq != 0u && v.kin(s, g.nk);
        const bool nW = act && pp.edge_i, nS = act && pp.edge_j;
        const GLOBAL uint64_t *pW = fbase + (nW ? pp.base_i + (uint32_t)s * FW : pp.own);
        const GLOBAL uint64_t *pS = fbase + (nS ? pp.base_j + (uint32_t)s * FW : pp.own);
        Halo<2 * NV> h;
        halo_issue(h, pW, pS);
        if (!halo_wait(h, nW, pW, nS, pS, tag, ctl, a.timeout_ticks)) aborted = true;
        U3 hW0, hW1, hS0, hS1;
        from_words(&h.a[0], hW0.n);
        from_words(&h.a[2], hW0.e);
        from_words(&h.a[4], hW0.t);
        from_words(&h.a[6], hW1.n);
        from_words(&h.a[8], hW1.e);
        from_words(&h.a[10], hW1.t);
        from_words(&h.b[0], hS0.n);
        from_words(&h.b[2], hS0.e);
        from_words(&h.b[4], hS0.t);
        from_words(&h.b[6], hS1.n);
        from_words(&h.b[8], hS1.e);
        from_words(&h.b[10], hS1.t);
        const U3 z{0.0, 0.0, 0.0};
        const int pr = (s - 1) & 1;
        auto nb = [&](int q, int l) { return U3{ubuf[pr][0][q][l], ubuf[pr][1][q][l], ubuf[pr][2][q][l]}; };
        const U3 W0 = dW ? nb(1, lane - 1) : (nW ? hW0 : z);    // W of quadrant (0,0)
        const U3 W2 = dW ? nb(3, lane - 1) : (nW ? hW1 : z);    // W of quadrant (0,1)
        const U3 S0 = dS ? nb(2, lane - LI) : (nS ? hS0 : z);   // S of quadrant (0,0)
        const U3 S1 = dS ? nb(3, lane - LI) : (nS ? hS1 : z);   // S of quadrant (1,0)
        const bool kin = v.kin(s, g.nk);
        Fac f[NQ];
        f[0] = stone(Ac[0], uB[0], W0, S0, alpha, kin && (v.inq & 1u), broke);
        f[1] = stone(Ac[1], uB[1], f[0].u, S1, alpha, kin && (v.inq & 2u), broke);
        f[2] = stone(Ac[2], uB[2], W2, f[0].u, alpha, kin && (v.inq & 4u), broke);
        f[3] = stone(Ac[3], uB[3], f[2].u, f[1].u, alpha, kin && (v.inq & 8u), broke);
        const uint32_t e = base + (uint32_t)s * PLANE;
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            uB[q] = f[q].u;
            ubuf[s & 1][0][q][lane] = f[q].u.n;
            ubuf[s & 1][1][q][lane] = f[q].u.e;
            ubuf[s & 1][2][q][lane] = f[q].u.t;
            const uint32_t eq = e + (uint32_t)(q * TT);
            const F lv[4] = {(F)f[q].lb, (F)f[q].lw, (F)f[q].ls, (F)f[q].ilp};
            if constexpr (Grp<F>::N == 1) {
                stg(LG[0], eq, flt4{lv[0], lv[1], lv[2], lv[3]});
            } else {
                stg(LG[0], eq, dbl2{lv[0], lv[1]});
                stg(LG[Grp<F>::N - 1], eq, dbl2{lv[2], lv[3]});
            }
            stg(UG[0], eq, (F)f[q].u.n);
            stg(UG[1], eq, (F)f[q].u.e);
            stg(UG[2], eq, (F)f[q].u.t);
        }
        const uint32_t rec = (uint32_t)v.t * (uint32_t)fstride + (uint32_t)s * FW;
#pragma unroll
        for (int m = 0; m < 3; m++) {
            uint32_t wd[2];
            to_words(ubuf[s & 1][rd[m]][rq[m]][rsrc[m]], wd);
            ll_store(fbase + rec + (uint32_t)(lane + WAVE * m), tag, rh[m] ? wd[1] : wd[0]);
        }
#pragma unroll
        for (int q = 0; q < NQ; q++)
#pragma unroll
            for (int d = 0; d < 7; d++) Ac[q][d] = An[q][d];
    }
    if (__any(broke) && lane == 0) __hip_atomic_fetch_or(&ctl->err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    if (job_last(J, s_buf) && lane == 0) {
        Ctl *cc = J.ctl;
        if (cc->err) cc->stop = (cc->err & 2u) ? BREAKDOWN : TIMEOUT;
        cc->epoch = tag + 1u;
        cc->done = 0u;
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

// The layout copies stage one tile column through LDS, so that both the
// natural-order side (rows of TI cells) and the sheared side (whole local
// planes of PLANE elements) are read and written in contiguous runs.  Local
// plane s of a tile holds the cells with k = s - i' - j', i' + j' in
// [0, SHEAR_SPAN], so a chunk of local planes needs SHEAR_SPAN more natural
// planes than it has, and a chunk of natural planes as many more local ones.
constexpr int SHEAR_SPAN = LI + LJ - 2;
constexpr int TO_KC = 16;     // local planes (margins included) per workgroup of k_to_sheared
constexpr int FROM_KC = 32;   // natural planes per workgroup of k_from_sheared

// Copies narr natural-order FP64 arrays into the sheared layout `shear`
// (T = float for SHEAR_F32 and SHEAR_COEF32, rounding to nearest): plain
// arrays at dst + a * dst_stride, or the 7 coefficient arrays P..T with the
// couplings that point out of the block zeroed, in the interleaved, symmetric
// (P, E, N, T only) or FP32 group storage (sip_internal.h).  Workgroup =
// (tile, chunk of TO_KC local planes); every slot of the chunk is written,
// margins and padding with zeros.
template <typename T>
__global__ __launch_bounds__(256) void k_to_sheared(Geom g, int narr, SrcPtrs src, T *dst, long long dst_stride,
                                                    int shear)
{
    __shared__ double st[(TO_KC + SHEAR_SPAN) * TI * TJ];
    const bool coef = shear == SHEAR_COEF || shear == SHEAR_SYM || shear == SHEAR_COEF32;
    const int nch = (g.planes + TO_KC - 1) / TO_KC;
    const int tile = blockIdx.x / nch, p0 = (blockIdx.x % nch) * TO_KC;
    const int p1 = min(p0 + TO_KC, g.planes);
    const int kbase = p0 - 1 - SHEAR_SPAN;              // natural plane of st[0]
    const int nkl = p1 - p0 + SHEAR_SPAN;               // natural planes staged
    const int ti = tile % g.nti, tj = tile / g.nti;
    const int t = threadIdx.x;
    // this thread's slot in every local plane of the chunk
    const int q = t / TT, ln = t % TT, ip = ln % LI, jp = ln / LI;
    const int il = 2 * ip + (q & 1), jl = 2 * jp + (q >> 1);
    const int i = ti * TI + il, j = tj * TJ + jl;
    const bool inij = i < g.ni && j < g.nj;
    for (int a = 0; a < narr; a++) {
        const double *sa = src.p[a];
        for (int r = t; r < nkl * TI * TJ; r += 256) {
            const int k = kbase + r / (TI * TJ), ri = ti * TI + r % TI, rj = tj * TJ + (r / TI) % TJ;
            st[r] = (k >= 0 && k < g.nk && ri < g.ni && rj < g.nj) ? sa[((long long)k * g.nj + rj) * g.ni + ri] : 0.0;
        }
        __syncthreads();
        for (int p = p0; p < p1; p++) {
            const int k = p - 1 - ip - jp;
            const bool ok = inij && k >= 0 && k < g.nk;
            double v = ok ? st[((k - kbase) * TJ + jl) * TI + il] : 0.0;
            if (coef && ok) {
                // couplings that point out of the block are ignored
                if ((a == 1 && i == 0) || (a == 2 && i == g.ni - 1) || (a == 3 && j == 0) ||
                    (a == 4 && j == g.nj - 1) || (a == 5 && k == 0) || (a == 6 && k == g.nk - 1))
                    v = 0.0;
            }
            const long long e = (long long)tile * g.tile_elems + (long long)p * PLANE + t;
            if (shear == SHEAR_PAIR_F64 || shear == SHEAR_PAIR_F32) {
                dst[2 * e + a] = (T)v;
            } else if (shear == SHEAR_SYM) {
                if (a == 0 || a == 2 || a == 4 || a == 6) dst[sym_index(a, e, dst_stride)] = (T)v;
            } else if (shear == SHEAR_COEF32) {
                dst[coef32_index(a, e, dst_stride)] = (T)v;
                if (a == 6) dst[coef32_index(7, e, dst_stride)] = T(0);   // pad of the second group
            } else {
                dst[coef ? coef_index(a, e, dst_stride) : a * dst_stride + e] = (T)v;
            }
        }
        __syncthreads();   // st is refilled for the next array
    }
}

// A symmetric system has A_W(i,j,k) = A_E(i-1,j,k), A_S = A_N of (i,j-1,k) and
// A_B = A_T of (i,j,k-1) for every interior coupling (bitwise).
__global__ void k_check_symmetric(int ni, int nj, int nk, SrcPtrs a, unsigned *bad)
{
    const long long n = (long long)ni * nj * nk, plane = (long long)ni * nj;
    const long long stride = (long long)gridDim.x * blockDim.x;
    unsigned cnt = 0u;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n; c += stride) {
        const int i = (int)(c % ni);
        const int j = (int)((c / ni) % nj);
        const int k = (int)(c / plane);
        if (i > 0 && !(a.p[1][c] == a.p[2][c - 1])) cnt++;
        if (j > 0 && !(a.p[3][c] == a.p[4][c - ni])) cnt++;
        if (k > 0 && !(a.p[5][c] == a.p[6][c - plane])) cnt++;
    }
    if (cnt) atomicAdd(bad, cnt);
}

// Copies x out of the sheared layout (element `which` of groups of `comp`)
// into natural order as FP64; zeros when the solve found a zero right-hand
// side.  Workgroup = (tile, chunk of FROM_KC natural planes).
template <typename T>
__global__ __launch_bounds__(256) void k_from_sheared(Geom g, const T *src, double *dst, const Ctl *ctl, int comp,
                                                      int which)
{
    __shared__ double st[FROM_KC * TI * TJ];
    const bool zero = ctl != nullptr && ctl->stop == ZERO_RHS;
    const int nch = (g.nk + FROM_KC - 1) / FROM_KC;
    const int tile = blockIdx.x / nch, k0 = (blockIdx.x % nch) * FROM_KC;
    const int k1 = min(k0 + FROM_KC, g.nk);
    const int ti = tile % g.nti, tj = tile / g.nti;
    const int t = threadIdx.x;
    const int q = t / TT, ln = t % TT, ip = ln % LI, jp = ln / LI;
    const int il = 2 * ip + (q & 1), jl = 2 * jp + (q >> 1);
    // local planes k0 .. k1 - 1 + SHEAR_SPAN hold the chunk's cells
    for (int s = k0; s < k1 + SHEAR_SPAN; s++) {
        const int k = s - ip - jp;
        if (k >= k0 && k < k1) {
            const long long e = (long long)tile * g.tile_elems + (long long)(s + 1) * PLANE + t;
            st[((k - k0) * TJ + jl) * TI + il] = (double)src[comp * e + which];
        }
    }
    __syncthreads();
    for (int r = t; r < (k1 - k0) * TI * TJ; r += 256) {
        const int k = k0 + r / (TI * TJ), i = ti * TI + r % TI, j = tj * TJ + (r / TI) % TJ;
        if (i < g.ni && j < g.nj) dst[((long long)k * g.nj + j) * g.ni + i] = zero ? 0.0 : st[r];
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
        const long long e = sheared_of(g, i, j, k);
#pragma unroll
        for (int d = 0; d < 7; d++) {
            const double v = (double)LU[factor_index<F>(d, e, g.elems)];
            out.p[d][c] = (d == 3) ? 1.0 / v : v;
        }
    }
}

__global__ void k_init_flags(uint32_t *f)
{
    if (threadIdx.x < 2) f[threadIdx.x] = 0u;
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

// ------------------------------------------------------ multi-block domain

// (the box lies inside the domain: nk is not needed for the indexing)
__global__ void k_box_copy(const double *src, double *dst, int ni, int nj, int /*nk*/, int i0, int j0, int k0, int bi,
                           int bj, int bk, int to_block)
{
    const long long nc = (long long)bi * bj * bk;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < nc; c += stride) {
        const int i = (int)(c % bi);
        const int j = (int)((c / bi) % bj);
        const int k = (int)(c / ((long long)bi * bj));
        const long long gidx = ((long long)(k + k0) * nj + (j + j0)) * ni + (i + i0);
        if (to_block) dst[c] = src[gidx];
        else dst[gidx] = src[c];
    }
}

__global__ void k_gather_coef(XTerm *terms, long long nterms, const uint8_t *dir, const long long *gidx, SrcPtrs a)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < nterms; t += stride)
        terms[t].coef = a.p[dir[t]][gidx[t]];
}

// beff = b - sum of the couplings into other blocks times their x (every
// block's x is the same iterate: the exchange runs between two sweeps).
__global__ void k_exchange(const XCell *cells, long long ncells, const XTerm *terms, BlockPtrs p)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < ncells; c += stride) {
        const XCell xc = cells[c];
        double v = p.b[xc.block][xc.e];
        for (uint32_t t = xc.begin; t < xc.end; t++) {
            const XTerm xt = terms[t];
            v -= xt.coef * p.x[xt.block][xt.e];
        }
        p.beff[xc.block][xc.e] = v;
    }
}

// ||b||^2 of the domain's b (natural order): SUMSQ_BLOCKS fixed partials,
// then one workgroup adds them in order (the result does not depend on timing).
constexpr int SUMSQ_BLOCKS = 256;
__global__ void k_sumsq(const double *v, long long n, double *part)
{
    __shared__ double s_w[4];
    double a = 0.0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x)
        a += v[c] * v[c];
    a = wave_sum(a);
    if ((threadIdx.x & (WAVE - 1)) == 0) s_w[threadIdx.x / WAVE] = a;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((s_w[0] + s_w[1]) + s_w[2]) + s_w[3];
}

__global__ void k_sumsq_final(const double *part, Ctl *g)
{
    if (threadIdx.x != 0) return;
    double a = 0.0;
    for (int q = 0; q < SUMSQ_BLOCKS; q++) a += part[q];
    g->bnorm2 = a;
}

// The blocks' forward finalisers left sum r^2 of their cells in ctl->rho.
__global__ void k_blocks_control(BlockPtrs p, int nblk, Ctl *g, double *hist)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double sr = 0.0;
    uint32_t err = 0u;
    const uint32_t iter = p.ctl[0]->iter;
    for (int q = 0; q < nblk; q++) {   // fixed block order: the norm does not depend on timing
        sr += p.ctl[q]->rho;
        err |= p.ctl[q]->err;
    }
    const double nb2 = g->bnorm2;   // of the domain's b (the blocks sweep on beff)
    uint32_t st = RUN;
    double rho = 0.0;
    if (err) {
        st = (err & 2u) ? BREAKDOWN : TIMEOUT;
    } else if (!finite_val(nb2)) {
        st = BAD_INPUT;
        rho = __builtin_nan("");
    } else if (nb2 == 0.0) {
        st = ZERO_RHS;
    } else {
        rho = sqrt(sr) / sqrt(nb2);
        if (!finite_val(rho)) st = iter == 0 ? BAD_INPUT : DIVERGED;
        else if (g->rtol > 0.0 && rho <= g->rtol) st = CONVERGED;
        else if (iter >= g->max_iter) st = MAXITER;
    }
    g->rho = rho;
    g->iter = iter;
    g->stop = st;
    if (hist) hist[iter] = rho;
    for (int q = 0; q < nblk; q++) p.ctl[q]->stop = st;
}

int grid_for(long long n)
{
    long long b = (n + 255) / 256;
    if (b > 256 * 64) b = 256 * 64;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

hipError_t launch_box_copy(const double *src, double *dst, int ni, int nj, int nk, int i0, int j0, int k0, int bi,
                           int bj, int bk, int to_block, hipStream_t s)
{
    hipLaunchKernelGGL(k_box_copy, dim3(grid_for((long long)bi * bj * bk)), dim3(256), 0, s, src, dst, ni, nj, nk, i0,
                       j0, k0, bi, bj, bk, to_block);
    return hipGetLastError();
}

hipError_t launch_gather_coef(XTerm *terms, long long nterms, const uint8_t *dir, const long long *gidx,
                              const double *const *a, hipStream_t s)
{
    if (nterms == 0) return hipSuccess;
    SrcPtrs sp{};
    for (int d = 0; d < 7; d++) sp.p[d] = a[d];
    hipLaunchKernelGGL(k_gather_coef, dim3(grid_for(nterms)), dim3(256), 0, s, terms, nterms, dir, gidx, sp);
    return hipGetLastError();
}

hipError_t launch_exchange(const XCell *cells, long long ncells, const XTerm *terms, BlockPtrs p, hipStream_t s)
{
    if (ncells == 0) return hipSuccess;
    hipLaunchKernelGGL(k_exchange, dim3(grid_for(ncells)), dim3(256), 0, s, cells, ncells, terms, p);
    return hipGetLastError();
}

hipError_t launch_sumsq(const double *v, long long n, double *part, Ctl *domain, hipStream_t s)
{
    hipLaunchKernelGGL(k_sumsq, dim3(SUMSQ_BLOCKS), dim3(256), 0, s, v, n, part);
    hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(64), 0, s, part, domain);
    return hipGetLastError();
}

hipError_t launch_blocks_control(BlockPtrs p, int nblk, Ctl *domain, double *hist, hipStream_t s)
{
    hipLaunchKernelGGL(k_blocks_control, dim3(1), dim3(64), 0, s, p, nblk, domain, hist);
    return hipGetLastError();
}

hipError_t launch_init_flags(uint32_t *flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_flags, dim3(1), dim3(64), 0, s, flags);
    return hipGetLastError();
}

hipError_t launch_init_ctl(Ctl *ctl, int n, uint32_t max_iter, double rtol, int reset_epoch, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_ctl, dim3((n + 63) / 64), dim3(64), 0, s, ctl, n, max_iter, rtol, reset_epoch);
    return hipGetLastError();
}

hipError_t launch_to_sheared(const Geom &g, int narr, const double *const *src, void *dst, long long dst_stride,
                             int shear, hipStream_t s)
{
    SrcPtrs sp{};
    for (int a = 0; a < narr && a < 9; a++) sp.p[a] = src[a];
    const dim3 grid((unsigned)g.ntiles * (unsigned)((g.planes + TO_KC - 1) / TO_KC));
    if (shear == SHEAR_F32 || shear == SHEAR_COEF32 || shear == SHEAR_PAIR_F32)
        hipLaunchKernelGGL(k_to_sheared<float>, grid, dim3(256), 0, s, g, narr, sp, (float *)dst, dst_stride, shear);
    else
        hipLaunchKernelGGL(k_to_sheared<double>, grid, dim3(256), 0, s, g, narr, sp, (double *)dst, dst_stride,
                           shear);
    return hipGetLastError();
}

hipError_t launch_check_symmetric(int ni, int nj, int nk, const double *const *a, unsigned *bad, hipStream_t s)
{
    SrcPtrs sp{};
    for (int d = 0; d < 7; d++) sp.p[d] = a[d];
    hipLaunchKernelGGL(k_check_symmetric, dim3(grid_for((long long)ni * nj * nk)), dim3(256), 0, s, ni, nj, nk, sp, bad);
    return hipGetLastError();
}

hipError_t launch_from_sheared(const Geom &g, const void *src, int src_f32, double *dst, const Ctl *ctl,
                               hipStream_t s, int comp, int which)
{
    const dim3 grid((unsigned)g.ntiles * (unsigned)((g.nk + FROM_KC - 1) / FROM_KC));
    if (src_f32)
        hipLaunchKernelGGL(k_from_sheared<float>, grid, dim3(256), 0, s, g, (const float *)src, dst, ctl, comp, which);
    else
        hipLaunchKernelGGL(k_from_sheared<double>, grid, dim3(256), 0, s, g, (const double *)src, dst, ctl, comp,
                           which);
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
        hipLaunchKernelGGL(k_factor<float>, dim3(a.total), dim3(WAVE), 0, s, a);
    else
        hipLaunchKernelGGL(k_factor<double>, dim3(a.total), dim3(WAVE), 0, s, a);
    return hipGetLastError();
}

template <typename F, typename R, int NP, int M, int PD, bool ST = false>
static hipError_t launch_sweep_t(const LaunchArgs &a, int backward, hipStream_t s)
{
    const dim3 block(WAVE * (1 + NQ * NP));
    if (backward)
        hipLaunchKernelGGL((k_backward<F, R, NP, M, PD>), dim3(a.total), block, 0, s, a);
    else
        hipLaunchKernelGGL((k_forward<F, R, NP, M, PD, ST>), dim3(a.total), block, 0, s, a);
    return hipGetLastError();
}

// One right-hand side: every poll distance with two or three phases; one
// phase and two right-hand sides come with the default distance only.
template <typename F, typename R, int NP>
static hipError_t launch_sweep_pd(const LaunchArgs &a, int poll, int backward, hipStream_t s)
{
    if constexpr (NP >= 2) {
        switch (poll) {
        case 1: return launch_sweep_t<F, R, NP, 1, 1>(a, backward, s);
        case 3: return launch_sweep_t<F, R, NP, 1, 3>(a, backward, s);
        default: break;
        }
    }
    return launch_sweep_t<F, R, NP, 1, 2>(a, backward, s);
}

template <int NP>
static hipError_t launch_sweep_np(const LaunchArgs &a, int arith, int nrhs, int poll, int backward, hipStream_t s)
{
    if (nrhs == 2) {   // FP32 factors only: a pair of FP32 values fills a face record entry
        switch (arith) {
        case ARITH_MIXED: return launch_sweep_t<float, double, NP, 2, 2>(a, backward, s);
        case ARITH_F32: return launch_sweep_t<float, float, NP, 2, 2>(a, backward, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (nrhs != 1) return hipErrorInvalidValue;
    switch (arith) {
    case ARITH_F64: return launch_sweep_pd<double, double, NP>(a, poll, backward, s);
    case ARITH_MIXED: return launch_sweep_pd<float, double, NP>(a, poll, backward, s);
    case ARITH_F32: return launch_sweep_pd<float, float, NP>(a, poll, backward, s);
    default: return hipErrorInvalidValue;
    }
}

// The default plan of a single large system (three phases, poll distance 2)
// also comes with the non-temporal streams of the forward sweep.
static hipError_t launch_sweep_st(const LaunchArgs &a, int arith, int nrhs, int backward, hipStream_t s)
{
    if (nrhs == 2) {
        switch (arith) {
        case ARITH_MIXED: return launch_sweep_t<float, double, 3, 2, 2, true>(a, backward, s);
        case ARITH_F32: return launch_sweep_t<float, float, 3, 2, 2, true>(a, backward, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (nrhs != 1) return hipErrorInvalidValue;
    switch (arith) {
    case ARITH_F64: return launch_sweep_t<double, double, 3, 1, 2, true>(a, backward, s);
    case ARITH_MIXED: return launch_sweep_t<float, double, 3, 1, 2, true>(a, backward, s);
    case ARITH_F32: return launch_sweep_t<float, float, 3, 1, 2, true>(a, backward, s);
    default: return hipErrorInvalidValue;
    }
}

static hipError_t launch_sweep(const LaunchArgs &a, int arith, int nrhs, int backward, const SweepPlan &p,
                               hipStream_t s)
{
    if (p.poll < 1 || p.poll > MAX_POLL) return hipErrorInvalidValue;
    if (p.stream && p.phases == 3 && p.poll == DEFAULT_POLL) return launch_sweep_st(a, arith, nrhs, backward, s);
    switch (p.phases) {
    case 1: return launch_sweep_np<1>(a, arith, nrhs, p.poll, backward, s);
    case 2: return launch_sweep_np<2>(a, arith, nrhs, p.poll, backward, s);
    case 3: return launch_sweep_np<3>(a, arith, nrhs, p.poll, backward, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename F, typename R, int NP, int M, bool ST>
static hipError_t launch_persist_t(const PersistArgs &a, int wgs, hipStream_t s)
{
    // dataflow and whole-sweep publication are separate kernels, so that the
    // one does not change the other's register allocation
    if (a.dep)
        hipLaunchKernelGGL((k_persist<F, R, NP, M, true, ST>), dim3(wgs), dim3(WAVE * (1 + NQ * NP)), 0, s, a);
    else
        hipLaunchKernelGGL((k_persist<F, R, NP, M, false, ST>), dim3(wgs), dim3(WAVE * (1 + NQ * NP)), 0, s, a);
    return hipGetLastError();
}

template <int NP, bool ST>
static hipError_t launch_persist_np(const PersistArgs &a, int arith, int nrhs, int wgs, hipStream_t s)
{
    if (nrhs == 2) {
        switch (arith) {
        case ARITH_MIXED: return launch_persist_t<float, double, NP, 2, ST>(a, wgs, s);
        case ARITH_F32: return launch_persist_t<float, float, NP, 2, ST>(a, wgs, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (nrhs != 1) return hipErrorInvalidValue;
    switch (arith) {
    case ARITH_F64: return launch_persist_t<double, double, NP, 1, ST>(a, wgs, s);
    case ARITH_MIXED: return launch_persist_t<float, double, NP, 1, ST>(a, wgs, s);
    case ARITH_F32: return launch_persist_t<float, float, NP, 1, ST>(a, wgs, s);
    default: return hipErrorInvalidValue;
    }
}

// The persistent sweeps poll two steps ahead whatever the plan says.
hipError_t launch_persist(const PersistArgs &a, int arith, const SweepPlan &p, int wgs, hipStream_t s, int nrhs)
{
    if (wgs < 1) return hipErrorInvalidValue;
    switch (p.phases) {
    case 2: return launch_persist_np<2, false>(a, arith, nrhs, wgs, s);
    case 3: return p.stream ? launch_persist_np<3, true>(a, arith, nrhs, wgs, s)
                            : launch_persist_np<3, false>(a, arith, nrhs, wgs, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_forward(const LaunchArgs &a, int arith, const SweepPlan &p, hipStream_t s, int nrhs)
{
    return launch_sweep(a, arith, nrhs, 0, p, s);
}

hipError_t launch_backward(const LaunchArgs &a, int arith, const SweepPlan &p, hipStream_t s, int nrhs)
{
    return launch_sweep(a, arith, nrhs, 1, p, s);
}

}  // namespace sipk
