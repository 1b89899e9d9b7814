// Internal declarations shared by the gfx950 kernels and the host runtime.
//
// Data layout ("tile-sheared hyperplane order, 2 x 2 cells per lane").  A
// block of ni x nj x nk cells is cut into tile columns of TI x TJ = 16 x 16
// cells in (i, j) that run through all of k.  A tile is worked by one wave of
// LI x LJ = 8 x 8 lanes; lane (i', j') owns the 2 x 2 cells (2 i' + a, 2 j' + b)
// of the tile, "quadrant" q = 2 b + a.  Cell (i', j', q, k) belongs to the
// local hyperplane (step) s = i' + j' + k and is stored at
//     tile * tile_elems + (s + 1) * PLANE + q * TT + j' * LI + i'
// (TT = 64 lanes, PLANE = 4 * TT), so the cells one step touches are 256
// contiguous elements, 64 per quadrant.  Planes -1 and steps (= nk + LI + LJ
// - 2) are zero margins; slots whose k falls outside [0, nk) or whose (i, j)
// falls outside the block are zero padding.
//
// Why this order computes the SIP recurrences: cell (i, j, k) depends on its
// W, S and B neighbours.  Inside a lane, quadrant (1, b) follows (0, b) and
// (a, 1) follows (a, 0) in the same step; across lanes, the W neighbour of a
// quadrant with a = 0 is lane i' - 1's quadrant (1, b) one step earlier, and
// likewise in j; the B neighbour is the same slot one step earlier.  Any order
// that visits W, S and B before P gives the values of the lexicographic one.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace sipk {

constexpr int LI = 8;              // lanes of a tile in i
constexpr int LJ = 8;              // lanes of a tile in j
constexpr int TT = LI * LJ;        // one wave: lane = j' * LI + i'
constexpr int NQ = 4;              // cells per lane (2 x 2), quadrant q = 2 b + a
constexpr int TI = 2 * LI;         // tile extent in cells (i)
constexpr int TJ = 2 * LJ;         // tile extent in cells (j)
constexpr int PLANE = NQ * TT;     // elements per local step of a tile

// Coefficient storage, 7 * elems doubles (pairs of 16 bytes, so the forward
// sweep loads six coefficients with three 16-byte loads):
//     (A_P, A_W) interleaved in [0, 2 elems), (A_E, A_S) in [2 elems, 4 elems),
//     (A_N, A_B) in [4 elems, 6 elems), A_T in [6 elems, 7 elems).
// Factor storage, 7 * elems of F: Lb, Lw, Ls, 1/Lp of a cell in 16-byte
// groups (FP32: one group of four; FP64: (Lb, Lw) in [0, 2 elems) and
// (Ls, 1/Lp) in [2 elems, 4 elems)), then Un, Ue, Ut as plain arrays.
// Kernels address arrays with 32-bit byte offsets of 16-byte elements, so
// elems stays below MAX_ELEMS.
constexpr long long MAX_ELEMS = 1ll << 28;
// Symmetric coefficient storage (A_W(P) = A_E(W), A_S(P) = A_N(S),
// A_B(P) = A_T(B)), 4 * elems doubles: A_P in [0, elems), (A_E, A_N)
// interleaved in [elems, 3 elems), A_T in [3 elems, 4 elems).  The forward
// sweep reads A_W, A_S, A_B from the neighbours' A_E, A_N, A_T.
__host__ __device__ inline long long sym_index(int a, long long e, long long elems)
{
    // a in the full order P, W, E, S, N, B, T; only P, E, N, T are stored
    return a == 0 ? e : a == 2 ? elems + 2 * e : a == 4 ? elems + 2 * e + 1 : 3 * elems + e;
}

// FP32 coefficient storage of the all-FP32 arithmetic, 8 * elems floats in
// two 16-byte groups per cell: (A_P, A_W, A_E, A_S) in [0, 4 elems) and
// (A_N, A_B, A_T, 0) in [4 elems, 8 elems), so the forward sweep loads the
// seven coefficients with two loads.
__host__ __device__ inline long long coef32_index(int a, long long e, long long elems)
{
    return a < 4 ? 4 * e + a : 4 * elems + 4 * e + (a - 4);
}

__host__ __device__ inline long long coef_index(int a, long long e, long long elems)
{
    return a < 6 ? (long long)(a >> 1) * 2 * elems + 2 * e + (a & 1) : 6 * elems + e;
}

template <typename F>
__host__ __device__ inline long long factor_index(int d, long long e, long long elems)
{
    constexpr int W = 16 / (int)sizeof(F);   // factors per 16-byte group
    return d < 4 ? (long long)(d / W) * W * elems + W * e + d % W : d * elems + e;
}

// Arithmetic of the sweeps (the values of sip_precision):
//   ARITH_F64    factors, sweeps, residual and update in FP64;
//   ARITH_MIXED  FP32 factors and sweeps; residual, norm and update in FP64;
//   ARITH_F32    FP32 coefficients, factors, b and x: the whole relaxation in
//                FP32 (the factors are still computed in FP64 and rounded).
enum Arith : int { ARITH_F64 = 0, ARITH_MIXED = 1, ARITH_F32 = 2 };
constexpr int NARITH = 3;

enum Stop : uint32_t {
    RUN = 0,
    CONVERGED = 1,
    MAXITER = 2,
    ZERO_RHS = 3,
    BREAKDOWN = 4,
    TIMEOUT = 5,
    BAD_INPUT = 6,   // non-finite ||b|| or residual of the start vector
    DIVERGED = 7,    // non-finite residual after the first update
    PARTNER = 8,     // swept right-hand sides with the split flag: one has stopped, the others go on alone
};

struct Geom {
    int ni, nj, nk;
    int nti, ntj, ntiles;
    int steps;                 // nk + LI + LJ - 2 local hyperplanes per tile
    int planes;                // steps + 2 (with the two margins)
    long long tile_elems;      // planes * PLANE
    long long elems;           // ntiles * tile_elems
};

// Sheared index of cell (i, j, k) (the layout at the top of this file).
__host__ __device__ inline long long sheared_of(const Geom &g, int i, int j, int k)
{
    const int ti = i / TI, tj = j / TJ, ii = i % TI, jj = j % TJ;
    const int ip = ii >> 1, jp = jj >> 1, q = (jj & 1) * 2 + (ii & 1);
    const int t = tj * g.nti + ti;
    return (long long)t * g.tile_elems + (long long)(k + ip + jp + 1) * PLANE + q * TT + jp * LI + ip;
}

// Per-system control block in device memory.  Written by the last
// workgroup of each sweep ("finaliser") and read by the next launch.
struct Ctl {
    uint32_t done;             // workgroups of this job finished in the current launch
    uint32_t epoch;            // sequence tag of the current sweep (face words)
    uint32_t iter;             // iteration index n of the next forward sweep
    uint32_t max_iter;
    uint32_t stop;             // Stop
    uint32_t err;              // sticky: 1 device wait timed out, 2 breakdown
    uint32_t pad0, pad1;
    double rtol;               // <= 0: never converge (fixed iteration count)
    double bnorm2;             // sum of b^2
    double rho;                // relative residual of the last forward sweep
};

// One block of a batched launch (a single solve is a batch of one).
struct Job {
    Geom g;
    const double *A;           // coefficients P,W,E,S,N,B,T (sheared; FP32 groups in ARITH_F32 sweeps)
    const void *b;             // elems FP64 (FP32 in ARITH_F32)
    void *x;                   // elems FP64 (FP32 in ARITH_F32)
    void *LU;                  // 7 * elems factors Lb,Lw,Ls,1/Lp,Un,Ue,Ut (FP64 or FP32)
    void *y;                   // elems forward-sweep result (FP64 or FP32)
    uint64_t *face;            // ntiles * steps * FACE_WORDS tagged face words
    double *part;              // 2 * ntiles per-tile partial sums
    double *hist;              // max_iter + 1 relative residuals
    Ctl *ctl;                  // m = 1: the control block; m > 1: ctl[0] the sweep's, ctl[1 + r] right-hand side r's
    double alpha;
    int fw;                    // face words per local step (FACE_WORDS_SWEEP or FACE_WORDS)
    int sym;                   // A in the symmetric storage (sweeps only; the factorisation reads the full one)
    int m;                     // right-hand sides swept together (b, x, y hold m values per cell)
    int coupled;               // m = 1: block of a multi-block domain: the forward finaliser leaves the stop
                               // decision to the domain's control kernel (rho <- sum r^2, bnorm2 <- sum b^2);
                               // m > 1 (split flag): the sweeps stop (PARTNER) once any right-hand side
                               // has stopped while another runs, which then goes on in one-RHS sweeps
    int hstride;               // m > 1: history of right-hand side r at hist + r * hstride
};

// Launch-wide ticket and completion counters (reset by the last workgroup).
struct LaunchCtl {
    uint32_t ticket;
    uint32_t done;
};

struct LaunchArgs {
    const Job *jobs;
    const int2 *order;         // ticket -> (job, tile), topological per job
    LaunchCtl *lc;
    int total;                 // number of workgroups = sum of ntiles
    uint64_t timeout_ticks;    // wall-clock ticks before a wait gives up
    uint32_t jitter;           // 0, or a seed: race testing pauses waves at random steps
};

// Persistent batched sweeps (k_persist): one launch in which every job runs
// its own sequence of sweeps (forward, backward, forward, ...) on its own
// control block, and leaves when it stops or when the host asks for a pause.
// Workgroups loop over a queue of tile tasks: ticket t lives in slot t % cap
// and is valid once its high half reads t + 1; a consumer frees the slot (0).  The
// workgroup that finishes a job's sweep runs its finaliser and publishes the
// job's next sweep, either as one block of tasks in the job's own topological
// order, so every task only waits for tasks with earlier tickets, which are
// held by running workgroups or done (no co-residency assumed), or
// (dataflow) as the sweep's first tile only, each tile's task then being
// published when the tiles it depends on have been taken, so every task only
// waits for tiles that running workgroups hold or have finished.  At most one
// sweep per job is published and unconsumed at any time, so cap > total
// tiles of all jobs guarantees a publisher finds its slots free.
// A task is one 64-bit word, written and read whole: ticket + 1 in the high
// half (0 while the slot is free), then job (12 bits), kind (1 bit: 0 forward,
// 1 backward sweep) and tile (19 bits).
typedef uint64_t Task;
constexpr int TASK_JOB_BITS = 12, TASK_TILE_BITS = 19;
__host__ __device__ inline Task make_task(uint32_t ticket, int job, int kind, int tile)
{
    return ((uint64_t)(ticket + 1u) << 32) | ((uint64_t)job << (TASK_TILE_BITS + 1)) |
           ((uint64_t)kind << TASK_TILE_BITS) | (uint64_t)tile;
}
struct PersistCtl {
    uint32_t head;             // tickets taken
    uint32_t alloc;            // tickets reserved by publishers
    uint32_t active;           // jobs that will still publish a sweep in this launch
    uint32_t err;              // sticky: 1 a queue wait timed out
};
struct PersistArgs {
    const Job *jobs;
    const int *tile_order;     // job j: forward tile order at 2 off[j], backward at 2 off[j] + ntiles
    const int *off;            // prefix sums of the jobs' tile counts
    Task *tasks;
    uint32_t cap;
    PersistCtl *pc;
    const uint32_t *pause;     // host-mapped: nonzero asks every job to leave at its next iteration boundary
    uint32_t *stopped;         // host-mapped: jobs that reached a stop decision (convergence, limit, error)
    uint64_t timeout_ticks;
    uint32_t jitter;
    // Dataflow publication (nonzero dep): a sweep is published tile by tile,
    // each tile once the tiles it depends on have been taken by workgroups;
    // dep holds, per job, 2 * ntiles counters (forward then backward) of
    // upstream tiles taken, zero at launch.  nullptr: every sweep is published
    // whole, in the job's tile order.
    uint32_t *dep;
};
// Face records.  At every local step a tile publishes the values its
// downstream neighbours need: FACE_ENTRIES entries, entry e < TJ for cell row
// j = e of the tile column facing the i neighbour, entry TJ + i for cell
// column i of the tile row facing the j neighbour.
constexpr int FACE_ENTRIES = TI + TJ;
// Words per step: the factorisation sends U triples (3 FP64 values, 2 words
// each); the sweeps one value (1 word FP32, 2 words FP64).
constexpr int FACE_WORDS = FACE_ENTRIES * 6;
constexpr int FACE_WORDS_SWEEP = FACE_ENTRIES * 2;
// Behind the sweeps' ntiles * steps * FACE_WORDS_SWEEP words (inside the
// buffer sized for the factorisation) each tile owns SINK_WORDS words that
// absorb the face-record stores of steps past its last one.
constexpr int SINK_WORDS = FACE_WORDS_SWEEP;
static_assert(SINK_WORDS <= FACE_WORDS - FACE_WORDS_SWEEP, "sink lines must fit behind the sweep face words");

Geom make_geom(int ni, int nj, int nk);

// Multi-block domain: exchange tables.  For every cell of a block with a
// coupling into another block, the effective right-hand side of the block's
// sweeps is b - sum over those couplings of A_nb x_nb, with x_nb the
// neighbour block's current iterate.
struct XCell {
    uint32_t block, e;         // destination block and its sheared index
    uint32_t begin, end;       // its terms
};
struct XTerm {
    uint32_t block, e;         // source block and sheared index of x_nb
    double coef;               // A_nb of the destination cell
};
// Per-block pointers used by the domain kernels (device arrays of nblk).
struct BlockPtrs {
    const double *const *b;    // sheared b of each block
    double *const *beff;       // effective right-hand side
    const double *const *x;    // sheared x
    Ctl *const *ctl;           // control blocks
};
// Copies a box of nc = bi x bj x bk cells between a natural-order domain array
// (dims ni x nj x nk, box origin i0, j0, k0) and a contiguous natural-order
// block array: to_block = 1 gathers into the block array, 0 scatters out.
hipError_t launch_box_copy(const double *src, double *dst, int ni, int nj, int nk, int i0, int j0, int k0, int bi,
                           int bj, int bk, int to_block, hipStream_t s);
// Coefficients of the exchange terms: coef[t] = a[dir[t]][gidx[t]].
hipError_t launch_gather_coef(XTerm *terms, long long nterms, const uint8_t *dir, const long long *gidx,
                              const double *const *a, hipStream_t s);
hipError_t launch_exchange(const XCell *cells, long long ncells, const XTerm *terms, BlockPtrs p, hipStream_t s);
// domain->bnorm2 = sum of v^2 over n values (deterministic; part: 256 doubles).
hipError_t launch_sumsq(const double *v, long long n, double *part, Ctl *domain, hipStream_t s);
// Sums the blocks' partial norms (block order), records rho_n in hist and
// decides the stop for the whole domain, copied into every block's control.
hipError_t launch_blocks_control(BlockPtrs p, int nblk, Ctl *domain, double *hist, hipStream_t s);

// Kernel launchers (sip_kernels.hip).  All are asynchronous on `s`.
hipError_t launch_init_ctl(Ctl *ctl, int n, uint32_t max_iter, double rtol, int reset_epoch, hipStream_t s);
// Zeroes the two flags of a persistent launch without a host (pause, stopped).
hipError_t launch_init_flags(uint32_t *flags, hipStream_t s);
// Layouts written by launch_to_sheared: plain FP64 or FP32 arrays (array a
// at dst + a * dst_stride elements), or the 7 coefficient arrays (masked at
// the block boundary) in the interleaved FP64, symmetric FP64 or FP32 group
// storage.
// SHEAR_PAIR_F64 / SHEAR_PAIR_F32 interleave two arrays per cell (dst[2 e + a],
// narr = 2): the b or x pairs of a two-right-hand-side sweep.
enum Shear : int {
    SHEAR_F64 = 0, SHEAR_COEF = 1, SHEAR_SYM = 2, SHEAR_F32 = 3, SHEAR_COEF32 = 4, SHEAR_PAIR_F64 = 5, SHEAR_PAIR_F32 = 6
};
hipError_t launch_to_sheared(const Geom &g, int narr, const double *const *src, void *dst,
                             long long dst_stride, int shear, hipStream_t s);
// Counts the cells whose W, S or B coupling differs from the neighbour's E, N
// or T one (bitwise) into *bad (device, zeroed by the caller).
hipError_t launch_check_symmetric(int ni, int nj, int nk, const double *const *a, unsigned *bad, hipStream_t s);
// Natural-order FP64 copy of a sheared FP64 (src_f32 = 0) or FP32 array;
// with comp = 2, component `which` of a pair array.
hipError_t launch_from_sheared(const Geom &g, const void *src, int src_f32, double *dst, const Ctl *zero_if_zero_rhs,
                               hipStream_t s, int comp = 1, int which = 0);
hipError_t launch_export_factors(const Geom &g, const void *LU, int fp32, double *const *dst, hipStream_t s);
hipError_t launch_factor(const LaunchArgs &a, int fp32, hipStream_t s);
// Launch shape of the sweeps: loader phases per tile (1 to 3).  Each phase
// is NQ loader waves (one per quadrant); phases take turns step by step.
// With one or two phases a loader's whole turn falls in one step interval and
// its loads have `phases` intervals to arrive; with three the turn is split
// over two intervals (the loads keep two intervals of lead), which shortens
// the step of a lone tile by about a quarter but costs occupancy.  Single
// systems default to three; the solve server takes three only for a launch
// with no more tiles than compute units, else two, like multi-block domains.
constexpr int MAX_PHASES = 3;
constexpr int SINGLE_SYSTEM_PHASES = 3;
// poll: how many steps ahead the recurrence wave polls the upstream tiles'
// face records (1 to 3; two or three phases and one right-hand side take any,
// the others 2).  A poll sees fresh data once the tile runs about 7 + poll
// steps behind its upstream neighbour, so the distance sets the lag per tile
// hop; it must also cover the poll's round trip.
constexpr int MAX_POLL = 3;
constexpr int DEFAULT_POLL = 2;
// stream: the forward sweep loads the coefficients, the factors and b with
// the non-temporal hint (three phases and the default poll distance only).
// Single systems of at least STREAM_HINT_CELLS cells take it: their data per
// iteration (124 B per cell, mixed) is far beyond the caches, so these
// streams would only displace the x planes that are read again.  Smaller
// systems, and the solve server's launches of many smaller blocks, measured
// faster without it.
constexpr long long STREAM_HINT_CELLS = 1ll << 22;
struct SweepPlan {
    int phases = 2;
    int poll = DEFAULT_POLL;
    int stream = 0;
};
// nrhs: right-hand sides per job (1, or 2 with FP32 factors: ARITH_MIXED,
// ARITH_F32); every job of the launch must have Job::m == nrhs.
constexpr int MAX_SWEEP_RHS = 2;
hipError_t launch_forward(const LaunchArgs &a, int arith, const SweepPlan &p, hipStream_t s, int nrhs = 1);
hipError_t launch_backward(const LaunchArgs &a, int arith, const SweepPlan &p, hipStream_t s, int nrhs = 1);
// Launches k_persist with `wgs` persistent workgroups for jobs of one
// arithmetic and right-hand-side count, `p.phases` loader phases (2 or 3).
hipError_t launch_persist(const PersistArgs &a, int arith, const SweepPlan &p, int wgs, hipStream_t s, int nrhs = 1);

}  // namespace sipk
