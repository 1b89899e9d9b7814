/*
 * sip.h -- C ABI of the MI355X (gfx950) implementation of Stone's strongly
 * implicit procedure (SIP) on structured 3D blocks with the 7-point stencil.
 *
 * The method is the linear solver of FASTEST-3D in arXiv:1303.4538: an
 * incomplete-LU (Stone) factorisation followed by relaxation sweeps (Sec. 1),
 * redesigned in Sec. 4.1 as a modular solver that owns its coefficient
 * memory, computes the factorisation once in advance, reuses it for all
 * later iterations and time steps, and relaxes with single-precision sweeps.
 *
 * Conventions shared by every entry point:
 *   - A block has ni x nj x nk cells.  Every grid array is C-contiguous
 *     [nk][nj][ni] FP64 (i fastest) in DEVICE memory of the current HIP device.
 *   - Row P of the system reads  A_P x_P + sum_nb A_nb x_nb = b_P  with signed
 *     coefficients (the paper's listing in Sec. 4.1 stores a_nb = -A_nb).
 *     Couplings that point out of the block are ignored.
 *   - Streams are hipStream_t passed as void* (NULL = the legacy default
 *     stream).  Work is stream-ordered on the caller's stream.
 *   - Errors come back as sip_status; no call aborts or throws.  Detail text
 *     for the calling thread is available from sip_last_error().
 *   - The library never frees caller memory.  Handles are freed only by the
 *     matching *_destroy call.
 */
#ifndef SIP_H
#define SIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SIP_OK = 0,
    SIP_PENDING = 1,        /* sip_batch_poll: request not finished yet            */
    SIP_EINVAL = -1,        /* bad argument (dims < 1, alpha outside [0,1], NULL,
                               non-finite b or start vector)                      */
    SIP_ENOMEM = -2,        /* device allocation or HBM budget exhausted           */
    SIP_EBREAKDOWN = -3,    /* zero/non-finite pivot or zero denominator, or a
                               non-finite residual after an update (divergence)   */
    SIP_ENOTCONV = -4,      /* iteration limit reached before the tolerance        */
    SIP_EDEVICE = -5,       /* HIP error or a device-side wait timed out           */
    SIP_EBUSY = -6,         /* server queue full                                   */
    SIP_ECANCELLED = -7     /* request cancelled / server shut down                */
} sip_status;

typedef enum {
    SIP_FP64 = 0,           /* factors and sweeps in FP64                          */
    SIP_MIXED = 1,          /* factors and sweeps in FP32; residual, norm and the
                               solution update in FP64 (defect correction)         */
    SIP_FP32 = 2            /* the single-precision relaxation of Sec. 4.1: b and
                               x converted to FP32 on entry and x back to FP64 on
                               exit; coefficients, factors (computed in FP64),
                               residual, sweeps and update all in FP32.  The
                               residual stalls near 1e-7 relative; the norm is
                               that of the FP32 residual, summed in FP64.  Not
                               with SIP_STORAGE_SYMMETRIC.                        */
} sip_precision;

/* Storage of the coefficients during the sweeps (the paper's section 4.1,
 * residual for a symmetric system matrix).  SIP_STORAGE_SYMMETRIC keeps only
 * A_P, A_E, A_N, A_T and reads A_W, A_S, A_B from the neighbours' A_E, A_N,
 * A_T, which cuts the forward sweep's coefficient traffic from 56 to 32 bytes
 * per cell.  It requires A_W(i,j,k) = A_E(i-1,j,k), A_S(i,j,k) = A_N(i,j-1,k)
 * and A_B(i,j,k) = A_T(i,j,k-1) bitwise for every interior coupling (checked
 * on the device; SIP_EINVAL otherwise); results are bitwise those of the full
 * storage. */
typedef enum {
    SIP_STORAGE_FULL = 0,
    SIP_STORAGE_SYMMETRIC = 1
} sip_storage;

typedef struct sip_system_s *sip_system;   /* factorised system resident on a GPU */
typedef struct sip_server_s *sip_server;   /* continuous-batching solve server    */

/* One block.  a[d] are device pointers in the order P, W, E, S, N, B, T, each
 * ni*nj*nk FP64 values.  alpha is Stone's cancellation parameter in [0, 1]. */
typedef struct {
    int32_t ni, nj, nk;
    const double *a[7];
    double alpha;
    int32_t precision;      /* sip_precision */
    int32_t storage;        /* sip_storage (0: full) */
} sip_problem;

typedef struct {
    int32_t iters;          /* updates applied                                     */
    double rel_res;         /* ||b - A x||_2 / ||b||_2 of the returned x (FP64;
                               SIP_FP32: the FP32 residual of the FP32 iterate)   */
    double seconds;         /* host wall time of the call                          */
} sip_info;

/* sip_factor -- copy A into the library's own layout and compute the SIP
 * factorisation (Sec. 4.1: the solver owns the coefficient memory and
 * computes the incomplete factorisation in advance, once).
 *   p       problem description; p->a are read during the call only (the
 *           caller may free them afterwards).
 *   stream  HIP stream; the call synchronises it before returning so that a
 *           breakdown can be reported.
 *   out     receives the new handle (unchanged on error).
 * Errors: SIP_EINVAL (dims < 1, NULL pointers, alpha outside [0,1], unknown
 * precision), SIP_ENOMEM, SIP_EBREAKDOWN (zero or non-finite pivot),
 * SIP_EDEVICE. */
sip_status sip_factor(const sip_problem *p, void *stream, sip_system *out);

/* sip_iterate -- apply exactly n_iter SIP updates to x (Sec. 4.1: the
 * original driver relaxes a fixed number of iterations):
 *   r = b - A x (FP64), forward sweep L y = r, backward sweep U d = y,
 *   x += d (residual and update in FP32 with SIP_FP32).
 *   b        device, read only.
 *   x        device, read as the start vector and overwritten.
 *   n_iter   >= 0.
 *   rel_res_hist  NULL, or HOST memory of n_iter+1 doubles that receives
 *           rho_n = ||b - A x_n|| / ||b|| for n = 0..n_iter.  With NULL the
 *           call only enqueues work and does not synchronise the stream (and
 *           so reports none of the stop decisions below).
 * b == 0 everywhere gives x = 0.  Non-finite values: the device computes
 * ||b||^2 and the start residual before any update; if either is not finite
 * (NaN or Inf in b, x or A x), nothing is updated, the history reads NaN and
 * the call returns SIP_EINVAL.  A residual that becomes non-finite later
 * stops the iteration there (x holds that iterate, the history reads NaN
 * from it on) with SIP_EBREAKDOWN.  The squared norms are FP64: entries
 * above about 1e150 in magnitude overflow them and count as non-finite.
 * Errors: SIP_EINVAL, SIP_EBREAKDOWN, SIP_EDEVICE. */
sip_status sip_iterate(sip_system h, const double *b, double *x, int32_t n_iter,
                       double *rel_res_hist, void *stream);

/* sip_iterate_noalloc -- sip_iterate for callers that cannot allocate device
 * memory (work captured into a HIP graph, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, iterates, history and statuses as
 * sip_iterate (bitwise); the call allocates nothing: the per-call state of
 * its sweeps (job descriptor, control block, launch counters, per-tile
 * partial norms, the residual history before it is copied out) lives in a
 * static device array of SIP_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends.  It launches its iterations one by one (no graph of its own).
 *   Limit: 1024 + 16 * tiles (rounded up to 256) + (rel_res_hist ? 8 *
 *   (n_iter + 1) : 0) bytes <= SIP_NOALLOC_SCRATCH_BYTES, where tiles =
 *   ceil(ni / 16) * ceil(nj / 16); beyond it the call returns SIP_EINVAL and
 *   does nothing.  (1 MiB: e.g. a 512 x 512 block with a history of up to
 *   about 128 k iterations.)
 *   The current device must be the system's (SIP_EINVAL otherwise).
 * Every call on one GPU shares that GPU's array, which keeps the last
 * call's contents: calls that overlap on one GPU (several streams or threads)
 * race and must be serialised by the caller. */
#define SIP_NOALLOC_SCRATCH_BYTES (1 << 20)
sip_status sip_iterate_noalloc(sip_system h, const double *b, double *x, int32_t n_iter,
                               double *rel_res_hist, void *stream);

/* sip_solve -- iterate until rho_n <= rtol and return that x_n (the paper
 * evaluates residuals through a global reduction and keeps such evaluations
 * cheap, Sec. 3.2; here the norm and the stop test run on the device).
 *   rtol > 0, max_iter >= 0; info (nullable, host) receives iterations,
 *   final relative residual and wall time.  Synchronises the stream.
 * Non-finite values stop the solve as in sip_iterate (info->rel_res NaN).
 * The whole solve runs as one persistent launch (the sweeps follow each
 * other on the device, which also takes the stop decision); with the
 * environment variable SIP_SOLVE_PERSISTENT=0 (read at every call), or a
 * plan with one loader phase or a poll distance other than 2, it replays
 * graph-captured chunks of 8 iterations instead, with the same results.
 * Every device-side wait (a tile for its neighbours' face records, a
 * workgroup for its next task) is bounded, by 2 s of device wall clock or
 * by SIP_WAIT_LIMIT_MS (read by every factorisation, iterate, solve, profile
 * and tune call, of a single system or of a multi-block domain;
 * 0 makes every wait that is not met at once time out, a hook for testing
 * the error path): a wait that times out ends the call with SIP_EDEVICE, and
 * the handle stays usable (later calls use fresh face-record tags).
 * Errors: SIP_EINVAL (also non-finite b or start vector), SIP_EBREAKDOWN,
 * SIP_ENOTCONV (x holds x_max_iter), SIP_EDEVICE. */
sip_status sip_solve(sip_system h, const double *b, double *x, double rtol, int32_t max_iter,
                     sip_info *info, void *stream);

/* sip_iterate_multi / sip_solve_multi -- nrhs right-hand sides of one
 * factorised system.  The paper reuses one factorisation for all later
 * solves (Sec. 4.1); here two right-hand sides also share one pass of the
 * sweeps over the coefficients and factors, which halves that traffic per
 * right-hand side.  Pairs (r, r + 1) are swept together with SIP_MIXED and
 * SIP_FP32; an odd last one, and every one with SIP_FP64, goes through the
 * one-right-hand-side path.
 *   b[r], x[r]  device arrays as in sip_iterate / sip_solve (r < nrhs).
 *   Every right-hand side gets exactly the iterates, residual history and
 *   stop decision it would get alone (bitwise): in sip_solve_multi each one
 *   stops at its own first n with rho_n <= rtol and keeps that x_n; once one
 *   of a pair has stopped, the other goes on through the one-right-hand-side
 *   path from its current iterate.  sip_solve_multi runs a pair as one
 *   persistent launch up to that point when sip_solve does (SIP_SOLVE_PERSISTENT
 *   unset or not "0"), else in chunks of launches; the results are the same.
 *   rel_res_hist  NULL, or HOST memory of nrhs * (n_iter + 1) doubles,
 *           right-hand side r's history at r * (n_iter + 1).
 *   info    NULL, or HOST memory of nrhs entries.
 * sip_solve_multi, and sip_iterate_multi with a history, synchronise the
 * stream.  A right-hand side whose norm or residual is not finite stops alone
 * (as in sip_iterate / sip_solve); the others run to their own end and the
 * call then returns that right-hand side's SIP_EINVAL or SIP_EBREAKDOWN
 * (before SIP_ENOTCONV).  Errors: SIP_EINVAL, SIP_ENOMEM (buffers for
 * the pairs are allocated on first use and kept by the handle), SIP_ENOTCONV
 * (sip_solve_multi: some right-hand side reached max_iter; the others are
 * still solved), SIP_EDEVICE. */
sip_status sip_iterate_multi(sip_system h, int32_t nrhs, const double *const *b, double *const *x, int32_t n_iter,
                             double *rel_res_hist, void *stream);
sip_status sip_solve_multi(sip_system h, int32_t nrhs, const double *const *b, double *const *x, double rtol,
                           int32_t max_iter, sip_info *info, void *stream);

/* ------------------------------------------------------------------------
 * Multi-block domain (Sec. 4.2: SIP runs per block; blocks are coupled only
 * through values at block boundaries, exchanged once per iteration, and with
 * the non-blocking exchange every block uses the values of the previous
 * exchange).  A domain of ni x nj x nk cells is cut into nb[0] x nb[1] x nb[2]
 * blocks at the planes cuts[d][0..nb[d]] (cuts[d][0] = 0, cuts[d][nb[d]] =
 * the extent, rising).  Each block is factorised on its own (couplings that
 * leave a block do not enter its factors); one iteration forms, for every
 * block, b - (couplings into the other blocks) x of the previous iterate,
 * runs the block's forward and backward sweeps on it (all blocks in one
 * launch per sweep) and updates x; rho_n is the relative residual of the
 * whole domain.  This is a different iteration from single-block SIP and
 * needs more iterations, the more blocks the more.
 * ------------------------------------------------------------------------ */
typedef struct sip_blocks_s *sip_blocks;

typedef struct {
    sip_problem domain;         /* dims, coefficients (device, read during the call only),
                                   alpha, precision (SIP_FP64 or SIP_MIXED), storage (the
                                   symmetric one needs a symmetric domain; results are
                                   bitwise those of the full storage) */
    int32_t nb[3];              /* blocks along i, j, k (nb[0] * nb[1] * nb[2] <= 4096) */
    const int32_t *cuts[3];     /* HOST arrays of nb[d] + 1 cut planes */
} sip_block_problem;

/* sip_blocks_factor -- copy and factorise every block.  Synchronises the
 * stream.  Errors: SIP_EINVAL (dims, cuts, precision SIP_FP32), SIP_ENOMEM,
 * SIP_EBREAKDOWN (in some block), SIP_EDEVICE. */
sip_status sip_blocks_factor(const sip_block_problem *p, void *stream, sip_blocks *out);
/* sip_blocks_iterate / sip_blocks_solve -- as sip_iterate / sip_solve for
 * the whole domain: b and x are natural-order arrays of the domain (device);
 * rel_res_hist (HOST, n_iter + 1 doubles) and info as there.  Both
 * synchronise the stream. */
sip_status sip_blocks_iterate(sip_blocks h, const double *b, double *x, int32_t n_iter, double *rel_res_hist,
                              void *stream);
sip_status sip_blocks_solve(sip_blocks h, const double *b, double *x, double rtol, int32_t max_iter, sip_info *info,
                            void *stream);
/* sip_blocks_info -- number of blocks and device bytes held. */
sip_status sip_blocks_info(sip_blocks h, int32_t *nblocks, size_t *device_bytes);
sip_status sip_blocks_destroy(sip_blocks h);

/* sip_export_factors -- the incomplete factors L and U of Stone's method
 * (Sec. 1; computed once, Sec. 4.1), written in natural [nk][nj][ni] order as
 * FP64 into seven device arrays of ni*nj*nk doubles, in the order
 * Lb, Lw, Ls, Lp, Un, Ue, Ut (Lp is the pivot, U has a unit diagonal).
 * In the mixed and FP32 precisions the FP32 factors are widened.
 * Stream-ordered. */
sip_status sip_export_factors(sip_system h, double *const out[7], void *stream);

/* sip_profile_sweeps -- measurement hook (Sec. 3 times the residual +
 * forward routine and the backward routine separately): runs n_iter iterations like
 * sip_iterate (x updated in place) with a HIP event recorded before and
 * after every sweep launch on `stream`, synchronises, and writes the average
 * device time in milliseconds of one forward sweep (ms[0]) and one backward
 * sweep (ms[1]) to host memory.  n_iter >= 1.  Errors: SIP_EINVAL,
 * SIP_EDEVICE. */
sip_status sip_profile_sweeps(sip_system h, const double *b, double *x, int32_t n_iter, double ms[2], void *stream);

/* sip_profile_sweeps_multi -- (Sec. 3, Sec. 4.1) sip_profile_sweeps for one pair of
 * right-hand sides (b[0], b[1], x[0], x[1]) swept together: the average
 * device time of one pair forward sweep (ms[0]) and one pair backward sweep
 * (ms[1]).  SIP_MIXED and SIP_FP32 only.  Errors: SIP_EINVAL, SIP_ENOMEM,
 * SIP_EDEVICE. */
sip_status sip_profile_sweeps_multi(sip_system h, const double *const *b, double *const *x, int32_t n_iter,
                                    double ms[2], void *stream);

/* sip_tune -- autotuner of the sweep launch plan (Sec. 2 sizes the paper's
 * blocks from about 12 thousand to 1.5 million control volumes per process,
 * so no single plan suits every block): times n_iter iterations from x = 0
 * with b (device, read only) for every plan the sweeps are compiled for --
 * the loader-phase count (1 to 3; each phase is a group of loader waves that
 * prefetch for alternate steps) and the poll distance (1 to 3 steps: how far
 * ahead a tile polls its upstream neighbours' boundary values, which sets the
 * lag per tile hop; the distances other than 2 with two or three phases) --
 * keeps the fastest for this handle and records it for the block shape,
 * precision and storage, so that later sip_factor calls and solve servers in
 * the process start with it.  Iterates and residual norms are unchanged
 * bitwise (the plan does not change the arithmetic).  *phases (nullable,
 * host) receives the chosen phase count; sip_system_plan reports the whole
 * plan.  Synchronises the stream.  The environment variables
 * SIP_SWEEP_PHASES (1..3) and SIP_POLL_DISTANCE (1..3), read by sip_factor
 * and sip_server_create, override tuned plans.
 * Errors: SIP_EINVAL, SIP_EDEVICE. */
sip_status sip_tune(sip_system h, const double *b, int32_t n_iter, int32_t *phases, void *stream);
/* sip_system_plan -- the sweep plan of a handle (Sec. 2; see sip_tune): loader
 * phases and poll distance (either pointer nullable, host).  Errors:
 * SIP_EINVAL (NULL handle). */
sip_status sip_system_plan(sip_system h, int32_t *phases, int32_t *poll);

/* sip_system_solve_ms -- device time of the persistent launches of the
 * handle's last sip_solve or sip_solve_multi call (Sec. 3 measures the
 * solver's kernels one by one; sip_solve runs a whole solve as one launch,
 * sip_solve_multi one per pair of right-hand sides plus one per one-RHS
 * continuation or odd last right-hand side): *ms (host) receives the sum,
 * over those launches, of the time between HIP events recorded on the
 * solve's stream just before and just after each; the layout copies, the
 * factorisation and any host work are outside it.  Errors: SIP_EINVAL (NULL
 * argument, or the last solve call ran no persistent launch: none has run
 * yet, or the chunked path of SIP_SOLVE_PERSISTENT=0 ran, which is not
 * timed). */
sip_status sip_system_solve_ms(sip_system h, double *ms);

/* sip_tune_save / sip_tune_load -- the autotuner's table (kept across
 * processes, like the factorisation that Sec. 4.1 computes once in advance) (block shape,
 * precision, storage -> loader phases and poll distance, as recorded by sip_tune) as a text
 * file, so that a later process starts with the plans an earlier one
 * measured (load it before sip_factor or sip_server_create).  One JSON
 * object per line:
 *   {"ni": 256, "nj": 256, "nk": 256, "precision": 1, "symmetric": 0, "phases": 3, "poll": 2}
 * sip_tune_save writes every entry of the process's table (overwriting
 * path).  sip_tune_load merges the file's entries into the table (the file's
 * win); blank lines are skipped; a line that is not such an entry (missing
 * key, dims < 1, unknown precision, phases or poll outside 1..3) fails the
 * whole load with SIP_EINVAL and merges nothing; a line without "poll" takes
 * the default distance 2.  Host only, thread-safe.
 * Errors: SIP_EINVAL (NULL path, unreadable or unwritable file, bad line). */
sip_status sip_tune_save(const char *path);
sip_status sip_tune_load(const char *path);

/* Race testing: when the environment variable SIP_SCHEDULE_SEED holds a
 * nonzero integer at sip_factor, sip_blocks_factor or sip_server_create, that
 * handle takes its tiles in a random order that still respects every tile's
 * upstream neighbours, and its kernels pause at pseudo-random steps.  The
 * results do not change (bitwise); only the run time grows.  Unset or 0: the
 * default schedule, at no cost. */

/* sip_system_info -- dims, precision and device bytes held by a handle
 * (Sec. 4.1: the solver module owns this memory). */
sip_status sip_system_info(sip_system h, int32_t dims[3], int32_t *precision, size_t *device_bytes);

/* sip_system_destroy -- free every device buffer of the handle (Sec. 4.1:
 * the redesigned solver allocates and releases the memory of its
 * coefficients and factors itself, through its own entry points).  The
 * caller must not have work in flight on it. */
sip_status sip_system_destroy(sip_system h);

/* ------------------------------------------------------------------------
 * Batched and served solves.  Sec. 4.1 turns SIP into a module that owns the
 * memory of its coefficients and factors, computes the factorisation in
 * advance and reuses it for all later iterations and time steps; Sec. 4.2
 * runs SIP on every block of a process one after another.  A server carries
 * both over to many blocks and right-hand sides on one GPU: its scheduler
 * thread admits requests while device memory (the HBM budget) and slots
 * allow, keeps SIP factors resident across requests of the same system, and
 * advances all admitted requests together in epochs of device launches
 * (continuous batching).  Requests that arrive while others run join the next
 * epoch.
 * ------------------------------------------------------------------------ */
typedef struct {
    size_t hbm_budget_bytes;    /* device bytes the server may hold (0 = 3/4 of free memory) */
    int32_t max_slots;          /* requests advanced together (<= 4096)      */
    int32_t epoch_iters;        /* iterations per epoch before re-admission  */
    int32_t max_queue;          /* pending requests before SIP_EBUSY         */
} sip_server_config;

typedef struct {
    uint64_t system_id;         /* caller's key: requests with the same id share factors */
    sip_problem problem;        /* coefficients (device); read when the system is first factorised */
    const double *b;            /* device right-hand side, read at admission  */
    double *x;                  /* device solution; written when done         */
    const double *x0;           /* device start vector or NULL (zeros)        */
    double rtol;
    int32_t max_iter;
    int32_t retain;             /* 1: keep this system's factors resident after the request
                                   (until evicted for room: least-recently-used first,
                                   never while a queued request names the system) */
    void *stream;               /* the caller's hipStream_t on which b, x0 and the
                                   coefficients were produced (NULL: the legacy default
                                   stream); the server reads them only after the work
                                   queued there before sip_batch_submit has run */
} sip_request;

typedef struct {
    sip_status status;          /* SIP_OK, SIP_ENOTCONV, SIP_EBREAKDOWN, SIP_EINVAL
                                   (non-finite b or x0) ...                   */
    sip_info info;
    double t_submit, t_admit, t_done;   /* seconds on the server's clock     */
    int32_t factorised;         /* 1 if this request triggered a factorisation */
} sip_result;

/* sip_server_create -- start a server on the current HIP device (Sec. 4.1:
 * the solver module sets up its own memory before the first solve).
 *   c     configuration (host, read during the call).  hbm_budget_bytes
 *         bounds the device bytes of resident systems plus running requests.
 *   out   receives the handle.
 * While no new request arrives, the admitted requests run in persistent
 * launches in which each iterates at its own pace, its sweeps published tile
 * by tile as the tiles they depend on are taken; while requests keep
 * arriving, in epochs of epoch_iters iterations.  Environment variables read
 * here: SIP_SERVER_PERSISTENT=1 / 0 forces one of the two modes;
 * SIP_SERVER_DATAFLOW=0 publishes whole sweeps in tile order instead; the
 * results are the same in every mode.  SIP_WAIT_LIMIT_MS (see sip_solve) is
 * read at every factorisation and step: a wait that times out fails the
 * requests of that launch with SIP_EDEVICE (a factorisation's with it too),
 * and the server goes on serving the others.
 * Errors: SIP_EINVAL (max_slots outside 1..4096, epoch_iters < 1,
 * max_queue < 1), SIP_ENOMEM (the server's own buffers), SIP_EDEVICE. */
sip_status sip_server_create(const sip_server_config *c, sip_server *out);

/* sip_batch_submit -- queue one solve (Sec. 4.1: the factorisation of a
 * system is computed once and reused for every later right-hand side;
 * requests with the same system_id share it while it stays resident).
 * Never blocks.  On success *ticket identifies the request.  The request's
 * device arrays must stay valid until sip_batch_poll reports it done; the
 * server reads them on its own stream after r->stream's earlier work.  A
 * resident system that a queued request names is not evicted.
 * Errors: SIP_EINVAL, SIP_EBUSY (queue full), SIP_ENOMEM (the request alone
 * exceeds the HBM budget), SIP_ECANCELLED (server shut down), SIP_EDEVICE
 * (the ordering event could not be recorded on r->stream). */
sip_status sip_batch_submit(sip_server s, const sip_request *r, uint64_t *ticket);

/* sip_batch_poll -- the result of a request (Sec. 3.2 / 4.1: the residual
 * norm the solver reports is the global one, here ||b - A x|| / ||b|| of the
 * returned x).  Returns SIP_PENDING while the request runs (waits up to
 * wait_ms milliseconds; 0 = do not wait, < 0 = wait until done), else SIP_OK
 * and fills *out (whose status field carries the solve outcome); x is then
 * written and visible to every stream.  A ticket can be collected once.
 * Errors: SIP_EINVAL (NULL, unknown or already collected ticket). */
sip_status sip_batch_poll(sip_server s, uint64_t ticket, int32_t wait_ms, sip_result *out);

/* sip_server_release -- drop a resident system's factors (no effect while
 * requests use it; Sec. 4.1: the module that computed the factorisation in
 * advance also frees it). */
sip_status sip_server_release(sip_server s, uint64_t system_id);

/* sip_server_stats -- counters of the server (Sec. 3: the paper measures
 * where the solver's time and memory traffic go; these count the work behind
 * them).  HOST array of SIP_SERVER_NSTATS: factorisations,
 * evictions, epochs, resident bytes, peak bytes, completed, admitted, sweep
 * launches, pairs formed, epochs replayed from a captured graph (an epoch's
 * sweeps are captured once the same launch parameters come up twice in a
 * row, i.e. while no request joins or leaves, and replayed until they
 * change; SIP_SERVER_GRAPHS=0, read by sip_server_create, launches every
 * epoch eagerly instead, with the same results).  With the environment variable SIP_SERVER_PAIRS=1
 * (read by sip_server_create), requests of one resident system with FP32
 * factors (SIP_MIXED, SIP_FP32), the same rtol and max_iter, admitted
 * together, are swept in pairs (the two-right-hand-side sweeps of
 * sip_solve_multi; each result is bitwise the one it gets alone).  It is off
 * by default: among many small concurrent blocks the pair sweeps' larger
 * register footprint (one workgroup per CU instead of two) costs more than
 * the shared coefficient traffic saves. */
#define SIP_SERVER_NSTATS 10
sip_status sip_server_stats(sip_server s, uint64_t out[SIP_SERVER_NSTATS]);

/* sip_server_shutdown -- stops the scheduler (Sec. 4.1: the solver module
 * ends its own work before its memory is released): the step in flight finishes,
 * then every request not yet done completes with status SIP_ECANCELLED (its
 * x is not written) and sip_batch_submit returns SIP_ECANCELLED.  Pollers
 * waiting on such requests wake up; every result stays pollable until
 * sip_server_destroy.  Returns once the server's kernels no longer touch any
 * request's arrays.  Thread-safe; later calls do nothing. */
sip_status sip_server_shutdown(sip_server s);

/* sip_server_destroy -- shuts the server down (if not yet) and frees it and
 * every resident factorisation (Sec. 4.1: the solver module releases the
 * coefficient and factor memory it allocated).  No other call on s may run
 * concurrently with it or follow it. */
sip_status sip_server_destroy(sip_server s);

/* Error reporting of every call above: the name of a status, the calling
 * thread's detail text of its last error, and the version of this ABI. */
const char *sip_status_str(sip_status st);
const char *sip_last_error(void);      /* thread-local detail of the last error */
int32_t sip_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SIP_H */
