// Multi-block domain on one GPU (include/sip.h, sip_blocks_*).
//
// The paper's solver runs SIP per block and couples the blocks only through
// values at block boundaries, exchanged once per iteration; with the
// non-blocking exchange every received value is the one of the previous
// exchange (Sec. 4.2).  Here every block is a factorised sip_system of its
// own; one iteration is
//   exchange: for each cell with a coupling into another block,
//             beff = b - sum A_nb x_nb (x_nb: the neighbour block's iterate),
//   forward sweep of every block on beff (one launch over all blocks),
//   domain control: the blocks' partial norms summed in block order, the
//             stop decision for the whole domain,
//   backward sweep + update of every block (one launch).
// The exchange tables (the paper's transfer tables between block patches)
// are built once on the host from the block cut planes.
#include "sip_internal.h"
#include "sip_runtime.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

using namespace sipk;

struct sip_blocks_s {
    int ni = 0, nj = 0, nk = 0;
    int nb[3] = {1, 1, 1};
    std::vector<int> cuts[3];
    int precision = 0;
    int nblk = 0;
    std::vector<sip_system> blk;
    std::vector<double *> beff;
    Job *d_jobs = nullptr;
    int2 *d_order_f = nullptr, *d_order_b = nullptr;
    int total = 0;
    LaunchCtl *lc = nullptr;
    XCell *d_cells = nullptr;
    XTerm *d_terms = nullptr;
    long long ncells = 0, nterms = 0;
    const double **d_b = nullptr;
    double **d_beff = nullptr;
    const double **d_x = nullptr;
    Ctl **d_ctl = nullptr;
    BlockPtrs ptrs{};
    Ctl *d_gctl = nullptr;
    Ctl *h_gctl = nullptr;   // pinned, 3 slots
    double *d_hist = nullptr, *h_hist = nullptr;
    int hist_cap = 0;
    double *tmp = nullptr;   // staging (7 block-sized natural-order arrays)
    size_t bytes = 0;
    uint64_t timeout_ticks = 0;
    uint32_t torture = 0;      // schedule_seed() at creation
    SweepPlan plan{};
};

namespace {

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

sip_status dalloc(void **p, size_t n, const char *what)
{
    if (hipMalloc(p, n ? n : 1) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return set_error(SIP_ENOMEM, "hipMalloc(%zu) for %s failed", n, what);
    }
    return SIP_OK;
}

void destroy(sip_blocks_s *h)
{
    if (!h) return;
    for (sip_system s : h->blk)
        if (s) sip_system_destroy(s);
    for (double *p : h->beff)
        if (p) (void)hipFree(p);
    for (void *p : {(void *)h->d_jobs, (void *)h->d_order_f, (void *)h->d_order_b, (void *)h->lc, (void *)h->d_cells,
                    (void *)h->d_terms, (void *)h->d_b, (void *)h->d_beff, (void *)h->d_x, (void *)h->d_ctl,
                    (void *)h->d_gctl, (void *)h->d_hist, (void *)h->tmp})
        if (p) (void)hipFree(p);
    if (h->h_gctl) (void)hipHostFree(h->h_gctl);
    if (h->h_hist) (void)hipHostFree(h->h_hist);
    delete h;
}

struct Box {
    int o[3], e[3];   // origin and extent in i, j, k
};

Box box_of(const sip_blocks_s *h, int q)
{
    const int bi = q % h->nb[0], bj = (q / h->nb[0]) % h->nb[1], bk = q / (h->nb[0] * h->nb[1]);
    const int b3[3] = {bi, bj, bk};
    Box x{};
    for (int d = 0; d < 3; d++) {
        x.o[d] = h->cuts[d][b3[d]];
        x.e[d] = h->cuts[d][b3[d] + 1] - x.o[d];
    }
    return x;
}

sip_status ensure_hist(sip_blocks_s *h, int n, hipStream_t s)
{
    if (n <= h->hist_cap) return SIP_OK;
    HIPTRY(hipStreamSynchronize(s));
    if (h->d_hist) (void)hipFree(h->d_hist);
    if (h->h_hist) (void)hipHostFree(h->h_hist);
    h->d_hist = nullptr;
    h->h_hist = nullptr;
    h->hist_cap = 0;
    const int cap = std::max(n, 64);
    TRY(dalloc((void **)&h->d_hist, (size_t)cap * 8, "history"));
    HIPTRY(hipHostMalloc((void **)&h->h_hist, (size_t)cap * 8, hipHostMallocDefault));
    h->hist_cap = cap;
    return SIP_OK;
}

// Exchange tables: every cell of a block with a coupling into another block,
// its terms (source block, source cell, direction, global index of the
// destination cell for the coefficient).
sip_status build_tables(sip_blocks_s *h, const sip_block_problem *p, hipStream_t s)
{
    std::vector<int> owner[3];
    for (int d = 0; d < 3; d++) {
        const int ext = d == 0 ? h->ni : d == 1 ? h->nj : h->nk;
        owner[d].resize(ext);
        for (int b = 0; b < h->nb[d]; b++)
            for (int c = h->cuts[d][b]; c < h->cuts[d][b + 1]; c++) owner[d][c] = b;
    }
    static const int off[7][3] = {{0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    std::vector<XCell> cells;
    std::vector<XTerm> terms;
    std::vector<uint8_t> dir;
    std::vector<long long> gidx;
    for (int q = 0; q < h->nblk; q++) {
        const Box bx = box_of(h, q);
        const Geom &g = h->blk[q]->g;
        for (int k = 0; k < bx.e[2]; k++)
            for (int j = 0; j < bx.e[1]; j++) {
                const bool face = k == 0 || k == bx.e[2] - 1 || j == 0 || j == bx.e[1] - 1;
                const int istep = face ? 1 : std::max(1, bx.e[0] - 1);
                for (int i = 0; i < bx.e[0]; i += istep) {
                    const int gi = bx.o[0] + i, gj = bx.o[1] + j, gk = bx.o[2] + k;
                    XCell xc{(uint32_t)q, (uint32_t)sheared_of(g, i, j, k), (uint32_t)terms.size(), 0u};
                    for (int d = 1; d < 7; d++) {
                        const int ni2 = gi + off[d][0], nj2 = gj + off[d][1], nk2 = gk + off[d][2];
                        if (ni2 < 0 || nj2 < 0 || nk2 < 0 || ni2 >= h->ni || nj2 >= h->nj || nk2 >= h->nk) continue;
                        const int sq = owner[0][ni2] + h->nb[0] * (owner[1][nj2] + h->nb[1] * owner[2][nk2]);
                        if (sq == q) continue;
                        const Box sb = box_of(h, sq);
                        const Geom &sg = h->blk[sq]->g;
                        terms.push_back(XTerm{(uint32_t)sq,
                                              (uint32_t)sheared_of(sg, ni2 - sb.o[0], nj2 - sb.o[1], nk2 - sb.o[2]),
                                              0.0});
                        dir.push_back((uint8_t)d);
                        gidx.push_back(((long long)gk * h->nj + gj) * h->ni + gi);
                    }
                    xc.end = (uint32_t)terms.size();
                    if (xc.end > xc.begin) cells.push_back(xc);
                }
            }
    }
    h->ncells = (long long)cells.size();
    h->nterms = (long long)terms.size();
    TRY(dalloc((void **)&h->d_cells, cells.size() * sizeof(XCell), "exchange cells"));
    TRY(dalloc((void **)&h->d_terms, terms.size() * sizeof(XTerm), "exchange terms"));
    uint8_t *d_dir = nullptr;
    long long *d_gidx = nullptr;
    sip_status st = dalloc((void **)&d_dir, dir.size(), "exchange setup");
    if (st == SIP_OK) st = dalloc((void **)&d_gidx, gidx.size() * sizeof(long long), "exchange setup");
    if (st == SIP_OK &&
        (hipMemcpyAsync(h->d_cells, cells.data(), cells.size() * sizeof(XCell), hipMemcpyHostToDevice, s) !=
             hipSuccess ||
         hipMemcpyAsync(h->d_terms, terms.data(), terms.size() * sizeof(XTerm), hipMemcpyHostToDevice, s) !=
             hipSuccess ||
         hipMemcpyAsync(d_dir, dir.data(), dir.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
         hipMemcpyAsync(d_gidx, gidx.data(), gidx.size() * sizeof(long long), hipMemcpyHostToDevice, s) !=
             hipSuccess ||
         launch_gather_coef(h->d_terms, h->nterms, d_dir, d_gidx, p->domain.a, s) != hipSuccess ||
         hipStreamSynchronize(s) != hipSuccess))
        st = set_error(SIP_EDEVICE, "exchange table setup failed");
    if (d_dir) (void)hipFree(d_dir);
    if (d_gidx) (void)hipFree(d_gidx);
    h->bytes += cells.size() * sizeof(XCell) + terms.size() * sizeof(XTerm);
    return st;
}

LaunchArgs args_of(const sip_blocks_s *h, bool backward)
{
    return LaunchArgs{h->d_jobs, backward ? h->d_order_b : h->d_order_f, h->lc, h->total, h->timeout_ticks,
                      h->torture};
}

sip_status stage_in(sip_blocks_s *h, const double *b, const double *x, uint32_t max_iter, double rtol, hipStream_t s)
{
    for (int q = 0; q < h->nblk; q++) {
        const Box bx = box_of(h, q);
        const long long m = (long long)bx.e[0] * bx.e[1] * bx.e[2];
        sip_system_s *bs = h->blk[q];
        double *tb = h->tmp, *tx = h->tmp + m;
        HIPTRY(launch_box_copy(b, tb, h->ni, h->nj, h->nk, bx.o[0], bx.o[1], bx.o[2], bx.e[0], bx.e[1], bx.e[2], 1, s));
        HIPTRY(launch_box_copy(x, tx, h->ni, h->nj, h->nk, bx.o[0], bx.o[1], bx.o[2], bx.e[0], bx.e[1], bx.e[2], 1, s));
        const double *src[2] = {tb, tx};
        HIPTRY(launch_to_sheared(bs->g, 2, src, bs->bx, bs->g.elems, SHEAR_F64, s));
        // cells without couplings into other blocks keep beff = b
        HIPTRY(hipMemcpyAsync(h->beff[q], bs->bx, (size_t)bs->g.elems * 8, hipMemcpyDeviceToDevice, s));
        HIPTRY(launch_init_ctl(bs->ctl, 1, max_iter, 0.0, 0, s));
    }
    HIPTRY(launch_init_ctl(h->d_gctl, 1, max_iter, rtol, 0, s));
    // ||b|| of the domain: the blocks' sweeps see beff, not b
    HIPTRY(launch_sumsq(b, (long long)h->ni * h->nj * h->nk, h->tmp, h->d_gctl, s));
    return SIP_OK;
}

sip_status stage_out(sip_blocks_s *h, double *x, hipStream_t s)
{
    for (int q = 0; q < h->nblk; q++) {
        const Box bx = box_of(h, q);
        sip_system_s *bs = h->blk[q];
        HIPTRY(launch_from_sheared(bs->g, bs->bx + bs->g.elems, 0, h->tmp, bs->ctl, s));
        HIPTRY(launch_box_copy(h->tmp, x, h->ni, h->nj, h->nk, bx.o[0], bx.o[1], bx.o[2], bx.e[0], bx.e[1], bx.e[2], 0,
                               s));
    }
    return SIP_OK;
}

// Exchange, forward sweep of all blocks, domain control; with `update`, then
// the backward sweep and x += d of all blocks.
sip_status step(sip_blocks_s *h, bool update, hipStream_t s)
{
    HIPTRY(launch_exchange(h->d_cells, h->ncells, h->d_terms, h->ptrs, s));
    HIPTRY(launch_forward(args_of(h, false), h->precision, h->plan, s));
    HIPTRY(launch_blocks_control(h->ptrs, h->nblk, h->d_gctl, h->d_hist, s));
    if (update) HIPTRY(launch_backward(args_of(h, true), h->precision, h->plan, s));
    return SIP_OK;
}

sip_status stop_status(uint32_t stop)
{
    switch (stop) {
    case RUN:
    case CONVERGED:
    case ZERO_RHS:
        return SIP_OK;
    case MAXITER:
        return SIP_ENOTCONV;
    case BREAKDOWN:
        return set_error(SIP_EBREAKDOWN, "SIP breakdown in a block");
    case BAD_INPUT:
        return set_error(SIP_EINVAL, "non-finite input: ||b|| or the residual of the start vector is not finite");
    case DIVERGED:
        return set_error(SIP_EBREAKDOWN, "the iteration diverged (non-finite residual)");
    default:
        return set_error(SIP_EDEVICE, "a device-side wait timed out");
    }
}

}  // namespace

extern "C" {

sip_status sip_blocks_factor(const sip_block_problem *p, void *stream, sip_blocks *out)
{
    const Range range("sip_blocks_factor");
    if (!p || !out) return set_error(SIP_EINVAL, "NULL argument");
    const sip_problem &dp = p->domain;
    if (dp.ni < 1 || dp.nj < 1 || dp.nk < 1) return set_error(SIP_EINVAL, "dims must be >= 1");
    if (dp.precision != SIP_FP64 && dp.precision != SIP_MIXED)
        return set_error(SIP_EINVAL, "a multi-block domain runs in SIP_FP64 or SIP_MIXED");
    for (int d = 0; d < 7; d++)
        if (!dp.a[d]) return set_error(SIP_EINVAL, "coefficient pointer %d is NULL", d);
    const int ext[3] = {dp.ni, dp.nj, dp.nk};
    for (int d = 0; d < 3; d++) {
        if (p->nb[d] < 1 || !p->cuts[d]) return set_error(SIP_EINVAL, "axis %d: need nb >= 1 and cut planes", d);
        if (p->cuts[d][0] != 0 || p->cuts[d][p->nb[d]] != ext[d])
            return set_error(SIP_EINVAL, "axis %d: cut planes must run from 0 to the extent", d);
        for (int b = 0; b < p->nb[d]; b++)
            if (p->cuts[d][b + 1] <= p->cuts[d][b]) return set_error(SIP_EINVAL, "axis %d: cut planes must rise", d);
    }
    const long long nblk = (long long)p->nb[0] * p->nb[1] * p->nb[2];
    if (nblk > 4096) return set_error(SIP_EINVAL, "at most 4096 blocks");
    hipStream_t s = (hipStream_t)stream;
    sip_blocks_s *h = new sip_blocks_s();
    h->ni = dp.ni;
    h->nj = dp.nj;
    h->nk = dp.nk;
    for (int d = 0; d < 3; d++) {
        h->nb[d] = p->nb[d];
        h->cuts[d].assign(p->cuts[d], p->cuts[d] + p->nb[d] + 1);
    }
    h->precision = dp.precision;
    h->nblk = (int)nblk;
    h->blk.assign(h->nblk, nullptr);
    h->beff.assign(h->nblk, nullptr);
    auto bail = [&](sip_status e) {
        (void)hipStreamSynchronize(s);
        destroy(h);
        return e;
    };
    long long maxc = 0;
    for (int q = 0; q < h->nblk; q++) {
        const Box bx = box_of(h, q);
        maxc = std::max(maxc, (long long)bx.e[0] * bx.e[1] * bx.e[2]);
    }
    // staging: 7 coefficient arrays of a block at set-up, b and x of a block
    // later, and the 256 partial sums of ||b||^2
    sip_status st = dalloc((void **)&h->tmp, (size_t)std::max(7 * maxc, 256ll) * 8, "block staging");
    if (st != SIP_OK) return bail(st);
    // every block: its coefficients gathered from the domain, factorised alone
    for (int q = 0; q < h->nblk; q++) {
        const Box bx = box_of(h, q);
        const long long m = (long long)bx.e[0] * bx.e[1] * bx.e[2];
        sip_problem bp = dp;
        bp.ni = bx.e[0];
        bp.nj = bx.e[1];
        bp.nk = bx.e[2];
        for (int d = 0; d < 7; d++) {
            double *dst = h->tmp + d * m;
            if (launch_box_copy(dp.a[d], dst, dp.ni, dp.nj, dp.nk, bx.o[0], bx.o[1], bx.o[2], bx.e[0], bx.e[1],
                                bx.e[2], 1, s) != hipSuccess)
                return bail(set_error(SIP_EDEVICE, "block gather failed"));
            bp.a[d] = dst;
        }
        st = sip_factor(&bp, stream, &h->blk[q]);   // synchronises the stream
        if (st != SIP_OK) return bail(st);
        h->bytes += h->blk[q]->bytes;
        st = dalloc((void **)&h->beff[q], (size_t)h->blk[q]->g.elems * 8, "effective right-hand side");
        if (st != SIP_OK) return bail(st);
        h->bytes += (size_t)h->blk[q]->g.elems * 8;
    }
    h->timeout_ticks = h->blk[0]->timeout_ticks;
    h->torture = h->blk[0]->torture;
    // all blocks sweep in one launch with many workgroups: the server's two
    // loader phases (SIP_SWEEP_PHASES overrides)
    h->plan = SweepPlan{};
    if (const char *e = getenv("SIP_SWEEP_PHASES")) {
        const int nl = atoi(e);
        if (nl >= 1 && nl <= MAX_PHASES) h->plan.phases = nl;
    }
    st = build_tables(h, p, s);
    if (st != SIP_OK) return bail(st);
    // one launch per sweep over all blocks
    std::vector<Job> jobs(h->nblk);
    std::vector<Geom> gs(h->nblk);
    std::vector<const double *> bp(h->nblk), xp(h->nblk);
    std::vector<Ctl *> cp(h->nblk);
    for (int q = 0; q < h->nblk; q++) {
        sip_system_s *bs = h->blk[q];
        jobs[q] = bs->job;
        jobs[q].b = h->beff[q];
        jobs[q].coupled = 1;
        gs[q] = bs->g;
        bp[q] = bs->bx;
        xp[q] = bs->bx + bs->g.elems;
        cp[q] = bs->ctl;
    }
    const std::vector<int2> of = topo_order(gs, false, h->torture), ob = topo_order(gs, true, h->torture);
    h->total = (int)of.size();
    if ((st = dalloc((void **)&h->d_jobs, jobs.size() * sizeof(Job), "jobs")) != SIP_OK ||
        (st = dalloc((void **)&h->d_order_f, of.size() * sizeof(int2), "order")) != SIP_OK ||
        (st = dalloc((void **)&h->d_order_b, ob.size() * sizeof(int2), "order")) != SIP_OK ||
        (st = dalloc((void **)&h->lc, sizeof(LaunchCtl), "launch control")) != SIP_OK ||
        (st = dalloc((void **)&h->d_b, h->nblk * sizeof(void *), "pointers")) != SIP_OK ||
        (st = dalloc((void **)&h->d_beff, h->nblk * sizeof(void *), "pointers")) != SIP_OK ||
        (st = dalloc((void **)&h->d_x, h->nblk * sizeof(void *), "pointers")) != SIP_OK ||
        (st = dalloc((void **)&h->d_ctl, h->nblk * sizeof(void *), "pointers")) != SIP_OK ||
        (st = dalloc((void **)&h->d_gctl, sizeof(Ctl), "control")) != SIP_OK)
        return bail(st);
    if (hipHostMalloc((void **)&h->h_gctl, 3 * sizeof(Ctl), hipHostMallocDefault) != hipSuccess)
        return bail(set_error(SIP_ENOMEM, "pinned control"));
    if (hipMemcpyAsync(h->d_jobs, jobs.data(), jobs.size() * sizeof(Job), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->d_order_f, of.data(), of.size() * sizeof(int2), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->d_order_b, ob.data(), ob.size() * sizeof(int2), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemsetAsync(h->lc, 0, sizeof(LaunchCtl), s) != hipSuccess ||
        hipMemcpyAsync(h->d_b, bp.data(), h->nblk * sizeof(void *), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->d_beff, h->beff.data(), h->nblk * sizeof(void *), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->d_x, xp.data(), h->nblk * sizeof(void *), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->d_ctl, cp.data(), h->nblk * sizeof(void *), hipMemcpyHostToDevice, s) != hipSuccess ||
        launch_init_ctl(h->d_gctl, 1, 0, 0.0, 1, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return bail(set_error(SIP_EDEVICE, "upload failed"));
    h->ptrs = BlockPtrs{h->d_b, h->d_beff, h->d_x, h->d_ctl};
    st = ensure_hist(h, 64, s);
    if (st != SIP_OK) return bail(st);
    *out = h;
    return SIP_OK;
}

sip_status sip_blocks_iterate(sip_blocks h, const double *b, double *x, int32_t n_iter, double *rel_res_hist,
                              void *stream)
{
    const Range range("sip_blocks_iterate");
    if (!h || !b || !x) return set_error(SIP_EINVAL, "NULL argument");
    if (n_iter < 0) return set_error(SIP_EINVAL, "n_iter must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    h->timeout_ticks = timeout_ticks_for(h->blk[0]->device, wait_limit_seconds());
    TRY(ensure_hist(h, n_iter + 1, s));
    TRY(stage_in(h, b, x, (uint32_t)n_iter, 0.0, s));
    for (int q = 0; q < n_iter; q++) TRY(step(h, true, s));
    TRY(step(h, false, s));   // residual of the final iterate
    TRY(stage_out(h, x, s));
    HIPTRY(hipMemcpyAsync(h->h_gctl, h->d_gctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    if (rel_res_hist) HIPTRY(hipMemcpyAsync(h->h_hist, h->d_hist, (size_t)(n_iter + 1) * 8, hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    const uint32_t stop = h->h_gctl->stop;
    if (rel_res_hist) {
        std::memcpy(rel_res_hist, h->h_hist, (size_t)(n_iter + 1) * 8);
        if (stop == ZERO_RHS)
            for (int q = 0; q <= n_iter; q++) rel_res_hist[q] = 0.0;
        if (stop == BAD_INPUT || stop == DIVERGED)   // no residual from the stopping iteration on
            for (int q = (int)h->h_gctl->iter; q <= n_iter; q++) rel_res_hist[q] = std::nan("");
    }
    if (stop == MAXITER || stop == RUN) return SIP_OK;
    return stop_status(stop);
}

sip_status sip_blocks_solve(sip_blocks h, const double *b, double *x, double rtol, int32_t max_iter, sip_info *info,
                            void *stream)
{
    const Range range("sip_blocks_solve");
    if (!h || !b || !x) return set_error(SIP_EINVAL, "NULL argument");
    if (!(rtol > 0.0) || max_iter < 0) return set_error(SIP_EINVAL, "need rtol > 0 and max_iter >= 0");
    hipStream_t s = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    h->timeout_ticks = timeout_ticks_for(h->blk[0]->device, wait_limit_seconds());
    TRY(ensure_hist(h, max_iter + 1, s));
    TRY(stage_in(h, b, x, (uint32_t)max_iter, rtol, s));
    hipEvent_t ev[2];
    HIPTRY(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    HIPTRY(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    long long launched = 0;
    sip_status st = SIP_OK;
    for (int c = 0; st == SIP_OK; c++) {
        for (int q = 0; q < CHUNK && st == SIP_OK; q++) st = step(h, true, s);
        if (st != SIP_OK) break;
        launched += CHUNK;
        if (hipMemcpyAsync(&h->h_gctl[c & 1], h->d_gctl, sizeof(Ctl), hipMemcpyDeviceToHost, s) != hipSuccess ||
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
            if (h->h_gctl[(c - 1) & 1].stop != RUN) break;
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (st != SIP_OK) {
        (void)hipStreamSynchronize(s);
        return st;
    }
    TRY(stage_out(h, x, s));
    HIPTRY(hipMemcpyAsync(&h->h_gctl[2], h->d_gctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    const Ctl &c = h->h_gctl[2];
    if (info) {
        info->iters = (int32_t)c.iter;
        info->rel_res = c.rho;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (c.stop == RUN) return set_error(SIP_EDEVICE, "solve ended without a stop decision");
    return stop_status(c.stop);
}

sip_status sip_blocks_info(sip_blocks h, int32_t *nblocks, size_t *device_bytes)
{
    if (!h) return set_error(SIP_EINVAL, "NULL handle");
    if (nblocks) *nblocks = h->nblk;
    if (device_bytes) *device_bytes = h->bytes;
    return SIP_OK;
}

sip_status sip_blocks_destroy(sip_blocks h)
{
    if (!h) return set_error(SIP_EINVAL, "NULL handle");
    destroy(h);
    return SIP_OK;
}

}  // extern "C"
