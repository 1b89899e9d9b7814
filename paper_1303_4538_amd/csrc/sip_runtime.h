// Host-side runtime structures of the SIP library.
#pragma once
#include "../../include/sip.h"
#include "sip_host.h"
#include "sip_internal.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <string>
#include <vector>

namespace sipk {

// Named host range around a library call (rocprofv3 --marker-trace shows it
// beside the kernels it launched); costs a function call when no tool listens.
struct Range {
    explicit Range(const char *name) { roctxRangePush(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

constexpr int CHUNK = 8;   // iterations per graph-captured launch chunk

uint64_t timeout_ticks_for(int device, double seconds);
// Bound of the device-side waits in seconds: 2, or SIP_WAIT_LIMIT_MS (a test
// hook: 0 makes every wait that is not met at once time out).
double wait_limit_seconds();
// Ticket order of a launch over the jobs gs: every tile after its upstream
// neighbours (W and S; E and N for the backward sweep).  seed 0: by
// anti-diagonal; otherwise a random order with the same property (race
// testing, see schedule_seed).
std::vector<int2> topo_order(const std::vector<Geom> &gs, bool backward, uint32_t seed = 0);
// Race testing: the environment variable SIP_SCHEDULE_SEED (read when a
// handle is created), when set to a nonzero integer, gives the handle a
// random ticket order and pauses the sweep and factorisation waves at
// pseudo-random steps.  Results must not change.
uint32_t schedule_seed();
size_t system_bytes(const Geom &g, int fp32);
// The sweep plan sip_tune chose for this shape and arithmetic, if any.
bool tuned_plan(const Geom &g, int arith, int sym, SweepPlan *out);

}  // namespace sipk

struct sip_system_s {
    sipk::Geom g{};
    int fp32 = 0;                   // factors stored in FP32
    int precision = 0;              // sip_precision = the sweeps' Arith
    int sym = 0;                    // coefficients in the symmetric storage for the sweeps
    double alpha = 0.0;
    int device = 0;
    uint64_t timeout_ticks = 0;
    uint32_t torture = 0;      // schedule_seed() at creation
    size_t bytes = 0;
    double *A = nullptr;            // 7 * elems
    void *LU = nullptr;             // 7 * elems of FP64 or FP32
    double *bx = nullptr;           // b then x, elems each (FP64, or FP32 in the all-FP32 arithmetic)
    void *y = nullptr;
    uint64_t *face = nullptr;
    double *part = nullptr;
    sipk::Ctl *ctl = nullptr;
    double *hist = nullptr;
    int hist_cap = 0;
    sipk::Job job{};                // sweeps
    sipk::Job job_factor{};         // factorisation (wider face words)
    sipk::Job *d_job = nullptr;
    sipk::Job *d_job_factor = nullptr;
    int2 *order_f = nullptr, *order_b = nullptr;
    sipk::LaunchCtl *lc = nullptr;
    sipk::Ctl *h_ctl = nullptr;     // pinned, 4 slots
    double *h_hist = nullptr;       // pinned
    // two right-hand sides swept together (allocated on first use): b pairs
    // then x pairs, y pairs, own face words and control blocks
    double *mbx = nullptr;
    void *my = nullptr;
    uint64_t *mface = nullptr;
    double *mpart = nullptr;
    sipk::Ctl *mctl = nullptr;      // 3: the sweep's, then one per right-hand side
    double *mhist = nullptr;        // 2 * mhist_cap
    int mhist_cap = 0;
    sipk::Job mjob{};
    sipk::Job *d_mjob = nullptr;
    sipk::Ctl *h_mctl = nullptr;    // pinned, 3 slots of 3
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t chunk_exec = nullptr;
    uint64_t chunk_ticks = 0;                 // the wait bound the chunk graph was captured with
    // persistent solves (allocated on first use): the tile orders, the task
    // queue and its control block with two device flags (pause, stopped)
    int num_cu = 0;
    int *p_tord = nullptr, *p_off = nullptr;
    sipk::Task *p_tasks = nullptr;
    sipk::PersistCtl *p_pc = nullptr;
    uint32_t *p_flags = nullptr;
    uint32_t p_cap = 0;
    std::vector<sipk::Task> p_host_tasks;   // host image of the queue uploaded before every solve
    sipk::PersistCtl p_host_pc{};
    hipEvent_t p_ev[2] = {nullptr, nullptr};  // recorded around the latest persistent solve launch
    bool p_timed = false;                     // the last solve call ran persistent launches
    double p_ms = 0.0;                        // their summed device time (ms)
    sipk::SweepPlan plan{};
};
