// Request scheduler of the SIP server (sip_server_* / sip_batch_* in
// include/sip.h).
//
// The paper's redesigned solver owns its coefficients and computes the
// factorisation once, in advance, for all later solves (Sec. 4.1).  The
// server serves many blocks and right-hand sides that way on one device; this
// part of it is the host logic: the request queue, admission under a
// device-memory budget, residency and least-recently-used eviction of
// factorised systems, retirement, cancellation and shutdown, on one
// scheduler thread.  It is plain C++ with no device code: every step that
// touches a device goes through a Backend.  The library's backend
// (sip_server.hip) runs the HIP kernels; a test backend can run the same
// scheduler on the CPU.
#pragma once
#include "../../include/sip.h"

#include <cstddef>
#include <cstdint>
#include <memory>
#include <vector>

namespace sipk {

// Most running requests of one server (sip_server_config.max_slots).
constexpr int SERVER_MAX_SLOTS = 4096;

// Indices into the counters of sip_server_stats.
enum ServerStat {
    STAT_FACTORISATIONS = 0,
    STAT_EVICTIONS = 1,
    STAT_EPOCHS = 2,
    STAT_RESIDENT_BYTES = 3,
    STAT_PEAK_BYTES = 4,
    STAT_COMPLETED = 5,
    STAT_ADMITTED = 6,
    STAT_LAUNCHES = 7,
    STAT_PAIRS = 8,
    STAT_GRAPH_EPOCHS = 9,
};

// A system whose coefficients and factors are resident.  A backend derives
// its own type with the device arrays.
struct Resident {
    virtual ~Resident() = default;
    uint64_t id = 0;
    int32_t ni = 0, nj = 0, nk = 0;
    size_t bytes = 0;              // budget bytes (Backend::system_bytes)
    int refs = 0;                  // running requests using it (and admission's pin)
    bool factored = false;
    bool retain = false;           // keep after the last request (until evicted)
    sip_status broken = SIP_OK;    // the factorisation failed: requests end with this status
    uint64_t last_use = 0;         // least-recently-used clock
};

// One request.  A backend derives its own type with the per-request device
// state.
struct Req {
    virtual ~Req() = default;
    uint64_t ticket = 0;
    sip_request r{};
    double t_submit = 0, t_admit = 0, t_done = 0;
    int state = 0;                 // 0 queued, 1 running, 2 done
    sip_result res{};
    Resident *sys = nullptr;
    int slot = -1;                 // running slot, 0 .. max_slots - 1
    size_t bytes = 0;              // budget bytes charged while it runs
    int factorised = 0;
};

// How a running request stands after a step.
struct Outcome {
    bool done = false;
    sip_status status = SIP_OK;
    int iters = 0;
    double rho = 0.0;
};

// What a backend may ask of the scheduler while it works; every call takes
// the scheduler's lock, so a backend calls none while it holds one of its own
// that the scheduler's callers could wait for.
class Host {
public:
    // whether a request was submitted since the previous call
    virtual bool arrivals_since_last_step() = 0;
    // whether queued requests wait and a running slot is free
    virtual bool admission_waiting() = 0;
    // whether the server is shutting down
    virtual bool quitting() = 0;
    virtual void count(ServerStat stat, uint64_t n = 1) = 0;

protected:
    ~Host() = default;
};

// The device side of the server.  The scheduler calls every member from its
// own thread, except that new_request, check_problem, system_bytes,
// request_bytes and now are also called from submitting threads, and
// free_system from sip_server_release and sip_server_destroy.  check_problem,
// system_bytes, request_bytes, new_system, free_system, alloc_request and
// release_request run under the scheduler's lock, the others without it.
class Backend {
public:
    virtual ~Backend() = default;
    Host *host = nullptr;   // set by the scheduler before its thread starts

    // seconds on the server's clock
    virtual double now() = 0;
    // on the scheduler thread before its first step
    virtual void thread_start() {}
    // limits of a new system beyond the checks of sip_batch_submit
    virtual sip_status check_problem(const sip_problem &p) = 0;
    // budget bytes of a resident system, and of a running request on a
    // resident system (resident) or on a new one (resident == nullptr)
    virtual size_t system_bytes(const sip_problem &p) = 0;
    virtual size_t request_bytes(const sip_problem &p, const Resident *resident) = 0;
    // a request object for r; orders later reads of r's arrays after the
    // caller's earlier work
    virtual sip_status new_request(const sip_request &r, std::unique_ptr<Req> *out) = 0;
    // a resident system for q's problem, its arrays allocated
    virtual sip_status new_system(const Req &q, std::unique_ptr<Resident> *out) = 0;
    // frees a system's arrays; the scheduler destroys the object
    virtual void free_system(Resident *s) = 0;
    // allocates the state of an admitted request
    virtual sip_status alloc_request(Req *q) = 0;
    // frees a finished request's state; returns the budget bytes that it
    // gives back now (a request may hold them for a partner it shares
    // buffers with, which gives both back)
    virtual size_t release_request(Req *q) = 0;
    // later work of the scheduler reads the admitted requests' arrays
    virtual void wait_for_callers(const std::vector<Req *> &admitted) = 0;
    // factorises new systems (owners[k] brought sys[k] in); result[k] is
    // SIP_OK, or the status its requests end with
    virtual void factor(const std::vector<Resident *> &sys, const std::vector<Req *> &owners,
                        std::vector<sip_status> &result) = 0;
    // copies b and x0 of newly admitted requests in
    virtual void stage(std::vector<Req *> &ready) = 0;
    // advances every running request; a failure ends them all with its status
    virtual sip_status step(std::vector<Req *> &act) = 0;
    // whether q stopped in the last step (st: what step returned)
    virtual Outcome outcome(const Req *q, sip_status st) = 0;
    // writes x of the stopped requests to their callers' arrays (st as
    // above: on a failed step nothing is written); complete on return
    virtual void retire(const std::vector<Req *> &fin, sip_status st) = 0;
    // waits for all work of the backend
    virtual void drain() = 0;
};

// The backend of a new server: the library's GPU backend, or a test's own
// (the function is defined once per program).  May fill in cfg's defaults
// (hbm_budget_bytes 0).
sip_status make_backend(sip_server_config &cfg, std::unique_ptr<Backend> *out);

}  // namespace sipk
