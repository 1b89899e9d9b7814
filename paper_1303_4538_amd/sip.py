"""Python binding of the SIP C ABI (include/sip.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream; every step of the method runs in the library's gfx950 kernels.  The
binding raises if the compiled library is missing; there is no CPU path.

Grid arrays are float64 CUDA (ROCm) tensors of shape (nk, nj, ni), C
contiguous; coefficients are a (7, nk, nj, ni) tensor in the order
P, W, E, S, N, B, T with signed entries (A_P x_P + sum A_nb x_nb = b_P).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsip.so")

SIP_OK, SIP_PENDING = 0, 1
SIP_EINVAL, SIP_ENOMEM, SIP_EBREAKDOWN, SIP_ENOTCONV = -1, -2, -3, -4
SIP_EDEVICE, SIP_EBUSY, SIP_ECANCELLED = -5, -6, -7
STATUS_NAMES = {0: "SIP_OK", 1: "SIP_PENDING", -1: "SIP_EINVAL", -2: "SIP_ENOMEM", -3: "SIP_EBREAKDOWN",
                -4: "SIP_ENOTCONV", -5: "SIP_EDEVICE", -6: "SIP_EBUSY", -7: "SIP_ECANCELLED"}
SIP_FP64, SIP_MIXED, SIP_FP32 = 0, 1, 2
PRECISIONS = {"fp64": SIP_FP64, "mixed": SIP_MIXED, "fp32": SIP_FP32,
              SIP_FP64: SIP_FP64, SIP_MIXED: SIP_MIXED, SIP_FP32: SIP_FP32}

# every symbol include/sip.h declares
EXPORTS = ("sip_factor", "sip_iterate", "sip_iterate_noalloc", "sip_solve", "sip_iterate_multi", "sip_solve_multi", "sip_export_factors",
           "sip_profile_sweeps", "sip_profile_sweeps_multi", "sip_tune", "sip_tune_save", "sip_tune_load",
           "sip_system_plan", "sip_system_solve_ms", "sip_system_info",
           "sip_system_destroy", "sip_blocks_factor", "sip_blocks_iterate", "sip_blocks_solve", "sip_blocks_info",
           "sip_blocks_destroy", "sip_server_create", "sip_batch_submit", "sip_batch_poll",
           "sip_server_release", "sip_server_stats", "sip_server_shutdown", "sip_server_destroy", "sip_status_str",
           "sip_last_error", "sip_abi_version")


class SipError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")


class Problem(ctypes.Structure):
    _fields_ = [("ni", ctypes.c_int32), ("nj", ctypes.c_int32), ("nk", ctypes.c_int32),
                ("a", ctypes.c_void_p * 7), ("alpha", ctypes.c_double), ("precision", ctypes.c_int32),
                ("storage", ctypes.c_int32)]


class BlockProblem(ctypes.Structure):
    _fields_ = [("domain", Problem), ("nb", ctypes.c_int32 * 3), ("cuts", ctypes.POINTER(ctypes.c_int32) * 3)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("rel_res", ctypes.c_double), ("seconds", ctypes.c_double)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("epoch_iters", ctypes.c_int32), ("max_queue", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("system_id", ctypes.c_uint64), ("problem", Problem), ("b", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("x0", ctypes.c_void_p), ("rtol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("retain", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("info", Info), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("factorised", ctypes.c_int32)]


_lib = None


def lib():
    """Load libsip.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"SIP HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    # torch first: the library must bind to the HIP runtime torch has loaded
    # (loaded before it, it can pull in a second runtime that sees no device)
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    L.sip_factor.argtypes = [ctypes.POINTER(Problem), vp, ctypes.POINTER(vp)]
    L.sip_iterate.argtypes = [vp, vp, vp, i32, ctypes.POINTER(dbl), vp]
    L.sip_iterate_noalloc.argtypes = [vp, vp, vp, i32, ctypes.POINTER(dbl), vp]
    L.sip_solve.argtypes = [vp, vp, vp, dbl, i32, ctypes.POINTER(Info), vp]
    L.sip_iterate_multi.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), i32, ctypes.POINTER(dbl), vp]
    L.sip_solve_multi.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), dbl, i32, ctypes.POINTER(Info), vp]
    L.sip_export_factors.argtypes = [vp, ctypes.POINTER(vp), vp]
    L.sip_tune.argtypes = [vp, vp, i32, ctypes.POINTER(i32), vp]
    L.sip_system_plan.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.sip_system_solve_ms.argtypes = [vp, ctypes.POINTER(dbl)]
    L.sip_tune_save.argtypes = [ctypes.c_char_p]
    L.sip_tune_load.argtypes = [ctypes.c_char_p]
    L.sip_blocks_factor.argtypes = [ctypes.POINTER(BlockProblem), vp, ctypes.POINTER(vp)]
    L.sip_blocks_iterate.argtypes = [vp, vp, vp, i32, ctypes.POINTER(dbl), vp]
    L.sip_blocks_solve.argtypes = [vp, vp, vp, dbl, i32, ctypes.POINTER(Info), vp]
    L.sip_blocks_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_size_t)]
    L.sip_blocks_destroy.argtypes = [vp]
    L.sip_profile_sweeps.argtypes = [vp, vp, vp, i32, ctypes.POINTER(dbl), vp]
    L.sip_profile_sweeps_multi.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), i32, ctypes.POINTER(dbl), vp]
    L.sip_system_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_size_t)]
    L.sip_system_destroy.argtypes = [vp]
    L.sip_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    L.sip_batch_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.sip_batch_poll.argtypes = [vp, ctypes.c_uint64, i32, ctypes.POINTER(Result)]
    L.sip_server_release.argtypes = [vp, ctypes.c_uint64]
    L.sip_server_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
    L.sip_server_shutdown.argtypes = [vp]
    L.sip_server_destroy.argtypes = [vp]
    for f in ("sip_factor", "sip_iterate", "sip_iterate_noalloc", "sip_solve", "sip_iterate_multi", "sip_solve_multi", "sip_export_factors",
              "sip_profile_sweeps", "sip_profile_sweeps_multi", "sip_tune", "sip_tune_save", "sip_tune_load",
              "sip_system_plan", "sip_system_solve_ms", "sip_system_info", "sip_system_destroy", "sip_blocks_factor", "sip_blocks_iterate", "sip_blocks_solve", "sip_blocks_info",
              "sip_blocks_destroy", "sip_server_create", "sip_batch_submit", "sip_batch_poll",
              "sip_server_release", "sip_server_stats", "sip_server_shutdown", "sip_server_destroy"):
        getattr(L, f).restype = ctypes.c_int32
    L.sip_status_str.argtypes = [ctypes.c_int32]
    L.sip_status_str.restype = ctypes.c_char_p
    L.sip_last_error.argtypes = []
    L.sip_last_error.restype = ctypes.c_char_p
    L.sip_abi_version.restype = ctypes.c_int32
    _lib = L
    return L


def _check(st, ok=(SIP_OK,)):
    if st not in ok:
        raise SipError(st, (lib().sip_last_error() or b"").decode())
    return st


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _grid(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor on the GPU")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


STORAGES = {"full": 0, "symmetric": 1}


def make_problem(A, alpha, precision, storage="full"):
    if A.dim() != 4 or A.shape[0] != 7:
        raise ValueError("A must have shape (7, nk, nj, ni)")
    _grid(A, A.shape, "A")
    nk, nj, ni = (int(v) for v in A.shape[1:])
    p = Problem()
    p.ni, p.nj, p.nk = ni, nj, nk
    for d in range(7):
        p.a[d] = A[d].data_ptr()
    p.alpha = float(alpha)
    p.precision = PRECISIONS[precision]
    p.storage = STORAGES[storage]
    return p


class System:
    """A factorised block resident on the GPU (owns its coefficient copy)."""

    def __init__(self, handle, dims, precision):
        self._h = handle
        self.ni, self.nj, self.nk = dims
        self.precision = precision

    @property
    def shape(self):
        return (self.nk, self.nj, self.ni)

    def info(self):
        dims = (ctypes.c_int32 * 3)()
        prec = ctypes.c_int32()
        nbytes = ctypes.c_size_t()
        _check(lib().sip_system_info(self._h, dims, ctypes.byref(prec), ctypes.byref(nbytes)))
        return dict(dims=tuple(dims), precision=prec.value, device_bytes=nbytes.value)

    def close(self):
        if self._h:
            lib().sip_system_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sip_factor(A, alpha=0.92, precision="fp64", stream=None, storage="full"):
    """Copy A (7, nk, nj, ni) into the library and factorise it (Stone).
    storage="symmetric" keeps only A_P, A_E, A_N, A_T for the sweeps."""
    p = make_problem(A, alpha, precision, storage)
    h = ctypes.c_void_p()
    _check(lib().sip_factor(ctypes.byref(p), _stream(stream), ctypes.byref(h)))
    return System(h, (p.ni, p.nj, p.nk), PRECISIONS[precision])


def sip_iterate(system, b, x, n_iter, history=True, stream=None, accept=()):
    """Apply n_iter SIP updates to x in place; returns rho_0..rho_n (numpy) or None.
    Statuses in accept (besides SIP_OK) return instead of raising SipError."""
    pb, px = _grid(b, system.shape, "b"), _grid(x, system.shape, "x")
    hist = np.zeros(int(n_iter) + 1) if history else None
    hp = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if history else None
    _check(lib().sip_iterate(system._h, pb, px, int(n_iter), hp, _stream(stream)), (SIP_OK,) + tuple(accept))
    return hist


def sip_iterate_noalloc(system, b, x, n_iter, history=True, stream=None, accept=()):
    """sip_iterate through the entry point that allocates no device memory
    (its per-call state lives in a static per-GPU scratch array)."""
    pb, px = _grid(b, system.shape, "b"), _grid(x, system.shape, "x")
    hist = np.zeros(int(n_iter) + 1) if history else None
    hp = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if history else None
    _check(lib().sip_iterate_noalloc(system._h, pb, px, int(n_iter), hp, _stream(stream)), (SIP_OK,) + tuple(accept))
    return hist


def _ok(raise_on_notconv, accept):
    return ((SIP_OK,) if raise_on_notconv else (SIP_OK, SIP_ENOTCONV)) + tuple(accept)


def sip_solve(system, b, x, rtol=1e-8, max_iter=100000, stream=None, raise_on_notconv=True, accept=()):
    """Iterate until ||b - A x|| <= rtol ||b||; x in/out.  Returns (status, iters, rel_res, seconds)."""
    pb, px = _grid(b, system.shape, "b"), _grid(x, system.shape, "x")
    info = Info()
    st = lib().sip_solve(system._h, pb, px, float(rtol), int(max_iter), ctypes.byref(info), _stream(stream))
    _check(st, _ok(raise_on_notconv, accept))
    return st, info.iters, info.rel_res, info.seconds


def _grids(ts, shape, name):
    ptrs = [_grid(t, shape, f"{name}[{r}]").value for r, t in enumerate(ts)]
    return (ctypes.c_void_p * len(ptrs))(*ptrs)


def sip_iterate_multi(system, bs, xs, n_iter, history=True, stream=None, accept=()):
    """n_iter SIP updates of several right-hand sides (pairs share one pass of
    the sweeps); xs updated in place.  Returns hist[r, n] (numpy) or None."""
    if len(bs) != len(xs) or not bs:
        raise ValueError("need as many x as b, at least one")
    pb, px = _grids(bs, system.shape, "b"), _grids(xs, system.shape, "x")
    hist = np.zeros((len(bs), int(n_iter) + 1)) if history else None
    hp = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if history else None
    _check(lib().sip_iterate_multi(system._h, len(bs), pb, px, int(n_iter), hp, _stream(stream)),
           (SIP_OK,) + tuple(accept))
    return hist


def sip_solve_multi(system, bs, xs, rtol=1e-8, max_iter=100000, stream=None, raise_on_notconv=True, accept=()):
    """Solve several right-hand sides (each stops at its own tolerance).
    Returns (status, [(iters, rel_res, seconds) per right-hand side])."""
    if len(bs) != len(xs) or not bs:
        raise ValueError("need as many x as b, at least one")
    pb, px = _grids(bs, system.shape, "b"), _grids(xs, system.shape, "x")
    info = (Info * len(bs))()
    st = lib().sip_solve_multi(system._h, len(bs), pb, px, float(rtol), int(max_iter), info, _stream(stream))
    _check(st, _ok(raise_on_notconv, accept))
    return st, [(i.iters, i.rel_res, i.seconds) for i in info]


def sip_export_factors(system, stream=None):
    """Factors in natural order as a (7, nk, nj, ni) float64 tensor: Lb, Lw, Ls, Lp, Un, Ue, Ut."""
    import torch
    out = torch.empty((7,) + system.shape, dtype=torch.float64, device="cuda")
    ptrs = (ctypes.c_void_p * 7)(*[out[d].data_ptr() for d in range(7)])
    _check(lib().sip_export_factors(system._h, ptrs, _stream(stream)))
    return out


def sip_profile_sweeps(system, b, x, n_iter, stream=None):
    """Average device milliseconds of one forward and one backward sweep over
    n_iter iterations (x updated in place).  Returns (fwd_ms, bwd_ms)."""
    pb, px = _grid(b, system.shape, "b"), _grid(x, system.shape, "x")
    ms = (ctypes.c_double * 2)()
    _check(lib().sip_profile_sweeps(system._h, pb, px, int(n_iter), ms, _stream(stream)))
    return ms[0], ms[1]


def sip_tune(system, b, n_iter=5, stream=None):
    """Time the sweep launch shapes on this system and keep the fastest
    (recorded for later systems of the same shape).  Returns the phase count."""
    pb = _grid(b, system.shape, "b")
    ph = ctypes.c_int32()
    _check(lib().sip_tune(system._h, pb, int(n_iter), ctypes.byref(ph), _stream(stream)))
    return ph.value


def sip_system_plan(system):
    """The handle's sweep plan: (loader phases, poll distance)."""
    ph, pd = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().sip_system_plan(system._h, ctypes.byref(ph), ctypes.byref(pd)))
    return ph.value, pd.value


def sip_system_solve_ms(system):
    """Device time (ms) of the persistent launches of the handle's last
    sip_solve / sip_solve_multi call (summed over its launches)."""
    ms = ctypes.c_double()
    _check(lib().sip_system_solve_ms(system._h, ctypes.byref(ms)))
    return ms.value


def sip_tune_save(path):
    """Write the process's tuning table (sip_tune results) to path, one JSON object per line."""
    _check(lib().sip_tune_save(os.fsencode(path)))


def sip_tune_load(path):
    """Merge a tuning table written by sip_tune_save into this process's table."""
    _check(lib().sip_tune_load(os.fsencode(path)))


def sip_profile_sweeps_multi(system, bs, xs, n_iter, stream=None):
    """sip_profile_sweeps for one pair of right-hand sides swept together."""
    if len(bs) != 2 or len(xs) != 2:
        raise ValueError("one pair of right-hand sides")
    pb, px = _grids(bs, system.shape, "b"), _grids(xs, system.shape, "x")
    ms = (ctypes.c_double * 2)()
    _check(lib().sip_profile_sweeps_multi(system._h, pb, px, int(n_iter), ms, _stream(stream)))
    return ms[0], ms[1]


# ----------------------------------------------------------------- multi-block domain

class Blocks:
    """A domain cut into blocks, each factorised alone and coupled through
    boundary values once per iteration (sip_blocks_*)."""

    def __init__(self, handle, dims, nblocks):
        self._h = handle
        self.ni, self.nj, self.nk = dims
        self.nblocks = nblocks

    @property
    def shape(self):
        return (self.nk, self.nj, self.ni)

    def iterate(self, b, x, n_iter, history=True, stream=None, accept=()):
        pb, px = _grid(b, self.shape, "b"), _grid(x, self.shape, "x")
        hist = np.zeros(int(n_iter) + 1) if history else None
        hp = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if history else None
        _check(lib().sip_blocks_iterate(self._h, pb, px, int(n_iter), hp, _stream(stream)), (SIP_OK,) + tuple(accept))
        return hist

    def solve(self, b, x, rtol=1e-8, max_iter=100000, stream=None, raise_on_notconv=True, accept=()):
        pb, px = _grid(b, self.shape, "b"), _grid(x, self.shape, "x")
        info = Info()
        st = lib().sip_blocks_solve(self._h, pb, px, float(rtol), int(max_iter), ctypes.byref(info), _stream(stream))
        _check(st, _ok(raise_on_notconv, accept))
        return st, info.iters, info.rel_res, info.seconds

    def info(self):
        n = ctypes.c_int32()
        nbytes = ctypes.c_size_t()
        _check(lib().sip_blocks_info(self._h, ctypes.byref(n), ctypes.byref(nbytes)))
        return dict(nblocks=n.value, device_bytes=nbytes.value)

    def close(self):
        if self._h:
            lib().sip_blocks_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sip_blocks_factor(A, cuts, alpha=0.92, precision="mixed", stream=None, storage="full"):
    """Cut the domain A (7, nk, nj, ni) at the planes cuts = (ci, cj, ck) (each
    from 0 to the extent) and factorise every block."""
    bp = BlockProblem()
    bp.domain = make_problem(A, alpha, precision, storage)
    arrs = [(ctypes.c_int32 * len(c))(*[int(v) for v in c]) for c in cuts]
    for d in range(3):
        bp.nb[d] = len(cuts[d]) - 1
        bp.cuts[d] = ctypes.cast(arrs[d], ctypes.POINTER(ctypes.c_int32))
    h = ctypes.c_void_p()
    _check(lib().sip_blocks_factor(ctypes.byref(bp), _stream(stream), ctypes.byref(h)))
    nblk = (len(cuts[0]) - 1) * (len(cuts[1]) - 1) * (len(cuts[2]) - 1)
    return Blocks(h, (bp.domain.ni, bp.domain.nj, bp.domain.nk), nblk)


# ----------------------------------------------------------------- server

class Server:
    """Continuous-batching SIP server (sip_server_create / sip_batch_*)."""

    def __init__(self, hbm_budget_bytes=0, max_slots=256, epoch_iters=8, max_queue=100000):
        c = ServerConfig(int(hbm_budget_bytes), int(max_slots), int(epoch_iters), int(max_queue))
        h = ctypes.c_void_p()
        _check(lib().sip_server_create(ctypes.byref(c), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, system_id, A, b, x, alpha=0.92, precision="mixed", rtol=1e-8, max_iter=100000,
               x0=None, retain=False, storage="full", stream=None):
        """Submit a solve; returns a ticket.  A may be None when the system is
        resident.  The server reads A, b and x0 after the work queued on
        `stream` (default: torch's current stream) before this call."""
        r = Request()
        r.system_id = int(system_id)
        if A is not None:
            r.problem = make_problem(A, alpha, precision, storage)
        else:
            nk, nj, ni = b.shape
            r.problem.ni, r.problem.nj, r.problem.nk = ni, nj, nk
            r.problem.alpha = float(alpha)
            r.problem.precision = PRECISIONS[precision]
        r.b = _grid(b, b.shape, "b").value
        r.x = _grid(x, b.shape, "x").value
        r.x0 = _grid(x0, b.shape, "x0").value if x0 is not None else None
        r.rtol = float(rtol)
        r.max_iter = int(max_iter)
        r.retain = 1 if retain else 0
        r.stream = _stream(stream).value
        t = ctypes.c_uint64()
        _check(lib().sip_batch_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = (A, b, x, x0)     # device arrays must outlive the request
        return t.value

    def poll(self, ticket, wait_ms=-1):
        """Returns None while pending, else a dict with the request outcome."""
        res = Result()
        st = lib().sip_batch_poll(self._h, ctypes.c_uint64(ticket), int(wait_ms), ctypes.byref(res))
        if st == SIP_PENDING:
            return None
        _check(st)
        self._keep.pop(ticket, None)
        return dict(status=res.status, iters=res.info.iters, rel_res=res.info.rel_res,
                    seconds=res.info.seconds, t_submit=res.t_submit, t_admit=res.t_admit,
                    t_done=res.t_done, factorised=res.factorised)

    def release(self, system_id):
        _check(lib().sip_server_release(self._h, ctypes.c_uint64(int(system_id))))

    def stats(self):
        out = (ctypes.c_uint64 * 10)()
        _check(lib().sip_server_stats(self._h, out))
        keys = ("factorisations", "evictions", "epochs", "resident_bytes", "peak_bytes", "completed",
                "admitted", "launches", "pairs", "graph_epochs")
        return dict(zip(keys, [int(v) for v in out]))

    def shutdown(self):
        """Stop scheduling: requests not done complete with SIP_ECANCELLED and
        stay pollable; later submissions are refused."""
        _check(lib().sip_server_shutdown(self._h))

    def close(self):
        if self._h:
            lib().sip_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
