"""ctypes front end of the plain-C FP64 SIP oracle (``sip_oracle.c``).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
baseline of the benchmark; never by the library path.  The C source states the
equations (Stone's construction of the SIP factorisation, the residual, the
forward/backward substitutions and the defect-correction update) and the
conventions; this module only marshals numpy arrays.

Array conventions: a grid of ``ni x nj x nk`` cells is a numpy array of shape
``(nk, nj, ni)`` (C order, i fastest).  Coefficients ``A`` have shape
``(7, nk, nj, ni)`` in the order P, W, E, S, N, B, T; factors ``LU`` have shape
``(7, nk, nj, ni)`` in the order Lb, Lw, Ls, Lp, Un, Ue, Ut.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sip_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)


def build(force=True):
    """Compile the oracle with gcc (-O2, no FP contraction, no fast-math)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([
        "gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
        "-shared", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i, l, d = ctypes.c_int, ctypes.c_long, ctypes.c_double
    lib.oracle_factor.argtypes = [i, i, i, _D, d, _D]
    lib.oracle_factor.restype = i
    lib.oracle_residual.argtypes = [i, i, i, _D, _D, _D, _D]
    lib.oracle_residual.restype = None
    lib.oracle_residual_f32.argtypes = [i, i, i, _F, _F, _F, _F]
    lib.oracle_residual_f32.restype = None
    lib.oracle_norm2.argtypes = [_D, ctypes.c_size_t]
    lib.oracle_norm2.restype = d
    lib.oracle_forward.argtypes = [i, i, i, _D, _D, _D]
    lib.oracle_forward.restype = None
    lib.oracle_backward.argtypes = [i, i, i, _D, _D, _D]
    lib.oracle_backward.restype = None
    lib.oracle_forward_f32.argtypes = [i, i, i, _F, _F, _F]
    lib.oracle_forward_f32.restype = None
    lib.oracle_backward_f32.argtypes = [i, i, i, _F, _F, _F]
    lib.oracle_backward_f32.restype = None
    lib.oracle_iterate.argtypes = [i, i, i, _D, _D, _D, _D, l, i, _D]
    lib.oracle_iterate.restype = l
    lib.oracle_solve.argtypes = [i, i, i, _D, _D, _D, _D, d, l, i, _D, _D]
    lib.oracle_solve.restype = l
    _I = ctypes.POINTER(ctypes.c_int)
    lib.oracle_blocks_run.argtypes = [i, i, i, _D, d, _D, _D, i, _I, i, _I, i, _I, l, d, i, _D, _D]
    lib.oracle_blocks_run.restype = l
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_D):
    return a.ctypes.data_as(t)


def _dims(a):
    nk, nj, ni = a.shape[-3:]
    return int(ni), int(nj), int(nk)


def factor(A, alpha):
    """Stone factorisation; returns LU (7, nk, nj, ni).  Raises on breakdown."""
    A = _f64(A)
    ni, nj, nk = _dims(A)
    LU = np.zeros_like(A)
    rc = _load().oracle_factor(ni, nj, nk, _ptr(A), float(alpha), _ptr(LU))
    if rc != 0:
        raise FloatingPointError("SIP factorisation breakdown")
    return LU


def residual(A, b, x):
    """r = b - A x (FP64)."""
    A, b, x = _f64(A), _f64(b), _f64(x)
    ni, nj, nk = _dims(A)
    r = np.empty_like(b)
    _load().oracle_residual(ni, nj, nk, _ptr(A), _ptr(b), _ptr(x), _ptr(r))
    return r


def residual_f32(A, b, x):
    """All-FP32 form: r = b - A x with FP32 inputs and FP32 arithmetic."""
    A = np.ascontiguousarray(A, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32)
    ni, nj, nk = _dims(A)
    r = np.empty_like(b)
    _load().oracle_residual_f32(ni, nj, nk, _ptr(A, _F), _ptr(b, _F), _ptr(x, _F), _ptr(r, _F))
    return r


def _mode(mixed, fp32):
    if mixed and fp32:
        raise ValueError("choose one of mixed and fp32")
    return 2 if fp32 else 1 if mixed else 0


def norm2(v):
    v = _f64(v).ravel()
    return _load().oracle_norm2(_ptr(v), v.size)


def forward(LU, r):
    LU, r = _f64(LU), _f64(r)
    ni, nj, nk = _dims(LU)
    y = np.empty_like(r)
    _load().oracle_forward(ni, nj, nk, _ptr(LU), _ptr(r), _ptr(y))
    return y


def backward(LU, y):
    LU, y = _f64(LU), _f64(y)
    ni, nj, nk = _dims(LU)
    d = np.empty_like(y)
    _load().oracle_backward(ni, nj, nk, _ptr(LU), _ptr(y), _ptr(d))
    return d


def forward_f32(LU32, r32):
    LU32 = np.ascontiguousarray(LU32, dtype=np.float32)
    r32 = np.ascontiguousarray(r32, dtype=np.float32)
    ni, nj, nk = _dims(LU32)
    y = np.empty_like(r32)
    _load().oracle_forward_f32(ni, nj, nk, _ptr(LU32, _F), _ptr(r32, _F), _ptr(y, _F))
    return y


def backward_f32(LU32, y32):
    LU32 = np.ascontiguousarray(LU32, dtype=np.float32)
    y32 = np.ascontiguousarray(y32, dtype=np.float32)
    ni, nj, nk = _dims(LU32)
    d = np.empty_like(y32)
    _load().oracle_backward_f32(ni, nj, nk, _ptr(LU32, _F), _ptr(y32, _F), _ptr(d, _F))
    return d


def iterate(A, LU, b, x0, n_iter, mixed=False, fp32=False):
    """Run n_iter SIP updates from x0.  Returns (x, hist) with hist[n] = rho_n,
    n = 0..n_iter (relative residual of the n-th iterate).  mixed: FP32 sweeps
    with FP64 residual and update; fp32: everything in FP32 (x returned as
    FP64)."""
    A, LU, b = _f64(A), _f64(LU), _f64(b)
    x = _f64(x0).copy()
    ni, nj, nk = _dims(A)
    hist = np.zeros(int(n_iter) + 1)
    rc = _load().oracle_iterate(ni, nj, nk, _ptr(A), _ptr(LU), _ptr(b), _ptr(x),
                                int(n_iter), _mode(mixed, fp32), _ptr(hist))
    if rc < 0:
        raise MemoryError("oracle allocation failed")
    return x, hist


def solve(A, LU, b, x0, rtol, max_iter, mixed=False, fp32=False):
    """Iterate until rho_n <= rtol (or max_iter updates).
    Returns (x, iterations, rel_res, hist[0..iterations])."""
    A, LU, b = _f64(A), _f64(LU), _f64(b)
    x = _f64(x0).copy()
    ni, nj, nk = _dims(A)
    hist = np.zeros(int(max_iter) + 1)
    rr = ctypes.c_double(0.0)
    it = _load().oracle_solve(ni, nj, nk, _ptr(A), _ptr(LU), _ptr(b), _ptr(x), float(rtol),
                              int(max_iter), _mode(mixed, fp32), _ptr(hist), ctypes.byref(rr))
    if it < 0:
        raise MemoryError("oracle allocation failed")
    return x, int(it), float(rr.value), hist[: it + 1]


def blocks(A, alpha, b, x0, cuts, n_iter, rtol=0.0, mixed=False):
    """Multi-block domain: the block cut planes ``cuts = (ci, cj, ck)`` (each
    starting at 0 and ending at the extent) split the domain into blocks, each
    factorised on its own and coupled through the residual of the whole
    domain once per iteration.  Runs n_iter updates, or stops at the first
    rho_n <= rtol (rtol > 0).  Returns (x, iterations, rel_res, hist)."""
    A, b = _f64(A), _f64(b)
    x = _f64(x0).copy()
    ni, nj, nk = _dims(A)
    cs = [np.ascontiguousarray(c, dtype=np.intc) for c in cuts]
    for c, ext in zip(cs, (ni, nj, nk)):
        if c[0] != 0 or c[-1] != ext or np.any(np.diff(c) < 1):
            raise ValueError("cut planes must rise from 0 to the extent")
    hist = np.zeros(int(n_iter) + 1)
    rr = ctypes.c_double(0.0)
    P = ctypes.POINTER(ctypes.c_int)
    it = _load().oracle_blocks_run(ni, nj, nk, _ptr(A), float(alpha), _ptr(b), _ptr(x),
                                   len(cs[0]) - 1, cs[0].ctypes.data_as(P), len(cs[1]) - 1, cs[1].ctypes.data_as(P),
                                   len(cs[2]) - 1, cs[2].ctypes.data_as(P), int(n_iter), float(rtol),
                                   1 if mixed else 0, _ptr(hist), ctypes.byref(rr))
    if it == -2:
        raise FloatingPointError("SIP factorisation breakdown in a block")
    if it < 0:
        raise MemoryError("oracle allocation failed")
    return x, int(it), float(rr.value), hist[: it + 1]
