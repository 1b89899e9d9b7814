"""Property tests of the CPU oracle over random tiny blocks (hypothesis):
extents 1..5 per axis (lines, planes, single cells and primes included),
alpha anywhere in [0, 1], random diagonally dominant M-matrices, symmetric or
not.  Each property is fixed by the method or by linear algebra, not by the
oracle's own formulas:

* L U - A is exactly Stone's partial-cancellation matrix N (the fill entries
  of L U and their alpha-weighted cancellation, nothing else);
* the forward and backward sweeps are the dense triangular solves with L, U;
* one SIP update is x + (L U)^-1 (b - A x), computed densely;
* the iteration's fixed point is the dense solution of A x = b.

The examples are derandomized, so every run checks the same cases.
"""
import numpy as np
import pytest

from tests import dense

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st   # noqa: E402

EXT = st.integers(min_value=1, max_value=5)
ALPHA = st.floats(min_value=0.0, max_value=1.0, allow_nan=False)
SEED = st.integers(min_value=0, max_value=2**32 - 1)


def scale(M):
    return max(1.0, np.abs(M).max())


@settings(max_examples=60, deadline=None, derandomize=True)
@given(ni=EXT, nj=EXT, nk=EXT, alpha=ALPHA, seed=SEED, sym=st.booleans())
def test_partial_cancellation(ora, ni, nj, nk, alpha, seed, sym):
    A = dense.random_mmatrix(ni, nj, nk, np.random.default_rng(seed), symmetric=sym)
    L, U = dense.dense_LU(ora.factor(A, alpha))
    M = L @ U
    assert np.abs((M - dense.dense_A(A)) - dense.stone_N(M, ni, nj, nk, alpha)).max() <= 1e-13 * scale(M)


@settings(max_examples=40, deadline=None, derandomize=True)
@given(ni=EXT, nj=EXT, nk=EXT, alpha=ALPHA, seed=SEED)
def test_sweeps_and_update_are_dense_solves(ora, ni, nj, nk, alpha, seed):
    rng = np.random.default_rng(seed)
    A = dense.random_mmatrix(ni, nj, nk, rng)
    LU = ora.factor(A, alpha)
    L, U = dense.dense_LU(LU)
    shape = (nk, nj, ni)
    r = rng.uniform(-1, 1, shape)
    y = ora.forward(LU, r)
    assert np.abs(L @ y.ravel() - r.ravel()).max() <= 1e-12 * scale(L) * max(1, np.abs(y).max())
    d = ora.backward(LU, y)
    assert np.abs(U @ d.ravel() - y.ravel()).max() <= 1e-12 * scale(U) * max(1, np.abs(d).max())
    b = rng.uniform(-1, 1, shape)
    x0 = rng.uniform(-0.5, 0.5, shape)
    x1, _ = ora.iterate(A, LU, b, x0, 1)
    Ad = dense.dense_A(A)
    want = x0.ravel() + np.linalg.solve(L @ U, b.ravel() - Ad @ x0.ravel())
    assert np.abs(x1.ravel() - want).max() <= 1e-11 * max(1, np.abs(want).max())


@settings(max_examples=25, deadline=None, derandomize=True)
@given(ni=EXT, nj=EXT, nk=EXT, seed=SEED)
def test_fixed_point_is_the_dense_solution(ora, ni, nj, nk, seed):
    rng = np.random.default_rng(seed)
    A = dense.random_mmatrix(ni, nj, nk, rng)
    b = rng.uniform(-1, 1, (nk, nj, ni))
    x, it, rr, _ = ora.solve(A, ora.factor(A, 0.92), b, np.zeros_like(b), 1e-12, 500)
    assert rr <= 1e-12
    xs = np.linalg.solve(dense.dense_A(A), b.ravel())
    assert np.abs(x.ravel() - xs).max() <= 1e-9 * max(1, np.abs(xs).max())
