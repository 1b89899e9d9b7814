"""Pins of the oracle's mixed form (FP32 factors and sweeps, FP64 residual and
update: the defect-correction reading of the paper's single-precision
relaxation, Sec. 4.1) against facts fixed by floating-point arithmetic.

Both mixed drivers are covered: the single-block iteration and the
multi-block domain iteration (Sec. 4.2).  None of these checks re-types the
oracle: they use closed forms of two-precision iterative refinement on
diagonal systems, the representability of the first update in FP32, and the
dense defect correction with the FP32-rounded factors.

A mixed form that ran its sweeps in FP64, or skipped the rounding of r or of
the factors to FP32, gives x_1 = b / A_P on the diagonal systems and an x_1
with more than 24 significant bits in general, and fails the first two groups.
"""
import numpy as np
import pytest

from tests import dense
from paper_1303_4538_amd import problems

U32 = 2.0 ** -24          # unit roundoff of FP32 (round to nearest)


def _diagonal_system(ni, nj, nk, seed):
    """A = diag(A_P) with A_P a power of two per cell; b in [-1, 1] drawn in
    FP64, so almost no entry is an FP32 number."""
    rng = np.random.default_rng(seed)
    A = np.zeros((7, nk, nj, ni))
    A[0] = 2.0 ** rng.integers(-4, 5, (nk, nj, ni))
    b = rng.uniform(-1, 1, (nk, nj, ni))
    return A, b


def _fp32_exact(v):
    return np.array_equal(v.astype(np.float32).astype(np.float64), v)


def _check_refinement(x1, x2, x3, b, ap):
    """Iterative refinement of diag(ap) x = b with the correction solved in
    FP32 and the residual and update in FP64.  From x_0 = 0, r_0 = b is rounded
    to FP32 and divided exactly by the power of two: x_1 = fl32(b) / ap.  Each
    later residual b - ap x_n is exact in FP64 (Sterbenz) and its FP32 rounding
    keeps 24 more bits, so |x_2 - b/ap| <= 2^-48 |b/ap| and x_3 = b / ap
    exactly (the last residual has at most 5 significant bits)."""
    exact = b / ap
    assert np.array_equal(x1, b.astype(np.float32).astype(np.float64) / ap)
    assert _fp32_exact(x1 * ap)
    # the pin discriminates: FP64 sweeps would give b / ap already
    assert np.count_nonzero(x1 != exact) > 0.9 * b.size
    assert np.all(np.abs(x1 - exact) <= U32 * np.abs(exact))
    assert np.all(np.abs(x2 - exact) <= U32 * U32 * np.abs(exact))
    assert np.array_equal(x3, exact)


def test_mixed_diagonal_is_two_precision_refinement(ora):
    ni, nj, nk = 5, 4, 6
    A, b = _diagonal_system(ni, nj, nk, 70)
    LU = ora.factor(A, 0.92)
    xs = [ora.iterate(A, LU, b, np.zeros_like(b), n, mixed=True)[0] for n in (1, 2, 3)]
    _check_refinement(*xs, b, A[0])
    _, hist = ora.iterate(A, LU, b, np.zeros_like(b), 3, mixed=True)
    assert hist[0] == 1.0
    assert 0.0 < hist[1] <= U32 and hist[2] <= U32 * U32 and hist[3] == 0.0
    # the FP64 form solves the diagonal system in one update
    x64, h64 = ora.iterate(A, LU, b, np.zeros_like(b), 1)
    assert np.array_equal(x64, b / A[0]) and h64[1] == 0.0


def test_blocks_mixed_diagonal_is_two_precision_refinement(ora):
    ni, nj, nk = 6, 4, 6
    A, b = _diagonal_system(ni, nj, nk, 71)
    cuts = ([0, 3, 6], [0, 2, 4], [0, 2, 4, 6])
    xs = [ora.blocks(A, 0.92, b, np.zeros_like(b), cuts, n, mixed=True)[0] for n in (1, 2, 3)]
    _check_refinement(*xs, b, A[0])
    x64 = ora.blocks(A, 0.92, b, np.zeros_like(b), cuts, 1)[0]
    assert np.array_equal(x64, b / A[0])


def _system(kind, ni, nj, nk, rng):
    if kind == "cd":
        return problems.convection_diffusion(ni, nj, nk, rng)
    if kind == "poisson":
        return problems.poisson(ni, nj, nk)
    return problems.stretched_poisson(ni, nj, nk)


@pytest.mark.parametrize("kind", ["cd", "poisson", "stretched"])
def test_mixed_first_update_is_single_precision(ora, kind):
    """From x_0 = 0 the first update is the FP32 correction widened to FP64,
    so every entry of x_1 is an FP32 number; the FP64 form's x_1 is not."""
    ni, nj, nk = 7, 6, 5
    rng = np.random.default_rng(72)
    A = _system(kind, ni, nj, nk, rng)
    b = rng.uniform(-1, 1, (nk, nj, ni))
    LU = ora.factor(A, 0.92)
    x1, _ = ora.iterate(A, LU, b, np.zeros_like(b), 1, mixed=True)
    assert _fp32_exact(x1)
    x64, _ = ora.iterate(A, LU, b, np.zeros_like(b), 1)
    assert not _fp32_exact(x64)
    # and the correction is the FP32 solve of the rounded residual with the
    # rounded factors, within a few FP32 roundings
    L, U = dense.dense_LU(LU.astype(np.float32).astype(np.float64))
    d = np.linalg.solve(L @ U, b.astype(np.float32).astype(np.float64).ravel())
    assert np.abs(x1.ravel() - d).max() <= 32 * U32 * np.abs(d).max()


def test_blocks_mixed_first_update_is_single_precision(ora):
    ni, nj, nk = 8, 6, 5
    A = problems.convection_diffusion(ni, nj, nk, np.random.default_rng(73))
    b = np.random.default_rng(74).uniform(-1, 1, (nk, nj, ni))
    cuts = ([0, 4, 8], [0, 3, 6], [0, 5])
    x1 = ora.blocks(A, 0.92, b, np.zeros_like(b), cuts, 1, mixed=True)[0]
    assert _fp32_exact(x1)
    assert not _fp32_exact(ora.blocks(A, 0.92, b, np.zeros_like(b), cuts, 1)[0])


# The bound below is also the GPU parity bar of the mixed form: the GPU rounds
# the same operands (FP64 factors to FP32, r to FP32) and differs from the
# oracle only in the order of its FP32 operations and in multiplying by a
# rounded 1/Lp where the oracle divides by Lp, so each side is within MIXED_B
# of the exact defect correction and the two within 2 MIXED_B of each other.
MIXED_B = 2e-6            # about 32 u32 of max |x_n|


@pytest.mark.parametrize("kind", ["cd", "poisson", "stretched"])
def test_mixed_tracks_dense_defect_correction(ora, kind):
    """Eight mixed updates stay within MIXED_B max|x| of the defect correction
    x_{n+1} = x_n + (L32 U32)^-1 fl32(b - A x_n) computed densely in FP64 from
    the FP32-rounded factors; rho_n is the FP64 residual norm of x_n."""
    ni, nj, nk = 6, 5, 7
    rng = np.random.default_rng(42)
    A = _system(kind, ni, nj, nk, rng)
    b = rng.uniform(-1, 1, (nk, nj, ni))
    LU = ora.factor(A, 0.92)
    n = 8
    x, hist = ora.iterate(A, LU, b, np.zeros_like(b), n, mixed=True)
    L, U = dense.dense_LU(LU.astype(np.float32).astype(np.float64))
    M = L @ U
    Ad = dense.dense_A(A)
    nb = np.linalg.norm(b.ravel())
    xr = np.zeros(b.size)
    for m in range(n + 1):
        xm = ora.iterate(A, LU, b, np.zeros_like(b), m, mixed=True)[0].ravel()
        assert np.abs(xm - xr).max() <= MIXED_B * max(np.abs(xr).max(), 1e-300)
        r = b.ravel() - Ad @ xm
        assert abs(hist[m] - np.linalg.norm(r) / nb) <= 1e-14
        if m < n:
            r = b.ravel() - Ad @ xr
            xr = xr + np.linalg.solve(M, r.astype(np.float32).astype(np.float64))
    assert np.array_equal(x.ravel(), xm)


def test_blocks_mixed_is_dense_block_jacobi_with_rounded_factors(ora):
    """Multi-block mixed iterates: x_{n+1} = x_n + M32^-1 fl32(b - A x_n) with
    M32 the block-diagonal matrix of each block's own FP32-rounded SIP factors."""
    ni, nj, nk = 6, 4, 5
    A = problems.convection_diffusion(ni, nj, nk, np.random.default_rng(75))
    b = np.random.default_rng(76).uniform(-1, 1, (nk, nj, ni))
    ci, cj, ck = [0, 3, 6], [0, 2, 4], [0, 5]
    n = 5
    M = np.zeros((b.size, b.size))
    idx = np.arange(b.size).reshape(nk, nj, ni)
    for bk in range(len(ck) - 1):
        for bj in range(len(cj) - 1):
            for bi in range(len(ci) - 1):
                box = (slice(ck[bk], ck[bk + 1]), slice(cj[bj], cj[bj + 1]), slice(ci[bi], ci[bi + 1]))
                Ab = np.ascontiguousarray(A[(slice(None),) + box])
                L, U = dense.dense_LU(ora.factor(Ab, 0.92).astype(np.float32).astype(np.float64))
                ids = idx[box].ravel()
                M[np.ix_(ids, ids)] = L @ U
    Ad = dense.dense_A(A)
    xr = np.zeros(b.size)
    for m in range(n + 1):
        xm = ora.blocks(A, 0.92, b, np.zeros_like(b), (ci, cj, ck), m, mixed=True)[0].ravel()
        assert np.abs(xm - xr).max() <= MIXED_B * max(np.abs(xr).max(), 1e-300)
        r = b.ravel() - Ad @ xr
        xr = xr + np.linalg.solve(M, r.astype(np.float32).astype(np.float64))
