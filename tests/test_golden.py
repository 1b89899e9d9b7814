"""Stored values written by hand from closed forms (tests/golden/, each file
states its derivation and the passage it rests on), checked against the
oracle on the CPU and against the library's factors on the GPU."""
import os

import numpy as np
import pytest

from paper_1303_4538_amd import problems
from tests import dense

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def column_pivots():
    rows = np.loadtxt(os.path.join(GOLDEN, "poisson_column_pivots.txt"), dtype=np.int64)
    k, u, um1 = rows.T
    assert list(k) == list(range(1, len(k) + 1))
    return u.astype(float), um1.astype(float)


def expected_column_factors(nk):
    u, um1 = column_pivots()
    assert len(u) == nk
    E = np.zeros((7, nk))
    E[dense.LB, 1:] = -1.0
    E[dense.LP] = u / um1
    E[dense.UT, :-1] = -um1[:-1] / u[:-1]
    return E


@pytest.mark.parametrize("alpha", [0.0, 0.5, 0.92, 1.0])
def test_oracle_column_factors(ora, alpha):
    A = problems.poisson(1, 1, 8)
    LU = ora.factor(A, alpha)[:, :, 0, 0]
    E = expected_column_factors(8)
    assert np.abs(LU - E).max() <= 2e-15 * np.abs(E).max()


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_library_column_factors(precision):
    torch = pytest.importorskip("torch")
    from paper_1303_4538_amd import sip
    sip.lib()
    A = torch.from_numpy(problems.poisson(1, 1, 8)).cuda()
    S = sip.sip_factor(A, 0.92, precision)
    LU = sip.sip_export_factors(S).cpu().numpy()[:, :, 0, 0]
    S.close()
    E = expected_column_factors(8)
    tol = 2e-15 if precision == "fp64" else 2 ** -24   # FP32 factors: rounding of the FP64 values
    assert np.abs(LU - E).max() <= tol * np.abs(E).max()
