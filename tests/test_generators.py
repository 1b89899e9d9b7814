"""Checks of the seeded input generators (no SIP arithmetic involved)."""
import numpy as np

from paper_1303_4538_amd import problems
from tests import dense


def test_fluxes_divergence_free_and_scaled():
    fx, fy, fz = problems.solenoidal_fluxes(12, 9, 7, np.random.default_rng(0))
    div = (fx[:, :, 1:] - fx[:, :, :-1]) + (fy[:, 1:, :] - fy[:, :-1, :]) + (fz[1:] - fz[:-1])
    assert np.abs(div).max() <= 1e-14
    m = max(np.abs(fx).max(), np.abs(fy).max(), np.abs(fz).max())
    assert abs(m - 2.0) <= 1e-15
    # no flux through the walls
    assert np.all(fx[:, :, 0] == 0) and np.all(fx[:, :, -1] == 0)
    assert np.all(fy[:, 0, :] == 0) and np.all(fy[:, -1, :] == 0)
    assert np.all(fz[0] == 0) and np.all(fz[-1] == 0)


def test_cd_is_m_matrix_with_zero_interior_row_sums():
    A = problems.convection_diffusion(10, 8, 6, np.random.default_rng(1))
    assert np.all(A[1:] <= 0) and np.all(A[0] > 0)
    rs = A.sum(axis=0)
    assert rs.min() >= -1e-13
    assert np.abs(rs[1:-1, 1:-1, 1:-1]).max() <= 1e-13
    # upwinding makes it non-symmetric
    Ad = dense.dense_A(problems.convection_diffusion(4, 4, 4, np.random.default_rng(1)))
    assert np.abs(Ad - Ad.T).max() > 1e-3


def test_poisson_and_stretched_are_symmetric():
    for A in (problems.poisson(4, 3, 5), problems.stretched_poisson(4, 3, 5)):
        Ad = dense.dense_A(A)
        assert np.abs(Ad - Ad.T).max() <= 1e-15
        assert A.sum(axis=0).min() >= -1e-13
    A = problems.poisson(5, 5, 5)
    assert np.all(A[0] == 6.0)
    S = problems.stretched_poisson(3, 3, 5, ratio=1.0)
    assert np.allclose(S[0], 6.0) and np.allclose(S[1:][S[1:] != 0], -1.0)


def test_stretched_middle_cell_is_cube():
    A = problems.stretched_poisson(2, 2, 5)
    # middle layer: dz = 1, so the lateral couplings are -1
    assert np.allclose(A[1, 2, :, 1:], -1.0)
    assert np.allclose(A[2, 0, :, :-1], -(1.05 ** -2))


def test_seeds_are_reproducible():
    c1 = problems.config1()
    c1b = problems.config1()
    assert np.array_equal(c1["b"], c1b["b"])
    assert np.array_equal(c1["b"], np.random.default_rng(1234).uniform(-1, 1, (16, 16, 16)))
    m1 = problems.config3_meta()
    m2 = problems.config3_meta()
    assert [(d, k) for d, k, _ in m1] == [(d, k) for d, k, _ in m2]
    assert all(32 <= v <= 160 for d, _, _ in m1 for v in d)
    kinds = [k for _, k, _ in m1]
    assert 16 <= kinds.count("poisson") <= 48


def test_serving_stream_shape():
    systems, reqs = problems.serving_stream(n_systems=20, rhs_per_system=8)
    assert len(reqs) == 160
    assert all(24 <= v <= 192 for d, _, _ in systems for v in d)
    t = [r[0] for r in reqs]
    assert all(b > a for a, b in zip(t, t[1:]))
    per = {}
    for _, s, m, _ in reqs:
        per.setdefault(s, set()).add(m)
    assert all(v == set(range(8)) for v in per.values())
