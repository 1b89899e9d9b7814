"""Several right-hand sides of one factorised system (sip_iterate_multi,
sip_solve_multi): pairs share one pass of the sweeps over A and the factors.

Bar: every right-hand side gets bitwise the iterates, residual history,
iteration count and stop decision it gets from sip_iterate / sip_solve alone
(the pair kernels do each right-hand side's arithmetic in the same order),
and those single-right-hand-side paths are the ones held to the oracle by the
parity tests.  A right-hand side that stops keeps its x while its partner
goes on.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1303_4538_amd import problems

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def sip():
    from paper_1303_4538_amd import sip as s
    s.lib()
    assert torch.cuda.is_available()
    return s


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def system(kind, dims, rng):
    ni, nj, nk = dims
    if kind == "poisson":
        return problems.poisson(ni, nj, nk)
    if kind == "stretched":
        return problems.stretched_poisson(ni, nj, nk)
    return problems.convection_diffusion(ni, nj, nk, rng)


def smooth(dims):
    """A low-frequency right-hand side (converges at another rate than noise)."""
    ni, nj, nk = dims
    k, j, i = np.meshgrid(np.arange(nk), np.arange(nj), np.arange(ni), indexing="ij")
    return (np.sin(math.pi * (i + 1) / (ni + 1)) * np.sin(math.pi * (j + 1) / (nj + 1))
            * np.sin(math.pi * (k + 1) / (nk + 1)))


DIMS = [(16, 16, 16), (17, 9, 5), (33, 31, 7), (5, 40, 12), (1, 1, 9), (40, 3, 1), (64, 9, 2)]


@pytest.mark.parametrize("precision", ["mixed", "fp32"])
@pytest.mark.parametrize("kind", ["cd", "stretched"])
@pytest.mark.parametrize("dims", DIMS)
def test_pair_iterates_equal_solo(sip, dims, kind, precision):
    rng = np.random.default_rng(sum(dims) + 3)
    A = system(kind, dims, rng)
    shape = A.shape[1:]
    bs = [rng.uniform(-1, 1, shape), smooth(dims)]
    x0 = [rng.uniform(-0.5, 0.5, shape), np.zeros(shape)]
    log(f"pair iterate {dims} {kind} {precision}")
    S = sip.sip_factor(dev(A), 0.92, precision)
    n = 6
    xs = [dev(x) for x in x0]
    hp = sip.sip_iterate_multi(S, [dev(b) for b in bs], xs, n)
    for r in range(2):
        xa = dev(x0[r])
        ha = sip.sip_iterate(S, dev(bs[r]), xa, n)
        assert torch.equal(xs[r], xa), f"right-hand side {r}"
        assert np.array_equal(hp[r], ha)
    S.close()


# FP32 stalls near u32 |A| |x| / |b|, about 2e-5 for the smooth right-hand side here
@pytest.mark.parametrize("persistent", ["1", "0"])
@pytest.mark.parametrize("precision,rtol", [("mixed", 1e-8), ("fp32", 1e-4)])
def test_pair_solves_stop_independently(sip, precision, rtol, persistent, monkeypatch):
    """Two right-hand sides solved together (one persistent launch, or
    chunks of iterations): the pair sweeps stop once one side has stopped and
    the other goes on alone; each result bitwise its solo solve."""
    monkeypatch.setenv("SIP_SOLVE_PERSISTENT", persistent)
    dims = (40, 36, 30)
    rng = np.random.default_rng(5)
    A = system("cd", dims, rng)
    bs = [dev(rng.uniform(-1, 1, A.shape[1:])), dev(smooth(dims))]
    S = sip.sip_factor(dev(A), 0.92, precision)
    solo = []
    for b in bs:
        x = torch.zeros_like(b)
        st, it, rr, _ = sip.sip_solve(S, b, x, rtol, 5000)
        solo.append((x, it, rr))
    assert solo[0][1] != solo[1][1], "the two right-hand sides should need different iteration counts"
    xs = [torch.zeros_like(b) for b in bs]
    st, info = sip.sip_solve_multi(S, bs, xs, rtol, 5000)
    S.close()
    assert st == sip.SIP_OK
    for r in range(2):
        assert info[r][0] == solo[r][1] and info[r][1] == solo[r][2]
        assert torch.equal(xs[r], solo[r][0])
    # and the result really solves the system (FP64 residual by the oracle)
    if precision == "mixed":
        for r in range(2):
            bn = bs[r].cpu().numpy()
            rc = oracle.norm2(oracle.residual(A, bn, xs[r].cpu().numpy())) / oracle.norm2(bn)
            assert rc <= rtol * (1 + 1e-9)


@pytest.mark.parametrize("persistent", ["1", "0"])
def test_odd_count_and_zero_rhs(sip, persistent, monkeypatch):
    monkeypatch.setenv("SIP_SOLVE_PERSISTENT", persistent)
    dims = (24, 20, 18)
    rng = np.random.default_rng(8)
    A = system("cd", dims, rng)
    bs = [dev(rng.uniform(-1, 1, A.shape[1:])), torch.zeros(A.shape[1:], dtype=torch.float64, device="cuda"),
          dev(smooth(dims))]
    S = sip.sip_factor(dev(A), 0.92, "mixed")
    xs = [torch.ones_like(b) for b in bs]
    st, info = sip.sip_solve_multi(S, bs, xs, 1e-8, 5000)
    assert st == sip.SIP_OK
    assert info[1][0] == 0 and info[1][1] == 0.0 and float(xs[1].abs().max()) == 0.0
    for r in (0, 2):
        x = torch.ones_like(bs[r])
        _, it, rr, _ = sip.sip_solve(S, bs[r], x, 1e-8, 5000)
        assert info[r][0] == it and torch.equal(xs[r], x)
    # histories: the zero right-hand side reports zeros; a fixed iteration
    # count keeps its partner in the pair sweeps to the end (after a solve
    # on the same handle, whose pairs stop when one side stops)
    xs = [torch.zeros_like(b) for b in bs]
    h = sip.sip_iterate_multi(S, bs, xs, 4)
    x0 = torch.zeros_like(bs[0])
    h0 = sip.sip_iterate(S, bs[0], x0, 4)
    S.close()
    assert np.all(h[1] == 0.0) and h[0][0] == 1.0 and h[2][0] == 1.0
    assert np.array_equal(h[0], h0) and torch.equal(xs[0], x0)


@pytest.mark.parametrize("persistent", ["1", "0"])
def test_max_iter_on_one_side(sip, persistent, monkeypatch):
    monkeypatch.setenv("SIP_SOLVE_PERSISTENT", persistent)
    dims = (30, 28, 26)
    rng = np.random.default_rng(9)
    A = system("cd", dims, rng)
    bs = [dev(rng.uniform(-1, 1, A.shape[1:])), dev(smooth(dims))]
    S = sip.sip_factor(dev(A), 0.92, "mixed")
    its = []
    for b in bs:
        x = torch.zeros_like(b)
        its.append(sip.sip_solve(S, b, x, 1e-8, 5000)[1])
    cap = (min(its) + max(its)) // 2     # one side converges, the other is cut off
    solo = []
    for b in bs:
        x = torch.zeros_like(b)
        st, it, rr, _ = sip.sip_solve(S, b, x, 1e-8, cap, raise_on_notconv=False)
        solo.append((st, it, x))
    xs = [torch.zeros_like(b) for b in bs]
    st, info = sip.sip_solve_multi(S, bs, xs, 1e-8, cap, raise_on_notconv=False)
    S.close()
    assert st == sip.SIP_ENOTCONV
    for r in range(2):
        assert info[r][0] == solo[r][1] and torch.equal(xs[r], solo[r][2])


def test_fp64_and_symmetric_pairs(sip):
    dims = (20, 17, 13)
    rng = np.random.default_rng(10)
    A = problems.poisson(*dims)
    bs = [dev(rng.uniform(-1, 1, A.shape[1:])), dev(smooth(dims))]
    for precision, storage in (("fp64", "full"), ("mixed", "symmetric")):
        S = sip.sip_factor(dev(A), 0.92, precision, storage=storage)
        xs = [torch.zeros_like(b) for b in bs]
        hp = sip.sip_iterate_multi(S, bs, xs, 5)
        for r in range(2):
            x = torch.zeros_like(bs[r])
            ha = sip.sip_iterate(S, bs[r], x, 5)
            assert torch.equal(xs[r], x) and np.array_equal(hp[r], ha), (precision, storage, r)
        S.close()


def test_pair_after_single_solves_and_back(sip):
    """The pair path keeps its own face words and control blocks: single and
    pair solves interleave on one handle without disturbing each other."""
    dims = (33, 20, 11)
    rng = np.random.default_rng(12)
    A = system("cd", dims, rng)
    bs = [dev(rng.uniform(-1, 1, A.shape[1:])) for _ in range(2)]
    S = sip.sip_factor(dev(A), 0.92, "mixed")
    ref = []
    for b in bs:
        x = torch.zeros_like(b)
        sip.sip_solve(S, b, x, 1e-8, 5000)
        ref.append(x)
    for rep in range(2):
        xs = [torch.zeros_like(b) for b in bs]
        sip.sip_solve_multi(S, bs, xs, 1e-8, 5000)
        assert all(torch.equal(xs[r], ref[r]) for r in range(2))
        x = torch.zeros_like(bs[0])
        sip.sip_solve(S, bs[0], x, 1e-8, 5000)
        assert torch.equal(x, ref[0])
    S.close()


def test_profile_pair_matches_iterate(sip):
    dims = (20, 18, 9)
    rng = np.random.default_rng(13)
    A = system("cd", dims, rng)
    bs = [dev(rng.uniform(-1, 1, A.shape[1:])) for _ in range(2)]
    S = sip.sip_factor(dev(A), 0.92, "mixed")
    xs = [torch.zeros_like(b) for b in bs]
    fwd, bwd = sip.sip_profile_sweeps_multi(S, bs, xs, 3)
    ys = [torch.zeros_like(b) for b in bs]
    sip.sip_iterate_multi(S, bs, ys, 3)
    S.close()
    assert fwd > 0 and bwd > 0
    assert all(torch.equal(xs[r], ys[r]) for r in range(2))
