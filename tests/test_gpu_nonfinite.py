"""Non-finite values.  Before any update the device forms ||b||^2 and the
residual of the start vector; if either is not finite (NaN or Inf in b, x0
or A x0), the solve stops at iteration 0 with SIP_EINVAL, x keeps its start
value and the history reads NaN.  A residual that turns non-finite after an
update (here: the FP32 sweeps of the mixed precision overflow on a right-hand
side of 1e38, which the oracle's mixed iteration shows as well, while FP64
solves the same system) stops at that iteration with SIP_EBREAKDOWN.  With
several right-hand sides, or requests in the server, only the one with the
bad values stops; the others get their normal results.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1303_4538_amd import problems

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DIMS = (17, 9, 5)
CELL = (2, 4, 11)   # k, j, i


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


def same(xt, expect):
    """Equal values, NaN where expect has NaN (payloads aside)."""
    x = xt.cpu().numpy()
    nan = np.isnan(expect)
    return bool(np.array_equal(np.isnan(x), nan) and np.array_equal(x[~nan], expect[~nan]))


def system(rng):
    A = problems.convection_diffusion(*DIMS, rng)
    shape = A.shape[1:]
    return A, rng.uniform(-1, 1, shape), rng.uniform(-0.5, 0.5, shape)


def spoil(b, x0, where):
    b, x0 = b.copy(), x0.copy()
    v = math.nan if where.endswith("nan") else -math.inf
    (b if where.startswith("b") else x0)[CELL] = v
    return b, x0


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
@pytest.mark.parametrize("where", ["b_nan", "b_inf", "x0_nan", "x0_inf"])
def test_bad_input_stops_before_any_update(sip, precision, where):
    rng = np.random.default_rng(21)
    A, b, x0 = system(rng)
    bb, xb = spoil(b, x0, where)
    log(f"non-finite {where} {precision}")
    S = sip.sip_factor(dev(A), 0.92, precision)
    # x is written back unchanged (FP32 keeps x in FP32)
    keep = xb.astype(np.float32).astype(np.float64) if precision == "fp32" else xb
    x = dev(xb)
    with pytest.raises(sip.SipError) as e:
        sip.sip_iterate(S, dev(bb), x, 5)
    assert e.value.status == sip.SIP_EINVAL
    assert same(x, keep)
    x = dev(xb)
    h = sip.sip_iterate(S, dev(bb), x, 5, accept=(sip.SIP_EINVAL,))
    assert np.all(np.isnan(h)) and same(x, keep)
    x = dev(xb)
    st, it, rr, _ = sip.sip_solve(S, dev(bb), x, 1e-8, 100, accept=(sip.SIP_EINVAL,))
    assert st == sip.SIP_EINVAL and it == 0 and math.isnan(rr) and same(x, keep)
    # the handle stays usable: a clean solve equals one on a fresh handle
    xa = dev(x0)
    ra = sip.sip_solve(S, dev(b), xa, 1e-6, 300, raise_on_notconv=False)
    S.close()
    S2 = sip.sip_factor(dev(A), 0.92, precision)
    xf = dev(x0)
    rf = sip.sip_solve(S2, dev(b), xf, 1e-6, 300, raise_on_notconv=False)
    S2.close()
    assert torch.equal(xa, xf) and ra[1] == rf[1] and ra[2] == rf[2]


@pytest.mark.parametrize("bad", [0, 1])
def test_pair_with_one_bad_right_hand_side(sip, bad):
    rng = np.random.default_rng(22)
    A, b, x0 = system(rng)
    b2 = rng.uniform(-1, 1, b.shape)
    bn, _ = spoil(b2, x0, "b_nan")
    bs = [dev(b), dev(b)]
    bs[bad] = dev(bn)
    good = 1 - bad
    log(f"pair, right-hand side {bad} NaN")
    S = sip.sip_factor(dev(A), 0.92, "mixed")
    xs_ = dev(x0)
    solo = sip.sip_solve(S, bs[good], xs_, 1e-8, 5000)
    xh = dev(x0)
    hsolo = sip.sip_iterate(S, bs[good], xh, 6)
    xs = [dev(x0), dev(x0)]
    st, info = sip.sip_solve_multi(S, bs, xs, 1e-8, 5000, accept=(sip.SIP_EINVAL,))
    assert st == sip.SIP_EINVAL
    assert info[bad][0] == 0 and math.isnan(info[bad][1]) and same(xs[bad], x0)
    assert info[good][0] == solo[1] and info[good][1] == solo[2] and torch.equal(xs[good], xs_)
    xs = [dev(x0), dev(x0)]
    h = sip.sip_iterate_multi(S, bs, xs, 6, accept=(sip.SIP_EINVAL,))
    assert np.all(np.isnan(h[bad])) and same(xs[bad], x0)
    assert np.array_equal(h[good], hsolo) and torch.equal(xs[good], xh)
    with pytest.raises(sip.SipError) as e:
        sip.sip_iterate_multi(S, bs, [dev(x0), dev(x0)], 2)
    assert e.value.status == sip.SIP_EINVAL
    S.close()


def test_odd_right_hand_side_bad(sip):
    rng = np.random.default_rng(23)
    A, b, x0 = system(rng)
    bn, _ = spoil(b, x0, "b_inf")
    log("three right-hand sides, the unpaired one Inf")
    S = sip.sip_factor(dev(A), 0.92, "mixed")
    bs = [dev(b), dev(b[::-1]), dev(bn)]
    xs = [dev(x0) for _ in bs]
    st, info = sip.sip_solve_multi(S, bs, xs, 1e-8, 5000, accept=(sip.SIP_EINVAL,))
    assert st == sip.SIP_EINVAL and info[2][0] == 0 and same(xs[2], x0)
    for r in range(2):
        x = dev(x0)
        _, it, rr, _ = sip.sip_solve(S, bs[r], x, 1e-8, 5000)
        assert info[r][0] == it and info[r][1] == rr and torch.equal(xs[r], x)
    S.close()


def test_blocks_bad_input(sip):
    rng = np.random.default_rng(24)
    A, b, x0 = system(rng)
    bb, _ = spoil(b, x0, "b_nan")
    log("blocks, NaN in b")
    B = sip.sip_blocks_factor(dev(A), ([0, 9, 17], [0, 9], [0, 2, 5]), 0.92, "fp64")
    x = dev(x0)
    h = B.iterate(dev(bb), x, 4, accept=(sip.SIP_EINVAL,))
    assert np.all(np.isnan(h)) and same(x, x0)
    st, it, rr, _ = B.solve(dev(bb), x, 1e-8, 100, accept=(sip.SIP_EINVAL,))
    assert st == sip.SIP_EINVAL and it == 0 and math.isnan(rr) and same(x, x0)
    # a clean solve on the same handle still matches the oracle's first iterates
    x = dev(x0)
    hg = B.iterate(dev(b), x, 2)
    B.close()
    xo, _, _, ho = oracle.blocks(A, 0.92, b, x0, ([0, 9, 17], [0, 9], [0, 2, 5]), 2)
    assert np.abs(x.cpu().numpy() - xo).max() <= 1e-12 * np.abs(xo).max()
    assert np.abs(hg - ho).max() <= 1e-12


@pytest.mark.parametrize("pairs", [False, True])
def test_server_bad_request_alone_fails(sip, monkeypatch, pairs):
    rng = np.random.default_rng(25)
    A, b, x0 = system(rng)
    bn, _ = spoil(b, x0, "b_nan")
    log(f"server: one request with NaN in b among good ones, pairing {pairs}")
    monkeypatch.setenv("SIP_SERVER_PAIRS", "1" if pairs else "0")
    At = dev(A)
    srv = sip.Server(max_slots=16, epoch_iters=4)
    # the first request is admitted alone; the others queue up while it
    # factorises and, with pairing on, are swept in pairs (the bad one too)
    bad = 2
    bs = [dev(bn) if q == bad else dev(b) for q in range(5)]
    xs = [torch.zeros_like(At[0]) for _ in bs]
    tickets = [srv.submit(7, At, bs[q], xs[q], precision="mixed", rtol=1e-8, max_iter=5000) for q in range(5)]
    res = [srv.poll(t) for t in tickets]
    paired = srv.stats()["pairs"]
    srv.close()
    assert (paired >= 1) == pairs
    assert res[bad]["status"] == sip.SIP_EINVAL and res[bad]["iters"] == 0 and math.isnan(res[bad]["rel_res"])
    S = sip.sip_factor(At, 0.92, "mixed")
    x = torch.zeros_like(At[0])
    _, it, rr, _ = sip.sip_solve(S, bs[0], x, 1e-8, 5000)
    S.close()
    for q in (0, 1, 3, 4):
        assert res[q]["status"] == sip.SIP_OK and res[q]["iters"] == it and torch.equal(xs[q], x)


def test_fp32_sweep_overflow_is_reported(sip):
    A = problems.poisson(16, 16, 16)
    b = np.full(A.shape[1:], 1.5e38)
    # the oracle's mixed iteration overflows in its FP32 sweeps; FP64 does not
    xo, ho = oracle.iterate(A, oracle.factor(A, 0.92), b, np.zeros_like(b), 1, mixed=True)
    assert not np.isfinite(xo).all() and ho[0] == 1.0
    log("mixed sweeps overflow on b = 1.5e38")
    S = sip.sip_factor(dev(A), 0.92, "mixed")
    x = torch.zeros_like(dev(b))
    with pytest.raises(sip.SipError) as e:
        sip.sip_iterate(S, dev(b), x, 3)
    assert e.value.status == sip.SIP_EBREAKDOWN
    x = torch.zeros_like(dev(b))
    h = sip.sip_iterate(S, dev(b), x, 3, accept=(sip.SIP_EBREAKDOWN,))
    assert h[0] == 1.0 and np.all(np.isnan(h[1:])) and not bool(torch.isfinite(x).all())
    x = torch.zeros_like(dev(b))
    st, it, rr, _ = sip.sip_solve(S, dev(b), x, 1e-8, 100, accept=(sip.SIP_EBREAKDOWN,))
    S.close()
    assert st == sip.SIP_EBREAKDOWN and it == 1 and math.isnan(rr)
    S = sip.sip_factor(dev(A), 0.92, "fp64")
    x = torch.zeros_like(dev(b))
    st, it, rr, _ = sip.sip_solve(S, dev(b), x, 1e-8, 1000)
    S.close()
    assert st == sip.SIP_OK and rr <= 1e-8 and bool(torch.isfinite(x).all())
