"""sip_solve runs a single system as one persistent launch (the finalisers
publish the sweeps one after the other and stop on the device); with
SIP_SOLVE_PERSISTENT=0 it replays chunks of iterations from a captured graph.
Both must give bitwise the same x, iteration count and residual, in every
precision and storage, on blocks with ragged tiles, a single tile, a thin
block, and with a limit reached before the tolerance."""
import numpy as np
import pytest

from paper_1303_4538_amd import problems

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sip():
    from paper_1303_4538_amd import sip as s
    s.lib()
    assert torch.cuda.is_available()
    return s


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def solve(sip, A, b, precision, rtol, max_iter, storage="full"):
    S = sip.sip_factor(dev(A), 0.92, precision, storage=storage)
    x = torch.zeros_like(dev(b))
    st, it, rr, _ = sip.sip_solve(S, dev(b), x, rtol, max_iter, raise_on_notconv=False)
    S.close()
    return st, it, rr, x.cpu().numpy()


@pytest.mark.parametrize("precision,rtol", [("mixed", 1e-8), ("fp64", 1e-8), ("fp32", 1e-5)])
@pytest.mark.parametrize("dims,kind", [((53, 37, 29), "cd"), ((16, 16, 40), "poisson"), ((33, 17, 3), "cd"),
                                       ((70, 9, 31), "stretched")])
def test_persistent_equals_chunked(sip, monkeypatch, precision, rtol, dims, kind):
    A, b = problems.make_block(dims, kind, np.random.SeedSequence(sum(dims)))
    print(f"persistent solve {dims} {kind} {precision}", flush=True)
    out = []
    for mode in ("1", "0"):
        monkeypatch.setenv("SIP_SOLVE_PERSISTENT", mode)
        out.append(solve(sip, A, b, precision, rtol, 5000))
    (st1, it1, rr1, x1), (st0, it0, rr0, x0) = out
    assert st1 == st0 == sip.SIP_OK
    assert it1 == it0 and rr1 == rr0 and np.array_equal(x1, x0)
    assert rr1 <= rtol


def test_persistent_limit_and_symmetric(sip, monkeypatch):
    A, b = problems.make_block((40, 36, 20), "poisson", np.random.SeedSequence(5))
    out = []
    for mode in ("1", "0"):
        monkeypatch.setenv("SIP_SOLVE_PERSISTENT", mode)
        out.append(solve(sip, A, b, "mixed", 1e-12, 7))                       # the limit comes first
        out.append(solve(sip, A, b, "mixed", 1e-8, 5000, storage="symmetric"))
    assert out[0][0] == out[2][0] == sip.SIP_ENOTCONV and out[0][1] == out[2][1] == 7
    for a, c in ((out[0], out[2]), (out[1], out[3])):
        assert a[1] == c[1] and a[2] == c[2] and np.array_equal(a[3], c[3])


def test_solve_launch_time(sip, monkeypatch):
    """sip_system_solve_ms: the device time of the last solve call's
    persistent launches, positive and within the call's wall time (a pair of
    right-hand sides: the pair launch plus the continuation of the one that
    runs longer, about as long as the longer solo solve or more); refused before any persistent solve
    and after a chunked one."""
    A, b = problems.make_block((48, 40, 24), "cd", np.random.SeedSequence(9))
    b2 = problems.rhs_uniform(48, 40, 24, np.random.default_rng(5))
    S = sip.sip_factor(dev(A), 0.92, "mixed")
    with pytest.raises(sip.SipError):
        sip.sip_system_solve_ms(S)
    monkeypatch.setenv("SIP_SOLVE_PERSISTENT", "1")
    _, it, _, secs = sip.sip_solve(S, dev(b), torch.zeros_like(dev(b)), 1e-8, 5000)
    ms = sip.sip_system_solve_ms(S)
    assert it > 0 and 0.0 < ms <= secs * 1e3
    _, it2, _, secs2 = sip.sip_solve(S, dev(b2), torch.zeros_like(dev(b)), 1e-8, 5000)
    ms2 = sip.sip_system_solve_ms(S)
    assert 0.0 < ms2 <= secs2 * 1e3
    _, info = sip.sip_solve_multi(S, [dev(b), dev(b2)], [torch.zeros_like(dev(b)) for _ in range(2)], 1e-8, 5000)
    assert [i[0] for i in info] == [it, it2]
    msp = sip.sip_system_solve_ms(S)
    assert 0.9 * max(ms, ms2) < msp <= max(i[2] for i in info) * 1e3
    S.close()
    monkeypatch.setenv("SIP_SOLVE_PERSISTENT", "0")
    S = sip.sip_factor(dev(A), 0.92, "mixed")
    sip.sip_solve(S, dev(b), torch.zeros_like(dev(b)), 1e-8, 5000)
    with pytest.raises(sip.SipError):
        sip.sip_system_solve_ms(S)
    S.close()


@pytest.mark.parametrize("persistent", ["1", "0"])
def test_stream_loads_change_nothing(sip, persistent, monkeypatch):
    """The forward sweep's non-temporal streams (taken by systems of 4 M
    cells and more, forced here on a small ragged block) leave x, iteration
    counts and residuals bitwise unchanged, in every precision, for one
    right-hand side and for a pair."""
    monkeypatch.setenv("SIP_SOLVE_PERSISTENT", persistent)
    dims = (40, 36, 30)
    A, b = problems.make_block(dims, "cd", np.random.SeedSequence(31))
    b2 = problems.rhs_uniform(*dims, np.random.default_rng(32))
    for precision, rtol in (("mixed", 1e-8), ("fp64", 1e-8), ("fp32", 1e-5)):
        out = {}
        for st in ("0", "1"):
            monkeypatch.setenv("SIP_STREAM_LOADS", st)
            S = sip.sip_factor(dev(A), 0.92, precision)
            x = torch.zeros_like(dev(b))
            _, it, rr, _ = sip.sip_solve(S, dev(b), x, rtol, 3000)
            xs = [torch.zeros_like(dev(b)) for _ in range(2)]
            _, info = sip.sip_solve_multi(S, [dev(b), dev(b2)], xs, rtol, 3000)
            S.close()
            out[st] = (x, it, rr, xs, [i[:2] for i in info])
        a, c = out["0"], out["1"]
        assert a[1:3] == c[1:3] and a[4] == c[4], precision
        assert torch.equal(a[0], c[0]) and all(torch.equal(p, q) for p, q in zip(a[3], c[3])), precision
