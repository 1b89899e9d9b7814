"""Every compiled sweep plan -- loader-phase count (SIP_SWEEP_PHASES = 1, 2,
3; with three the loader turns are split over two intervals) and poll
distance (SIP_POLL_DISTANCE = 1, 2, 3 with two or three phases) -- computes
bitwise the same iterates, residual norms and stop decisions: the launch
shape does not change the arithmetic (the squares of the residual are summed per quadrant
and lane plane by plane, in plane order, whichever loader wave stages a
plane).  Covered: the three precisions, a pair of right-hand sides, the
symmetric storage, a multi-block domain and a server batch, on shapes with
ragged tile edges, a single tile and a thin block.
"""
import numpy as np
import pytest

from paper_1303_4538_amd import problems

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (phases, poll distance); the first is the reference
PLANS = [("2", "2"), ("1", "2"), ("3", "2"), ("2", "1"), ("2", "3"), ("3", "1"), ("3", "3")]


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


def close(h, ref):
    return np.array_equal(h, ref)


def each_phase(monkeypatch, run):
    out = []
    for ph, pd in PLANS:
        monkeypatch.setenv("SIP_SWEEP_PHASES", ph)
        monkeypatch.setenv("SIP_POLL_DISTANCE", pd)
        out.append(run())
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
@pytest.mark.parametrize("dims", [(70, 50, 20), (16, 16, 40), (33, 17, 3)])
def test_single_system(sip, monkeypatch, precision, dims):
    rng = np.random.default_rng(sum(dims))
    A = problems.convection_diffusion(*dims, rng)
    b = rng.uniform(-1, 1, A.shape[1:])
    log(f"phases: single {dims} {precision}")

    def run():
        S = sip.sip_factor(dev(A), 0.92, precision)
        x = torch.zeros_like(dev(b))
        h = sip.sip_iterate(S, dev(b), x, 10)
        xs = torch.zeros_like(dev(b))
        st = sip.sip_solve(S, dev(b), xs, 1e-8 if precision != "fp32" else 1e-4, 5000)[:3]
        S.close()
        return x, h, xs, st

    out = each_phase(monkeypatch, run)
    for x, h, xs, st in out[1:]:
        assert torch.equal(x, out[0][0]) and close(h, out[0][1])
        assert torch.equal(xs, out[0][2]) and st[:2] == out[0][3][:2] and close(st[2], out[0][3][2])


@pytest.mark.parametrize("precision", ["mixed", "fp32"])
def test_pair(sip, monkeypatch, precision):
    dims = (40, 36, 30)
    rng = np.random.default_rng(61)
    A = problems.convection_diffusion(*dims, rng)
    bs = [dev(rng.uniform(-1, 1, A.shape[1:])) for _ in range(2)]
    log(f"phases: pair {precision}")

    def run():
        S = sip.sip_factor(dev(A), 0.92, precision)
        xs = [torch.zeros_like(b) for b in bs]
        h = sip.sip_iterate_multi(S, bs, xs, 8)
        S.close()
        return xs, h

    out = each_phase(monkeypatch, run)
    for xs, h in out[1:]:
        assert all(torch.equal(xs[r], out[0][0][r]) for r in range(2)) and close(h, out[0][1])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_symmetric_storage(sip, monkeypatch, precision):
    dims = (37, 29, 17)
    A = problems.stretched_poisson(*dims)
    b = np.random.default_rng(62).uniform(-1, 1, A.shape[1:])
    log(f"phases: symmetric {precision}")

    def run():
        S = sip.sip_factor(dev(A), 0.92, precision, storage="symmetric")
        x = torch.zeros_like(dev(b))
        h = sip.sip_iterate(S, dev(b), x, 10)
        S.close()
        return x, h

    out = each_phase(monkeypatch, run)
    for x, h in out[1:]:
        assert torch.equal(x, out[0][0]) and close(h, out[0][1])


def test_blocks_and_server(sip, monkeypatch):
    rng = np.random.default_rng(63)
    A = problems.convection_diffusion(40, 33, 14, rng)
    b = rng.uniform(-1, 1, A.shape[1:])
    cuts = ([0, 20, 40], [0, 17, 33], [0, 14])
    others = [problems.convection_diffusion(*d, rng) for d in ((24, 30, 9), (50, 12, 7))]
    obs = [rng.uniform(-1, 1, a.shape[1:]) for a in others]
    log("phases: blocks and server")

    def run():
        B = sip.sip_blocks_factor(dev(A), cuts, 0.92, "mixed")
        xb = torch.zeros_like(dev(b))
        hb = B.iterate(dev(b), xb, 8)
        B.close()
        srv = sip.Server(max_slots=8, epoch_iters=4)
        sysA = [dev(A)] + [dev(a) for a in others]
        sysb = [dev(b)] + [dev(v) for v in obs]
        xs = [torch.zeros_like(v) for v in sysb]
        ts = [srv.submit(q, sysA[q], sysb[q], xs[q], rtol=1e-8, max_iter=5000) for q in range(3)]
        res = [(r["status"], r["iters"], r["rel_res"]) for r in (srv.poll(t) for t in ts)]
        srv.close()
        return xb, hb, xs, res

    out = each_phase(monkeypatch, run)
    for xb, hb, xs, res in out[1:]:
        assert torch.equal(xb, out[0][0]) and close(hb, out[0][1])
        assert [r[:2] for r in res] == [r[:2] for r in out[0][3]]
        assert all(close(r[2], r0[2]) for r, r0 in zip(res, out[0][3]))
        assert all(torch.equal(xs[q], out[0][2][q]) for q in range(3))
