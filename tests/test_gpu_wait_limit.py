"""The device-side waits (a tile polling its neighbours' face records, a
persistent workgroup waiting for its next task) are all bounded.  Forced from
the host with SIP_WAIT_LIMIT_MS=0, every wait that is not met at once times
out: the call reports SIP_EDEVICE, every kernel exits, and the handle then
solves exactly as a fresh handle does (bitwise x, iteration count and
residual), which needs the face records of the aborted sweep to be told from
the new ones by their tags.  Covers the persistent and the chunked single
solve, a pair of right-hand sides and a fixed iteration count."""
import numpy as np
import pytest

from paper_1303_4538_amd import problems

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DIMS = (96, 80, 40)   # 6 x 5 tiles: every sweep has tiles that must wait for others


@pytest.fixture(scope="module")
def sip():
    from paper_1303_4538_amd import sip as s
    s.lib()
    assert torch.cuda.is_available()
    return s


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module")
def system():
    A, b = problems.make_block(DIMS, "cd", np.random.SeedSequence(21))
    b2 = problems.rhs_uniform(DIMS[0], DIMS[1], DIMS[2], np.random.default_rng(22))
    return dev(A), dev(b), dev(b2)


def fresh_solve(sip, A, b):
    S = sip.sip_factor(A, 0.92, "mixed")
    x = torch.zeros_like(b)
    _, it, rr, _ = sip.sip_solve(S, b, x, 1e-8, 5000)
    S.close()
    return x, it, rr


@pytest.mark.parametrize("persistent", ["1", "0"])
def test_solve_times_out_then_recovers(sip, system, persistent, monkeypatch):
    A, b, _ = system
    monkeypatch.setenv("SIP_SOLVE_PERSISTENT", persistent)
    x_ref, it_ref, rr_ref = fresh_solve(sip, A, b)
    S = sip.sip_factor(A, 0.92, "mixed")
    for attempt in range(2):   # twice in a row: the second starts from the first one's leftovers
        monkeypatch.setenv("SIP_WAIT_LIMIT_MS", "0")
        with pytest.raises(sip.SipError) as e:
            sip.sip_solve(S, b, torch.zeros_like(b), 1e-8, 5000)
        assert e.value.status == sip.SIP_EDEVICE, str(e.value)
        monkeypatch.delenv("SIP_WAIT_LIMIT_MS")
        x = torch.zeros_like(b)
        _, it, rr, _ = sip.sip_solve(S, b, x, 1e-8, 5000)
        assert it == it_ref and rr == rr_ref, (attempt, it, it_ref, rr, rr_ref)
        assert torch.equal(x, x_ref), attempt
    S.close()


def test_pair_times_out_then_recovers(sip, system, monkeypatch):
    A, b, b2 = system
    monkeypatch.setenv("SIP_SOLVE_PERSISTENT", "1")
    refs = [fresh_solve(sip, A, r) for r in (b, b2)]
    S = sip.sip_factor(A, 0.92, "mixed")
    monkeypatch.setenv("SIP_WAIT_LIMIT_MS", "0")
    with pytest.raises(sip.SipError) as e:
        sip.sip_solve_multi(S, [b, b2], [torch.zeros_like(b) for _ in range(2)], 1e-8, 5000)
    assert e.value.status == sip.SIP_EDEVICE, str(e.value)
    monkeypatch.delenv("SIP_WAIT_LIMIT_MS")
    xs = [torch.zeros_like(b) for _ in range(2)]
    _, info = sip.sip_solve_multi(S, [b, b2], xs, 1e-8, 5000)
    for (x_ref, it_ref, rr_ref), x, (it, rr, _) in zip(refs, xs, info):
        assert it == it_ref and rr == rr_ref
        assert torch.equal(x, x_ref)
    S.close()


def test_iterate_times_out_then_recovers(sip, system, monkeypatch):
    A, b, _ = system
    S0 = sip.sip_factor(A, 0.92, "mixed")
    x_ref = torch.zeros_like(b)
    h_ref = sip.sip_iterate(S0, b, x_ref, 20)
    S0.close()
    S = sip.sip_factor(A, 0.92, "mixed")
    monkeypatch.setenv("SIP_WAIT_LIMIT_MS", "0")
    with pytest.raises(sip.SipError) as e:
        sip.sip_iterate(S, b, torch.zeros_like(b), 20)
    assert e.value.status == sip.SIP_EDEVICE, str(e.value)
    monkeypatch.delenv("SIP_WAIT_LIMIT_MS")
    x = torch.zeros_like(b)
    h = sip.sip_iterate(S, b, x, 20)
    assert np.array_equal(h, h_ref) and torch.equal(x, x_ref)
    S.close()


@pytest.mark.parametrize("persistent", ["1", "0"])
def test_server_times_out_then_serves(sip, system, persistent, monkeypatch):
    """The solve server reads the bound at every factorisation and step: a
    resident system's solve that times out, and a new system's factorisation
    that does, fail their requests with SIP_EDEVICE; the next requests for
    both systems are served bitwise as solo solves.  (The variable is only
    changed while the server has no request, so its thread never reads the
    environment while it is being changed.)"""
    A, b, _ = system
    monkeypatch.setenv("SIP_SOLVE_PERSISTENT", "1")
    x_ref, it_ref, rr_ref = fresh_solve(sip, A, b)
    monkeypatch.setenv("SIP_SERVER_PERSISTENT", persistent)
    srv = sip.Server(max_slots=16)

    def run(system_id):
        x = torch.zeros_like(b)
        r = srv.poll(srv.submit(system_id, A, b, x, rtol=1e-8, max_iter=5000, retain=True))
        return r, x

    def exact(r, x):
        assert r["status"] == 0 and r["iters"] == it_ref and r["rel_res"] == rr_ref, r
        assert torch.equal(x, x_ref)

    exact(*run(7))
    for system_id in (7, 8):   # 7: resident, its solve times out; 8: its factorisation does
        monkeypatch.setenv("SIP_WAIT_LIMIT_MS", "0")
        r, _ = run(system_id)
        assert r["status"] == sip.SIP_EDEVICE, (system_id, r)
        monkeypatch.delenv("SIP_WAIT_LIMIT_MS")
        exact(*run(system_id))
    srv.close()


def test_blocks_time_out_then_recover(sip, system, monkeypatch):
    """A multi-block domain (2 x 2 x 2 blocks coupled through boundary
    values): the blocks' sweeps time out, the domain control stops every block
    and the solve reports SIP_EDEVICE; the next solve is bitwise a fresh one."""
    A, b, _ = system
    cuts = [[0, 48, 96], [0, 32, 80], [0, 16, 40]]
    B0 = sip.sip_blocks_factor(A, cuts, 0.92, "mixed")
    x_ref = torch.zeros_like(b)
    _, it_ref, rr_ref, _ = B0.solve(b, x_ref, 1e-8, 5000)
    B0.close()
    B = sip.sip_blocks_factor(A, cuts, 0.92, "mixed")
    monkeypatch.setenv("SIP_WAIT_LIMIT_MS", "0")
    with pytest.raises(sip.SipError) as e:
        B.solve(b, torch.zeros_like(b), 1e-8, 5000)
    assert e.value.status == sip.SIP_EDEVICE, str(e.value)
    monkeypatch.delenv("SIP_WAIT_LIMIT_MS")
    x = torch.zeros_like(b)
    _, it, rr, _ = B.solve(b, x, 1e-8, 5000)
    assert it == it_ref and rr == rr_ref and torch.equal(x, x_ref)
    B.close()


def test_factorisation_times_out(sip, system, monkeypatch):
    """sip_factor's face-record waits are bounded the same way: SIP_EDEVICE,
    no handle; the next factorisation gives the same factors (solve bitwise)."""
    A, b, _ = system
    x_ref, it_ref, rr_ref = fresh_solve(sip, A, b)
    monkeypatch.setenv("SIP_WAIT_LIMIT_MS", "0")
    with pytest.raises(sip.SipError) as e:
        sip.sip_factor(A, 0.92, "mixed")
    assert e.value.status == sip.SIP_EDEVICE, str(e.value)
    monkeypatch.delenv("SIP_WAIT_LIMIT_MS")
    x, it, rr = fresh_solve(sip, A, b)
    assert it == it_ref and rr == rr_ref and torch.equal(x, x_ref)
