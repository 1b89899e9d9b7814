"""Batched and served solves (sip_batch_submit / sip_batch_poll) on the GPU.

Bar: every request's result equals the same block solved alone through
sip_solve (bitwise: identical per-block arithmetic and reduction order; the
per-tile norms are summed plane by plane whatever the launch shape, so the
residual and the stop iteration are bitwise too), its final residual
re-checked by the oracle in FP64 is <= rtol, and its iteration count is
within 2 of the mixed-form oracle's.  The server runs every request at its
own pace in one persistent launch (default) or, with
SIP_SERVER_PERSISTENT=0, in epochs of per-iteration launches; the first test
covers both.
"""
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
    return s


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


BLOCKS = [((20, 17, 13), "cd"), ((33, 8, 21), "poisson"), ((9, 40, 12), "cd"), ((16, 16, 16), "stretched"),
          ((25, 30, 6), "cd"), ((12, 12, 35), "poisson")]


def block(dims, kind, seed):
    ni, nj, nk = dims
    rng = np.random.default_rng(seed)
    if kind == "poisson":
        A = problems.poisson(ni, nj, nk)
    elif kind == "stretched":
        A = problems.stretched_poisson(ni, nj, nk)
    else:
        A = problems.convection_diffusion(ni, nj, nk, rng)
    b = rng.uniform(-1, 1, (nk, nj, ni))
    return A, b


def alone(sip, A, b, precision, rtol=1e-8):
    S = sip.sip_factor(dev(A), 0.92, precision)
    x = torch.zeros_like(dev(b))
    st, it, rr, _ = sip.sip_solve(S, dev(b), x, rtol, 5000)
    S.close()
    return x.cpu().numpy(), it, rr


@pytest.mark.parametrize("mode", ["dataflow", "whole", "epochs"])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_batch_equals_alone_and_oracle(sip, precision, mode, monkeypatch):
    """Persistent launches that publish sweeps tile by tile as upstream tiles
    are taken, or whole sweeps in tile order, and per-iteration epochs: every
    result bitwise its solo solve."""
    monkeypatch.setenv("SIP_SERVER_PERSISTENT", "0" if mode == "epochs" else "1")
    monkeypatch.setenv("SIP_SERVER_DATAFLOW", "0" if mode == "whole" else "1")
    data = [block(d, k, 100 + q) for q, (d, k) in enumerate(BLOCKS)]
    log(f"server batch of {len(data)} blocks, {precision}, {mode}")
    srv = sip.Server(max_slots=64, epoch_iters=8)
    At = [dev(A) for A, _ in data]
    bt = [dev(b) for _, b in data]
    xt = [torch.zeros_like(b) for b in bt]
    tickets = [srv.submit(q, At[q], bt[q], xt[q], precision=precision) for q in range(len(data))]
    res = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["factorisations"] == len(data)
    for q, (A, b) in enumerate(data):
        r = res[q]
        assert r["status"] == sip.SIP_OK and r["rel_res"] <= 1e-8, r
        xg = xt[q].cpu().numpy()
        xa, ita, rra = alone(sip, A, b, precision)
        assert r["iters"] == ita and np.array_equal(xg, xa), f"block {q} differs from its solo solve"
        assert r["rel_res"] == rra, f"block {q}: residual differs from its solo solve"
        rc = oracle.norm2(oracle.residual(A, b, xg)) / oracle.norm2(b)
        assert rc <= 1e-8 * (1 + 1e-9)
        LU = oracle.factor(A, 0.92)
        _, ito, _, _ = oracle.solve(A, LU, b, np.zeros_like(b), 1e-8, 5000, mixed=(precision == "mixed"))
        assert abs(r["iters"] - ito) <= 2


def test_resident_factors_reused(sip):
    A, _ = block((24, 20, 18), "cd", 7)
    At = dev(A)
    srv = sip.Server(max_slots=8, epoch_iters=4)
    outs = []
    for m in range(4):
        b = np.random.default_rng(50 + m).uniform(-1, 1, A.shape[1:])
        bt = dev(b)
        xt = torch.zeros_like(bt)
        t = srv.submit(42, At if m == 0 else None, bt, xt, retain=True)
        r = srv.poll(t)
        assert r["status"] == sip.SIP_OK and r["factorised"] == (1 if m == 0 else 0)
        outs.append((b, xt.cpu().numpy(), r))
    st = srv.stats()
    assert st["factorisations"] == 1
    srv.release(42)
    srv.close()
    for b, xg, r in outs:
        assert oracle.norm2(oracle.residual(A, b, xg)) / oracle.norm2(b) <= 1e-8 * (1 + 1e-9)


def test_budget_forces_eviction_and_waiting(sip):
    data = [block(d, k, 200 + q) for q, (d, k) in enumerate(BLOCKS[:4])]
    At = [dev(A) for A, _ in data]
    bt = [dev(b) for _, b in data]
    xt = [torch.zeros_like(b) for b in bt]
    # the largest single-request footprint, measured by the server itself
    probe = sip.Server(max_slots=16, epoch_iters=4)
    for q in range(len(data)):
        probe.poll(probe.submit(900 + q, At[q], bt[q], torch.zeros_like(bt[q]), retain=True))
        probe.release(900 + q)
    one = probe.stats()["peak_bytes"]
    probe.close()
    # room for roughly one block at a time
    budget = int(one * 1.5)
    srv = sip.Server(hbm_budget_bytes=budget, max_slots=16, epoch_iters=4)
    tickets = [srv.submit(100 + q, At[q], bt[q], xt[q], retain=True) for q in range(len(data))]
    res = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["peak_bytes"] <= budget
    assert st["evictions"] >= 1
    for q, (A, b) in enumerate(data):
        assert res[q]["status"] == sip.SIP_OK
        xa, ita, _ = alone(sip, A, b, "mixed")
        assert np.array_equal(xt[q].cpu().numpy(), xa)


def test_queued_request_keeps_its_resident_system(sip):
    """A request naming a resident system without coefficients keeps that
    system from eviction while it waits: here a new system queued ahead of it
    needs the room, is held back, and is admitted (evicting the first system)
    once that request is done."""
    (A, b), (A2, b2) = block((24, 20, 18), "cd", 301), block((24, 20, 18), "poisson", 302)
    Ar, br = block((12, 10, 9), "cd", 303)
    At, bt, A2t, b2t, Art, brt = dev(A), dev(b), dev(A2), dev(b2), dev(Ar), dev(br)
    probe = sip.Server(max_slots=4, epoch_iters=4)
    probe.poll(probe.submit(1, At, bt, torch.zeros_like(bt), retain=True))
    sys_and_slot = probe.stats()["peak_bytes"]
    probe.close()
    srv = sip.Server(hbm_budget_bytes=int(sys_and_slot * 1.5), max_slots=1, epoch_iters=4)
    x1 = torch.zeros_like(bt)
    assert srv.poll(srv.submit(7, At, bt, x1, retain=True))["status"] == sip.SIP_OK
    # a long request takes the only slot while the next two queue behind it
    tr = srv.submit(9, Art, brt, torch.zeros_like(brt), rtol=1e-300, max_iter=20000)
    x2, x3 = torch.zeros_like(b2t), torch.zeros_like(bt)
    t2 = srv.submit(8, A2t, b2t, x2)              # new system: needs the room system 7 holds
    t3 = srv.submit(7, None, bt, x3)              # resident system 7, no coefficients
    assert srv.poll(tr)["status"] == sip.SIP_ENOTCONV
    r3, r2 = srv.poll(t3), srv.poll(t2)
    st = srv.stats()
    srv.close()
    assert r3["status"] == sip.SIP_OK and r3["factorised"] == 0
    assert r2["status"] == sip.SIP_OK and r2["factorised"] == 1
    assert r2["t_admit"] >= r3["t_done"] - 1e-3
    assert st["evictions"] >= 1 and st["factorisations"] == 3
    assert torch.equal(x3, x1)
    xa, _, _ = alone(sip, A2, b2, "mixed")
    assert np.array_equal(x2.cpu().numpy(), xa)


def test_server_reads_inputs_after_the_callers_stream(sip):
    """b is written on a side stream behind a long queue of work just before
    submit; the server, told that stream, reads the new b (with no ordering it
    would see the zeros still there and return x = 0)."""
    A, b = block((20, 18, 16), "cd", 305)
    At, bsrc = dev(A), dev(b)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bt = torch.zeros_like(bsrc)
        m = torch.ones((4096, 4096), dtype=torch.float32, device="cuda") / 4096
        for _ in range(40):
            m = m @ m
        bt.copy_(bsrc)
    xt = torch.zeros_like(bsrc)
    srv = sip.Server(max_slots=4, epoch_iters=4)
    r = srv.poll(srv.submit(3, At, bt, xt, stream=side))
    srv.close()
    torch.cuda.synchronize()
    assert r["status"] == sip.SIP_OK and r["iters"] > 0
    xa, ita, _ = alone(sip, A, b, "mixed")
    assert r["iters"] == ita and np.array_equal(xt.cpu().numpy(), xa)


def test_breakdown_and_bad_requests(sip):
    A, b = block((10, 9, 8), "poisson", 3)
    A[0, 0, 0, 0] = 0.0
    srv = sip.Server(max_slots=4, epoch_iters=4)
    bt = dev(b)
    xt = torch.zeros_like(bt)
    t = srv.submit(1, dev(A), bt, xt)
    r = srv.poll(t)
    assert r["status"] == sip.SIP_EBREAKDOWN
    # a request for an unknown system without coefficients is rejected
    with pytest.raises(sip.SipError) as e:
        srv.submit(2, None, bt, xt)
    assert e.value.status == sip.SIP_EINVAL
    with pytest.raises(sip.SipError):
        srv.submit(3, dev(A), bt, xt, rtol=-1.0)
    # a request larger than the whole budget is refused at submission
    small = sip.Server(hbm_budget_bytes=1 << 16, max_slots=4, epoch_iters=4)
    with pytest.raises(sip.SipError) as e:
        small.submit(4, dev(A), bt, xt)
    assert e.value.status == sip.SIP_ENOMEM
    small.close()
    srv.close()


def test_arrivals_while_running_join_the_mix(sip):
    """Continuous batching: requests submitted while others run are admitted
    at the next epoch and finish with the same result as alone."""
    import time
    data = [block(d, k, 300 + q) for q, (d, k) in enumerate(BLOCKS)]
    srv = sip.Server(max_slots=64, epoch_iters=2)
    At = [dev(A) for A, _ in data]
    bt = [dev(b) for _, b in data]
    xt = [torch.zeros_like(b) for b in bt]
    tickets = []
    for q in range(len(data)):
        tickets.append(srv.submit(q, At[q], bt[q], xt[q]))
        time.sleep(0.002)
    res = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["epochs"] >= 2
    overlapped = sum(1 for q in range(1, len(res)) if res[q]["t_admit"] < res[q - 1]["t_done"])
    log(f"  epochs {st['epochs']}, requests admitted while an earlier one ran: {overlapped}")
    for q, (A, b) in enumerate(data):
        xa, ita, _ = alone(sip, A, b, "mixed")
        assert res[q]["status"] == sip.SIP_OK and res[q]["iters"] == ita
        assert np.array_equal(xt[q].cpu().numpy(), xa)


@pytest.mark.parametrize("precision,rtol", [("mixed", 1e-8), ("fp32", 1e-4)])
def test_requests_of_one_system_run_in_pairs(sip, precision, rtol, monkeypatch):
    """Requests of one system admitted together are swept in pairs; each
    result is bitwise its solo solve (also a zero right-hand side and one
    with its own tolerance, which stays single)."""
    A, _ = block((30, 26, 22), "cd", 400)
    rng = np.random.default_rng(401)
    bs = [rng.uniform(-1, 1, A.shape[1:]) for _ in range(5)]
    bs[3] = np.zeros(A.shape[1:])
    At = dev(A)
    bt = [dev(b) for b in bs]
    tols = [rtol] * 5 + [rtol * 10]
    bt.append(dev(rng.uniform(-1, 1, A.shape[1:])))
    xt = [torch.zeros_like(b) for b in bt]
    monkeypatch.setenv("SIP_SERVER_PAIRS", "1")
    srv = sip.Server(max_slots=16, epoch_iters=4)
    tickets = [srv.submit(7, At, bt[q], xt[q], precision=precision, rtol=tols[q], retain=True)
               for q in range(len(bt))]
    res = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    log(f"  {precision}: pairs formed {st['pairs']}")
    assert st["pairs"] >= 2
    S = sip.sip_factor(At, 0.92, precision)
    for q in range(len(bt)):
        xa = torch.zeros_like(bt[q])
        _, it, rr, _ = sip.sip_solve(S, bt[q], xa, tols[q], 100000)
        assert res[q]["status"] == sip.SIP_OK, res[q]
        assert res[q]["iters"] == it and torch.equal(xt[q], xa), f"request {q}"
    S.close()
    assert res[3]["iters"] == 0 and float(xt[3].abs().max()) == 0.0


def test_pairing_off_gives_the_same_results(sip, monkeypatch):
    A, _ = block((20, 17, 13), "poisson", 402)
    rng = np.random.default_rng(403)
    n = 5   # the first is admitted alone; the others queue up while it factorises
    bt = [dev(rng.uniform(-1, 1, A.shape[1:])) for _ in range(n)]
    out = []
    for flag in ("1", "0"):
        monkeypatch.setenv("SIP_SERVER_PAIRS", flag)
        srv = sip.Server(max_slots=8, epoch_iters=4)
        xt = [torch.zeros_like(b) for b in bt]
        tickets = [srv.submit(3, dev(A), bt[q], xt[q]) for q in range(n)]
        res = [srv.poll(t) for t in tickets]
        pairs = srv.stats()["pairs"]
        srv.close()
        out.append((xt, res, pairs))
    assert out[0][2] >= 1 and out[1][2] == 0
    for q in range(n):
        assert out[0][1][q]["iters"] == out[1][1][q]["iters"] and torch.equal(out[0][0][q], out[1][0][q])


def test_shutdown_cancels_what_is_not_done(sip):
    """sip_server_shutdown: requests still queued or running complete with
    SIP_ECANCELLED and their x is not written, a poller blocked on one wakes
    up, finished ones keep their results (equal to the solo solve), and later
    submissions are refused with SIP_ECANCELLED."""
    import threading
    data = [block((40, 36, 30), "cd", 600 + q) for q in range(12)]
    keep = [(dev(A), dev(b)) for A, b in data]
    xs = [torch.full_like(b, 7.0) for _, b in keep]
    srv = sip.Server(max_slots=1, epoch_iters=4)   # one request at a time: the others queue
    tickets = [srv.submit(q, A, b, xs[q], rtol=1e-10, max_iter=100000) for q, (A, b) in enumerate(keep)]
    got = {}
    waiter = threading.Thread(target=lambda: got.setdefault("last", srv.poll(tickets[-1])))
    waiter.start()
    srv.shutdown()
    waiter.join(timeout=60)
    assert not waiter.is_alive()
    res = [srv.poll(t) for t in tickets[:-1]] + [got["last"]]
    with pytest.raises(sip.SipError) as e:
        srv.submit(99, keep[0][0], keep[0][1], torch.zeros_like(keep[0][1]))
    assert e.value.status == sip.SIP_ECANCELLED
    srv.shutdown()   # a second call does nothing
    srv.close()
    status = [r["status"] for r in res]
    log(f"  statuses after shutdown: {status}")
    assert set(status) <= {sip.SIP_OK, sip.SIP_ECANCELLED}
    assert status.count(sip.SIP_ECANCELLED) >= 6 and status[-1] == sip.SIP_ECANCELLED
    for q, (A, b) in enumerate(data):
        if status[q] == sip.SIP_ECANCELLED:
            assert bool((xs[q] == 7.0).all()), f"request {q}: cancelled, x written"
        else:
            xa, it, _ = alone(sip, A, b, "mixed", rtol=1e-10)
            assert res[q]["iters"] == it and np.array_equal(xs[q].cpu().numpy(), xa)


def test_full_queue_refuses_with_busy(sip):
    """max_queue bounds the requests waiting for admission: with one slot and
    room for three in the queue, a burst of six gets SIP_EBUSY for some; the
    accepted ones finish with their solo results."""
    data = [block((40, 36, 30), "cd", 700 + q) for q in range(6)]
    keep = [(dev(A), dev(b)) for A, b in data]
    xs = [torch.zeros_like(b) for _, b in keep]
    srv = sip.Server(max_slots=1, epoch_iters=4, max_queue=3)
    accepted, busy = [], 0
    for q, (A, b) in enumerate(keep):
        try:
            accepted.append((q, srv.submit(q, A, b, xs[q], rtol=1e-8)))
        except sip.SipError as e:
            assert e.status == sip.SIP_EBUSY
            busy += 1
    res = [(q, srv.poll(t)) for q, t in accepted]
    srv.close()
    log(f"  accepted {len(accepted)}, busy {busy}")
    assert busy >= 1 and len(accepted) >= 3
    for q, r in res:
        xa, it, _ = alone(sip, *data[q], "mixed")
        assert r["status"] == sip.SIP_OK and r["iters"] == it and np.array_equal(xs[q].cpu().numpy(), xa)


@pytest.mark.parametrize("pairs", ["0", "1"])
def test_epochs_replayed_from_a_graph(sip, monkeypatch, pairs):
    """While no request joins or leaves, the server replays its epoch's sweeps
    from a captured graph (the job lists and ticket orders are uploaded before
    every replay, with the host's own bookkeeping in between); results stay
    bitwise the solo solves.  Epochs exist in the per-iteration launch mode."""
    monkeypatch.setenv("SIP_SERVER_PAIRS", pairs)
    monkeypatch.setenv("SIP_SERVER_PERSISTENT", "0")
    data = [block(d, k, 800 + q) for q, (d, k) in enumerate(BLOCKS[:4])]
    A0, _ = data[0]
    data += [(A0, np.random.default_rng(900 + q).uniform(-1, 1, A0.shape[1:])) for q in range(2)]
    keep = [(dev(A), dev(b)) for A, b in data]
    xs = [torch.zeros_like(b) for _, b in keep]
    srv = sip.Server(max_slots=16, epoch_iters=2)
    ids = [0, 1, 2, 3, 0, 0]   # the last two share the first system (pairs when on)
    tickets = [srv.submit(ids[q], A, b, xs[q], rtol=1e-10, max_iter=100000, retain=True)
               for q, (A, b) in enumerate(keep)]
    res = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    log(f"  pairs {pairs}: epochs {st['epochs']}, replayed from a graph {st['graph_epochs']}")
    assert st["graph_epochs"] >= 1
    for q, (A, b) in enumerate(data):
        xa, it, _ = alone(sip, A, b, "mixed", rtol=1e-10)
        assert res[q]["status"] == sip.SIP_OK and res[q]["iters"] == it, f"request {q}"
        assert np.array_equal(xs[q].cpu().numpy(), xa), f"request {q}"
