"""Race testing: with SIP_SCHEDULE_SEED set, a handle takes its tiles in a
random order that still lists every tile after its upstream neighbours, and
the factorisation and sweep waves pause at pseudo-random steps.  Results
must be bitwise those of the default schedule: the factors, every iterate,
the residual history and the stop decision, for single systems (every
precision), pairs of right-hand sides, multi-block domains and batches in the
solve server.  A difference would mean a result that depends on timing, i.e.
a missing wait somewhere in the cross-tile or cross-wave synchronisation.
"""
import numpy as np
import pytest

from paper_1303_4538_amd import problems

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SEEDS = [1, 7, 123457]


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


def solve_once(sip, A, b, precision, n_iter=None):
    S = sip.sip_factor(dev(A), 0.92, precision)
    LU = sip.sip_export_factors(S)
    x = torch.zeros_like(dev(b))
    if n_iter is None:
        out = sip.sip_solve(S, dev(b), x, 1e-8 if precision != "fp32" else 1e-4, 5000)[1:3]
    else:
        out = sip.sip_iterate(S, dev(b), x, n_iter)
    S.close()
    return LU, x, out


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
def test_single_system_under_random_schedules(sip, monkeypatch, precision):
    dims = (70, 50, 20)   # 5 x 4 tiles, a ragged tile edge on both axes
    rng = np.random.default_rng(31)
    A = problems.convection_diffusion(*dims, rng)
    b = rng.uniform(-1, 1, A.shape[1:])
    monkeypatch.delenv("SIP_SCHEDULE_SEED", raising=False)
    ref_it = solve_once(sip, A, b, precision, n_iter=12)
    ref_sv = solve_once(sip, A, b, precision)
    for seed in SEEDS:
        log(f"single {precision} seed {seed}")
        monkeypatch.setenv("SIP_SCHEDULE_SEED", str(seed))
        LU, x, h = solve_once(sip, A, b, precision, n_iter=12)
        assert torch.equal(LU, ref_it[0]) and torch.equal(x, ref_it[1]) and np.array_equal(h, ref_it[2])
        _, x, (it, rr) = solve_once(sip, A, b, precision)
        assert torch.equal(x, ref_sv[1]) and (it, rr) == ref_sv[2]


def sweep_ms(sip, A, b):
    S = sip.sip_factor(dev(A), 0.92, "mixed")
    ms = sip.sip_profile_sweeps(S, dev(b), torch.zeros_like(dev(b)), 20)
    S.close()
    return ms


def test_random_schedule_is_active(sip, monkeypatch):
    """The pauses really happen (else the tests above would prove nothing)."""
    rng = np.random.default_rng(35)
    A = problems.convection_diffusion(70, 50, 20, rng)
    b = rng.uniform(-1, 1, A.shape[1:])
    monkeypatch.delenv("SIP_SCHEDULE_SEED", raising=False)
    plain = sweep_ms(sip, A, b)
    monkeypatch.setenv("SIP_SCHEDULE_SEED", "7")
    paused = sweep_ms(sip, A, b)
    log(f"sweep ms plain {plain}, random schedule {paused}")
    assert paused[0] > 1.2 * plain[0] and paused[1] > 1.2 * plain[1]


def test_pair_under_random_schedules(sip, monkeypatch):
    dims = (40, 36, 30)
    rng = np.random.default_rng(32)
    A = problems.convection_diffusion(*dims, rng)
    bs = [dev(rng.uniform(-1, 1, A.shape[1:])), dev(rng.uniform(-1, 1, A.shape[1:]) ** 3)]

    def run():
        S = sip.sip_factor(dev(A), 0.92, "mixed")
        xs = [torch.zeros_like(b) for b in bs]
        st, info = sip.sip_solve_multi(S, bs, xs, 1e-8, 5000)
        S.close()
        return xs, [i[:2] for i in info]

    monkeypatch.delenv("SIP_SCHEDULE_SEED", raising=False)
    ref = run()
    for seed in SEEDS:
        log(f"pair seed {seed}")
        monkeypatch.setenv("SIP_SCHEDULE_SEED", str(seed))
        xs, info = run()
        assert all(torch.equal(xs[r], ref[0][r]) for r in range(2)) and info == ref[1]


def test_blocks_under_random_schedules(sip, monkeypatch):
    dims = (50, 40, 12)
    rng = np.random.default_rng(33)
    A = problems.convection_diffusion(*dims, rng)
    b = dev(rng.uniform(-1, 1, A.shape[1:]))
    cuts = ([0, 20, 50], [0, 17, 40], [0, 5, 12])

    def run():
        B = sip.sip_blocks_factor(dev(A), cuts, 0.92, "mixed")
        x = torch.zeros_like(b)
        h = B.iterate(b, x, 10)
        B.close()
        return x, h

    monkeypatch.delenv("SIP_SCHEDULE_SEED", raising=False)
    ref = run()
    for seed in SEEDS:
        log(f"blocks seed {seed}")
        monkeypatch.setenv("SIP_SCHEDULE_SEED", str(seed))
        x, h = run()
        assert torch.equal(x, ref[0]) and np.array_equal(h, ref[1])


def test_server_batch_under_random_schedules(sip, monkeypatch):
    rng = np.random.default_rng(34)
    dims = [(33, 20, 11), (17, 40, 9), (50, 18, 6), (24, 24, 24), (9, 9, 30), (40, 33, 5)]
    systems = []
    for q, d in enumerate(dims):
        A = problems.poisson(*d) if q % 2 else problems.convection_diffusion(*d, rng)
        systems.append((dev(A), dev(rng.uniform(-1, 1, A.shape[1:]))))

    def run():
        srv = sip.Server(max_slots=64, epoch_iters=4)
        xs = [torch.zeros_like(b) for _, b in systems]
        ts = [srv.submit(q, A, b, xs[q], precision="mixed" if q % 3 else "fp64", rtol=1e-8, max_iter=5000)
              for q, (A, b) in enumerate(systems)]
        res = [srv.poll(t) for t in ts]
        srv.close()
        return xs, [(r["status"], r["iters"], r["rel_res"]) for r in res]

    monkeypatch.delenv("SIP_SCHEDULE_SEED", raising=False)
    ref = run()
    for seed in SEEDS:
        log(f"server seed {seed}")
        monkeypatch.setenv("SIP_SCHEDULE_SEED", str(seed))
        xs, res = run()
        assert res == ref[1]
        assert all(torch.equal(xs[q], ref[0][q]) for q in range(len(dims)))
