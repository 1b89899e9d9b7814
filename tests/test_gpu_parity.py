"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar (FP64): factors elementwise within 1e-13 relative; every iterate x_n
within 1e-12 * max|x_n(oracle)|; residual history within 1e-12 absolute
(rho is already normalised by ||b||).  Mixed form: every iterate x_n within
MIXED_TOL * max|x_n(oracle)| of the mixed-form oracle, with rho_n the oracle's
FP64 residual norm of the GPU's own x_n (1e-12 absolute); solves reach the
same final residual bar (<= rtol, re-checked by the oracle's FP64 residual)
with an iteration count within 2 of the mixed-form oracle.
"""
import numpy as np
import pytest

import oracle
from paper_1303_4538_amd import problems
from tests import dense
from tests.mixed_check import MIXED_TOL, mixed_iterates_agree  # noqa: F401

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


def factors_close(Lg, Lo, tol=1e-13):
    scale = np.maximum(np.abs(Lo), 1e-300)
    rel = np.abs(Lg - Lo) / scale
    # entries that are exactly zero in the oracle must be (near) zero on the GPU
    zero = Lo == 0
    return float(np.where(zero, np.abs(Lg), rel).max())


def make(kind, dims, seed=0):
    ni, nj, nk = dims
    rng = np.random.default_rng(seed)
    if kind == "poisson":
        A = problems.poisson(ni, nj, nk)
    elif kind == "cd":
        A = problems.convection_diffusion(ni, nj, nk, rng)
    elif kind == "stretched":
        A = problems.stretched_poisson(ni, nj, nk)
    else:
        A = dense.random_mmatrix(ni, nj, nk, rng)
    b = rng.uniform(-1, 1, (nk, nj, ni))
    return A, b


@pytest.mark.parametrize("dims,kind", [((16, 16, 16), "cd"), ((33, 20, 13), "random"), ((17, 35, 9), "poisson"),
                                       ((1, 40, 21), "cd"), ((37, 1, 18), "stretched"), ((23, 19, 1), "cd"),
                                       ((48, 47, 5), "cd")])
def test_mixed_iterates_match_mixed_oracle(sip, dims, kind):
    A, b = make(kind, dims, 17)
    LU = oracle.factor(A, 0.92)
    log(f"mixed iterates {kind} {dims}")
    S = sip.sip_factor(dev(A), 0.92, "mixed")
    worst = mixed_iterates_agree(sip, S, A, LU, b, 6)
    log(f"  worst x_n rel diff {worst:.2e}")


def test_config1_factors(sip):
    c = problems.config1()
    log("config1 factor fp64")
    S = sip.sip_factor(dev(c["A"]), c["alpha"], "fp64")
    Lg = sip.sip_export_factors(S).cpu().numpy()
    Lo = oracle.factor(c["A"], c["alpha"])
    assert factors_close(Lg, Lo) <= 1e-13


def test_config1_every_iteration(sip):
    """16^3 Poisson, alpha 0.92, 50 iterations: x_n and rho_n after every update."""
    c = problems.config1()
    A, b = c["A"], c["b"]
    LU = oracle.factor(A, c["alpha"])
    log("config1 factor + 50 single-iteration calls")
    S = sip.sip_factor(dev(A), c["alpha"], "fp64")
    bt = dev(b)
    xt = torch.zeros_like(bt)
    xo = np.zeros_like(b)
    for n in range(c["n_iter"]):
        hg = sip.sip_iterate(S, bt, xt, 1)
        xo, ho = oracle.iterate(A, LU, b, xo, 1)
        xg = xt.cpu().numpy()
        assert np.abs(xg - xo).max() <= 1e-12 * np.abs(xo).max(), f"iteration {n + 1}"
        assert np.abs(hg - ho).max() <= 1e-12, f"rho at iteration {n + 1}"
    # the same 50 iterations in one call give the same history
    xt2 = torch.zeros_like(bt)
    hg = sip.sip_iterate(S, bt, xt2, c["n_iter"])
    _, ho = oracle.iterate(A, LU, b, np.zeros_like(b), c["n_iter"])
    assert np.abs(hg - ho).max() <= 1e-12
    assert np.abs(xt2.cpu().numpy() - xo).max() <= 1e-12 * np.abs(xo).max()


DIMS = [(8, 8, 8), (17, 5, 3), (9, 13, 11), (1, 1, 7), (7, 1, 1), (1, 7, 1), (33, 20, 7), (16, 24, 5),
        (5, 3, 40), (25, 17, 1), (64, 9, 2)]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("kind", ["poisson", "cd", "random"])
def test_parity_dims(sip, dims, kind):
    """Several tiles, ragged edges and degenerate axes; 6 updates."""
    A, b = make(kind, dims, seed=sum(dims))
    alpha = 0.92 if kind != "random" else 0.6
    log(f"parity {kind} {dims}")
    S = sip.sip_factor(dev(A), alpha, "fp64")
    LU = oracle.factor(A, alpha)
    assert factors_close(sip.sip_export_factors(S).cpu().numpy(), LU) <= 1e-13
    x0 = np.random.default_rng(5).uniform(-0.5, 0.5, b.shape)
    xt = dev(x0)
    hg = sip.sip_iterate(S, dev(b), xt, 6)
    xo, ho = oracle.iterate(A, LU, b, x0, 6)
    assert np.abs(xt.cpu().numpy() - xo).max() <= 1e-12 * np.abs(xo).max()
    assert np.abs(hg - ho).max() <= 1e-12


def test_zero_iterations_round_trip_bitexact(sip):
    A, b = make("cd", (19, 11, 6), 3)
    S = sip.sip_factor(dev(A), 0.92, "fp64")
    x0 = np.random.default_rng(1).standard_normal(b.shape)
    xt = dev(x0)
    hg = sip.sip_iterate(S, dev(b), xt, 0)
    assert np.array_equal(xt.cpu().numpy(), x0)
    ro = oracle.norm2(oracle.residual(A, b, x0)) / oracle.norm2(b)
    assert abs(hg[0] - ro) <= 1e-12


def test_zero_rhs_gives_zero(sip):
    A, _ = make("poisson", (10, 9, 8))
    S = sip.sip_factor(dev(A), 0.92, "fp64")
    bt = torch.zeros((8, 9, 10), dtype=torch.float64, device="cuda")
    xt = torch.ones_like(bt)
    st, it, rr, _ = sip.sip_solve(S, bt, xt, 1e-8, 10)
    assert st == sip.SIP_OK and it == 0 and rr == 0.0
    assert float(xt.abs().max()) == 0.0


def test_breakdown_reported(sip):
    A, _ = make("poisson", (6, 6, 6))
    A[0, 0, 0, 0] = 0.0
    with pytest.raises(sip.SipError) as e:
        sip.sip_factor(dev(A), 0.92, "fp64")
    assert e.value.status == sip.SIP_EBREAKDOWN


def test_invalid_arguments(sip):
    A, b = make("poisson", (6, 5, 4))
    with pytest.raises(sip.SipError) as e:
        sip.sip_factor(dev(A), 1.5, "fp64")
    assert e.value.status == sip.SIP_EINVAL
    S = sip.sip_factor(dev(A), 0.92, "fp64")
    with pytest.raises(sip.SipError) as e:
        sip.sip_solve(S, dev(b), dev(b), -1.0, 10)
    assert e.value.status == sip.SIP_EINVAL


@pytest.mark.parametrize("dims,kind", [((16, 16, 16), "cd"), ((24, 20, 18), "cd"), ((20, 22, 17), "poisson"),
                                       ((30, 12, 25), "stretched")])
def test_mixed_solve_matches_mixed_oracle(sip, dims, kind):
    A, b = make(kind, dims, 11)
    LU = oracle.factor(A, 0.92)
    xo, ito, rro, _ = oracle.solve(A, LU, b, np.zeros_like(b), 1e-8, 5000, mixed=True)
    x64, it64, _, _ = oracle.solve(A, LU, b, np.zeros_like(b), 1e-8, 5000)
    log(f"mixed solve {kind} {dims}")
    S = sip.sip_factor(dev(A), 0.92, "mixed")
    xt = torch.zeros((dims[2], dims[1], dims[0]), dtype=torch.float64, device="cuda")
    st, it, rr, _ = sip.sip_solve(S, dev(b), xt, 1e-8, 5000)
    assert st == sip.SIP_OK and rr <= 1e-8
    assert abs(it - ito) <= 2
    xg = xt.cpu().numpy()
    r_cpu = oracle.norm2(oracle.residual(A, b, xg)) / oracle.norm2(b)
    assert r_cpu <= 1e-8 * (1 + 1e-9) and abs(r_cpu - rr) <= 1e-12
    # stated error against the FP64 oracle solution at the same tolerance
    err = np.abs(xg - x64).max() / np.abs(x64).max()
    log(f"  iters gpu {it} oracle-mixed {ito} oracle-fp64 {it64}; max rel err vs fp64 {err:.2e}")
    assert err <= 1e-6


@pytest.mark.parametrize("dims,kind", [((16, 16, 16), "cd"), ((33, 20, 13), "random")])
def test_fp64_solve_matches_oracle(sip, dims, kind):
    A, b = make(kind, dims, 21)
    LU = oracle.factor(A, 0.92)
    xo, ito, rro, ho = oracle.solve(A, LU, b, np.zeros_like(b), 1e-10, 5000)
    log(f"fp64 solve {kind} {dims}")
    S = sip.sip_factor(dev(A), 0.92, "fp64")
    xt = torch.zeros((dims[2], dims[1], dims[0]), dtype=torch.float64, device="cuda")
    st, it, rr, _ = sip.sip_solve(S, dev(b), xt, 1e-10, 5000)
    assert st == sip.SIP_OK
    assert it == ito and abs(rr - rro) <= 1e-12
    assert np.abs(xt.cpu().numpy() - xo).max() <= 1e-12 * np.abs(xo).max()


def test_not_converged_status(sip):
    A, b = make("cd", (20, 20, 20), 2)
    S = sip.sip_factor(dev(A), 0.92, "fp64")
    xt = torch.zeros((20, 20, 20), dtype=torch.float64, device="cuda")
    st, it, rr, _ = sip.sip_solve(S, dev(b), xt, 1e-14, 5, raise_on_notconv=False)
    assert st == sip.SIP_ENOTCONV and it == 5
    LU = oracle.factor(A, 0.92)
    xo, ho = oracle.iterate(A, LU, b, np.zeros_like(b), 5)
    assert abs(rr - ho[5]) <= 1e-12
    assert np.abs(xt.cpu().numpy() - xo).max() <= 1e-12 * np.abs(xo).max()


def test_config2_full_size(sip):
    """256^3 convection-diffusion at the benchmark's size: factors and the first
    two iterates against the oracle; then the mixed solve to 1e-8 with its
    final residual re-checked by the oracle in FP64."""
    c = problems.config2()
    A, b = c["A"], c["b"]
    log("config2 256^3 factor fp64")
    S = sip.sip_factor(dev(A), c["alpha"], "fp64")
    LU = oracle.factor(A, c["alpha"])
    Lg = sip.sip_export_factors(S).cpu().numpy()
    assert factors_close(Lg, LU) <= 1e-13
    del Lg
    log("config2 2 iterations fp64")
    xt = torch.zeros_like(dev(b))
    hg = sip.sip_iterate(S, dev(b), xt, 2)
    xo, ho = oracle.iterate(A, LU, b, np.zeros_like(b), 2)
    assert np.abs(xt.cpu().numpy() - xo).max() <= 1e-12 * np.abs(xo).max()
    assert np.abs(hg - ho).max() <= 1e-12
    S.close()
    log("config2 mixed solve to 1e-8")
    S = sip.sip_factor(dev(A), c["alpha"], "mixed")
    xt = torch.zeros_like(dev(b))
    st, it, rr, secs = sip.sip_solve(S, dev(b), xt, 1e-8, 20000)
    log(f"  mixed: {it} iterations, rho {rr:.3e}, {secs:.2f} s")
    assert st == sip.SIP_OK and rr <= 1e-8
    r_cpu = oracle.norm2(oracle.residual(A, b, xt.cpu().numpy())) / oracle.norm2(b)
    assert r_cpu <= 1e-8 * (1 + 1e-9)


def test_tune_keeps_results_and_records_the_plan(sip, tmp_path):
    """The autotuner picks a launch shape; solves before and after it, and on
    a new system of the same shape (which starts with the tuned plan), are
    bitwise the same; the plan is in the saved tuning table."""
    import json
    A, b = make("cd", (40, 33, 21), 17)
    S = sip.sip_factor(dev(A), 0.92, "mixed")
    x1 = torch.zeros_like(dev(b))
    _, it1, _, _ = sip.sip_solve(S, dev(b), x1, 1e-8, 5000)
    ph = sip.sip_tune(S, dev(b), 3)
    assert 1 <= ph <= 3
    tuned = sip.sip_system_plan(S)
    assert tuned[0] == ph and 1 <= tuned[1] <= 3
    sip.sip_tune_save(tmp_path / "tune.jsonl")
    saved = [json.loads(line) for line in (tmp_path / "tune.jsonl").read_text().splitlines()]
    assert dict(ni=40, nj=33, nk=21, precision=1, symmetric=0, phases=ph, poll=tuned[1]) in saved
    x2 = torch.zeros_like(dev(b))
    _, it2, _, _ = sip.sip_solve(S, dev(b), x2, 1e-8, 5000)
    S.close()
    S = sip.sip_factor(dev(A), 0.92, "mixed")
    assert sip.sip_system_plan(S) == tuned   # a new system of the shape starts with the tuned plan
    x3 = torch.zeros_like(dev(b))
    _, it3, _, _ = sip.sip_solve(S, dev(b), x3, 1e-8, 5000)
    S.close()
    assert it1 == it2 == it3 and torch.equal(x1, x2) and torch.equal(x1, x3)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
def test_graph_replays_equal_eager_launches(sip, precision):
    """sip_iterate replays a captured graph for every 8 iterations; 24
    iterations that way (three replays, host work in between) equal 24 eager
    single iterations, each restaging x (exact: x is stored at the
    precision the sweeps update it in), bitwise, residual history included;
    the same call twice gives the same bits (deterministic norms)."""
    A, b = make("cd", (37, 29, 17), 21)
    S = sip.sip_factor(dev(A), 0.92, precision)
    bt = dev(b)
    xg = torch.zeros_like(bt)
    hg = sip.sip_iterate(S, bt, xg, 24)
    xg2 = torch.zeros_like(bt)
    hg2 = sip.sip_iterate(S, bt, xg2, 24)
    assert torch.equal(xg, xg2) and np.array_equal(hg, hg2)
    xe = torch.zeros_like(bt)
    he = []
    for n in range(24):
        h = sip.sip_iterate(S, bt, xe, 1)
        he.append(h[0])
    he.append(sip.sip_iterate(S, bt, xe, 0)[0])
    S.close()
    assert torch.equal(xg, xe)
    assert np.array_equal(hg, np.array(he))
