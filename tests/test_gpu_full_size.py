"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times.

* 512 x 512 x 256 stretched-grid Poisson (67 M cells): FP64 factors and the
  first two iterates elementwise against the oracle (1e-13 / 1e-12), then
  mixed iterates with the FP64 residual of the result re-checked by the
  oracle on every cell.
* 64 uneven blocks through one solve server (mixed to 1e-8): every block's
  result equals its solo solve bitwise and its FP64 residual, re-checked by
  the oracle, is <= 1e-8.
* 256^3 with the all-FP32 relaxation, a pair of right-hand sides and the
  domain cut into 2^3 blocks: first iterates against the oracle (all-FP32,
  multi-block) or against the solo solves (pair, bitwise).
* 256^3 convection-diffusion, mixed: the first iterates elementwise against
  the mixed-form oracle (2 x the CPU-pinned bound), and the 2^3-block domain's
  mixed iterates against the multi-block oracle.
* The largest block the layout takes at a 1024^2 cross-section
  (1024 x 1024 x 239): FP64 factors and iterates against the oracle.
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
    assert torch.cuda.is_available()
    return s


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_config4_large_block(sip):
    c = problems.config4()
    A, b = c["A"], c["b"]
    log("512x512x256 stretched Poisson: factor fp64")
    At, bt = dev(A), dev(b)
    S = sip.sip_factor(At, c["alpha"], "fp64")
    LU = oracle.factor(A, c["alpha"])
    Lg = sip.sip_export_factors(S).cpu().numpy()
    zero = LU == 0
    rel = np.where(zero, np.abs(Lg), np.abs(Lg - LU) / np.maximum(np.abs(LU), 1e-300))
    assert float(rel.max()) <= 1e-13
    del Lg, rel, zero
    log("  2 iterations fp64")
    xt = torch.zeros_like(bt)
    hg = sip.sip_iterate(S, bt, xt, 2)
    S.close()
    xo, ho = oracle.iterate(A, LU, b, np.zeros_like(b), 2)
    assert np.abs(xt.cpu().numpy() - xo).max() <= 1e-12 * np.abs(xo).max()
    assert np.abs(hg - ho).max() <= 1e-12
    del xo
    log("  40 mixed iterations, residual re-checked")
    S = sip.sip_factor(At, c["alpha"], "mixed")
    xt = torch.zeros_like(bt)
    hg = sip.sip_iterate(S, bt, xt, 40)
    S.close()
    r = oracle.norm2(oracle.residual(A, b, xt.cpu().numpy())) / oracle.norm2(b)
    assert abs(r - hg[-1]) <= 1e-12
    assert hg[-1] < hg[0]


@pytest.mark.timeout(600)
def test_largest_block(sip):
    """The largest block the tile-sheared layout takes at a 1024 x 1024 cross
    section: 1024 x 1024 x 239 (250.6 M cells, just under 2^28 sheared
    elements, where the byte offsets of the 16-byte coefficient pairs come
    within 0.4 % of 2^32).  FP64 factors and two iterates elementwise against
    the oracle."""
    A = problems.poisson(1024, 1024, 239)
    b = np.random.default_rng(239).uniform(-1, 1, A.shape[1:])
    log("1024x1024x239 Poisson: factor fp64 + 2 iterations")
    At, bt = dev(A), dev(b)
    S = sip.sip_factor(At, 0.92, "fp64")
    del At
    Lg = sip.sip_export_factors(S).cpu().numpy()
    xt = torch.zeros_like(bt)
    hg = sip.sip_iterate(S, bt, xt, 2)
    S.close()
    xg = xt.cpu().numpy()
    del xt, bt
    log("  oracle factor")
    LU = oracle.factor(A, 0.92)
    zero = LU == 0
    rel = np.where(zero, np.abs(Lg), np.abs(Lg - LU) / np.maximum(np.abs(LU), 1e-300))
    assert float(rel.max()) <= 1e-13
    del Lg, rel, zero
    log("  oracle iterations")
    xo, ho = oracle.iterate(A, LU, b, np.zeros_like(b), 2)
    assert np.abs(xg - xo).max() <= 1e-12 * np.abs(xo).max()
    assert np.abs(hg - ho).max() <= 1e-12


def test_config3_batched_blocks(sip):
    meta = problems.config3_meta()
    blocks = []
    for dims, kind, ss in meta:
        A, b = problems.make_block(dims, kind, ss)
        blocks.append((A, b, dev(A), dev(b)))
    log(f"64 blocks, {sum(A.shape[1] * A.shape[2] * A.shape[3] for A, _, _, _ in blocks)} cells, one server")
    srv = sip.Server(max_slots=256, epoch_iters=8)
    xs = [torch.zeros_like(bt) for _, _, _, bt in blocks]
    tickets = [srv.submit(q, At, bt, xs[q], precision="mixed", rtol=1e-8, max_iter=200000)
               for q, (_, _, At, bt) in enumerate(blocks)]
    res = [srv.poll(t) for t in tickets]
    srv.close()
    for q, (A, b, At, bt) in enumerate(blocks):
        assert res[q]["status"] == sip.SIP_OK and res[q]["rel_res"] <= 1e-8
        S = sip.sip_factor(At, 0.92, "mixed")
        xa = torch.zeros_like(bt)
        _, it, rr, _ = sip.sip_solve(S, bt, xa, 1e-8, 200000)
        S.close()
        assert res[q]["iters"] == it and torch.equal(xs[q], xa), f"block {q}"
        # the server's launch (thousands of tiles, two loader phases) and the
        # solo solve (three phases) sum the residual norms in the same order
        assert res[q]["rel_res"] == rr, f"block {q}"
        rc = oracle.norm2(oracle.residual(A, b, xs[q].cpu().numpy())) / oracle.norm2(b)
        assert rc <= 1e-8 * (1 + 1e-9), f"block {q}"


@pytest.fixture(scope="module")
def cube():
    return problems.config2()


def test_config2_all_fp32(sip, cube):
    A, b = cube["A"], cube["b"]
    log("256^3 all-FP32: 2 iterations against the oracle")
    S = sip.sip_factor(dev(A), cube["alpha"], "fp32")
    xt = torch.zeros_like(dev(b))
    hg = sip.sip_iterate(S, dev(b), xt, 2)
    S.close()
    xo, ho = oracle.iterate(A, oracle.factor(A, cube["alpha"]), b, np.zeros_like(b), 2, fp32=True)
    assert np.abs(xt.cpu().numpy() - xo).max() <= 4e-6 * np.abs(xo).max()
    assert np.abs(hg - ho).max() <= 2e-6


def test_config2_pair(sip, cube):
    A, b = cube["A"], cube["b"]
    log("256^3 pair of right-hand sides: 3 iterations against the solo solves")
    b2 = np.ascontiguousarray(b[::-1])
    S = sip.sip_factor(dev(A), cube["alpha"], "mixed")
    bs = [dev(b), dev(b2)]
    xs = [torch.zeros_like(bs[0]), torch.zeros_like(bs[0])]
    hp = sip.sip_iterate_multi(S, bs, xs, 3)
    for r in range(2):
        xa = torch.zeros_like(bs[0])
        ha = sip.sip_iterate(S, bs[r], xa, 3)
        assert torch.equal(xs[r], xa) and np.array_equal(hp[r], ha)
    S.close()


def test_config2_blocks(sip, cube):
    A, b = cube["A"], cube["b"]
    cuts = ([0, 128, 256],) * 3
    log("256^3 in 2^3 blocks: 2 iterations against the multi-block oracle")
    B = sip.sip_blocks_factor(dev(A), cuts, cube["alpha"], "fp64")
    xt = torch.zeros_like(dev(b))
    hg = B.iterate(dev(b), xt, 2)
    B.close()
    xo, _, _, ho = oracle.blocks(A, cube["alpha"], b, np.zeros_like(b), cuts, 2)
    assert np.abs(xt.cpu().numpy() - xo).max() <= 1e-12 * np.abs(xo).max()
    assert np.abs(hg - ho).max() <= 1e-12


def test_config2_mixed_iterates(sip, cube):
    """Mixed iterates at the benchmark's size, in its launch configuration
    (single system, default plan): x_1..x_3 elementwise against the mixed
    oracle within 4e-6 max|x_n| (twice the pinned bound)."""
    from tests.mixed_check import mixed_iterates_agree
    A, b, alpha = cube["A"], cube["b"], cube["alpha"]
    log("256^3 mixed: factor, 3 single iterations against the mixed oracle")
    S = sip.sip_factor(dev(A), alpha, "mixed")
    LU = oracle.factor(A, alpha)
    worst = mixed_iterates_agree(sip, S, A, LU, b, 3, log_every=True)
    S.close()
    log(f"  worst {worst:.2e}")


def test_config2_blocks_mixed_iterates(sip, cube):
    """The 256^3 domain in 2^3 blocks, mixed: x_1, x_2 elementwise against the
    multi-block mixed oracle (same 4e-6 bar)."""
    A, b, alpha = cube["A"], cube["b"], cube["alpha"]
    cuts = ([0, 128, 256], [0, 128, 256], [0, 128, 256])
    log("256^3 in 2^3 blocks, mixed: 2 iterations against the multi-block mixed oracle")
    D = sip.sip_blocks_factor(dev(A), cuts, alpha, "mixed")
    bt = dev(b)
    xt = torch.zeros_like(bt)
    xo = np.zeros_like(b)
    for n in (1, 2):
        D.iterate(bt, xt, 1)
        xo = oracle.blocks(A, alpha, b, xo, cuts, 1, mixed=True)[0]
        err = float(np.abs(xt.cpu().numpy() - xo).max() / np.abs(xo).max())
        log(f"  x_{n}: max rel diff {err:.2e}")
        assert err <= 4e-6
    D.close()


@pytest.mark.timeout(600)
def test_config4_mixed_solve(sip):
    """The 512 x 512 x 256 block solved in the mixed form to 1e-8 (about 15 k
    iterations); the returned x is re-checked with the oracle's FP64 residual
    on every cell."""
    c = problems.config4()
    A, b = c["A"], c["b"]
    log("512x512x256 stretched Poisson: mixed solve to 1e-8")
    At, bt = dev(A), dev(b)
    S = sip.sip_factor(At, c["alpha"], "mixed")
    xt = torch.zeros_like(bt)
    st, it, rr, _ = sip.sip_solve(S, bt, xt, 1e-8, 200000)
    S.close()
    log(f"  {it} iterations, rel_res {rr:.3e}; oracle FP64 residual")
    assert st == sip.SIP_OK and rr <= 1e-8
    r = oracle.norm2(oracle.residual(A, b, xt.cpu().numpy())) / oracle.norm2(b)
    assert abs(r - rr) <= 1e-12
    assert r <= 1e-8 * (1 + 1e-9)
