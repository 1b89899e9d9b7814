"""Seeded synthetic linear systems shaped like the paper's pressure and momentum
systems (Sec. 2.2 test problems; Sec. 4.1: symmetric pressure-correction
systems versus non-symmetric convection-diffusion momentum systems).

This module only builds inputs.  It holds none of SIP's arithmetic and is the
one piece shared by the GPU path and the CPU oracle, which both receive the
arrays it returns.

Conventions: a block of ``ni x nj x nk`` cells is an array of shape
``(nk, nj, ni)`` (C order, i fastest).  Coefficients have shape
``(7, nk, nj, ni)`` in the order P, W, E, S, N, B, T, with signed entries: row P
reads ``A_P x_P + sum_nb A_nb x_nb = b_P``.  Couplings that would point out of
the block are stored as 0; the wall face still contributes to ``A_P``
(ghost-cell Dirichlet-0 walls, so the uniform Poisson stencil is 6 / -1).
"""
import math

import numpy as np

P, W, E, S, N, B, T = range(7)
MASTER_SEED = 1234
ALPHA = 0.92


def _mask_outward(A):
    """Zero the couplings that point out of the block."""
    A[W, :, :, 0] = 0.0
    A[E, :, :, -1] = 0.0
    A[S, :, 0, :] = 0.0
    A[N, :, -1, :] = 0.0
    A[B, 0, :, :] = 0.0
    A[T, -1, :, :] = 0.0
    return A


def poisson(ni, nj, nk):
    """7-point Poisson: A_P = 6, neighbours -1, Dirichlet-0 walls."""
    A = np.empty((7, nk, nj, ni), dtype=np.float64)
    A[P] = 6.0
    A[1:] = -1.0
    return _mask_outward(A)


def solenoidal_fluxes(ni, nj, nk, rng, fmax=2.0):
    """Face fluxes of a divergence-free random field with zero wall flux.

    A vector potential psi lives on cell edges (uniform[-1, 1] from ``rng``,
    zero on edges that lie in the block surface); the fluxes are its discrete
    curl, so every cell's net outflow is zero exactly and no flux crosses the
    walls.  The fluxes are scaled so that max |F| == fmax.

    Returns (Fx, Fy, Fz) with shapes (nk, nj, ni+1), (nk, nj+1, ni),
    (nk+1, nj, ni); Fx[k, j, f] is the flux in +x through the face between
    cells f-1 and f.
    """
    px = rng.uniform(-1.0, 1.0, size=(nk + 1, nj + 1, ni))   # edges along x
    py = rng.uniform(-1.0, 1.0, size=(nk + 1, nj, ni + 1))   # edges along y
    pz = rng.uniform(-1.0, 1.0, size=(nk, nj + 1, ni + 1))   # edges along z
    px[0], px[-1], px[:, 0], px[:, -1] = 0.0, 0.0, 0.0, 0.0
    py[0], py[-1], py[:, :, 0], py[:, :, -1] = 0.0, 0.0, 0.0, 0.0
    pz[:, 0], pz[:, -1], pz[:, :, 0], pz[:, :, -1] = 0.0, 0.0, 0.0, 0.0
    fx = (pz[:, 1:, :] - pz[:, :-1, :]) - (py[1:, :, :] - py[:-1, :, :])
    fy = (px[1:, :, :] - px[:-1, :, :]) - (pz[:, :, 1:] - pz[:, :, :-1])
    fz = (py[:, :, 1:] - py[:, :, :-1]) - (px[:, 1:, :] - px[:, :-1, :])
    m = max(np.abs(fx).max(initial=0.0), np.abs(fy).max(initial=0.0), np.abs(fz).max(initial=0.0))
    if m > 0.0:
        s = fmax / m
        fx *= s
        fy *= s
        fz *= s
    return fx, fy, fz


def convection_diffusion(ni, nj, nk, rng, diff=1.0, fmax=2.0):
    """First-order upwind convection-diffusion coefficients (non-symmetric).

    For each face f of cell P with outward flux F: A_nb = -(D + max(-F, 0)),
    and A_P = sum over the six faces of (D + max(F, 0)).  Wall faces carry no
    flux and keep their diffusive part D in A_P.
    """
    fx, fy, fz = solenoidal_fluxes(ni, nj, nk, rng, fmax)
    out = {
        E: fx[:, :, 1:], W: -fx[:, :, :-1],
        N: fy[:, 1:, :], S: -fy[:, :-1, :],
        T: fz[1:, :, :], B: -fz[:-1, :, :],
    }
    A = np.empty((7, nk, nj, ni), dtype=np.float64)
    A[P] = 0.0
    for d in (W, E, S, N, B, T):
        f = out[d]
        A[d] = -(diff + np.maximum(-f, 0.0))
        A[P] += diff + np.maximum(f, 0.0)
    return _mask_outward(A)


def stretched_poisson(ni, nj, nk, ratio=1.05):
    """Poisson on a grid stretched geometrically in z (dx = dy = 1,
    dz_k = ratio ** (k - (nk-1)/2)); face coefficients are area / distance,
    wall faces use the distance to a mirrored ghost (the cell's own width).
    Symmetric: A_T at cell k equals A_B at cell k+1."""
    k = np.arange(nk, dtype=np.float64)
    dz = ratio ** (k - (nk - 1) / 2.0)
    A = np.empty((7, nk, nj, ni), dtype=np.float64)
    lat = dz[:, None, None] * np.ones((1, nj, ni))          # area dy*dz over distance dx = 1
    A[W] = -lat
    A[E] = -lat
    A[S] = -lat
    A[N] = -lat
    dzt = np.empty(nk)
    dzt[:-1] = 1.0 / (0.5 * (dz[:-1] + dz[1:]))              # top face, interior
    dzt[-1] = 1.0 / dz[-1]                                   # top wall
    dzb = np.empty(nk)
    dzb[1:] = dzt[:-1]                                       # bottom face = top of k-1
    dzb[0] = 1.0 / dz[0]                                     # bottom wall
    A[T] = -dzt[:, None, None]
    A[B] = -dzb[:, None, None]
    A[P] = 4.0 * lat + dzt[:, None, None] + dzb[:, None, None]
    return _mask_outward(A)


def rhs_uniform(ni, nj, nk, rng):
    """Right-hand side with entries uniform[-1, 1]."""
    return rng.uniform(-1.0, 1.0, size=(nk, nj, ni))


# --------------------------------------------------------------------------
# The five workload recipes.  Every random draw comes from numpy's
# default_rng fed from SeedSequence(1234) (or a child of it).
# --------------------------------------------------------------------------

def config1():
    """16^3 Poisson, b uniform[-1,1] from default_rng(1234), alpha 0.92,
    50 iterations, plain FP64."""
    rng = np.random.default_rng(MASTER_SEED)
    b = rhs_uniform(16, 16, 16, rng)
    return dict(A=poisson(16, 16, 16), b=b, alpha=ALPHA, n_iter=50)


def config2(n=256, seed=MASTER_SEED):
    """n^3 upwind convection-diffusion (D = 1, max|F| = 2), b uniform[-1,1].
    The field uses the first child of SeedSequence(seed), b the second."""
    c_field, c_rhs = np.random.SeedSequence(seed).spawn(2)
    A = convection_diffusion(n, n, n, np.random.default_rng(c_field))
    b = rhs_uniform(n, n, n, np.random.default_rng(c_rhs))
    return dict(A=A, b=b, alpha=ALPHA, rtol=1e-8)


def config3_meta(n_blocks=64, lo=32, hi=160, seed=MASTER_SEED):
    """Dims and kinds of the batched workload: child 0 of SeedSequence(seed)
    draws dims uniform in {lo..hi} per axis and kind ('poisson' if u < 0.5
    else 'cd'); block b uses child b+1 for its field and right-hand side."""
    children = np.random.SeedSequence(seed).spawn(n_blocks + 1)
    meta = np.random.default_rng(children[0])
    dims = meta.integers(lo, hi + 1, size=(n_blocks, 3))
    kinds = np.where(meta.random(n_blocks) < 0.5, "poisson", "cd")
    return [(tuple(int(v) for v in dims[q]), str(kinds[q]), children[q + 1]) for q in range(n_blocks)]


def make_block(dims, kind, seedseq):
    """Coefficients and right-hand side of one block of a batched or served
    workload ('poisson', 'cd' or 'stretched')."""
    ni, nj, nk = dims
    rng = np.random.default_rng(seedseq)
    if kind == "poisson":
        A = poisson(ni, nj, nk)
    elif kind == "cd":
        A = convection_diffusion(ni, nj, nk, rng)
    elif kind == "stretched":
        A = stretched_poisson(ni, nj, nk)
    else:
        raise ValueError(kind)
    b = rhs_uniform(ni, nj, nk, rng)
    return A, b


def config3(n_blocks=64, lo=32, hi=160, seed=MASTER_SEED):
    """64 independent blocks, dims uniform {32..160} per axis, half Poisson
    and half convection-diffusion, b uniform[-1,1]."""
    out = []
    for dims, kind, ss in config3_meta(n_blocks, lo, hi, seed):
        A, b = make_block(dims, kind, ss)
        out.append(dict(dims=dims, kind=kind, A=A, b=b))
    return out


def config4(ni=512, nj=512, nk=256, seed=MASTER_SEED):
    """512 x 512 x 256 stretched-grid Poisson (z ratio 1.05), b uniform."""
    A = stretched_poisson(ni, nj, nk)
    b = rhs_uniform(ni, nj, nk, np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0]))
    return dict(A=A, b=b, alpha=ALPHA, rtol=1e-8)


def serving_stream(n_systems=250, rhs_per_system=8, rate_hz=200.0, lo=24, hi=192,
                   seed=MASTER_SEED + 5):
    """Request stream of the serving workload.

    System s: dims per axis lognormal with median sqrt(lo*hi) and sigma
    ln(hi/lo)/4 (so [lo, hi] is +-2 sigma), rounded and clipped to [lo, hi];
    kind Poisson or convection-diffusion with probability 1/2.  Each system
    receives ``rhs_per_system`` requests; all requests are shuffled and given
    Poisson arrivals (exponential gaps, mean 1/rate_hz seconds).

    Returns (systems, requests): systems[s] = (dims, kind, seedseq);
    requests[q] = (t_arrival_s, system_index, rhs_index, rhs_seedseq).
    """
    c_meta, c_sys, c_rhs = np.random.SeedSequence(seed).spawn(3)
    rng = np.random.default_rng(c_meta)
    med, sig = math.sqrt(lo * hi), math.log(hi / lo) / 4.0
    dims = np.clip(np.rint(rng.lognormal(math.log(med), sig, size=(n_systems, 3))), lo, hi).astype(int)
    kinds = np.where(rng.random(n_systems) < 0.5, "poisson", "cd")
    sys_ss = c_sys.spawn(n_systems)
    systems = [(tuple(int(v) for v in dims[s]), str(kinds[s]), sys_ss[s]) for s in range(n_systems)]
    order = rng.permutation(n_systems * rhs_per_system)
    gaps = rng.exponential(1.0 / rate_hz, size=order.size)
    t = np.cumsum(gaps)
    rhs_ss = c_rhs.spawn(order.size)
    requests = []
    for q, code in enumerate(order):
        s, m = divmod(int(code), rhs_per_system)
        requests.append((float(t[q]), s, m, rhs_ss[s * rhs_per_system + m]))
    return systems, requests


def system_coefficients(dims, kind, seedseq):
    """Coefficients of a served system (drawn from its own seed)."""
    ni, nj, nk = dims
    if kind == "poisson":
        return poisson(ni, nj, nk)
    return convection_diffusion(ni, nj, nk, np.random.default_rng(seedseq))


def request_rhs(dims, seedseq):
    ni, nj, nk = dims
    return rhs_uniform(ni, nj, nk, np.random.default_rng(seedseq))
