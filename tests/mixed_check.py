"""Elementwise comparison of mixed-form GPU iterates with the mixed-form oracle
(shared by the GPU parity tests)."""
import numpy as np

import oracle

# Twice the bound pinned on the CPU (tests/test_oracle_mixed.py, MIXED_B):
# the oracle's mixed iterates stay within MIXED_B max|x| of the exact defect
# correction with the FP32-rounded factors, and the GPU rounds the same
# operands, differing only in the order of its FP32 operations (FMA, a
# multiply by a rounded 1/Lp where the oracle divides by Lp).
MIXED_TOL = 4e-6


def mixed_iterates_agree(sip, S, A, LU, b, n_iter, log_every=False):
    """n_iter single mixed updates on the GPU and in the oracle from x = 0,
    compared after every update: x_n elementwise within MIXED_TOL, and the
    GPU's rho_n equal to the oracle's FP64 residual norm of the GPU's x_n."""
    import torch
    bt = torch.from_numpy(np.ascontiguousarray(b)).to("cuda")
    xt = torch.zeros_like(bt)
    xo = np.zeros_like(b)
    nb = oracle.norm2(b)
    worst = 0.0
    for n in range(1, n_iter + 1):
        hg = sip.sip_iterate(S, bt, xt, 1)
        xo, _ = oracle.iterate(A, LU, b, xo, 1, mixed=True)
        xg = xt.cpu().numpy()
        err = float(np.abs(xg - xo).max() / np.abs(xo).max())
        worst = max(worst, err)
        if log_every:
            print(f"  x_{n}: max rel diff vs mixed oracle {err:.2e}", flush=True)
        assert err <= MIXED_TOL, f"x_{n} differs from the mixed oracle by {err:.3e}"
        rho = oracle.norm2(oracle.residual(A, b, xg)) / nb
        assert abs(hg[1] - rho) <= 1e-12
    return worst
