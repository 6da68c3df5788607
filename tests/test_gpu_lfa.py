"""The GPU two-grid cycle against local Fourier analysis (Section 4).

On a constant-coefficient grid without absorbing layer, the two-grid cycle
(red-black full Vanka, one pre- and one post-smoothing, dense exact coarse
solve) used as a stationary iteration on the shifted operator,
e <- e - V(H_s e), converges at the rate the LFA two-grid factor rho_loc
predicts (Definition of rho_loc).  Every cycle and residual runs on the GPU
through the C ABI; the oracle's two-grid cycle, iterated from the same
start, gives the same rate.
"""
import numpy as np
import pytest
import torch

from oracle import lfa
from oracle import grid as G
from oracle import cycle as C
from synthetic import constant_media

pytestmark = pytest.mark.gpu


def test_two_grid_rate_matches_lfa_2d():
    """64^2 cells, lam = 20, mu = rho = 1, 10 points per shear wavelength,
    alpha = 0.3: beta = 2/3 (w 0.65) converges at rho_loc within 0.05
    (boundaries), beta = 1 (w 0.75) clearly slower; the GPU and oracle
    rates agree to 1e-6"""
    from paper_2307_03242_amd import Problem
    n, om = 64, np.pi / 5
    m = constant_media((n, n), 20.0, 1.0, 1.0)
    med = [torch.from_numpy(m[k]) for k in ("lam", "mu", "rho")]
    rates, orates = {}, {}
    for beta, w in ((2 / 3, 0.65), (1.0, 0.75)):
        prob = Problem(*med, h=1.0, omega=om, gamma=0.0, alpha=0.3, beta=beta, abl_width=0.0, abl_amp=0.0,
                       levels=2, nu1=1, nu2=1, cycle="V", damping=(w,), coarse_mode="dense",
                       precond_dtype=torch.complex128)
        lv = G.Level((n, n), 1.0, om, 0.0, beta, m["lam"], m["mu"], m["rho"])
        e0 = np.random.default_rng(0).standard_normal(lv.nunknowns()) + 0j
        e = torch.from_numpy(G.unpack(lv, e0)[None]).cuda()
        zero = torch.zeros_like(e)
        norms = []
        for _ in range(40):
            e = e + prob.vcycle(prob.residual(zero, e, shifted=True))
            norms.append(torch.linalg.vector_norm(e).item())
        rates[beta] = (norms[-1] / norms[19]) ** (1 / 20)
        hier = C.Hierarchy(lv, C.CycleParams(levels=2, alpha=0.3, damping=(w,), coarse="direct"))
        eo, onorms = e0, []
        for _ in range(40):
            eo = hier.two_grid_error_matrix_action(eo)
            onorms.append(np.linalg.norm(eo))
        orates[beta] = (onorms[-1] / onorms[19]) ** (1 / 20)
        prob.close()
    rho = lfa.LFA(2, h=1.0, omega=om, gamma=0.0, beta=2 / 3, lam=20.0, mu=1.0, rho=1.0, alpha=0.3,
                  w=0.65).rho_loc(step=2 * np.pi / n)
    for beta in rates:
        assert abs(rates[beta] - orates[beta]) <= 1e-6, (rates, orates)
    assert abs(rates[2 / 3] - rho) <= 0.05, (rates, rho)
    assert rates[1.0] > rates[2 / 3] + 0.1
