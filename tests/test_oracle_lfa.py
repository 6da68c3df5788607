"""Pins of the two-grid local Fourier analysis (Section 4) and of the
oracle's multigrid cycle against it."""
import itertools

import numpy as np
import pytest

from oracle import lfa
from oracle import grid as G
from oracle import cycle as C
from synthetic import constant_media
from golden_io import load


def _low_grid(N):
    """the periodic N-grid's frequencies inside T_low = [-pi/2, pi/2)"""
    return [2 * np.pi * k / N for k in range(-N, N) if -np.pi / 2 - 1e-12 <= 2 * np.pi * k / N < np.pi / 2 - 1e-12]


@pytest.mark.parametrize("dim,N,beta,w,nu", [
    (2, 8, 2 / 3, 0.55, (1, 1)),
    (2, 12, 1.0, 0.75, (1, 1)),
    (2, 8, 0.6, 0.7, (2, 1)),
    (3, 4, 2 / 3, 0.55, (1, 1)),
    (3, 4, 1.0, 0.6, (1, 2))])
def test_lfa_equals_exact_periodic_two_grid(dim, N, beta, w, nu):
    """P8: on a periodic grid the two-grid operator decouples into the LFA
    symbol blocks, so the LFA maximum over the grid's low frequencies equals
    the exact spectral radius of the assembled two-grid operator."""
    kw = dict(h=0.9, omega=0.7, gamma=0.01, beta=beta, lam=3.0, mu=1.3, rho=1.1)
    prob = lfa.PeriodicProblem(N, dim, **kw)
    TG = lfa.periodic_two_grid(prob, alpha=0.3, w=w, nu1=nu[0], nu2=nu[1])
    exact = np.abs(np.linalg.eigvals(TG)).max()
    L = lfa.LFA(dim, alpha=0.3, w=w, nu1=nu[0], nu2=nu[1], **kw)
    ks = _low_grid(N)
    assert abs(L.rho_loc(thetas=itertools.product(ks, repeat=dim)) - exact) <= 1e-10


def test_periodic_operator_matches_symbol():
    """the periodic assembly acts on every discrete plane wave exactly as the
    closed-form symbol (no boundary rows at all)"""
    from oracle import symbols as S
    N, d = 8, 2
    kw = dict(h=0.7, omega=1.1, gamma=0.05, beta=2 / 3, lam=2.0, mu=1.5, rho=0.8)
    prob = lfa.PeriodicProblem(N, d, **kw)
    A = prob.operator(0.2).toarray()
    th = np.array([2 * np.pi * 3 / N, -2 * np.pi * 1 / N])
    i2, i1 = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    amp = np.array([0.3 + 0.1j, -0.7j, 1.2])
    x = []
    for f in range(3):
        ph = th[0] * (i1 + (0 if f == 0 else 0.5)) + th[1] * (i2 + (0 if f == 1 else 0.5))
        x.append(amp[f] * np.exp(1j * ph).ravel())
    x = np.concatenate(x)
    Hs = S.operator_symbol(th, kw["h"], kw["omega"], kw["gamma"] + 0.2, kw["beta"], kw["lam"], kw["mu"], kw["rho"])
    yh = Hs @ amp
    y = A @ x
    for f in range(3):
        sl = slice(f * N * N, (f + 1) * N * N)
        assert np.allclose(y[sl], yh[f] * x[sl] / amp[f], atol=1e-12)


def test_measured_two_grid_factor_matches_lfa():
    """the oracle's two-grid cycle (red-black Vanka, exact coarse solve) on
    a 64^2 Dirichlet grid converges at the rate LFA predicts for beta = 2/3
    (lam = 20, mu = rho = 1, 10 points per wavelength, alpha = 0.3)"""
    n, om = 64, np.pi / 5
    m = constant_media((n, n), 20.0, 1.0, 1.0)
    rates = {}
    for beta, w in ((2 / 3, 0.65), (1.0, 0.75)):
        lv = G.Level((n, n), 1.0, om, 0.0, beta, m["lam"], m["mu"], m["rho"])
        hier = C.Hierarchy(lv, C.CycleParams(levels=2, alpha=0.3, damping=(w,), coarse="direct"))
        e = np.random.default_rng(0).standard_normal(lv.nunknowns()) + 0j
        norms = []
        for _ in range(40):
            e = hier.two_grid_error_matrix_action(e)
            norms.append(np.linalg.norm(e))
        rates[beta] = (norms[-1] / norms[19]) ** (1 / 20)
    L = lfa.LFA(2, h=1.0, omega=om, gamma=0.0, beta=2 / 3, lam=20.0, mu=1.0, rho=1.0, alpha=0.3, w=0.65)
    rho = L.rho_loc(step=2 * np.pi / n)
    assert abs(rates[2 / 3] - rho) <= 0.05, (rates, rho)
    assert rates[1.0] > rates[2 / 3] + 0.1


def test_lfa_reproduces_paper_trends():
    """P10 (range check; the paper's numbers are for lexicographic economic
    Vanka, so exact parity is unpinned): at the Table 1 settings (lam = 500,
    mu = rho = 1, h = 1/1024) the LFA-tuned beta = 2/3 has a much smaller
    two-grid factor than beta = 1, the beta = 2/3 factors are of the
    paper's magnitude, and the optimum of rho_loc over beta lies in
    [0.55, 0.75] (Section 4.3: 0.667)."""
    gold = load("paper_numbers.txt")
    h = 1 / 1024
    rb1, rb23 = [], []
    for om_div, alpha in ((5, 0.15), (4, 0.2), (3.3, 0.3)):
        for beta, w, store in ((1.0, 0.75, rb1), (2 / 3, 0.65, rb23)):
            L = lfa.LFA(2, h=h, omega=np.pi / (om_div * h), gamma=0.0, beta=beta, lam=500.0, mu=1.0, rho=1.0,
                        alpha=alpha, w=w)
            store.append(L.rho_loc(step=0.1))
    for a, b in zip(rb23, rb1):
        assert a < 0.7 * b
    for a, g in zip(rb23, gold["table1_rho_loc_beta23"][0]):
        assert abs(a - g) <= 0.2
    betas = [0.5, 0.6, 0.667, 0.75, 0.9, 1.0]
    r = [lfa.LFA(2, h=h, omega=np.pi / (5 * h), gamma=0.0, beta=b, lam=500.0, mu=1.0, rho=1.0, alpha=0.1,
                 w=0.7).rho_loc(step=0.1) for b in betas]
    assert 0.55 <= betas[int(np.argmin(r))] <= 0.75
    assert min(r) <= gold["lfa_rho_loc_beta_opt"][0, 0] + 0.15
