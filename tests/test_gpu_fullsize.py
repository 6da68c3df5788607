"""Parity at the benchmark's full size (3D 256^3, seed 3, the benchmark's
solver settings and launch configuration: stencil autotuner on, graphs on).

Every output of the float32 residual that the benchmark's roofline times,
of the float64 apply and of the float32-input float64 outer operator is
compared with the oracle's matrix-free operator on the whole grid (about
35 s of host time per oracle apply); the benchmark's mixed-precision solve
is checked by recomputing its true residual with the oracle.  Tolerances as
in the small-grid parity tests.
"""
import numpy as np
import pytest
import torch

from oracle import grid as G
from oracle import operator as O
from synthetic import make_media, random_field, point_source, omega_for_ppw

pytestmark = pytest.mark.gpu

N = 256
SHAPE = (N, N, N)
ALPHA = 0.5
ABL = 16.0


@pytest.fixture(scope="module")
def bench_problem():
    from paper_2307_03242_amd import Problem
    m = make_media(SHAPE, 3)
    om = omega_for_ppw(m["vs"].min(), 1.0, 10)
    med = [torch.from_numpy(m[k]) for k in ("lam", "mu", "rho")]
    prob = Problem(*med, h=1.0, omega=om, gamma=0.01, alpha=ALPHA, beta=2 / 3, abl_width=ABL, abl_amp=2.0,
                   levels=4, nu1=1, nu2=1, cycle="K", damping=(0.6, 0.5, 0.4, 0.4), coarse_mode="krylov",
                   coarse_sweeps=1, coarse_restart=5, coarse_maxit=2, coarse_rtol=0.0,
                   precond_dtype=torch.complex64)
    lv = G.Level(tuple(reversed(SHAPE)), 1.0, om, 0.01, 2 / 3, m["lam"], m["mu"], m["rho"],
                 abl_width=ABL, abl_amp=2.0)
    yield prob, lv
    prob.close()
    torch.cuda.empty_cache()


def _maxrel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_residual_f32_full_size(bench_problem):
    """the benchmark's roofline kernel: b - H_s x in complex64 at 256^3"""
    prob, lv = bench_problem
    x = random_field(SHAPE, 41, nrhs=1).astype(np.complex64)
    b = random_field(SHAPE, 42, nrhs=1).astype(np.complex64)
    xg, bg = torch.from_numpy(x).cuda(), torch.from_numpy(b).cuda()
    prob.residual(bg, xg, shifted=True)  # first use: the autotuner picks the x_3 chunk
    r = prob.residual(bg, xg, shifted=True).cpu().numpy()[0].astype(np.complex128)
    del xg, bg
    ref = b[0].astype(np.complex128) - O.apply(lv, x[0].astype(np.complex128), shift=ALPHA)
    assert _maxrel(r, ref) <= 3e-5


def test_apply_f64_and_f32_input_full_size(bench_problem):
    """the float64 operator (plain solver) and the outer operator on the
    float32 preconditioned vector (mixed solver) at 256^3"""
    prob, lv = bench_problem
    x = random_field(SHAPE, 43, nrhs=1)
    ref = O.apply(lv, x[0])
    y = prob.apply(torch.from_numpy(x).cuda()).cpu().numpy()[0]
    assert _maxrel(y, ref) <= 1e-12
    x32 = x.astype(np.complex64)
    ref32 = O.apply(lv, x32[0].astype(np.complex128))
    y32 = prob.apply_f32_input(torch.from_numpy(x32).cuda()).cpu().numpy()[0]
    assert _maxrel(y32, ref32) <= 1e-12


def test_mixed_precision_solve_full_size(bench_problem):
    """the benchmark's solve (float32 K-cycle inside float64 FGMRES(5) to
    1e-6): its true residual recomputed with the oracle's operator"""
    prob, lv = bench_problem
    q = point_source(SHAPE)[None]
    u, info, code = prob.solve(torch.from_numpy(q).cuda(), rtol=1e-6, maxit=400)
    assert code == 0 and info[0]["status"] == 0
    un = u.cpu().numpy()[0]
    r = q[0] - O.apply(lv, un)
    rel = np.linalg.norm(r.ravel()) / np.linalg.norm(q.ravel())
    assert rel <= 1e-6 * (1 + 1e-3)
    assert abs(rel - info[0]["relres"]) <= 1e-9
