"""Forward error of the mixed-precision solve (float32 K-cycle inside
float64 FGMRES) against the oracle at 32^3, beyond the sizes a sparse direct
solve reaches in a test.

The oracle runs the same algorithm in float64 (its matrix-free operator,
its K-cycle hierarchy, its FGMRES(5)): once to the solve's tolerance 1e-6
and once to 1e-11, which stands in for the exact solution.  A 1e-6 residual
leaves a forward error of a few 1e-5 on this operator in any precision, so
the precision bar compares like with like:
- the float32-cycle solution differs from the oracle's float64 solution at
  the same tolerance by at most 1e-5 (the mixed-precision bar of the
  method's design: a preconditioner in single precision inside a double
  precision outer solve);
- its error against the 1e-11 solution is within 1 % of the oracle's own
  (single precision in the cycle costs no accuracy beyond the tolerance's);
- the plain float64 solver matches the oracle's float64 solution to 1e-9."""
import numpy as np
import pytest
import torch

from oracle import grid as G
from oracle import operator as O
from oracle import cycle as C
from oracle.krylov import fgmres
from synthetic import make_media, point_source, omega_for_ppw

pytestmark = pytest.mark.gpu

N = 32
LEVELS = 3
DAMP = (0.6, 0.5, 0.4)


def test_mixed_precision_forward_error_32cubed():
    from paper_2307_03242_amd import Problem
    shape = (N, N, N)
    m = make_media(shape, 3)
    om = omega_for_ppw(m["vs"].min(), 1.0, 10)
    abl = 4.0 * N / 64
    lv = G.Level(shape, 1.0, om, 0.01, 2 / 3, m["lam"], m["mu"], m["rho"], abl_width=abl, abl_amp=2.0)
    hier = C.Hierarchy(lv, C.CycleParams(levels=LEVELS, alpha=0.5, damping=DAMP, coarse="krylov",
                                         coarse_sweeps=1, coarse_maxit=2, coarse_rtol=0.0, calls=3))
    A = O.assemble(lv)
    q = point_source(shape)
    b = G.pack(lv, q)
    x6, i6 = fgmres(lambda v: A @ v, b, precond=hier.vcycle, restart=5, tol=1e-6, maxit=400)
    xs, _ = fgmres(lambda v: A @ v, b, precond=hier.vcycle, restart=5, tol=1e-11, maxit=600)
    print("oracle iterations (1e-6):", i6["iters"], flush=True)
    cfg = dict(h=1.0, omega=om, gamma=0.01, alpha=0.5, beta=2 / 3, abl_width=abl, abl_amp=2.0, levels=LEVELS,
               nu1=1, nu2=1, cycle="K", damping=DAMP, coarse_mode="krylov", coarse_sweeps=1, coarse_restart=5,
               coarse_maxit=2, coarse_rtol=0.0)
    med = [torch.from_numpy(m[k]) for k in ("lam", "mu", "rho")]
    qd = torch.from_numpy(q[None]).cuda()
    sols = {}
    for name, dt in (("f32", torch.complex64), ("f64", torch.complex128)):
        prob = Problem(*med, precond_dtype=dt, **cfg)
        u, info, code = prob.solve(qd, restart=5, maxit=400, rtol=1e-6)
        assert code == 0, info
        print(name, "iterations:", info[0]["iters"], flush=True)
        sols[name] = G.pack(lv, u.cpu().numpy()[0])
        prob.close()

    def rel(a, ref):
        return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))

    err64 = rel(x6, xs)
    err32 = rel(sols["f32"], xs)
    print("forward errors vs the 1e-11 oracle solution: oracle f64 %.3e, gpu f32-cycle %.3e, gpu f64 %.3e; "
          "f32-cycle vs oracle f64 at 1e-6: %.3e" % (err64, err32, rel(sols["f64"], xs), rel(sols["f32"], x6)),
          flush=True)
    assert rel(sols["f32"], x6) <= 1e-5
    assert err32 <= 1.01 * err64
    assert rel(sols["f64"], x6) <= 1e-9
