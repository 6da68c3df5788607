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


def _solver(m, shape, precond, levels, alpha=0.5, abl=ABL):
    from paper_2307_03242_amd import Problem
    om = omega_for_ppw(m["vs"].min(), 1.0, 10)
    args = dict(h=1.0, omega=om, gamma=0.01, alpha=alpha, beta=2 / 3, abl_width=abl, abl_amp=2.0, levels=levels,
                nu1=1, nu2=1, cycle="K", damping=(0.6, 0.5, 0.4, 0.4), coarse_mode="krylov", coarse_sweeps=1,
                coarse_restart=5, coarse_maxit=2, coarse_rtol=0.0)
    med = [torch.from_numpy(m[k]) for k in ("lam", "mu", "rho")]
    prob = Problem(*med, precond_dtype=precond, **args)
    lv = G.Level(tuple(reversed(shape)), 1.0, om, 0.01, 2 / 3, m["lam"], m["mu"], m["rho"],
                 abl_width=abl, abl_amp=2.0)
    return prob, lv


def _oracle_relres(lv, q, u):
    r = q - O.apply(lv, u)
    return np.linalg.norm(r.ravel()) / np.linalg.norm(q.ravel())


def _oracle_relres_many(cases, workers=8):
    """_oracle_relres over (lv, q, u) triples in host threads (the oracle's
    array arithmetic releases the interpreter lock)"""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda c: _oracle_relres(*c), cases))


def test_fp64_solve_128_full_size():
    """plain float64 solve at 128^3 (seed 2, one centred source) to 1e-8:
    true residual recomputed with the oracle's operator"""
    shape = (128, 128, 128)
    prob, lv = _solver(make_media(shape, 2), shape, torch.complex128, levels=3)
    q = point_source(shape)[None]
    u, info, code = prob.solve(torch.from_numpy(q).cuda(), rtol=1e-8, maxit=500)
    assert code == 0
    rel = _oracle_relres(lv, q[0], u.cpu().numpy()[0])
    assert rel <= 1e-8 * (1 + 1e-3)
    prob.close()


def test_batched_sources_160_full_size():
    """32 point sources on 160^3 in one batched mixed-precision solve to
    1e-6: every source's true residual recomputed by the oracle, and each
    agrees with the residual the solve reports"""
    from synthetic import lattice_sources
    shape = (160, 160, 160)
    prob, lv = _solver(make_media(shape, 4), shape, torch.complex64, levels=4)
    q = lattice_sources(shape, 4, 8, depth_index=int(ABL) + 2, margin=int(ABL))
    u, info, code = prob.solve(torch.from_numpy(q).cuda(), rtol=1e-6, maxit=400)
    assert code == 0 and all(i["status"] == 0 for i in info)
    un = u.cpu().numpy()
    prob.close()
    rels = _oracle_relres_many([(lv, q[s], un[s]) for s in range(q.shape[0])])
    for s, rel in enumerate(rels):
        assert rel <= 1e-6 * (1 + 1e-3), (s, rel)
        assert abs(rel - info[s]["relres"]) <= 1e-3 * rel, (s, rel, info[s]["relres"])


def test_uneven_batch_full_size():
    """the 12 uneven problems (64^3 .. 192^3, seeds 100-111) in one batch
    handle, as the benchmark runs them: every problem's true residual
    recomputed by the oracle, and the problems' reported residuals agree
    with them"""
    from paper_2307_03242_amd import Batch
    sizes = [64, 80, 96, 112, 128, 144, 160, 176, 192, 96, 128, 160]
    specs, lvs, qs = [], [], []
    for i, n in enumerate(sizes):
        sh = (n, n, n)
        m = make_media(sh, 100 + i)
        om = omega_for_ppw(m["vs"].min(), 1.0, 10)
        specs.append(dict(lam=torch.from_numpy(m["lam"]), mu=torch.from_numpy(m["mu"]), rho=torch.from_numpy(m["rho"]),
                          h=1.0, omega=om, gamma=0.01, alpha=ALPHA, beta=2 / 3, abl_width=ABL, abl_amp=2.0,
                          levels=4, nu1=1, nu2=1, cycle="K", damping=(0.6, 0.5, 0.4, 0.4), coarse_mode="krylov",
                          coarse_sweeps=1, coarse_restart=5, coarse_maxit=2, coarse_rtol=0.0,
                          precond_dtype=torch.complex64))
        lvs.append(G.Level(sh, 1.0, om, 0.01, 2 / 3, m["lam"], m["mu"], m["rho"], abl_width=ABL, abl_amp=2.0))
        qs.append(torch.from_numpy(point_source(sh)[None]).cuda())
    batch = Batch(specs)
    us, infos, code = batch.solve(qs, rtol=1e-6, maxit=400)
    assert code == 0
    rels = _oracle_relres_many([(lvs[i], qs[i].cpu().numpy()[0], us[i].cpu().numpy()[0]) for i in range(len(sizes))])
    for i, rel in enumerate(rels):
        assert rel <= 1e-6 * (1 + 1e-3), (i, rel)
        assert abs(rel - infos[i][0]["relres"]) <= 1e-3 * rel
    batch.close()


def test_fwi_gradient_128_finite_differences():
    """the FWI-style gradient at 128^3 (true medium seed 500, start = true
    with an 8 % central Gaussian anomaly, 8 sources at depth 18, receivers
    on the plane at depth 18): directional derivatives along 20 smooth
    random directions (seed 502) equal central finite differences to 1e-4.

    Step: the misfit is strongly nonlinear along these directions (a blob of
    the full medium's size per unit step): the central difference's
    O(eps^2) error is 1e-3..2e-3 relative at eps = 1e-4 and grows 100-fold
    per decade of eps, independent of the solve tolerance (1e-12 and 1e-13
    give the same differences).  eps = 5e-6 puts it near 5e-6; the solves'
    misfit noise (2.5e-18 between tolerances 1e-12 and 1e-13, against
    differences of 1e-13 and more) stays below 2e-5."""
    from paper_2307_03242_amd.autograd import misfit
    from synthetic import lattice_sources
    n = 128
    shape = (n, n, n)
    mt = make_media(shape, 500)
    prob, _ = _solver(mt, shape, torch.complex128, levels=3)
    src = torch.from_numpy(lattice_sources(shape, 2, 4, depth_index=18, margin=int(ABL))).cuda()
    mask = torch.zeros((4,) + shape, dtype=torch.bool, device="cuda")
    a = int(ABL)
    mask[:3, 18, a:-a, a:-a] = True
    true = [torch.from_numpy(mt[k]).cuda() for k in ("lam", "mu", "rho")]
    prob.set_media(*true)
    d_obs, _, code = prob.solve(src, rtol=1e-12, maxit=3000)
    assert code == 0
    d_obs = d_obs * mask
    z, y, x = torch.meshgrid(*[torch.arange(n, dtype=torch.float64, device="cuda") + 0.5] * 3, indexing="ij")
    blob = 1.0 - 0.08 * torch.exp(-((z - n / 2) ** 2 + (y - n / 2) ** 2 + (x - n / 2) ** 2) / (2 * 12.0 ** 2))
    base = [t * blob for t in true]
    params = [b.clone().requires_grad_(True) for b in base]
    phi = misfit(prob, *params, src, mask, d_obs, rtol=1e-12, maxit=3000)
    phi.backward()
    grads = [p.grad.clone() for p in params]
    rng = np.random.default_rng(502)
    worst = 0.0
    for trial in range(20):
        dirs = []
        for b in base:
            c = rng.uniform(0.3 * n, 0.7 * n, 3)
            d = torch.exp(-((z - c[0]) ** 2 + (y - c[1]) ** 2 + (x - c[2]) ** 2) / (2 * (n / 10.0) ** 2))
            dirs.append(d * float(rng.uniform(-1, 1)) * float(b.abs().max()))
        eps = 5e-6
        with torch.no_grad():
            pp = misfit(prob, *[b + eps * d for b, d in zip(base, dirs)], src, mask, d_obs, rtol=1e-12, maxit=3000)
            pm = misfit(prob, *[b - eps * d for b, d in zip(base, dirs)], src, mask, d_obs, rtol=1e-12, maxit=3000)
        fd = (pp - pm).item() / (2 * eps)
        an = sum(float((g * d).sum()) for g, d in zip(grads, dirs))
        worst = max(worst, abs(fd - an) / abs(an))
    assert worst <= 1e-4, worst
    prob.close()
