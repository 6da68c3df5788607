"""GPU parity of the adjoint-state parameter gradient (elh_gradient and the
autograd wrapper) against the oracle and against finite differences."""
import numpy as np
import pytest
import torch
import scipy.sparse.linalg as spla

from oracle import grid as G
from oracle import operator as O
from oracle import adjoint as AD
from synthetic import make_media, random_field, point_source, omega_for_ppw, lattice_sources

pytestmark = pytest.mark.gpu


def _problem(m, shape, **kw):
    from paper_2307_03242_amd import Problem
    args = dict(h=1.0, omega=omega_for_ppw(m["vs"].min(), 1.0, 10), gamma=0.01, alpha=0.5,
                abl_width=0.25 * min(shape), abl_amp=2.0, levels=3, cycle="W",
                damping=(0.55, 0.35, 0.25), coarse_mode="krylov", coarse_sweeps=2, coarse_maxit=6)
    args.update(kw)
    return Problem(torch.from_numpy(m["lam"]), torch.from_numpy(m["mu"]), torch.from_numpy(m["rho"]), **args), args


def _level(m, shape, args):
    return G.Level(tuple(reversed(shape)), args["h"], args["omega"], args["gamma"], 2 / 3,
                   m["lam"], m["mu"], m["rho"], abl_width=args["abl_width"], abl_amp=args["abl_amp"])


@pytest.mark.parametrize("shape", [(8, 12, 16), (12, 20)])
def test_gradient_kernel_matches_oracle(shape):
    m = make_media(shape, 21)
    prob, args = _problem(m, shape, levels=2)
    lv = _level(m, shape, args)
    u = random_field(shape, 1, nrhs=3)
    v = random_field(shape, 2, nrhs=3)
    g = prob.gradient(torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda())
    ref = AD.gradient(lv, u, v)
    for a, b in zip(g, ref):
        a = a.cpu().numpy()
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_autograd_gradient_matches_oracle_direct():
    """misfit gradient through ElasticFWI (GPU solves to 1e-12) vs the
    oracle adjoint state with sparse direct solves"""
    from paper_2307_03242_amd.autograd import misfit
    shape = (16, 16, 16)
    mt = make_media(shape, 500)
    m0 = make_media(shape, 501)
    prob, args = _problem(m0, shape)
    q = lattice_sources(shape, 1, 2, depth_index=5)
    mask = np.zeros((4,) + shape, dtype=bool)
    mask[:3, 5, 2:-2, 2:-2] = True
    lvt = _level(mt, shape, args)
    At = O.assemble(lvt).tocsc()
    d_obs = np.stack([G.unpack(lvt, spla.spsolve(At, G.pack(lvt, qs))) for qs in q])
    lam, mu, rho = [torch.from_numpy(m0[k]).cuda().requires_grad_(True) for k in ("lam", "mu", "rho")]
    qd = torch.from_numpy(q).cuda()
    md = torch.from_numpy(mask).cuda()
    dd = torch.from_numpy(d_obs).cuda()
    phi = misfit(prob, lam, mu, rho, qd, md, dd, rtol=1e-12, maxit=2000)
    phi.backward()
    lv0 = _level(m0, shape, args)
    A0 = O.assemble(lv0).tocsc()
    u = np.stack([G.unpack(lv0, spla.spsolve(A0, G.pack(lv0, qs))) for qs in q])
    adj = AD.adjoint_source(u, d_obs, mask)
    v = np.stack([G.unpack(lv0, spla.spsolve(A0.conj().T.tocsc(), G.pack(lv0, r))) for r in adj])
    ref = AD.gradient(lv0, u, v)
    assert abs(phi.item() - AD.misfit(u, d_obs, mask)) <= 1e-9 * AD.misfit(u, d_obs, mask)
    for t, r in zip((lam.grad, mu.grad, rho.grad), ref):
        t = t.cpu().numpy()
        assert np.linalg.norm(t - r) <= 1e-6 * np.linalg.norm(r)


def test_autograd_gradient_finite_differences():
    """directional derivative of the misfit along smooth random directions
    equals central finite differences (relative error 1e-4)"""
    from paper_2307_03242_amd.autograd import misfit
    shape = (16, 16, 16)
    mt = make_media(shape, 500)
    m0 = make_media(shape, 501)
    prob, args = _problem(m0, shape)
    q = lattice_sources(shape, 1, 2, depth_index=5)
    mask = np.zeros((4,) + shape, dtype=bool)
    mask[:3, 5, 2:-2, 2:-2] = True
    lvt = _level(mt, shape, args)
    At = O.assemble(lvt).tocsc()
    d_obs = torch.from_numpy(np.stack([G.unpack(lvt, spla.spsolve(At, G.pack(lvt, qs))) for qs in q])).cuda()
    qd = torch.from_numpy(q).cuda()
    md = torch.from_numpy(mask).cuda()
    base = [torch.from_numpy(m0[k]).cuda() for k in ("lam", "mu", "rho")]
    params = [b.clone().requires_grad_(True) for b in base]
    phi = misfit(prob, *params, qd, md, d_obs, rtol=1e-12, maxit=2000)
    phi.backward()
    grads = [p.grad.clone() for p in params]
    rng = np.random.default_rng(502)
    z, y, x = np.meshgrid(*[np.arange(s) + 0.5 for s in shape], indexing="ij")
    for trial in range(3):
        dirs = []
        for b in base:
            c = rng.uniform(4, 12, 3)
            blob = np.exp(-((z - c[0]) ** 2 + (y - c[1]) ** 2 + (x - c[2]) ** 2) / (2 * 3.0 ** 2))
            dirs.append(torch.from_numpy(blob * rng.uniform(-1, 1)).cuda())
        eps = 1e-4 * min(float(b.abs().max()) for b in base) / max(float(d.abs().max()) for d in dirs)
        with torch.no_grad():
            pp = misfit(prob, *[b + eps * d for b, d in zip(base, dirs)], qd, md, d_obs, rtol=1e-12, maxit=2000)
            pm = misfit(prob, *[b - eps * d for b, d in zip(base, dirs)], qd, md, d_obs, rtol=1e-12, maxit=2000)
        fd = (pp - pm).item() / (2 * eps)
        an = sum(float((g * d).sum()) for g, d in zip(grads, dirs))
        assert abs(fd - an) <= 1e-4 * abs(an), (trial, fd, an)
