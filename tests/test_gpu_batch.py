"""Batching forms through the C ABI: the uneven-grid batch handle
(elh_batch_*) solving problems of different sizes side by side, and
right-hand sides that converge at different restarts (they leave the packed
batch).  Expected values: the oracle's true residuals, and the same solves
run one at a time (a problem of a batch runs the same kernels in the same
order on its own stream as a single solve, so its iterates are bitwise the
same)."""
import numpy as np
import pytest
import torch

from oracle import grid as G
from oracle import operator as O
from synthetic import make_media, point_source, random_field, omega_for_ppw

pytestmark = pytest.mark.gpu


def _cfg(shape, seed, precond=torch.complex64, levels=3):
    m = make_media(shape, seed)
    om = omega_for_ppw(m["vs"].min(), 1.0, 10)
    kw = dict(h=1.0, omega=om, gamma=0.01, alpha=0.4, beta=2 / 3, abl_width=4.0, abl_amp=2.0, levels=levels,
              damping=(0.6, 0.5, 0.4), cycle="K", coarse_mode="krylov", coarse_sweeps=1, coarse_restart=5,
              coarse_maxit=4, precond_dtype=precond)
    lv = G.Level(tuple(reversed(shape)), 1.0, om, 0.01, 2 / 3, m["lam"], m["mu"], m["rho"],
                 abl_width=4.0, abl_amp=2.0)
    return m, kw, lv


def _relres(lv, q, u):
    qn, un = q.cpu().numpy(), u.cpu().numpy()
    return [np.linalg.norm(G.pack(lv, qn[s] - O.apply(lv, un[s]))) / np.linalg.norm(G.pack(lv, qn[s]))
            for s in range(qn.shape[0])]


SHAPES = [(16, 16, 16), (24, 16, 32), (16, 32, 24), (32, 32)]


def test_batch_handle_uneven_grids():
    """four problems of different sizes (one 2D) in one batch handle: each
    solution equals the single solve bitwise and meets the tolerance by the
    oracle's true residual; problem views work with the other entry points"""
    from paper_2307_03242_amd import Batch, Problem
    probs, singles, lvs, qs = [], [], [], []
    for i, shp in enumerate(SHAPES):
        m, kw, lv = _cfg(shp, 20 + i, levels=3 if len(shp) == 3 else 2)
        med = {k: torch.from_numpy(m[k]) for k in ("lam", "mu", "rho")}
        probs.append(dict(med, **kw))
        singles.append(Problem(med["lam"], med["mu"], med["rho"], **kw))
        lvs.append(lv)
        nr = 2 if i % 2 == 0 else 1
        q = np.stack([point_source(shp), random_field(shp, 30 + i)])[:nr]
        qs.append(torch.from_numpy(q).cuda())
    batch = Batch(probs)
    assert len(batch) == len(SHAPES)
    us, infos, code = batch.solve(qs, rtol=1e-7, maxit=300)
    assert code == 0
    for i in range(len(SHAPES)):
        u1, info1, c1 = singles[i].solve(qs[i], rtol=1e-7, maxit=300)
        assert c1 == 0
        assert torch.equal(us[i], u1), i
        assert [x["iters"] for x in infos[i]] == [x["iters"] for x in info1]
        for s, r in enumerate(_relres(lvs[i], qs[i], us[i])):
            assert r <= 1e-7 * (1 + 1e-6), (i, s, r)
            assert abs(r - infos[i][s]["relres"]) <= 1e-6 * r
    # a problem view drives the other entry points on the batch's handle
    y = batch.problem(1).apply(us[1])
    ref = np.stack([O.apply(lvs[1], u) for u in us[1].cpu().numpy()])
    assert np.abs(y.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    batch.close()


def test_batch_handle_rejects_a_bad_problem():
    from paper_2307_03242_amd import Batch
    from paper_2307_03242_amd._lib import ElhError
    m, kw, _ = _cfg((16, 16, 16), 3)
    med = {k: torch.from_numpy(m[k]) for k in ("lam", "mu", "rho")}
    bad = dict(kw, levels=6)  # 16 not divisible by 2^5
    with pytest.raises(ElhError) as ei:
        Batch([dict(med, **kw), dict(med, **bad)])
    assert ei.value.code == -1 and "problem 1" in str(ei.value)


@pytest.mark.parametrize("precond", [torch.complex128, torch.complex64])
def test_converged_rhs_leave_the_batch(precond):
    """right-hand sides that converge at different restarts: the ones left
    are packed and solved on (compaction); each solution meets the tolerance
    by the oracle's true residual and agrees with its single solve"""
    from paper_2307_03242_amd import Problem
    shape = (16, 16, 24)
    m, kw, lv = _cfg(shape, 9, precond=precond)
    prob = Problem(torch.from_numpy(m["lam"]), torch.from_numpy(m["mu"]), torch.from_numpy(m["rho"]), **kw)
    q = np.stack([point_source(shape), random_field(shape, 41), 1e-3 * point_source(shape)
                  + random_field(shape, 42), random_field(shape, 43)])
    qd = torch.from_numpy(q).cuda()
    # rhs 2 starts from a guess close to its solution: it converges in the
    # first restart and leaves the others
    u2, _, _ = prob.solve(qd[2:3].contiguous(), rtol=1e-4, maxit=300)
    x0 = torch.zeros_like(qd)
    x0[2] = u2[0]
    u, info, code = prob.solve(qd, rtol=1e-8, maxit=400, x0=x0)
    assert code == 0
    its = [i["iters"] for i in info]
    assert its[2] < min(its[0], its[1], its[3]) and info[2]["restarts"] < info[0]["restarts"]
    for s, r in enumerate(_relres(lv, qd, u)):
        assert r <= 1e-8 * (1 + 1e-6), (s, r)
    for s in (0, 1, 3):
        us, infos, _ = prob.solve(qd[s:s + 1].contiguous(), rtol=1e-8, maxit=400)
        err = float(torch.linalg.vector_norm(us[0] - u[s]) / torch.linalg.vector_norm(us[0]))
        assert err <= 1e-6, (s, err)
