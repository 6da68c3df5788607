"""GPU tests of the solve entry points' options and failure paths, through
the C ABI: resuming from an initial guess, the precision of the stored
preconditioned vectors, ELH_NOT_CONVERGED with its iterate and statistics,
and the negative codes (non-finite media, invalid options).

Expected values come from the oracle (true residuals recomputed by its
matrix-free operator) or from the library's own uninterrupted run where the
property is an identity of the algorithm (a resume at a restart boundary
repeats the same float64 operations)."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import grid as G
from oracle import operator as O
from synthetic import make_media, point_source, random_field, omega_for_ppw

pytestmark = pytest.mark.gpu


def _problem(shape, precond=torch.complex128, cycle="K", media=None, levels=3):
    from paper_2307_03242_amd import Problem
    m = media if media is not None else make_media(shape, 7)
    om = omega_for_ppw(make_media(shape, 7)["vs"].min(), 1.0, 10)
    prob = Problem(torch.from_numpy(m["lam"]), torch.from_numpy(m["mu"]), torch.from_numpy(m["rho"]),
                   h=1.0, omega=om, gamma=0.01, alpha=0.4, beta=2 / 3, abl_width=4.0, abl_amp=2.0,
                   levels=levels, damping=(0.6, 0.5, 0.4), coarse_mode="krylov", coarse_sweeps=1,
                   coarse_restart=5, coarse_maxit=4, precond_dtype=precond, cycle=cycle)
    lv = G.Level(tuple(reversed(shape)), 1.0, om, 0.01, 2 / 3, m["lam"], m["mu"], m["rho"],
                 abl_width=4.0, abl_amp=2.0)
    return prob, lv


def _q(shape):
    return torch.from_numpy(np.stack([point_source(shape), random_field(shape, 23)])).cuda()


def _true_relres(lv, q, u):
    qn, un = q.cpu().numpy(), u.cpu().numpy()
    return [np.linalg.norm(G.pack(lv, qn[s] - O.apply(lv, un[s]))) / np.linalg.norm(G.pack(lv, qn[s]))
            for s in range(qn.shape[0])]


@pytest.mark.parametrize("precond", [torch.complex128, torch.complex64])
def test_resume_at_restart_boundary_continues_exactly(precond):
    """k restart cycles, then a resume from the returned iterate, give
    bitwise the solution and iteration count of one uninterrupted solve
    (the resume recomputes the true residual exactly as a restart does)"""
    shape = (16, 16, 24)
    prob, lv = _problem(shape, precond)
    q = _q(shape)
    full, info_f, code_f = prob.solve(q, restart=5, maxit=300, rtol=1e-8)
    assert code_f == 0
    assert all(i["iters"] > 10 for i in info_f)
    part, info_p, code_p = prob.solve(q, restart=5, maxit=10, rtol=1e-8)
    assert code_p == 1
    for i in info_p:
        assert i["status"] == 1 and i["iters"] == 10 and i["restarts"] == 2
    rel = _true_relres(lv, q, part)
    for s, i in enumerate(info_p):
        assert abs(i["relres"] - rel[s]) <= 1e-8 * rel[s]
    res, info_r, code_r = prob.solve(q, restart=5, maxit=300, rtol=1e-8, x0=part)
    assert code_r == 0
    for s in range(2):
        assert info_r[s]["iters"] + 10 == info_f[s]["iters"]
        assert info_r[s]["relres"] == info_f[s]["relres"]
    assert torch.equal(res, full)
    # resuming in place (x0 is the output buffer) gives the same
    part2, _, _ = prob.solve(q, restart=5, maxit=10, rtol=1e-8)
    res2, _, code2 = prob.solve(q, restart=5, maxit=300, rtol=1e-8, x0=part2, out=part2)
    assert code2 == 0 and torch.equal(res2, full)


def test_resume_from_converged_guess_does_nothing():
    """an initial guess that already meets the tolerance returns at once
    with no iteration and its true residual"""
    shape = (16, 16, 16)
    prob, lv = _problem(shape)
    q = _q(shape)
    u, info, code = prob.solve(q, rtol=1e-8, maxit=300)
    u2, info2, code2 = prob.solve(q, rtol=1e-6, maxit=300, x0=u)
    assert code2 == 0 and all(i["iters"] == 0 for i in info2)
    assert torch.equal(u2, u)
    rel = _true_relres(lv, q, u2)
    for s, i in enumerate(info2):
        # a residual 1e-8 below |q| carries ~1e-5 relative cancellation error
        assert i["relres"] <= 1e-8 * (1 + 1e-6) and abs(i["relres"] - rel[s]) <= 1e-3 * rel[s]


def test_store_z_widened_equals_float32_storage():
    """the float32 cycle's output is exact in complex128, so storing z_j
    widened or in complex64 gives the same iterations and solution"""
    shape = (16, 16, 24)
    prob, lv = _problem(shape, torch.complex64)
    q = _q(shape)
    u32, i32, c32 = prob.solve(q, rtol=1e-6, maxit=300, store_z_fp32=True)
    u64, i64, c64 = prob.solve(q, rtol=1e-6, maxit=300, store_z_fp32=False)
    assert c32 == 0 and c64 == 0
    for a, b in zip(i32, i64):
        assert a["iters"] == b["iters"]
    err = float(torch.linalg.vector_norm(u32 - u64) / torch.linalg.vector_norm(u64))
    assert err <= 1e-12
    assert max(_true_relres(lv, q, u64)) <= 1e-6 * (1 + 1e-6)


def test_not_converged_writes_iterate_and_stats():
    """maxit = 1: ELH_NOT_CONVERGED, one iteration, and the returned
    iterate's true residual (recomputed by the oracle) in the stats"""
    shape = (16, 16, 16)
    prob, lv = _problem(shape, torch.complex64)
    q = _q(shape)
    u, info, code = prob.solve(q, rtol=1e-8, maxit=1)
    assert code == 1
    rel = _true_relres(lv, q, u)
    for s, i in enumerate(info):
        assert i["status"] == 1 and i["iters"] == 1 and i["restarts"] == 1 and len(i["history"]) == 1
        assert 0 < i["relres"] < 1 and abs(i["relres"] - rel[s]) <= 1e-8 * rel[s]


def test_non_finite_media_is_a_numeric_error():
    """a NaN in the media makes the first norm non-finite: ELH_ERR_NUMERIC"""
    from paper_2307_03242_amd._lib import ElhError
    shape = (16, 16, 16)
    m = make_media(shape, 7)
    m = {k: v.copy() for k, v in m.items()}
    m["mu"][5, 6, 7] = np.nan
    prob, _ = _problem(shape, media=m)
    with pytest.raises(ElhError) as ei:
        prob.solve(_q(shape), rtol=1e-8, maxit=20)
    assert ei.value.code == -3
    # a non-finite right-hand side is caught before any iteration
    prob2, _ = _problem(shape)
    q = _q(shape)
    q[1, 0, 3, 3, 3] = complex(float("inf"), 0.0)
    with pytest.raises(ElhError) as ei:
        prob2.solve(q, rtol=1e-8, maxit=20)
    assert ei.value.code == -3


def test_solve_rejects_invalid_options():
    """bad options return ELH_ERR_ARG through the C ABI"""
    from paper_2307_03242_amd import _lib as L
    shape = (16, 16, 16)
    prob, _ = _problem(shape)
    q = _q(shape)
    u = torch.empty_like(q)
    lib = prob.lib

    def call(nrhs=2, **kw):
        o = dict(restart=5, maxit=10, rtol=1e-6, zero_x0=1, store_z_fp32=0)
        o.update(kw)
        opts = L.SolveOpts(o["restart"], o["maxit"], o["rtol"], o["zero_x0"], o["store_z_fp32"])
        return lib.elh_solve(prob.handle, nrhs, ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                             ctypes.byref(opts), None)

    assert call(restart=0) == L.ELH_ERR_ARG
    assert call(maxit=0) == L.ELH_ERR_ARG
    assert call(rtol=-1.0) == L.ELH_ERR_ARG
    assert call(zero_x0=2) == L.ELH_ERR_ARG
    assert call(store_z_fp32=1) == L.ELH_ERR_ARG     # float64 cycle
    assert call(nrhs=0) == L.ELH_ERR_ARG
    assert call(nrhs=65) == L.ELH_ERR_ARG
    assert lib.elh_solve(prob.handle, 2, ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(q.data_ptr()),
                         ctypes.byref(L.SolveOpts(5, 10, 1e-6, 1, 0)), None) == L.ELH_ERR_ARG
