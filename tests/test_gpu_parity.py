"""GPU parity: every C-ABI level operation against the CPU oracle.

Inputs come from the seeded generators in `synthetic`; expected values from
`oracle` only.  Float64 tolerances follow the operator's arithmetic
(a few hundred terms of size ~max|y| per output: 1e-12 relative), float32
ones the single-precision unit roundoff times the same term count.
"""
import numpy as np
import pytest
import torch
import scipy.sparse.linalg as spla

from oracle import grid as G
from oracle import operator as O
from oracle import transfer as T
from oracle import cycle as C
from oracle.smoother import Vanka
from synthetic import make_media, random_field, point_source, omega_for_ppw

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 3e-5


def _params(shape, levels=3, alpha=0.3, seed=3, abl=None, coarse="relax", beta=2 / 3):
    m = make_media(shape, seed)
    h = 1.0
    om = omega_for_ppw(m["vs"].min(), h, 10)
    abl_w = abl if abl is not None else 0.25 * min(shape) * h
    return dict(media=m, h=h, omega=om, gamma=0.01, alpha=alpha, beta=beta, abl_width=abl_w,
                abl_amp=2.0, levels=levels, damping=(0.55, 0.35, 0.25), coarse=coarse)


def _gpu_problem(P, shape, coarse_sweeps=2, coarse_maxit=6, precond=torch.complex128, cycle="V"):
    from paper_2307_03242_amd import Problem
    m = P["media"]
    return Problem(torch.from_numpy(m["lam"]), torch.from_numpy(m["mu"]), torch.from_numpy(m["rho"]),
                   h=P["h"], omega=P["omega"], gamma=P["gamma"], alpha=P["alpha"], beta=P["beta"],
                   abl_width=P["abl_width"], abl_amp=P["abl_amp"], levels=P["levels"],
                   damping=P["damping"], coarse_mode=P["coarse"], coarse_sweeps=coarse_sweeps,
                   coarse_restart=5, coarse_maxit=coarse_maxit, coarse_rtol=0.0,
                   precond_dtype=precond, cycle=cycle)


def _oracle_levels(P, shape):
    m = P["media"]
    lv = G.Level(tuple(reversed(shape)), P["h"], P["omega"], P["gamma"], P["beta"], m["lam"], m["mu"],
                 m["rho"], abl_width=P["abl_width"], abl_amp=P["abl_amp"])
    lvs = [lv]
    for _ in range(P["levels"] - 1):
        lvs.append(C.coarsen_level(lvs[-1]))
    return lvs


def _dev(a, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _host(t):
    return t.detach().cpu().to(torch.complex128).numpy()


def _relerr(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def _maxrel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


SHAPES = [(8, 12, 16), (6, 10, 14), (12, 20), (18, 26)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("shifted", [False, True])
@pytest.mark.parametrize("adjoint", [False, True])
def test_apply_f64(shape, shifted, adjoint):
    lvls = 2 if min(shape) % 4 else 3
    P = _params(shape, levels=lvls)
    prob = _gpu_problem(P, shape)
    lvs = _oracle_levels(P, shape)
    for level, lv in enumerate(lvs):
        lshape = lv.np_shape
        x = random_field(lshape, 11 + level, nrhs=2)
        y = _host(prob.apply(_dev(x), level=level, shifted=shifted, adjoint=adjoint))
        ref = O.apply(lv, x, shift=P["alpha"] if shifted else 0.0, adjoint=adjoint)
        assert _maxrel(y, ref) <= TOL64, (level, _maxrel(y, ref))


@pytest.mark.parametrize("shape", [(8, 12, 16), (12, 20)])
def test_apply_f32(shape):
    P = _params(shape, levels=2)
    prob = _gpu_problem(P, shape)
    lv = _oracle_levels(P, shape)[0]
    x = random_field(shape, 5, nrhs=3)
    for shifted in (False, True):
        for adj in (False, True):
            y = _host(prob.apply(_dev(x, torch.complex64), shifted=shifted, adjoint=adj))
            ref = O.apply(lv, x.astype(np.complex64).astype(np.complex128),
                          shift=P["alpha"] if shifted else 0.0, adjoint=adj)
            assert _relerr(y, ref) <= TOL32


@pytest.mark.parametrize("shape", [(8, 12, 16), (12, 20)])
def test_residual(shape):
    P = _params(shape, levels=2)
    prob = _gpu_problem(P, shape)
    lv = _oracle_levels(P, shape)[0]
    x = random_field(shape, 6, nrhs=2)
    b = random_field(shape, 7, nrhs=2)
    r = _host(prob.residual(_dev(b), _dev(x), shifted=True))
    ref = b - O.apply(lv, x, shift=P["alpha"])
    assert _maxrel(r, ref) <= TOL64


@pytest.mark.parametrize("shape", [(8, 12, 16), (12, 20)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_restrict_residual(shape, adjoint):
    P = _params(shape, levels=2)
    prob = _gpu_problem(P, shape)
    lv, lvc = _oracle_levels(P, shape)
    x = random_field(shape, 8, nrhs=2)
    b = random_field(shape, 9, nrhs=2)
    rc = _host(prob.restrict_residual(_dev(b), _dev(x), adjoint=adjoint))
    ref = np.stack([T.restrict(lv, b[s] - O.apply(lv, x[s], shift=P["alpha"], adjoint=adjoint), lvc)
                    for s in range(2)])
    assert _maxrel(rc, ref) <= TOL64
    rc0 = _host(prob.restrict_residual(_dev(b)))
    ref0 = np.stack([T.restrict(lv, b[s], lvc) for s in range(2)])
    assert _maxrel(rc0, ref0) <= 1e-14


@pytest.mark.parametrize("shape", [(8, 12, 16), (6, 10, 14), (12, 20)])
def test_prolong_add(shape):
    P = _params(shape, levels=2)
    prob = _gpu_problem(P, shape)
    lv, lvc = _oracle_levels(P, shape)
    x = random_field(shape, 10, nrhs=2)
    e = random_field(lvc.np_shape, 11, nrhs=2)
    out = _host(prob.prolong_add(_dev(e), _dev(x)))
    ref = np.stack([x[s] + T.prolong(lv, e[s], lvc) for s in range(2)])
    assert _maxrel(out, ref) <= 1e-14


@pytest.mark.parametrize("shape", [(8, 12, 16), (6, 10, 14), (12, 20)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_relax_half_sweep(shape, adjoint):
    P = _params(shape, levels=2)
    prob = _gpu_problem(P, shape)
    lv = _oracle_levels(P, shape)[0]
    A = O.assemble(lv, shift=P["alpha"])
    if adjoint:
        A = A.conj().T.tocsr()
    vk = Vanka(lv, A)
    x = random_field(shape, 12, nrhs=1)[0]
    b = random_field(shape, 13, nrhs=1)[0]
    xg = _dev(x)
    for colour in (0, 1):
        prob.relax(_dev(b), xg, colour, adjoint=adjoint)
        xr = vk.half_sweep(G.pack(lv, x), G.pack(lv, b), P["damping"][0], colour)
        x = G.unpack(lv, xr)
        assert _maxrel(_host(xg), x) <= 1e-12


@pytest.mark.parametrize("coarse", ["relax", "krylov"])
@pytest.mark.parametrize("shape,levels", [((8, 12, 16), 3), ((16, 16, 16), 2), ((24, 32), 3)])
def test_vcycle_f64(shape, levels, coarse):
    P = _params(shape, levels=levels, coarse=coarse)
    prob = _gpu_problem(P, shape, coarse_sweeps=2, coarse_maxit=6)
    lv = _oracle_levels(P, shape)[0]
    cp = C.CycleParams(levels=levels, alpha=P["alpha"], damping=P["damping"], coarse=coarse,
                       coarse_sweeps=2, coarse_restart=5, coarse_maxit=6, coarse_rtol=0.0)
    hier = C.Hierarchy(lv, cp)
    b = random_field(shape, 14, nrhs=2)
    x = _host(prob.vcycle(_dev(b)))
    ref = np.stack([hier.vcycle_storage(b[s]) for s in range(2)])
    assert _relerr(x, ref) <= 1e-11


@pytest.mark.parametrize("coarse", ["krylov", "relax"])
@pytest.mark.parametrize("shape,levels", [((16, 16, 24), 4), ((16, 16, 16), 3), ((32, 48), 3)])
def test_wcycle_f64(shape, levels, coarse):
    """W-cycle: two recursive calls on every level (above the coarsest, two
    coarsest solves, the second on the residual of the first)"""
    P = _params(shape, levels=levels, coarse=coarse)
    prob = _gpu_problem(P, shape, coarse_sweeps=2, coarse_maxit=6, cycle="W")
    lv = _oracle_levels(P, shape)[0]
    cp = C.CycleParams(levels=levels, alpha=P["alpha"], damping=P["damping"], coarse=coarse,
                       coarse_sweeps=2, coarse_restart=5, coarse_maxit=6, coarse_rtol=0.0, calls=2)
    hier = C.Hierarchy(lv, cp)
    b = random_field(shape, 17, nrhs=2)
    x = _host(prob.vcycle(_dev(b)))
    ref = np.stack([hier.vcycle_storage(b[s]) for s in range(2)])
    assert _relerr(x, ref) <= 1e-11


@pytest.mark.parametrize("coarse", ["relax", "krylov"])
@pytest.mark.parametrize("shape,levels", [((8, 12, 16), 3), ((16, 16, 16), 3), ((24, 32), 3)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_kcycle_f64(shape, levels, coarse, adjoint):
    """K-cycle (two flexible-GCR steps per coarse correction, coefficients
    computed on the device) against the oracle's K-cycle"""
    P = _params(shape, levels=levels, coarse=coarse)
    prob = _gpu_problem(P, shape, coarse_sweeps=2, coarse_maxit=6, cycle="K")
    lv = _oracle_levels(P, shape)[0]
    cp = C.CycleParams(levels=levels, alpha=P["alpha"], damping=P["damping"], coarse=coarse,
                       coarse_sweeps=2, coarse_restart=5, coarse_maxit=6, coarse_rtol=0.0, calls=3)
    hier = C.Hierarchy(lv, cp, adjoint=adjoint)
    b = random_field(shape, 18, nrhs=2)
    x = _host(prob.vcycle(_dev(b), adjoint=adjoint))
    ref = np.stack([hier.vcycle_storage(b[s]) for s in range(2)])
    assert _relerr(x, ref) <= 1e-10


@pytest.mark.parametrize("nrhs", [1, 3, 9])
def test_kcycle_reductions_any_batch(nrhs):
    """the K-cycle coefficients and the coarsest GMRES finish reductions of
    at most 16 values inside their bookkeeping kernels and larger ones in a
    separate pass: with 1 right-hand side every reduction takes the first
    path, with 3 both occur (GMRES columns from the third on, the second
    K-cycle stage), with 9 only the second; every column equals the
    oracle's K-cycle"""
    shape = (8, 12, 16)
    P = _params(shape, levels=3, coarse="krylov")
    prob = _gpu_problem(P, shape, coarse_sweeps=2, coarse_maxit=6, cycle="K")
    lv = _oracle_levels(P, shape)[0]
    cp = C.CycleParams(levels=3, alpha=P["alpha"], damping=P["damping"], coarse="krylov", coarse_sweeps=2,
                       coarse_restart=5, coarse_maxit=6, coarse_rtol=0.0, calls=3)
    hier = C.Hierarchy(lv, cp)
    b = random_field(shape, 19, nrhs=nrhs)
    x = _host(prob.vcycle(_dev(b)))
    ref = np.stack([hier.vcycle_storage(b[s]) for s in range(nrhs)])
    assert _relerr(x, ref) <= 1e-10


def test_kcycle_mixed_precision_solve():
    """float32 K-cycle inside float64 FGMRES: converges and agrees with the
    float64 direct solution to 1e-5"""
    shape = (16, 16, 16)
    P = _params(shape, levels=3, coarse="krylov")
    prob = _gpu_problem(P, shape, coarse_sweeps=2, coarse_maxit=6, precond=torch.complex64, cycle="K")
    lv = _oracle_levels(P, shape)[0]
    q = point_source(shape)[None]
    u, info, code = prob.solve(_dev(q), restart=5, maxit=300, rtol=1e-6)
    assert code == 0 and info[0]["relres"] <= 1e-6
    ref = spla.spsolve(O.assemble(lv).tocsc(), G.pack(lv, q[0]))
    err = np.linalg.norm(G.pack(lv, _host(u)[0]) - ref) / np.linalg.norm(ref)
    assert err <= 1e-5


@pytest.mark.parametrize("shape", [(8, 12, 16)])
def test_vcycle_adjoint_f64(shape):
    P = _params(shape, levels=3, coarse="relax")
    prob = _gpu_problem(P, shape)
    lv = _oracle_levels(P, shape)[0]
    cp = C.CycleParams(levels=3, alpha=P["alpha"], damping=P["damping"], coarse="relax", coarse_sweeps=2)
    hier = C.Hierarchy(lv, cp, adjoint=True)
    b = random_field(shape, 15, nrhs=1)
    x = _host(prob.vcycle(_dev(b), adjoint=True))
    assert _relerr(x[0], hier.vcycle_storage(b[0])) <= 1e-11


@pytest.mark.parametrize("shape", [(8, 12, 16)])
def test_vcycle_f32_close_to_f64(shape):
    P = _params(shape, levels=3, coarse="relax")
    prob = _gpu_problem(P, shape)
    lv = _oracle_levels(P, shape)[0]
    hier = C.Hierarchy(lv, C.CycleParams(levels=3, alpha=P["alpha"], damping=P["damping"],
                                         coarse="relax", coarse_sweeps=2))
    b = random_field(shape, 16, nrhs=1)
    x = _host(prob.vcycle(_dev(b, torch.complex64)))
    assert _relerr(x[0], hier.vcycle_storage(b[0])) <= 1e-4


@pytest.mark.parametrize("shape,levels", [((16, 16, 16), 3), ((32, 48), 3)])
def test_solve_f64_matches_direct(shape, levels):
    import scipy.sparse.linalg as spla
    P = _params(shape, levels=levels, coarse="krylov")
    prob = _gpu_problem(P, shape, coarse_sweeps=2, coarse_maxit=10)
    lv = _oracle_levels(P, shape)[0]
    q = point_source(shape)[None]
    u, info, code = prob.solve(_dev(q), restart=5, maxit=300, rtol=1e-10)
    assert code == 0 and info[0]["relres"] <= 1e-10
    ref = spla.spsolve(O.assemble(lv).tocsc(), G.pack(lv, q[0]))
    err = np.linalg.norm(G.pack(lv, _host(u)[0]) - ref) / np.linalg.norm(ref)
    assert err <= 1e-7
    # true residual in float64 through the oracle operator
    res = np.linalg.norm(G.pack(lv, q[0] - O.apply(lv, _host(u)[0]))) / np.linalg.norm(G.pack(lv, q[0]))
    assert res <= 1.5e-10


def test_solve_mixed_precision_matches_f64():
    """float32 cycle inside float64 FGMRES to 1e-6: forward error against
    the float64 direct solution within 1e-5."""
    import scipy.sparse.linalg as spla
    shape = (16, 16, 16)
    P = _params(shape, levels=3, coarse="krylov")
    prob = _gpu_problem(P, shape, coarse_sweeps=2, coarse_maxit=10, precond=torch.complex64)
    lv = _oracle_levels(P, shape)[0]
    q = point_source(shape)[None]
    u, info, code = prob.solve(_dev(q), restart=5, maxit=300, rtol=1e-6)
    assert code == 0 and info[0]["relres"] <= 1e-6
    ref = spla.spsolve(O.assemble(lv).tocsc(), G.pack(lv, q[0]))
    err = np.linalg.norm(G.pack(lv, _host(u)[0]) - ref) / np.linalg.norm(ref)
    assert err <= 1e-5


def test_solve_reports_history_and_time_split():
    """solve stats: one FGMRES residual estimate per iteration (ending at
    the tolerance), and a GPU time split that fits inside the wall time"""
    shape = (16, 16, 16)
    P = _params(shape, levels=3, coarse="krylov")
    prob = _gpu_problem(P, shape, coarse_sweeps=2, coarse_maxit=6, precond=torch.complex64, cycle="K")
    q = np.stack([point_source(shape), random_field(shape, 41)])
    u, info, code = prob.solve(_dev(q), restart=5, maxit=300, rtol=1e-6)
    assert code == 0
    for i in info:
        h = i["history"]
        assert len(h) == i["iters"] and h[-1] <= 1e-6 and all(v >= 0 for v in h)
        assert h[-1] < h[0]
        parts = i["t_precond_ms"] + i["t_apply_ms"] + i["t_orth_ms"]
        assert i["t_precond_ms"] > 0 and i["t_apply_ms"] > 0 and i["t_orth_ms"] > 0
        assert parts <= 1.05 * i["t_total_ms"]


def test_solve_batched_rhs_independent():
    shape = (16, 16, 16)
    P = _params(shape, levels=3, coarse="relax")
    prob = _gpu_problem(P, shape, coarse_sweeps=4)
    q = np.stack([point_source(shape), random_field(shape, 40)])
    ub, infob, _ = prob.solve(_dev(q), rtol=1e-8, maxit=300)
    for s in range(2):
        u1, info1, _ = prob.solve(_dev(q[s:s + 1]), rtol=1e-8, maxit=300)
        assert _relerr(_host(ub)[s], _host(u1)[0]) <= 1e-6
        assert infob[s]["relres"] <= 1e-8


def test_solve_degenerate_right_hand_sides():
    """a zero right-hand side has the zero solution, reported converged with
    no iterations, beside a live one in the same batch; an all-zero batch
    launches no iteration; the largest batch (64 right-hand sides) solves
    every column; one more is rejected before anything runs"""
    from paper_2307_03242_amd._lib import ElhError
    shape = (8, 8, 8)
    P = _params(shape, levels=2, coarse="relax")
    prob = _gpu_problem(P, shape, coarse_sweeps=4)
    q = np.stack([np.zeros((4,) + shape, dtype=np.complex128), point_source(shape)])
    u, info, code = prob.solve(_dev(q), rtol=1e-8, maxit=300)
    uh = _host(u)
    assert code == 0 and info[0]["status"] == 0 and info[0]["iters"] == 0 and info[0]["relres"] == 0.0
    assert np.all(uh[0] == 0)
    assert info[1]["status"] == 0 and info[1]["relres"] <= 1e-8
    u0, info0, code0 = prob.solve(_dev(q[:1]), rtol=1e-8, maxit=300)
    assert code0 == 0 and info0[0]["iters"] == 0 and np.all(_host(u0) == 0)
    q64 = random_field(shape, 50, nrhs=64)
    u64, info64, code64 = prob.solve(_dev(q64), rtol=1e-6, maxit=300)
    assert code64 == 0 and all(i["status"] == 0 and i["relres"] <= 1e-6 for i in info64)
    r = prob.residual(_dev(q64), u64)
    rel = torch.linalg.vector_norm(r.reshape(64, -1), dim=1) / torch.linalg.vector_norm(_dev(q64).reshape(64, -1), dim=1)
    assert float(rel.max()) <= 1e-6 * (1 + 1e-6)
    with pytest.raises(ElhError):
        prob.solve(torch.zeros((65, 4) + shape, dtype=torch.complex128, device="cuda"))


def test_argument_errors_on_gpu():
    shape = (8, 8, 8)
    P = _params(shape, levels=2)
    prob = _gpu_problem(P, shape)
    x = _dev(random_field(shape, 1))
    y = torch.empty_like(x)
    assert prob.lib.elh_apply(prob.handle, 5, 0, 2, 1, x.data_ptr(), y.data_ptr()) == -1
    assert prob.lib.elh_apply(prob.handle, 0, 0, 2, 1, x.data_ptr(), x.data_ptr()) == -1
    with pytest.raises(ValueError):
        prob.apply(_dev(random_field((8, 8, 6), 1)))
    # every extra vector must match x's layout before anything is launched
    with pytest.raises(ValueError):
        prob.apply(x, out=torch.empty(x.numel() // 2, dtype=x.dtype, device=x.device))
    with pytest.raises(ValueError):
        prob.residual(x.to(torch.complex64), x)
    with pytest.raises(ValueError):
        prob.residual(x, x, out=torch.empty_like(x)[..., :4].contiguous())
    with pytest.raises(ValueError):
        prob.relax(x[None].repeat(2, 1, 1, 1, 1).contiguous(), x, 0)
    with pytest.raises(ValueError):
        prob.prolong_add(x, x)  # e on the fine level instead of the coarse one


def test_cycle_right_hand_side_limits():
    """The K-cycle and the Krylov coarsest solve keep per-rhs state for at
    most 64 right-hand sides: 65 are rejected before any launch.  The
    W-cycle's own per-rhs coefficients grow with nrhs: 65 right-hand sides
    with a sweep coarsest solve match the oracle column by column."""
    from paper_2307_03242_amd._lib import ElhError
    shape = (16, 16, 16)
    b65 = random_field(shape, 60, nrhs=65)
    for cyc, coarse in (("K", "relax"), ("W", "krylov"), ("V", "krylov")):
        P = _params(shape, levels=3, coarse=coarse)
        prob = _gpu_problem(P, shape, cycle=cyc)
        with pytest.raises(ElhError) as ei:
            prob.vcycle(_dev(b65))
        assert ei.value.code == -1
    P = _params(shape, levels=3, coarse="relax")
    prob = _gpu_problem(P, shape, coarse_sweeps=2, cycle="W")
    x = _host(prob.vcycle(_dev(b65)))
    cp = C.CycleParams(levels=3, alpha=P["alpha"], damping=P["damping"], coarse="relax", coarse_sweeps=2, calls=2)
    hier = C.Hierarchy(_oracle_levels(P, shape)[0], cp)
    for s in (0, 37, 64):
        assert _relerr(x[s], hier.vcycle_storage(b65[s])) <= 1e-11, s


@pytest.mark.parametrize("precond", [torch.complex128, torch.complex64])
def test_graph_replays_match_eager(precond):
    """The preconditioner cycle (device-resident coarse GMRES) is recorded
    once into a hipGraph and replayed; every replayed solve, with eager work
    and synchronisations in between, equals the eagerly launched solve."""
    import os
    shape = (16, 16, 24)
    P = _params(shape, levels=3, coarse="krylov")
    old = os.environ.get("ELH_GRAPHS")
    os.environ["ELH_GRAPHS"] = "0"
    try:
        eager = _gpu_problem(P, shape, coarse_sweeps=2, coarse_maxit=7, precond=precond)
    finally:
        if old is None:
            del os.environ["ELH_GRAPHS"]
        else:
            os.environ["ELH_GRAPHS"] = old
    graphed = _gpu_problem(P, shape, coarse_sweeps=2, coarse_maxit=7, precond=precond)
    q = _dev(np.stack([point_source(shape), random_field(shape, 41)]))
    ue, infoe, _ = eager.solve(q, rtol=1e-8, maxit=200)
    ue = _host(ue)
    x = _dev(random_field(shape, 42))
    for rep in range(3):
        ug, infog, _ = graphed.solve(q, rtol=1e-8, maxit=200)
        torch.cuda.synchronize()
        assert [i["iters"] for i in infog] == [i["iters"] for i in infoe]
        assert np.array_equal(_host(ug), ue), rep
        graphed.apply(x)            # eager work between replays
        torch.cuda.synchronize()


def test_device_coarse_gmres_matches_oracle_krylov():
    """fixed-budget coarsest solve (device-resident GMRES + Vanka sweeps)
    against the oracle's GMRES with the same budget"""
    shape = (16, 16, 16)
    P = _params(shape, levels=2, coarse="krylov")
    prob = _gpu_problem(P, shape, coarse_sweeps=2, coarse_maxit=12)
    lv = _oracle_levels(P, shape)[0]
    hier = C.Hierarchy(lv, C.CycleParams(levels=2, alpha=P["alpha"], damping=P["damping"], coarse="krylov",
                                         coarse_sweeps=2, coarse_restart=5, coarse_maxit=12, coarse_rtol=0.0))
    lvc = hier.levels[-1]
    b = random_field(lvc.np_shape, 43, nrhs=3)
    x = _host(prob.coarse_solve(_dev(b)))
    ref = np.stack([G.unpack(lvc, hier.coarse_solve(G.pack(lvc, b[s]))) for s in range(3)])
    assert _relerr(x, ref) <= 1e-10


@pytest.mark.parametrize("shape,levels", [((16, 16), 2), ((8, 8, 8), 2), ((16, 24, 32), 3)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_coarse_dense_matches_sparse_lu(shape, levels, adjoint):
    """dense coarsest solve (inverse built on the GPU) equals a sparse LU
    solve of the coarsest shifted operator"""
    P = _params(shape, levels=levels, coarse="dense")
    prob = _gpu_problem(P, shape)
    lvc = _oracle_levels(P, shape)[-1]
    A = O.assemble(lvc, shift=P["alpha"])
    if adjoint:
        A = A.conj().T
    lu = spla.splu(A.tocsc())
    b = random_field(lvc.np_shape, 44, nrhs=2)
    x = _host(prob.coarse_solve(_dev(b), adjoint=adjoint))
    ref = np.stack([G.unpack(lvc, lu.solve(G.pack(lvc, b[s]))) for s in range(2)])
    assert _relerr(x, ref) <= 1e-11


@pytest.mark.parametrize("shape,levels", [((8, 12, 16), 2), ((24, 32), 3)])
def test_vcycle_dense_coarse(shape, levels):
    P = _params(shape, levels=levels, coarse="dense")
    prob = _gpu_problem(P, shape)
    lv = _oracle_levels(P, shape)[0]
    hier = C.Hierarchy(lv, C.CycleParams(levels=levels, alpha=P["alpha"], damping=P["damping"], coarse="direct"))
    b = random_field(shape, 45, nrhs=2)
    x = _host(prob.vcycle(_dev(b)))
    ref = np.stack([hier.vcycle_storage(b[s]) for s in range(2)])
    assert _relerr(x, ref) <= 1e-11


def test_config_2d_64_dense_fp64():
    """2D 64x64, constant media Vp=2, Vs=1, rho=1, 10 points per shear
    wavelength, gamma 0.01, absorbing layer 8 cells, centred point source;
    2 levels, alpha 0.1, dense coarsest solve; float64 FGMRES(5) to 1e-8
    against a sparse direct solve of the whole system"""
    from synthetic import constant_media
    from paper_2307_03242_amd import Problem
    shape = (64, 64)
    m = constant_media(shape, 2.0, 1.0, 1.0)
    om = omega_for_ppw(1.0, 1.0, 10)
    prob = Problem(torch.from_numpy(m["lam"]), torch.from_numpy(m["mu"]), torch.from_numpy(m["rho"]),
                   h=1.0, omega=om, gamma=0.01, alpha=0.1, abl_width=8.0, abl_amp=2.0, levels=2,
                   damping=(0.55,), coarse_mode="dense")
    q = point_source(shape)[None]
    u, info, code = prob.solve(_dev(q), rtol=1e-8, maxit=500)
    assert code == 0 and info[0]["relres"] <= 1e-8
    lv = G.Level((64, 64), 1.0, om, 0.01, 2 / 3, m["lam"], m["mu"], m["rho"], abl_width=8.0, abl_amp=2.0)
    ref = spla.spsolve(O.assemble(lv).tocsc(), G.pack(lv, q[0]))
    err = np.linalg.norm(G.pack(lv, _host(u)[0]) - ref) / np.linalg.norm(ref)
    assert err <= 1e-6
    # same preconditioned iteration in the oracle: counts agree within +-2
    _, oinfo = C.solve(lv, q[0], C.CycleParams(levels=2, alpha=0.1, damping=(0.55,), coarse="direct"),
                       tol=1e-8, maxit=500)
    assert abs(oinfo["iters"] - info[0]["iters"]) <= 2


def test_solve_batch_uneven_grids_equal_single_solves():
    """independent problems of different grid sizes, each on its own stream,
    solved together equal their individual solves exactly"""
    from paper_2307_03242_amd import Problem
    shapes = [(16, 16, 16), (24, 24, 24), (16, 24, 32)]
    probs, qs = [], []
    streams = [torch.cuda.Stream() for _ in shapes]
    for i, (shape, st) in enumerate(zip(shapes, streams)):
        P = _params(shape, levels=3, coarse="krylov", seed=100 + i)
        with torch.cuda.stream(st):
            probs.append(_gpu_problem(P, shape, coarse_sweeps=2, coarse_maxit=4, precond=torch.complex64,
                                      cycle="W"))
        qs.append(_dev(np.stack([point_source(shape)] * (1 + i % 2))))
    torch.cuda.synchronize()
    us, infos, code = Problem.solve_batch(probs, qs, rtol=1e-8, maxit=300)
    assert code == 0
    for p, q, u, info in zip(probs, qs, us, infos):
        u1, info1, _ = p.solve(q, rtol=1e-8, maxit=300)
        torch.cuda.synchronize()
        assert np.array_equal(_host(u), _host(u1))
        assert [i["iters"] for i in info] == [i["iters"] for i in info1]
