"""Pins of the oracle's coarsest-grid solver of Section 3.2 (Schur
complement of the pressure, FGMRES preconditioned by hybrid Kaczmarz
sweeps) against direct solves, the stencil structure and the defining
properties of row projections."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import grid as G
from oracle import operator as O
from oracle import cycle as C
from oracle import kaczmarz as K
from synthetic import make_media, random_field, omega_for_ppw


def _level(shape, seed=1, abl=(0.0, 0.0), omega=0.6):
    m = make_media(shape, seed)
    return G.Level(tuple(reversed(shape)), 1.0, omega, 0.01, 2 / 3,
                   m["lam"], m["mu"], m["rho"], abl_width=abl[0], abl_amp=abl[1])


def _rand(n, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(n) + 1j * r.standard_normal(n)


CASES = [((6, 5, 7), False), ((6, 5, 7), True), ((9, 11), False), ((9, 11), True)]


@pytest.mark.parametrize("shape,adjoint", CASES)
def test_schur_solve_equals_full_solve(shape, adjoint):
    """eliminating p through its diagonal block and back-substituting gives
    the solution of the full system (direct solves on both)"""
    lv = _level(shape, abl=(2.0, 1.5))
    A = O.assemble(lv, shift=0.4)
    if adjoint:
        A = A.conj().T.tocsr()
    b = _rand(A.shape[0], 3)
    x_full = spla.spsolve(A.tocsc(), b)
    S, Aup, Apu, dp = K.schur_blocks(lv, A)
    nu = S.shape[0]
    u = spla.spsolve(S.tocsc(), b[:nu] - Aup @ (b[nu:] / dp))
    p = (b[nu:] - Apu @ u) / dp
    x = np.concatenate([u, p])
    assert np.abs(x - x_full).max() <= 1e-10 * np.abs(x_full).max()


@pytest.mark.parametrize("shape,adjoint", CASES)
def test_pattern_is_the_structure_of_schur(shape, adjoint):
    """S has no entry outside the derived pattern, and on rows away from
    the boundary every pattern entry is a nonzero of S (random media)"""
    lv = _level(shape, seed=4, abl=(2.0, 1.5))
    A = O.assemble(lv, shift=0.4)
    if adjoint:
        A = A.conj().T.tocsr()
    S = K.schur_blocks(lv, A)[0]
    assert K.pattern_check(lv, S, adjoint)
    pat = K.pattern(lv, adjoint)
    full = 27 + 2 * 24 if lv.dim == 3 else 9 + 8
    interior = [i for i in range(S.shape[0]) if len(pat[i]) == full]
    assert len(interior) > 0
    for i in interior:
        a, b = S.indptr[i], S.indptr[i + 1]
        nz = np.sort(S.indices[a:b][S.data[a:b] != 0])
        assert np.array_equal(nz, pat[i])


def test_regions_partition_the_rows():
    lv = _level((6, 5, 7))
    nu = sum(lv.field_sizes()[:3])
    for box in (2, 3, 4, 8):
        regs = K.regions(lv, box)
        allr = np.sort(np.concatenate(regs))
        assert np.array_equal(allr, np.arange(nu))
        assert all(np.all(np.diff(r) > 0) for r in regs)


def _small_system(shape=(4, 5, 4), adjoint=False, seed=2):
    lv = _level(shape, seed=seed, abl=(1.0, 1.0))
    A = O.assemble(lv, shift=0.5)
    if adjoint:
        A = A.conj().T.tocsr()
    S = K.schur_blocks(lv, A)[0]
    return lv, S


@pytest.mark.parametrize("adjoint", [False, True])
def test_single_region_projection_zeroes_last_row(adjoint):
    """one region, w = 1: after the pass the last (nonzero) row's equation
    holds exactly, the defining property of a Kaczmarz projection"""
    lv, S = _small_system(adjoint=adjoint)
    kz = K.HybridKaczmarz(lv, S, box=64, omega=1.0, adjoint=adjoint)
    assert len(kz.regions) == 1
    b = _rand(S.shape[0], 5)
    x = kz.sweep(_rand(S.shape[0], 6), b)
    last = max(i for i in range(S.shape[0]) if kz.rowdata[i][2] > 0)
    r = b - S @ x
    assert abs(r[last]) <= 1e-12 * np.abs(b).max()
    assert abs(r[last - 1]) > 1e-6  # earlier rows are disturbed by later ones


@pytest.mark.parametrize("omega", [0.5, 1.0, 1.5])
def test_single_region_sweep_does_not_increase_error(omega):
    """a relaxed projection onto a hyperplane through the solution is
    non-expansive for 0 < w < 2; one pass is a chain of them"""
    lv, S = _small_system()
    kz = K.HybridKaczmarz(lv, S, box=64, omega=omega)
    b = _rand(S.shape[0], 7)
    xs = spla.spsolve(S.tocsc(), b)
    x = _rand(S.shape[0], 8)
    e0 = np.linalg.norm(x - xs)
    for _ in range(5):
        x = kz.sweep(x, b)
        e1 = np.linalg.norm(x - xs)
        assert e1 < e0
        e0 = e1


@pytest.mark.parametrize("box", [2, 3])
@pytest.mark.parametrize("adjoint", [False, True])
def test_solution_is_a_fixed_point_of_the_hybrid_sweep(box, adjoint):
    """every row equation holds at the solution, so every region's copy
    stays there and the component average returns it"""
    lv, S = _small_system(shape=(6, 4, 5), adjoint=adjoint)
    kz = K.HybridKaczmarz(lv, S, box=box, omega=0.8, adjoint=adjoint)
    assert len(kz.regions) > 4
    assert kz.counts.max() > 1  # regions share unknowns
    b = _rand(S.shape[0], 9)
    xs = spla.spsolve(S.tocsc(), b)
    x = kz.sweep(xs, b)
    assert np.abs(x - xs).max() <= 1e-10 * np.abs(xs).max()


def test_hybrid_sweeps_converge_on_a_consistent_system():
    """component-averaged projections converge for 0 < w < 2 on a
    consistent system; many regions, the paper's w = 0.8"""
    lv, S = _small_system(shape=(4, 4, 4))
    kz = K.HybridKaczmarz(lv, S, box=2, omega=0.8)
    b = _rand(S.shape[0], 10)
    xs = spla.spsolve(S.tocsc(), b)
    x = np.zeros_like(b)
    errs = []
    for _ in range(300):
        x = kz.sweep(x, b)
        errs.append(np.linalg.norm(x - xs))
    assert errs[-1] < 0.1 * errs[0]
    assert all(e1 <= e0 * (1 + 1e-12) for e0, e1 in zip(errs[::20], errs[20::20]))


@pytest.mark.parametrize("adjoint", [False, True])
def test_schur_kaczmarz_solver(adjoint):
    """the coarsest-grid solver: p rows hold exactly, the displacement
    residual drops by the requested factor within the sweep budget"""
    lv = _level((6, 6, 6), abl=(1.5, 1.5))
    A = O.assemble(lv, shift=0.5)
    if adjoint:
        A = A.conj().T.tocsr()
    sol = K.SchurKaczmarzSolver(lv, A, box=2, omega=0.8, sweeps=10, restart=5, rtol=0.1, maxit=25,
                                adjoint=adjoint)
    b = _rand(A.shape[0], 11)
    x = sol.solve(b)
    nu = sol.nu
    r = b - A @ x
    assert np.abs(r[nu:]).max() <= 1e-12 * np.abs(b).max()
    bs = sol.schur_rhs(b)
    assert np.linalg.norm(r[:nu]) <= 0.1 * np.linalg.norm(bs) * (1 + 1e-9)
    assert sol.last_info["iters"] <= 25


def test_cycle_with_kaczmarz_coarse_solve_converges():
    """a three-level K-cycle whose coarsest solve is the paper's solver
    preconditions FGMRES to 1e-6 on a 3D problem"""
    shape = (16, 16, 16)
    m = make_media(shape, 3)
    om = omega_for_ppw(m["vs"].min(), 1.0, 10)
    lv = G.Level(tuple(reversed(shape)), 1.0, om, 0.01, 2 / 3, m["lam"], m["mu"], m["rho"],
                 abl_width=3.0, abl_amp=2.0)
    cp = C.CycleParams(levels=3, alpha=0.5, damping=(0.6, 0.5, 0.4), coarse="kaczmarz",
                       coarse_sweeps=10, coarse_restart=5, coarse_maxit=25, coarse_rtol=0.1,
                       calls=3, kacz_box=2)
    assert cp.wc() == 0.8
    q = random_field(shape, 12, nrhs=1)[0]
    x, info = C.solve(lv, q, cp, tol=1e-6, restart=5, maxit=60)
    A = O.assemble(lv)
    assert info["converged"]
    qc = G.pack(lv, q)
    assert np.linalg.norm(qc - A @ G.pack(lv, x)) <= 1e-6 * np.linalg.norm(qc) * (1 + 1e-9)
