"""GPU parity of the marching 3D kernels against the CPU oracle.

The wavefront-march stencil (forward and adjoint, apply and residual, float64
and float32 input), the 19-cell Vanka half-sweep and the fixed-stencil
prolongation take over from the point-wise kernels from 16^3 cells up.  The
shapes here span several 62-lane x_1 segments with a ragged last one,
several x_3 chunks with a ragged last one and two right-hand sides, so every
boundary case of the tiling is exercised.  Expected values come from
`oracle` only.
"""
import numpy as np
import pytest
import torch

from oracle import grid as G
from oracle import operator as O
from oracle import transfer as T
from oracle import cycle as C
from oracle.smoother import Vanka
from synthetic import make_media, random_field, omega_for_ppw

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 3e-5
# (n_3, n_2, n_1): n_1 = 70 and 130 give one and two x_1 segments of 62 lanes and a remainder
# of 8 and 6 cells in 16-lane row groups (n_2 = 9 leaves three rows of the last group empty);
# n_3 = 10, 17 and 18 give ragged x_3 chunks
SHAPES = [(10, 12, 70), (17, 9, 130)]
# x_1 remainders at the edge of the row-group case: 76 = 62 + 14 (the largest
# remainder in 16-lane groups) and 77 = 62 + 15 (one more full segment);
# n_2 = 10 leaves two rows of the last group empty
EDGE_SHAPES = [(6, 10, 76), (6, 10, 77)]
EVEN_SHAPES = [(10, 12, 70), (18, 10, 130)]  # two-level hierarchies


def _setup(shape, seed=5, levels=1, alpha=0.3):
    from paper_2307_03242_amd import Problem
    m = make_media(shape, seed)
    om = omega_for_ppw(m["vs"].min(), 1.0, 10)
    abl = 3.0
    prob = Problem(torch.from_numpy(m["lam"]), torch.from_numpy(m["mu"]), torch.from_numpy(m["rho"]),
                   h=1.0, omega=om, gamma=0.01, alpha=alpha, beta=2 / 3, abl_width=abl, abl_amp=2.0,
                   levels=levels, damping=(0.55, 0.35), coarse_mode="relax", coarse_sweeps=2)
    lv = G.Level(tuple(reversed(shape)), 1.0, om, 0.01, 2 / 3, m["lam"], m["mu"], m["rho"],
                 abl_width=abl, abl_amp=2.0)
    return prob, lv


def _dev(a, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _host(t):
    return t.detach().cpu().to(torch.complex128).numpy()


def _maxrel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("shape", SHAPES + EDGE_SHAPES)
@pytest.mark.parametrize("adjoint", [False, True])
@pytest.mark.parametrize("shifted", [False, True])
def test_marching_apply_and_residual(shape, adjoint, shifted):
    prob, lv = _setup(shape)
    shift = 0.3 if shifted else 0.0
    x = random_field(shape, 11, nrhs=2)
    b = random_field(shape, 12, nrhs=2)
    ref = np.stack([O.apply(lv, x[s], shift=shift, adjoint=adjoint) for s in range(2)])
    y = _host(prob.apply(_dev(x), shifted=shifted, adjoint=adjoint))
    assert _maxrel(y, ref) <= TOL64
    ref32 = np.stack([O.apply(lv, x[s].astype(np.complex64).astype(np.complex128), shift=shift, adjoint=adjoint)
                      for s in range(2)])
    y32 = _host(prob.apply(_dev(x, torch.complex64), shifted=shifted, adjoint=adjoint))
    assert _maxrel(y32, ref32) <= TOL32
    r = _host(prob.residual(_dev(b), _dev(x), shifted=shifted, adjoint=adjoint))
    assert _maxrel(r, b - ref) <= TOL64
    r32 = _host(prob.residual(_dev(b, torch.complex64), _dev(x, torch.complex64), shifted=shifted,
                              adjoint=adjoint))
    assert _maxrel(r32, b - ref) <= TOL32


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("adjoint", [False, True])
def test_marching_relax(shape, adjoint):
    """residual + 19-cell Vanka half-sweeps of both colours on the shifted
    operator, against the oracle's block smoother"""
    prob, lv = _setup(shape)
    A = O.assemble(lv, shift=0.3)
    if adjoint:
        A = A.conj().T.tocsr()
    vk = Vanka(lv, A)
    x = random_field(shape, 21, nrhs=1)[0]
    b = random_field(shape, 22, nrhs=1)[0]
    xg = _dev(x)
    for colour in (0, 1):
        prob.relax(_dev(b), xg, colour, adjoint=adjoint)
        x = G.unpack(lv, vk.half_sweep(G.pack(lv, x), G.pack(lv, b), 0.55, colour))
        assert _maxrel(_host(xg), x) <= 1e-12


@pytest.mark.parametrize("shape", EVEN_SHAPES)
def test_marching_prolong_add(shape):
    prob, lv = _setup(shape, levels=2)
    lvc = C.coarsen_level(lv)
    x = random_field(shape, 31, nrhs=2)
    e = random_field(lvc.np_shape, 32, nrhs=2)
    out = _host(prob.prolong_add(_dev(e), _dev(x)))
    ref = np.stack([x[s] + T.prolong(lv, e[s], lvc) for s in range(2)])
    assert _maxrel(out, ref) <= 1e-14


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_prolong_add_unaligned_output_matches_aligned(dtype):
    """x one element past a pair boundary (a view into a larger buffer): the
    launcher takes the per-cell kernel instead of the pair kernel's wide
    accesses, with the same result"""
    shape = EVEN_SHAPES[0]
    prob, lv = _setup(shape, levels=2)
    lvc = C.coarsen_level(lv)
    x = _dev(random_field(shape, 41, nrhs=1), dtype)
    e = _dev(random_field(lvc.np_shape, 42, nrhs=1), dtype)
    aligned = prob.prolong_add(e, x.clone())
    big = torch.zeros(x.numel() + 1, dtype=dtype, device="cuda")
    xu = big[1:].view(x.shape)
    xu.copy_(x)
    assert xu.data_ptr() % (2 * x.element_size()) != 0
    prob.prolong_add(e, xu)
    tol = 1e-6 if dtype == torch.complex64 else 1e-14
    assert _maxrel(_host(xu), _host(aligned)) <= tol


@pytest.mark.parametrize("shape", EVEN_SHAPES)
def test_marching_vcycle_and_adjoint_vcycle(shape):
    """one V-cycle (and one adjoint V-cycle) built from the marching kernels
    against the oracle's cycle"""
    prob, lv = _setup(shape, levels=2)
    b = random_field(shape, 51, nrhs=1)
    for adjoint in (False, True):
        cp = C.CycleParams(levels=2, alpha=0.3, damping=(0.55, 0.35), coarse="relax", coarse_sweeps=2)
        hier = C.Hierarchy(lv, cp, adjoint=adjoint)
        ref = hier.vcycle_storage(b[0])
        got = _host(prob.vcycle(_dev(b), adjoint=adjoint))[0]
        assert _maxrel(got, ref) <= 1e-11


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("adjoint", [False, True])
def test_outer_operator_on_float32_input(shape, adjoint):
    """the mixed solve's outer operator: complex64 input, float64 arithmetic
    (forward through the march's float32-input variant, adjoint widened)"""
    prob, lv = _setup(shape)
    x = random_field(shape, 61, nrhs=2).astype(np.complex64)
    ref = np.stack([O.apply(lv, x[s].astype(np.complex128), adjoint=adjoint) for s in range(2)])
    y = _host(prob.apply_f32_input(_dev(x, torch.complex64), adjoint=adjoint))
    assert _maxrel(y, ref) <= TOL64


# n_1 = 70, 130 and 62: two, three and two x_1 segments of the 60-lane
# restriction tiles with ragged last ones (62 puts two fine cells in the
# last); n_3 = 10, 18 and 14 give 5, 9 and 7 coarse planes: ragged chunks
RR_SHAPES = [(10, 12, 70), (18, 10, 130), (14, 16, 62)]


@pytest.mark.parametrize("shape", RR_SHAPES)
@pytest.mark.parametrize("adjoint", [False, True])
def test_marching_restrict_residual(shape, adjoint):
    """R (b - H_s x) in one launch (fine residual never stored) against the
    oracle's restriction of its residual, float64 and float32, two
    right-hand sides"""
    prob, lv = _setup(shape, levels=2)
    lvc = C.coarsen_level(lv)
    x = random_field(shape, 71, nrhs=2)
    b = random_field(shape, 72, nrhs=2)
    ref = np.stack([T.restrict(lv, b[s] - O.apply(lv, x[s], shift=0.3, adjoint=adjoint), lvc) for s in range(2)])
    rc = _host(prob.restrict_residual(_dev(b), _dev(x), adjoint=adjoint))
    assert _maxrel(rc, ref) <= TOL64
    x32 = x.astype(np.complex64).astype(np.complex128)
    b32 = b.astype(np.complex64).astype(np.complex128)
    ref32 = np.stack([T.restrict(lv, b32[s] - O.apply(lv, x32[s], shift=0.3, adjoint=adjoint), lvc)
                      for s in range(2)])
    rc32 = _host(prob.restrict_residual(_dev(b, torch.complex64), _dev(x, torch.complex64), adjoint=adjoint))
    assert _maxrel(rc32, ref32) <= TOL32


@pytest.mark.parametrize("adjoint", [False, True])
def test_marching_restrict_residual_chunks_bitwise(adjoint, monkeypatch):
    """every forced x_3 chunk (in coarse planes) gives bitwise the output of
    the default chunk: the chunk only decides which workgroup marches which
    planes"""
    shape = (18, 10, 130)
    x = _dev(random_field(shape, 73, nrhs=2), torch.complex64)
    b = _dev(random_field(shape, 74, nrhs=2), torch.complex64)
    monkeypatch.setenv("ELH_TUNE", "0")
    prob, _ = _setup(shape, levels=2)
    ref = prob.restrict_residual(b, x, adjoint=adjoint)
    for c in (1, 2, 3, 4, 9):
        monkeypatch.setenv("ELH_ZCHUNK", str(-c))
        p2, _ = _setup(shape, levels=2)
        got = p2.restrict_residual(b, x, adjoint=adjoint)
        assert torch.equal(got, ref), c
