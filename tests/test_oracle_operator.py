"""Pins of the oracle's discrete operator against what the paper fixes.

Each test checks the oracle against something other than itself: the
stencils the paper prints (golden fixtures), closed-form Fourier symbols,
the continuum limit, or algebraic identities.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import grid as G
from oracle import operator as O
from oracle import symbols as S
from synthetic import make_media, constant_media, random_field, plane_wave_field
from golden_io import load


def _level(shape, h=0.7, omega=1.3, gamma=0.01, beta=2 / 3, media=None,
           abl=(0.0, 0.0), seed=1):
    m = media or make_media(shape, seed)
    return G.Level(tuple(reversed(shape)), h, omega, gamma, beta,
                   m["lam"], m["mu"], m["rho"], abl_width=abl[0], abl_amp=abl[1])


def _cidx(lv, f, pos):
    """compact index of field f at storage position pos (numpy order)."""
    offs = np.cumsum([0] + lv.field_sizes())
    p = list(pos)
    if f < lv.dim:
        p[lv.axis(f + 1)] -= 1
    return offs[f] + np.ravel_multi_index(tuple(p), lv.field_shape(f))


@pytest.mark.parametrize("shape", [(5, 6), (4, 5, 6)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_matrix_free_equals_assembled(shape, adjoint):
    lv = _level(shape, abl=(1.4, 2.0))
    H = O.assemble(lv, shift=0.3)
    if adjoint:
        H = H.conj().T
    x = random_field(shape, 2)
    y1 = G.unpack(lv, H @ G.pack(lv, x))
    y2 = O.apply(lv, x, shift=0.3, adjoint=adjoint)
    assert np.abs(y1 - y2).max() <= 1e-13 * np.abs(y1).max()


def _u1_stencil_2d(H, lv, i2, i1):
    row = _cidx(lv, 0, (i2, i1))
    st = np.zeros((3, 3), dtype=complex)
    for a, dy in enumerate((1, 0, -1)):
        for b, dx in enumerate((-1, 0, 1)):
            st[a, b] = H[row, _cidx(lv, 0, (i2 + dy, i1 + dx))]
    return st


def test_singer_turkel_stencil_2d():
    """P1: beta = 2/3, mu = rho = 1 reproduces eq. (HO) exactly."""
    gold = load("singer_turkel_HO.txt")
    shape = (8, 8)
    h, om, gam = 0.5, 1.7, 0.2
    med = constant_media(shape, 3.0, 1.0, 1.0)
    H0 = O.assemble(_level(shape, h=h, omega=0.0, gamma=gam, media=med))
    Hw = O.assemble(_level(shape, h=h, omega=om, gamma=gam, media=med))
    lap = _u1_stencil_2d(H0, _level(shape, h=h, media=med), 4, 4) * h * h
    mass = (_u1_stencil_2d(H0, _level(shape, h=h, media=med), 4, 4)
            - _u1_stencil_2d(Hw, _level(shape, h=h, media=med), 4, 4)) / (om ** 2 * (1 - 1j * gam))
    assert np.allclose(lap, gold["laplacian_times_h2"], atol=1e-14, rtol=0)
    assert np.allclose(mass, gold["mass_over_omega2_1mgi"], atol=1e-14, rtol=0)


@pytest.mark.parametrize("beta", [0.3, 0.8])
def test_laplacian_convex_combination_2d(beta):
    """P2: grad^T grad^beta = beta*standard + (1-beta)*skew/2 (eq. LapHO)."""
    gold = load("laplacian_beta_2d.txt")
    shape = (8, 8)
    h = 0.25
    med = constant_media(shape, 3.0, 1.0, 1.0)
    lv = _level(shape, h=h, omega=0.0, beta=beta, media=med)
    lap = _u1_stencil_2d(O.assemble(lv), lv, 3, 4) * h * h
    expect = beta * gold["standard_times_h2"] + (1 - beta) * gold["skew_times_2h2"] / 2
    assert np.allclose(lap, expect, atol=1e-14, rtol=0)


def test_beta_one_is_standard_mac():
    """P3: beta = 1 gives the 5-point Laplacian, the identity mass and the
    two-point divergence/gradient (standard MAC)."""
    gold = load("laplacian_beta_2d.txt")
    shape = (8, 8)
    h, om, gam = 0.5, 1.1, 0.05
    med = constant_media(shape, 3.0, 1.0, 1.0)
    lv0 = _level(shape, h=h, omega=0.0, beta=1.0, media=med)
    lvw = _level(shape, h=h, omega=om, gamma=gam, beta=1.0, media=med)
    H0, Hw = O.assemble(lv0), O.assemble(lvw)
    assert np.allclose(_u1_stencil_2d(H0, lv0, 4, 4) * h * h, gold["standard_times_h2"], atol=1e-14)
    mass = (_u1_stencil_2d(H0, lv0, 4, 4) - _u1_stencil_2d(Hw, lvw, 4, 4)) / (om ** 2 * (1 - 1j * gam))
    ident = np.zeros((3, 3))
    ident[1, 1] = 1
    assert np.allclose(mass, ident, atol=1e-14)
    # p-row: only the cell's own two faces, +-1/h
    prow = _cidx(lv0, 2, (4, 4))
    rowvals = H0[prow].toarray().ravel()
    nz = {int(j): rowvals[j] for j in np.nonzero(rowvals)[0]}
    expect = {_cidx(lv0, 0, (4, 4)): -1 / h, _cidx(lv0, 0, (4, 5)): 1 / h,
              _cidx(lv0, 1, (4, 4)): -1 / h, _cidx(lv0, 1, (5, 4)): 1 / h,
              prow: 1 / 4.0}
    assert set(nz) == set(expect)
    for j, v in expect.items():
        assert abs(nz[j] - v) < 1e-14


def test_spread_derivative_3d_stencil():
    """eq. (dxSkew3D): at beta = 0 the p-row coefficients on u_1 are the
    printed 18-point weights (1/16)[..]/h (with the 1/h of the 2D form)."""
    gold = load("spread_derivative_3d.txt")
    shape = (6, 6, 6)
    h = 0.5
    med = constant_media(shape, 3.0, 1.0, 1.0)
    lv = _level(shape, h=h, omega=0.0, beta=0.0, media=med)
    H = O.assemble(lv)
    c = (3, 3, 3)
    prow = _cidx(lv, 3, c)
    scale = gold["scale"][0, 0]
    for dz, name in ((-1, "slice_x3_m1"), (0, "slice_x3_0"), (1, "slice_x3_p1")):
        for a, dy in enumerate((1, 0, -1)):
            for b, face in enumerate((c[2], c[2] + 1)):
                col = _cidx(lv, 0, (c[0] + dz, c[1] + dy, face))
                assert abs(H[prow, col] - scale * gold[name][a, b] / h) < 1e-14


def test_spread_mass_3d_stencil():
    """eq. (massHO3D): centre beta, six face neighbours (1-beta)/6."""
    gold = load("spread_mass_3d.txt")
    shape = (6, 6, 6)
    beta, om, gam = 0.4, 0.9, 0.1
    med = constant_media(shape, 3.0, 1.0, 1.0)
    lv0 = _level(shape, h=1.0, omega=0.0, beta=beta, media=med)
    lvw = _level(shape, h=1.0, omega=om, gamma=gam, beta=beta, media=med)
    D = (O.assemble(lv0) - O.assemble(lvw)) / (om ** 2 * (1 - 1j * gam))
    row = _cidx(lv0, 1, (3, 3, 3))         # u_2 face
    nb = gold["neighbour_weight"][0, 0] * (1 - beta)
    for off in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        pos = (3 + off[0], 3 + off[1], 3 + off[2])
        assert abs(D[row, _cidx(lv0, 1, pos)] - nb) < 1e-14
    assert abs(D[row, row] - beta) < 1e-14
    assert abs(D[row].toarray()).sum() == pytest.approx(beta + 6 * nb, abs=1e-13)


@pytest.mark.parametrize("shape", [(12, 14), (9, 10, 11)])
@pytest.mark.parametrize("beta", [2 / 3, 1.0, 0.55])
def test_plane_wave_symbol(shape, beta):
    """P4: away from the boundary the operator acts on exp(i theta.x/h) as
    the closed-form symbol matrix."""
    rng = np.random.default_rng(7)
    dim = len(shape)
    h, om, gam = 0.8, 1.2, 0.07
    lam, mu, rho = 4.0, 1.5, 1.3
    lv = _level(shape, h=h, omega=om, gamma=gam, beta=beta,
                media=constant_media(shape, lam, mu, rho))
    for _ in range(3):
        theta = rng.uniform(-np.pi, np.pi, dim)
        amp = rng.standard_normal(dim + 1) + 1j * rng.standard_normal(dim + 1)
        x = plane_wave_field(shape, theta, amp)
        y = O.apply(lv, x, shift=0.0)
        Hs = S.operator_symbol(theta, h, om, gam, beta, lam, mu, rho)
        yhat = Hs @ amp
        phase = plane_wave_field(shape, theta, np.ones(dim + 1))
        inner = tuple(slice(2, s - 2) for s in shape)
        for f in range(dim + 1):
            got = y[f][inner]
            exp = yhat[f] * phase[f][inner]
            assert np.abs(got - exp).max() <= 1e-12 * max(1.0, np.abs(exp).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_schur_symbol_continuum_limit(dim):
    """P6: eliminating p from the symbol gives the (negated) continuum
    elastic operator mu|k|^2 I + (lam+mu) k k^T - rho omega^2 (1-i gamma)
    with a second-order error -- this fixes the sign of the coupling."""
    lam, mu, rho, om, gam = 3.0, 1.2, 1.4, 2.0, 0.05
    kvec = np.array([0.7, -0.4, 0.5][:dim])
    cont = mu * kvec @ kvec * np.eye(dim) + (lam + mu) * np.outer(kvec, kvec) \
        - rho * om ** 2 * (1 - 1j * gam) * np.eye(dim)
    errs = []
    for h in (0.1, 0.05, 0.025):
        Hs = S.operator_symbol(kvec * h, h, om, gam, 2 / 3, lam, mu, rho)
        A, B, C, Dm = Hs[:dim, :dim], Hs[:dim, dim:], Hs[dim:, :dim], Hs[dim:, dim:]
        schur = A - B @ np.linalg.inv(Dm) @ C
        errs.append(np.abs(schur - cont).max())
    assert errs[0] < 0.05 * np.abs(cont).max()
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.5 < e0 / e1 < 4.5


@pytest.mark.parametrize("shape", [(7, 9), (5, 6, 7)])
def test_adjoint_dot_product(shape):
    """P12: <H x, y> = <x, H^H y> with the matrix-free adjoint."""
    lv = _level(shape, abl=(2.0, 2.0))
    x = random_field(shape, 3)
    y = random_field(shape, 4)
    lhs = np.vdot(y, O.apply(lv, x, shift=0.4))
    rhs = np.vdot(O.apply(lv, y, shift=0.4, adjoint=True), x)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_abl_profile_values():
    """absorbing layer: zero in the interior, A at the outer boundary
    along one axis, quadratic in between."""
    lv = _level((20,), h=0.5) if False else _level((10, 20), h=0.5, abl=(2.0, 3.0))
    xs = [np.array([0.0, 1.0, 2.0, 5.0, 9.0, 10.0]), np.array([2.5])]
    g = G.abl_profile(lv, xs)
    assert np.allclose(g.ravel(), [3.0, 3.0 * 0.25, 0.0, 0.0, 3.0 * 0.25, 3.0])


def test_operator_nonsingular_with_shift():
    """with gamma + alpha > 0 the system has a unique solution; a direct
    solve reproduces the right-hand side."""
    lv = _level((6, 6, 6), abl=(2.0, 2.0))
    H = O.assemble(lv, shift=0.2)
    b = G.pack(lv, random_field((6, 6, 6), 5))
    x = spla.spsolve(H.tocsc(), b)
    assert np.linalg.norm(H @ x - b) <= 1e-10 * np.linalg.norm(b)
