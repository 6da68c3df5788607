"""Inter-grid transfers of the MAC multigrid.

Test infrastructure (see the package header).

Section 2.3, eqs. (pIntergrid) and (u2Intergrid); 3D is their tensor
product extension, which the paper calls straightforward:
  * pressure: restriction = mean of the 2^d child cells, prolongation =
    (bi/tri)linear interpolation with 1D weights (1 3 3 1)/4 (transposed
    stencil);
  * u_k: along x_k (normal direction) full weighting (1/4)[1 2 1] for
    restriction and linear interpolation ]1/2 1 1/2[ for prolongation;
    along the other axes the same pair mean / (1 3 3 1)/4 weights as the
    pressure.
Coarse face J coincides with fine face 2J; coarse cell I covers fine cells
2I, 2I+1.  Values outside the domain (and on boundary faces) are zero.
R is deliberately not a multiple of P^T (Section 3.2).
"""
import numpy as np
import scipy.sparse as sp

from . import grid as G


def fw_face(n):
    """coarse interior faces J=1..n/2-1 <- fine faces 2J-1, 2J, 2J+1."""
    nc = n // 2
    m = sp.lil_matrix((nc - 1, n - 1))
    for J in range(1, nc):
        for f, w in ((2 * J - 1, 0.25), (2 * J, 0.5), (2 * J + 1, 0.25)):
            m[J - 1, f - 1] = w
    return m.tocsr()


def pair_cell(n):
    """coarse cell I <- mean of fine cells 2I, 2I+1."""
    nc = n // 2
    m = sp.lil_matrix((nc, n))
    for I in range(nc):
        m[I, 2 * I] = 0.5
        m[I, 2 * I + 1] = 0.5
    return m.tocsr()


def lin_face(n):
    """fine interior faces f=1..n-1 <- coarse faces (linear interpolation)."""
    nc = n // 2
    m = sp.lil_matrix((n - 1, nc - 1))
    for f in range(1, n):
        if f % 2 == 0:
            J = f // 2
            if 1 <= J <= nc - 1:
                m[f - 1, J - 1] = 1.0
        else:
            for J in ((f - 1) // 2, (f + 1) // 2):
                if 1 <= J <= nc - 1:
                    m[f - 1, J - 1] = 0.5
    return m.tocsr()


def lin_cell(n):
    """fine cells <- coarse cells, weights 3/4 (parent) and 1/4 (the coarse
    neighbour on the same side), zero outside."""
    nc = n // 2
    m = sp.lil_matrix((n, nc))
    for I in range(nc):
        m[2 * I, I] += 0.75
        if I - 1 >= 0:
            m[2 * I, I - 1] += 0.25
        m[2 * I + 1, I] += 0.75
        if I + 1 <= nc - 1:
            m[2 * I + 1, I + 1] += 0.25
    return m.tocsr()


def _field_mats(lv, f, restrict):
    mats = {}
    for a in range(1, lv.dim + 1):
        n = lv.n[a - 1]
        if f == a - 1:
            mats[a] = fw_face(n) if restrict else lin_face(n)
        else:
            mats[a] = pair_cell(n) if restrict else lin_cell(n)
    return mats


def restriction_matrix(lv):
    """Block-diagonal R (fine compact -> coarse compact), sparse."""
    blocks = [G.kron_axes(lv, _field_mats(lv, f, True), {}) for f in range(lv.dim + 1)]
    return sp.block_diag(blocks, format="csr")


def prolongation_matrix(lv):
    """Block-diagonal P (coarse compact -> fine compact), sparse; lv is the
    FINE level."""
    blocks = [G.kron_axes(lv, _field_mats(lv, f, False), {}) for f in range(lv.dim + 1)]
    return sp.block_diag(blocks, format="csr")


def restrict(lv, x, lvc):
    """R x on storage arrays (fine level lv -> coarse level lvc)."""
    comp = G.field_views(lv, G.pack(lv, x))
    out = [G.apply_axes(lv, comp[f], _field_mats(lv, f, True)) for f in range(lv.dim + 1)]
    return G.unpack(lvc, np.concatenate([np.ravel(a) for a in out]))


def prolong(lv, e, lvc):
    """P e on storage arrays (coarse level lvc -> fine level lv)."""
    comp = G.field_views(lvc, G.pack(lvc, e))
    out = [G.apply_axes(lv, comp[f], _field_mats(lv, f, False)) for f in range(lv.dim + 1)]
    return G.unpack(lv, np.concatenate([np.ravel(a) for a in out]))
