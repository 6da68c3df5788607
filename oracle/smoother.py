"""Cell-wise Vanka relaxation.

Test infrastructure (see the package header).

Section 2.3 (Vanka box smoother, Figure 1b) and Section 3.2: every cell's
degrees of freedom -- the 2d faces of the cell that are unknowns (boundary
faces are not) and the cell's pressure -- are relaxed together by solving
with the submatrix of the operator on those DOFs ("full Vanka"), or with
the displacement part replaced by its diagonal ("economic Vanka"); the
correction is damped by w.

Orderings:
  * red-black (the parallel smoother used for the solver results):
    colour of cell (i_1..i_d) = (sum i_k) mod 2.  Reading of "red-black
    order": for one colour, the residual b - A x is formed once, every cell
    of that colour solves its block with it, and all corrections are added
    (cells of one colour share no DOF); red (colour 0) then black.
  * lexicographic (used for the paper's LFA comparison): cells in C order
    (x_1 fastest), each cell uses the current residual (Gauss-Seidel).
One "sweep" = both colours (red-black) or all cells (lexicographic).
"""
import numpy as np

from . import grid as G


def cell_dofs(lv):
    """(ncells, 2d+1) compact indices of each cell's DOFs in the order
    [u_1 left, u_1 right, ..., u_d left, u_d right, p]; -1 = not an unknown.
    Cells are listed in C order of the cell grid (x_1 fastest)."""
    d = lv.dim
    cshape = lv.np_shape
    idx = np.indices(cshape).reshape(d, -1)          # numpy-axis order
    ncell = idx.shape[1]
    out = -np.ones((ncell, 2 * d + 1), dtype=np.int64)
    offs = np.cumsum([0] + lv.field_sizes())
    for k in range(1, d + 1):
        ax = lv.axis(k)
        fshape = lv.field_shape(k - 1)
        ik = idx[ax]
        for side, face in ((0, ik), (1, ik + 1)):
            valid = (face >= 1) & (face <= lv.n[k - 1] - 1)
            pos = idx.copy()
            pos[ax] = np.where(valid, face - 1, 0)
            lin = np.ravel_multi_index(tuple(pos), fshape)
            out[:, 2 * (k - 1) + side] = np.where(valid, offs[k - 1] + lin, -1)
    out[:, 2 * d] = offs[d] + np.arange(ncell)
    return out


def cell_colours(lv):
    idx = np.indices(lv.np_shape).reshape(lv.dim, -1)
    return idx.sum(axis=0) % 2


def cell_blocks(A, dofs, economic=False):
    """Dense (ncells, m, m) submatrices of sparse A on each cell's DOFs;
    missing DOFs get an identity row/column (their correction is zero)."""
    nc, m = dofs.shape
    valid = dofs >= 0
    safe = np.where(valid, dofs, 0)
    rows = np.repeat(safe[:, :, None], m, axis=2)
    cols = np.repeat(safe[:, None, :], m, axis=1)
    vals = np.asarray(A[rows.ravel(), cols.ravel()]).reshape(nc, m, m)
    both = valid[:, :, None] & valid[:, None, :]
    vals = np.where(both, vals, 0.0)
    if economic:
        d = (m - 1) // 2
        for i in range(2 * d):
            for j in range(2 * d):
                if i != j:
                    vals[:, i, j] = 0.0
    eye = np.eye(m)[None]
    vals = vals + np.where(~valid[:, :, None], eye, 0.0)
    return vals


class Vanka:
    """Vanka relaxation for a sparse operator A (compact layout)."""

    def __init__(self, lv, A, economic=False):
        self.lv = lv
        self.A = A.tocsr()
        self.dofs = cell_dofs(lv)
        self.colour = cell_colours(lv)
        self.blocks = cell_blocks(self.A, self.dofs, economic)
        self.inv = np.linalg.inv(self.blocks)

    def half_sweep(self, x, b, w, colour):
        """one colour of red-black Vanka (compact vectors); returns new x."""
        sel = self.colour == colour
        r = b - self.A @ x
        dofs = self.dofs[sel]
        valid = dofs >= 0
        rc = np.where(valid, r[np.where(valid, dofs, 0)], 0.0)
        delta = np.einsum("cij,cj->ci", self.inv[sel], rc)
        x = x.copy()
        np.add.at(x, dofs[valid], w * delta[valid])
        return x

    def sweep_rb(self, x, b, w):
        x = self.half_sweep(x, b, w, 0)
        return self.half_sweep(x, b, w, 1)

    def sweep_lex(self, x, b, w):
        """lexicographic (Gauss-Seidel over cells) sweep."""
        x = x.copy()
        A = self.A
        for c in range(self.dofs.shape[0]):
            dofs = self.dofs[c]
            valid = dofs >= 0
            dv = dofs[valid]
            rc = np.zeros(dofs.shape[0], dtype=np.complex128)
            rc[valid] = b[dv] - A[dv] @ x
            delta = self.inv[c] @ rc
            x[dv] += w * delta[valid]
        return x
