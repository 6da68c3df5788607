"""The paper's coarsest-grid solver: FGMRES on the Schur complement of the
pressure, preconditioned by parallel hybrid Kaczmarz sweeps.

Test infrastructure (see the package header).

Section 3.2 ("Coarsest grid solution") and the 3D experiments of Section
5.3:
  * the pressure is eliminated through the diagonal p-p block, which leaves
    a system in the displacements only (the Schur complement
        S = A_uu - A_up diag(A_pp)^-1 A_pu,
    right-hand side b_u - A_up diag(A_pp)^-1 b_p, and p recovered as
    diag(A_pp)^-1 (b_p - A_pu u) afterwards);
  * that system is solved by restarted FGMRES(5) until the residual has
    dropped by a factor 10, with at most 250 Kaczmarz sweeps in all;
  * each preconditioner application is 10 hybrid Kaczmarz sweeps from a
    zero initial guess with relaxation 0.8.

Readings (the paper names the method and cites the component-averaging
row-projection methods of Gordon & Gordon, but gives no formula):
  * sub-regions are boxes of `box`^d cells; a displacement unknown belongs
    to the box that holds its storage index (face index along its own
    axis, cell index along the others);
  * one hybrid sweep: every sub-region starts from the same iterate, makes
    one forward Kaczmarz pass over its own rows in ascending global order
        x <- x + w (b_i - a_i x) / ||a_i||^2 conj(a_i)
    (rows with a_i = 0 are skipped), and the new iterate takes, for each
    unknown, the mean of the copies of the sub-regions whose rows reach it
    (component averaging); an unknown reached by no row keeps its value;
  * "reaches" is structural: row i reaches the columns of its stencil
    pattern (below), whatever the numerical values;
  * the sub-regions are many small boxes (the paper used 8, one per CPU
    core), so that a GPU can run one per wavefront.

Stencil pattern of S (derived from the operator's structure, Section 3.1
and its 3D form in Section 5.3): the u-u block couples u_k only with itself
within one cell in every direction; A_up couples the face of u_k with the
two cells beside it; A_pu couples a cell with the faces of every component
within one cell of it (the spread divergence).  Hence the row of u_k at
storage index c reaches
  * u_k at c + o, o in {-1, 0, 1}^d;
  * u_l (l != k) at c + o with o_l in {0, 1}, o_k in {-2, -1, 0, 1} and
    o_m in {-1, 0, 1} on the remaining axis;
and for the conjugate-transposed operator (adjoint solves) the row of u_k
reaches u_l at c - o for every o in the pattern of the row of u_l towards
u_k.  `pattern_check` pins that S has no entry outside this set.
"""
import itertools

import numpy as np
import scipy.sparse as sp

from . import grid as G
from .krylov import fgmres


# ----------------------------------------------------------------------------
# Schur complement of the pressure
# ----------------------------------------------------------------------------
def schur_blocks(lv, A):
    """(S, A_up, A_pu, diag(A_pp)) of the compact operator A (CSR)."""
    nu = int(sum(lv.field_sizes()[:lv.dim]))
    A = A.tocsr()
    Auu, Aup = A[:nu, :nu], A[:nu, nu:]
    Apu, App = A[nu:, :nu], A[nu:, nu:].tocsr()
    dp = App.diagonal()
    off = (App - sp.diags(dp)).tocsr()
    off.eliminate_zeros()
    if off.nnz:
        raise ValueError("p-p block is not diagonal")
    if np.any(dp == 0):
        raise ValueError("zero on the p-p diagonal")
    S = (Auu - Aup @ sp.diags(1.0 / dp) @ Apu).tocsr()
    return S, Aup.tocsr(), Apu.tocsr(), dp


# ----------------------------------------------------------------------------
# unknown geometry: storage coordinates and the row pattern
# ----------------------------------------------------------------------------
def _coords(lv, f):
    """x-order storage coordinates (d, count) of the compact unknowns of
    displacement field f (0-based)."""
    idx = np.indices(lv.field_shape(f)).reshape(lv.dim, -1)
    c = idx[::-1].copy()
    c[f] += 1  # faces 1..n_k-1 along x_k
    return c


def _offsets(dim, k, l, adjoint):
    """pattern offsets (x-order tuples) from a row of u_k to u_l."""
    def fwd(k, l):
        out = []
        rng = []
        for a in range(dim):
            if k == l:
                rng.append((-1, 0, 1))
            elif a == l:
                rng.append((0, 1))
            elif a == k:
                rng.append((-2, -1, 0, 1))
            else:
                rng.append((-1, 0, 1))
        for o in itertools.product(*rng):
            out.append(tuple(o))
        return out
    if not adjoint:
        return fwd(k, l)
    return [tuple(-v for v in o) for o in fwd(l, k)]


def pattern(lv, adjoint=False):
    """list over compact displacement rows of arrays of compact column
    indices reached by the row (the structural pattern above)."""
    d = lv.dim
    sizes = lv.field_sizes()
    base = np.concatenate([[0], np.cumsum(sizes[:d])])
    coords = [_coords(lv, f) for f in range(d)]
    # compact index lookup per field: storage coords -> compact index
    lut = []
    for f in range(d):
        shp = list(lv.n)  # x-order storage extents
        t = -np.ones(shp[::-1], dtype=np.int64)  # numpy order
        c = coords[f]
        t[tuple(c[::-1])] = base[f] + np.arange(c.shape[1])
        lut.append(t)
    rows = []
    for k in range(d):
        ck = coords[k]
        for i in range(ck.shape[1]):
            c = ck[:, i]
            cols = []
            for l in range(d):
                for o in _offsets(d, k, l, adjoint):
                    t = c + np.array(o)
                    if np.any(t < 0) or np.any(t >= np.array(lv.n)):
                        continue
                    j = lut[l][tuple(t[::-1])]
                    if j >= 0:
                        cols.append(j)
            rows.append(np.array(sorted(set(cols)), dtype=np.int64))
    return rows


def pattern_check(lv, S, adjoint=False):
    """True when every stored nonzero of S lies in the pattern."""
    pat = pattern(lv, adjoint)
    S = S.tocsr()
    for i in range(S.shape[0]):
        a, b = S.indptr[i], S.indptr[i + 1]
        nz = S.indices[a:b][S.data[a:b] != 0]
        if not np.all(np.isin(nz, pat[i])):
            return False
    return True


def regions(lv, box):
    """sub-regions: list of ascending arrays of compact displacement rows,
    one per box of box^d cells holding at least one row (boxes in
    lexicographic order, x_d slowest)."""
    d = lv.dim
    nb = [-(-n // box) for n in lv.n]
    rid_all = []
    for f in range(d):
        c = _coords(lv, f) // box
        rid = np.zeros(c.shape[1], dtype=np.int64)
        for a in reversed(range(d)):
            rid = rid * nb[a] + c[a]
        rid_all.append(rid)
    rid = np.concatenate(rid_all)
    out = []
    for r in np.unique(rid):
        out.append(np.nonzero(rid == r)[0])
    return out


# ----------------------------------------------------------------------------
# hybrid Kaczmarz
# ----------------------------------------------------------------------------
class HybridKaczmarz:
    """Component-averaged parallel Kaczmarz on S x = b (see the header)."""

    def __init__(self, lv, S, box=4, omega=0.8, adjoint=False):
        self.S = S.tocsr()
        self.omega = float(omega)
        self.regions = regions(lv, box)
        pat = pattern(lv, adjoint)
        n = self.S.shape[0]
        self.counts = np.zeros(n, dtype=np.int64)
        self.cols = []
        for rows in self.regions:
            c = np.unique(np.concatenate([pat[i] for i in rows]))
            self.cols.append(c)
            self.counts[c] += 1
        self.rowdata = []
        for i in range(n):
            a, b = self.S.indptr[i], self.S.indptr[i + 1]
            vals = self.S.data[a:b]
            self.rowdata.append((self.S.indices[a:b], vals, float(np.sum(np.abs(vals) ** 2))))

    def sweep(self, x, b):
        acc = np.zeros_like(x)
        for rows, cols in zip(self.regions, self.cols):
            xr = x.copy()
            for i in rows:
                idx, vals, nrm = self.rowdata[i]
                if nrm == 0.0:
                    continue
                res = b[i] - np.dot(vals, xr[idx])
                xr[idx] += (self.omega * res / nrm) * np.conj(vals)
            acc[cols] += xr[cols]
        out = x.copy()
        m = self.counts > 0
        out[m] = acc[m] / self.counts[m]
        return out

    def apply(self, b, sweeps):
        """`sweeps` hybrid sweeps from x = 0 (the preconditioner)."""
        x = np.zeros_like(b, dtype=np.complex128)
        for _ in range(sweeps):
            x = self.sweep(x, b)
        return x


# ----------------------------------------------------------------------------
# coarsest-grid solve
# ----------------------------------------------------------------------------
class SchurKaczmarzSolver:
    """x = approximate solution of A x = b on the coarsest grid (compact
    vectors): FGMRES(restart) on the Schur complement, each step
    preconditioned by `sweeps` hybrid Kaczmarz sweeps; stop at a relative
    residual drop `rtol` or after `maxit` steps (the paper: restart 5,
    sweeps 10, omega 0.8, rtol 0.1, maxit 25 = 250 sweeps)."""

    def __init__(self, lv, A, box=4, omega=0.8, sweeps=10, restart=5, rtol=0.1, maxit=25,
                 adjoint=False):
        self.S, self.Aup, self.Apu, self.dp = schur_blocks(lv, A)
        self.nu = self.S.shape[0]
        self.kz = HybridKaczmarz(lv, self.S, box=box, omega=omega, adjoint=adjoint)
        self.sweeps, self.restart, self.rtol, self.maxit = sweeps, restart, rtol, maxit
        self.last_info = None

    def schur_rhs(self, b):
        return b[:self.nu] - self.Aup @ (b[self.nu:] / self.dp)

    def solve(self, b):
        bs = self.schur_rhs(b)
        u, info = fgmres(lambda v: self.S @ v, bs,
                         precond=lambda v: self.kz.apply(v, self.sweeps),
                         restart=self.restart, tol=self.rtol, maxit=self.maxit)
        self.last_info = info
        p = (b[self.nu:] - self.Apu @ u) / self.dp
        return np.concatenate([u, p])
