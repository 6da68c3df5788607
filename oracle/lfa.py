"""Two-grid local Fourier analysis of the red-black Vanka multigrid cycle.

Test infrastructure (see the package header).

Section 4 (LFA): for a constant-coefficient problem the two-grid operator
TG = S^nu2 (I - P A_2h^{-1} R A_h) S^nu1 (eq. 2G, CGC) leaves the space of
2^d harmonics E(theta) = { theta + pi*a : a in {0,1}^d } invariant (Section
4.1, Definition of the 4 harmonics in 2D; 8 in 3D).  Its restriction to
E(theta) is the symbol matrix of eq. symbolTG, of size 2^d (d+1):
  * A_h, A_2h: closed-form operator symbols (module `symbols`), at theta^(a)
    on the fine grid and at 2 theta (spacing 2h) on the coarse grid;
  * R, P: closed-form transfer symbols; a coarse DOF sits at a multiple of
    2h along its face axis and at an odd multiple of h along the others,
    which gives harmonic a the sign s(a, f) = prod over those axes of
    (-1)^{a_b};
  * S: the smoother.  Two are analysed here.  The paper's LFA (Sections
    4.3 and 5.1) uses economic Vanka (the displacement part of each cell
    block replaced by its diagonal, Section 2.3) swept over the cells in
    lexicographic order; it omits the symbol's derivation, which is given
    in `LexVanka` below.  The build's production smoother is red-black
    full Vanka, whose symbol is derived next.  One colour's
    half-sweep e <- e - w B_c A e solves every cell block of colour c with
    the residual; on a plane wave it returns the same wave plus the wave
    shifted by (pi,...,pi), because the colour indicator is
    (1 + (-1)^(i_1+...+i_d))/2.  The block A_cell is the operator's
    submatrix on one cell's 2d+1 unknowns.
rho_loc = max over theta in T_low of the spectral radius of TG(theta)
(Definition of rho_loc, Section 4.1); mu_loc (Definition of mu_loc) is
the smoothing factor on the high frequencies.

A brute-force counterpart assembles the same two-grid operator on a small
periodic grid as a dense matrix (periodic_two_grid), so the LFA can be
checked against an exact spectral radius.
"""
import itertools

import numpy as np
import scipy.sparse as sp

from . import symbols as S


# ----------------------------------------------------------------------------
# periodic grid (constant media, no absorbing layer)
# ----------------------------------------------------------------------------
def _per_shift(n, k):
    """matrix of v -> v[(i + k) mod n]"""
    rows = np.arange(n)
    return sp.csr_matrix((np.ones(n), (rows, (rows + k) % n)), shape=(n, n))


def _kron(mats):
    """mats in x-order (x_1 first); C-order flattening with x_1 fastest."""
    out = None
    for m in reversed(mats):
        out = m if out is None else sp.kron(out, m, format="csr")
    return out.tocsr()


class PeriodicProblem:
    """n^d periodic cells, spacing h, constant media; every field has n^d
    unknowns (face i along x_k sits between cells i-1 and i)."""

    def __init__(self, n, dim, h, omega, gamma, beta, lam, mu, rho):
        self.n, self.dim, self.h = n, dim, h
        self.omega, self.gamma, self.beta = omega, gamma, beta
        self.lam, self.mu, self.rho = lam, mu, rho

    def I(self):
        return sp.identity(self.n, format="csr")

    def d_face_to_cell(self):
        return (_per_shift(self.n, 1) - self.I()) / self.h

    def d_cell_to_face(self):
        return (self.I() - _per_shift(self.n, -1)) / self.h

    def avg(self):
        return 0.5 * self.I() + 0.25 * (_per_shift(self.n, 1) + _per_shift(self.n, -1))

    def operator(self, shift=0.0):
        d, n, b = self.dim, self.n, self.beta
        N = n ** d
        I = self.I()
        blocks = [[None] * (d + 1) for _ in range(d + 1)]
        w2 = self.omega ** 2 * (1 - 1j * (self.gamma + shift))
        for k in range(d):
            lap = None
            for l in range(d):
                Dl = self.d_face_to_cell() if l == k else self.d_cell_to_face()
                base = [I] * d
                base[l] = Dl
                D = _kron(base)
                spr = [self.avg()] * d
                spr[l] = Dl
                Ds = b * D + (1 - b) * _kron(spr)
                term = self.mu * (D.T @ Ds)
                lap = term if lap is None else lap + term
            nb = sum(_kron([(_per_shift(n, 1) + _per_shift(n, -1)) if a == l else I for a in range(d)])
                     for l in range(d))
            mass = w2 * self.rho * (b * sp.identity(N) + (1 - b) / (2 * d) * nb)
            blocks[k][k] = (lap - mass).tocsr()
            g = [I] * d
            g[k] = self.d_cell_to_face()
            blocks[k][d] = _kron(g)
            dv = [I] * d
            dv[k] = self.d_face_to_cell()
            spr = [self.avg()] * d
            spr[k] = self.d_face_to_cell()
            blocks[d][k] = b * _kron(dv) + (1 - b) * _kron(spr)
        blocks[d][d] = sp.identity(N) / (self.lam + self.mu)
        return sp.bmat(blocks, format="csr").astype(np.complex128)

    def coarse(self):
        return PeriodicProblem(self.n // 2, self.dim, 2 * self.h, self.omega, self.gamma, self.beta,
                               self.lam, self.mu, self.rho)

    # transfers (Section 2.3 stencils with periodic wrap)
    def restriction(self):
        n, d = self.n, self.dim
        nc = n // 2
        fw = sp.lil_matrix((nc, n))
        pr = sp.lil_matrix((nc, n))
        for J in range(nc):
            for f, w in ((2 * J - 1, 0.25), (2 * J, 0.5), (2 * J + 1, 0.25)):
                fw[J, f % n] += w
            pr[J, 2 * J] += 0.5
            pr[J, 2 * J + 1] += 0.5
        blocks = []
        for f in range(d + 1):
            blocks.append(_kron([fw.tocsr() if a == f else pr.tocsr() for a in range(d)]))
        return sp.block_diag(blocks, format="csr")

    def prolongation(self):
        n, d = self.n, self.dim
        nc = n // 2
        lf = sp.lil_matrix((n, nc))
        lc = sp.lil_matrix((n, nc))
        for f in range(n):
            if f % 2 == 0:
                lf[f, (f // 2) % nc] += 1.0
            else:
                lf[f, ((f - 1) // 2) % nc] += 0.5
                lf[f, ((f + 1) // 2) % nc] += 0.5
        for I in range(nc):
            lc[2 * I, I] += 0.75
            lc[2 * I, (I - 1) % nc] += 0.25
            lc[2 * I + 1, I] += 0.75
            lc[2 * I + 1, (I + 1) % nc] += 0.25
        blocks = []
        for f in range(d + 1):
            blocks.append(_kron([lf.tocsr() if a == f else lc.tocsr() for a in range(d)]))
        return sp.block_diag(blocks, format="csr")

    def cell_dofs(self):
        """(ncells, 2d+1): [u_1 left, u_1 right, ..., p] with periodic wrap;
        cells in C order (x_1 fastest) and their colours."""
        n, d = self.n, self.dim
        N = n ** d
        idx = np.array(list(itertools.product(range(n), repeat=d)))[:, ::-1]  # x-order columns
        lin = lambda v: sum(int(v[a]) * n ** a for a in range(d))
        out = np.zeros((N, 2 * d + 1), dtype=np.int64)
        colours = np.zeros(N, dtype=np.int64)
        for c, v in enumerate(idx):
            assert lin(v) == c
            colours[c] = int(v.sum()) % 2
            for k in range(d):
                r = v.copy()
                r[k] = (r[k] + 1) % n
                out[c, 2 * k] = k * N + lin(v)
                out[c, 2 * k + 1] = k * N + lin(r)
            out[c, 2 * d] = d * N + c
        return out, colours


def vanka_cell_block(prob, shift):
    """the (2d+1)x(2d+1) block of the shifted operator on one cell (all
    cells are equal for constant media), slot order [L_1, R_1, ..., p]"""
    A = prob.operator(shift).tocsr()
    dofs, _ = prob.cell_dofs()
    c = 0
    return A[dofs[c]][:, dofs[c]].toarray()


def periodic_two_grid(prob, alpha, w, nu1=1, nu2=1):
    """dense two-grid error propagator on the periodic grid"""
    A = prob.operator(alpha).toarray()
    Ac = prob.coarse().operator(alpha).toarray()
    R = prob.restriction().toarray()
    P = prob.prolongation().toarray()
    dofs, col = prob.cell_dofs()
    n = A.shape[0]

    def half(c):
        B = np.zeros((n, n), dtype=complex)
        for cell in np.nonzero(col == c)[0]:
            dv = dofs[cell]
            B[np.ix_(dv, dv)] += np.linalg.inv(A[np.ix_(dv, dv)])
        return np.eye(n) - w * B @ A

    Ssweep = half(1) @ half(0)
    K = np.eye(n) - P @ np.linalg.solve(Ac, R @ A)
    return np.linalg.matrix_power(Ssweep, nu2) @ K @ np.linalg.matrix_power(Ssweep, nu1)


# ----------------------------------------------------------------------------
# harmonic (LFA) symbols
# ----------------------------------------------------------------------------
def _harmonics(d):
    return [np.array(a) for a in itertools.product((0, 1), repeat=d)]


def _sign(a, f, d):
    """(-1)^(sum of a_b over the axes b where field f is cell-centred)"""
    s = 1.0
    for b in range(d):
        if b != f and a[b]:
            s = -s
    return s


class LFA:
    def __init__(self, dim, h, omega, gamma, beta, lam, mu, rho, alpha, w, nu1=1, nu2=1, cell_block=None,
                 smoother="red-black", scalar_smoother=False):
        """smoother: "red-black" (full Vanka, the production smoother),
        "lex-economic" or "lex-full" (lexicographic sweeps, `LexVanka`).

        scalar_smoother (lexicographic smoothers only): the paper's reading
        of its smoothing symbol matrix (eq. smoothingSymbolMatrix), which
        puts one scalar per harmonic on the diagonal.  The scalar taken is
        the eigenvalue of largest modulus of the (d+1)x(d+1) sweep symbol at
        that harmonic, acting on all d+1 fields alike.  This is not the
        two-grid operator of the cycle (that is scalar_smoother=False, which
        the periodic assembly pins); it is the reading under which the
        two-grid factors printed in Table 1 are reproduced."""
        self.d = dim
        self.h, self.omega, self.gamma, self.beta = h, omega, gamma, beta
        self.lam, self.mu, self.rho = lam, mu, rho
        self.alpha, self.w, self.nu1, self.nu2 = alpha, w, nu1, nu2
        if cell_block is None:
            prob = PeriodicProblem(4, dim, h, omega, gamma, beta, lam, mu, rho)
            cell_block = vanka_cell_block(prob, alpha)
        self.Acell_inv = np.linalg.inv(cell_block)
        self.H = _harmonics(dim)
        assert smoother in ("red-black", "lex-economic", "lex-full")
        self.kind = smoother
        assert not (scalar_smoother and smoother == "red-black")
        self.scalar_smoother = scalar_smoother
        if smoother != "red-black":
            self.lex = LexVanka(PeriodicProblem(8, dim, h, omega, gamma, beta, lam, mu, rho), alpha, w,
                                economic=smoother == "lex-economic")

    def A_sym(self, th, shifted=True, coarse=False):
        g = self.gamma + (self.alpha if shifted else 0.0)
        h = 2 * self.h if coarse else self.h
        return S.operator_symbol(th, h, self.omega, g, self.beta, self.lam, self.mu, self.rho)

    def _idx(self, ai, f):
        return ai * (self.d + 1) + f

    def fine(self, theta):
        d, nf = self.d, self.d + 1
        M = np.zeros((len(self.H) * nf,) * 2, dtype=complex)
        for ai, a in enumerate(self.H):
            M[ai * nf:(ai + 1) * nf, ai * nf:(ai + 1) * nf] = self.A_sym(theta + np.pi * a)
        return M

    def restriction(self, theta):
        nf = self.d + 1
        R = np.zeros((nf, len(self.H) * nf))
        for ai, a in enumerate(self.H):
            rs = S.restriction_symbol(theta + np.pi * a)
            for f in range(nf):
                R[f, self._idx(ai, f)] = rs[f] * _sign(a, f, self.d)
        return R

    def prolongation(self, theta):
        nf = self.d + 1
        P = np.zeros((len(self.H) * nf, nf))
        for ai, a in enumerate(self.H):
            ps = S.prolongation_symbol(theta + np.pi * a)
            for f in range(nf):
                P[self._idx(ai, f), f] = ps[f] * _sign(a, f, self.d) / 2 ** self.d
        return P

    def half_sweep(self, theta, colour):
        """symbol of e <- e - w B_c A e on E(theta)"""
        d, nf = self.d, self.d + 1
        size = len(self.H) * nf
        M = np.zeros((size, size), dtype=complex)
        flip = {tuple(a): i for i, a in enumerate(self.H)}
        for ai, a in enumerate(self.H):
            th = theta + np.pi * a
            Ah = self.A_sym(th)
            ap = flip[tuple((a + 1) % 2)]
            for g in range(nf):
                r = Ah[:, g]
                # local residual on the 2d+1 slots of a cell centred at X_c
                rho_l = np.zeros(2 * d + 1, dtype=complex)
                for k in range(d):
                    rho_l[2 * k] = r[k] * np.exp(-0.5j * th[k])
                    rho_l[2 * k + 1] = r[k] * np.exp(0.5j * th[k])
                rho_l[2 * d] = r[d]
                dl = self.Acell_inv @ rho_l
                sc = -1.0 if colour else 1.0
                for k in range(d):
                    aL = np.exp(0.5j * th[k]) * dl[2 * k]
                    aR = np.exp(-0.5j * th[k]) * dl[2 * k + 1]
                    M[self._idx(ai, k), self._idx(ai, g)] += 0.5 * (aL + aR)
                    M[self._idx(ap, k), self._idx(ai, g)] += (0.5 * (aL - aR) * sc * np.exp(-0.5j * np.pi * (d - 1))
                                                              * _sign(a, k, d))
                apv = dl[2 * d]
                M[self._idx(ai, d), self._idx(ai, g)] += 0.5 * apv
                M[self._idx(ap, d), self._idx(ai, g)] += 0.5 * apv * sc * np.exp(-0.5j * np.pi * d) * _sign(a, d, d)
        return np.eye(size) - self.w * M

    def smoother(self, theta):
        if self.kind == "red-black":
            return self.half_sweep(theta, 1) @ self.half_sweep(theta, 0)
        # a lexicographic sweep maps each harmonic to itself
        nf = self.d + 1
        M = np.zeros((len(self.H) * nf,) * 2, dtype=complex)
        for ai, a in enumerate(self.H):
            Sa = self.lex.symbol(theta + np.pi * a)
            if self.scalar_smoother:
                ev = np.linalg.eigvals(Sa)
                Sa = ev[np.argmax(np.abs(ev))] * np.eye(nf)
            M[ai * nf:(ai + 1) * nf, ai * nf:(ai + 1) * nf] = Sa
        return M

    def two_grid(self, theta):
        theta = np.asarray(theta, dtype=float)
        Ah = self.fine(theta)
        Ac = self.A_sym(2 * theta, coarse=True)
        K = np.eye(Ah.shape[0]) - self.prolongation(theta) @ np.linalg.solve(Ac, self.restriction(theta) @ Ah)
        Sm = self.smoother(theta)
        return np.linalg.matrix_power(Sm, self.nu2) @ K @ np.linalg.matrix_power(Sm, self.nu1)

    def _lex_blocks(self, th):
        """(m, d+1, d+1) smoother blocks of a lexicographic sweep at the rows
        of th, under the chosen reading"""
        Sa = self.lex.symbol(th)
        if self.scalar_smoother:
            ev = np.linalg.eigvals(Sa)
            pick = ev[np.arange(len(ev)), np.argmax(np.abs(ev), axis=1)]
            Sa = pick[:, None, None] * np.eye(self.d + 1)
        return Sa

    def two_grid_many(self, thetas):
        """TG at every row of an (m, d) array (lexicographic smoothers): the
        same matrices as `two_grid`, built for all m frequencies at once"""
        th = np.atleast_2d(np.asarray(thetas, dtype=float))
        m, d, nf = th.shape[0], self.d, self.d + 1
        n = len(self.H) * nf
        Ah = np.zeros((m, n, n), dtype=complex)
        Sm = np.zeros((m, n, n), dtype=complex)
        R = np.zeros((m, nf, n))
        P = np.zeros((m, n, nf))
        for ai, a in enumerate(self.H):
            ta = th + np.pi * a
            sl = slice(ai * nf, (ai + 1) * nf)
            Ah[:, sl, sl] = np.moveaxis(self.A_sym(ta.T), -1, 0)
            rs = S.restriction_symbol(ta.T)
            ps = S.prolongation_symbol(ta.T)
            for f in range(nf):
                R[:, f, self._idx(ai, f)] = rs[f] * _sign(a, f, d)
                P[:, self._idx(ai, f), f] = ps[f] * _sign(a, f, d) / 2 ** d
            Sm[:, sl, sl] = self._lex_blocks(ta)
        Ac = np.moveaxis(self.A_sym((2 * th).T, coarse=True), -1, 0)
        K = np.eye(n) - P @ np.linalg.solve(Ac, R @ Ah)
        return np.linalg.matrix_power(Sm, self.nu2) @ K @ np.linalg.matrix_power(Sm, self.nu1)

    def rho_loc(self, step=None, thetas=None):
        """max spectral radius of TG(theta) over theta in T_low (a grid with
        spacing `step`, or the given list)."""
        if self.kind != "red-black":
            if thetas is None:
                g = np.arange(-np.pi / 2, np.pi / 2, step)
                thetas = np.array(list(itertools.product(g, repeat=self.d)))
            th = np.asarray(list(thetas), dtype=float)
            best = 0.0
            for c in range(0, len(th), 8192):
                ev = np.linalg.eigvals(self.two_grid_many(th[c:c + 8192]))
                best = max(best, float(np.abs(ev).max()))
            return best
        if thetas is None:
            g = np.arange(-np.pi / 2, np.pi / 2, step)
            thetas = itertools.product(g, repeat=self.d)
        best = 0.0
        for th in thetas:
            th = np.asarray(th, dtype=float)
            if np.allclose(th, 0.0):
                # the constant mode: A_2h is regular (shifted mass), keep it
                pass
            ev = np.linalg.eigvals(self.two_grid(th))
            best = max(best, float(np.abs(ev).max()))
        return best

    def mu_loc(self, step):
        """smoothing factor: max over high frequencies of the spectral radius
        of the smoother restricted to the high harmonics (ideal coarse-grid
        correction removes the low harmonic of every E(theta))."""
        g = np.arange(-np.pi / 2, np.pi / 2, step)
        if self.kind != "red-black":
            # the sweep keeps each harmonic: its high-frequency symbols directly
            th = np.array(list(itertools.product(g, repeat=self.d)))
            best = 0.0
            for a in self.H[1:]:
                for c in range(0, len(th), 65536):
                    ev = np.linalg.eigvals(self.lex.symbol(th[c:c + 65536] + np.pi * a))
                    best = max(best, float(np.abs(ev).max()))
            return best
        nf = self.d + 1
        Q = np.eye(len(self.H) * nf)
        Q[:nf, :nf] = 0.0                      # projector onto the high harmonics
        best = 0.0
        for th in itertools.product(g, repeat=self.d):
            Sm = self.smoother(np.asarray(th, dtype=float))
            ev = np.linalg.eigvals(Q @ Sm)
            best = max(best, float(np.abs(ev).max()))
        return best


# ----------------------------------------------------------------------------
# lexicographic cell-wise Vanka (full or economic)
# ----------------------------------------------------------------------------
def economic_block(block, dim):
    """economic Vanka's block (Section 2.3): the cell block with every
    displacement-displacement entry off the diagonal dropped; the pressure
    row and column are kept."""
    B = np.array(block, dtype=complex, copy=True)
    nu = 2 * dim
    for a in range(nu):
        for b in range(nu):
            if a != b:
                B[a, b] = 0.0
    return B


def lex_sweep(prob, shift, w, e, economic=True):
    """one lexicographic Vanka sweep on the error equation of the periodic
    grid, written out: cells in C order (x_1 fastest); each cell's 2d+1
    unknowns are corrected by w B^{-1} r with the residual r = -A e taken
    at that moment, so faces shared with an earlier cell see its update."""
    A = prob.operator(shift).tocsr()
    dofs, _ = prob.cell_dofs()
    e = np.array(e, dtype=complex, copy=True)
    for dv in dofs:
        blk = A[dv][:, dv].toarray()
        B = economic_block(blk, prob.dim) if economic else blk
        r = -(A[dv] @ e)
        e[dv] += w * np.linalg.solve(B, r)
    return e


class LexVanka:
    """Symbol of one lexicographic sweep of cell-wise Vanka.

    Cell c's block holds, for each axis k, the face on its low side L_k
    (shared with the earlier cell c - e_k) and on its high side R_k (shared
    with the later cell c + e_k), and its pressure.  A sweep therefore
    leaves every face in one of three states: old (no cell touched it yet),
    mid (its low-side cell corrected it) and new (both cells did); a
    pressure is old or new.  On an infinite grid with a plane-wave error
    exp(i theta.x/h) every state of every field is the same plane wave with
    its own amplitude.  When cell c is relaxed:
      * the residual on its block rows reads each stencil neighbour in the
        state the lexicographic order gives it at that moment;
      * L_k goes mid -> new, R_k old -> mid, p old -> new, by w B^{-1} r.
    These 2d+1 equations are linear in the unknown amplitudes
    z = (new_1..new_d, mid_1..mid_d, new_p) given the old ones o, and
    S(theta) is the map o -> (new_1..new_d, new_p).  The stencil and the
    block come from the periodic assembly, so the symbol uses the operator
    the cycle uses; `lex_sweep` is the direct counterpart it is checked
    against."""

    def __init__(self, prob, shift, w, economic=True):
        d, n = prob.dim, prob.n
        assert n >= 6
        self.d, self.w = d, w
        A = prob.operator(shift).tocsr()
        N = n ** d
        centre = np.full(d, n // 2)
        lin = lambda v: sum(int(v[a]) * n ** a for a in range(d))
        rows = []
        for g in range(d + 1):
            j = g * N + lin(centre)
            ent = []
            for ptr in range(A.indptr[j], A.indptr[j + 1]):
                f, q = divmod(int(A.indices[ptr]), N)
                idx = np.array([(q // n ** a) % n for a in range(d)])
                ent.append((f, idx - centre, A.data[ptr]))
            rows.append(ent)
        dofs, _ = prob.cell_dofs()
        blk = A[dofs[lin(centre)]][:, dofs[lin(centre)]].toarray()
        self.Binv = np.linalg.inv(economic_block(blk, d) if economic else blk)
        eye = np.eye(d, dtype=np.int64)
        slots = []
        for k in range(d):
            slots += [(k, np.zeros(d, dtype=np.int64)), (k, eye[k])]
        slots.append((d, np.zeros(d, dtype=np.int64)))
        self.slots = slots
        # each residual term: (slot, unknown vector 'z' or 'o', its index,
        # coefficient, the neighbour's position in units of h)
        self.terms = []
        for s, (g, j) in enumerate(slots):
            for f, off, a in rows[g]:
                i = j + off
                where, idx = self._amp(f, i)
                self.terms.append((s, where, idx, a, self._pos(f, i)))

    def _pos(self, f, i):
        x = i.astype(float)
        if f < self.d:
            x[f] -= 0.5
        return x

    @staticmethod
    def _before(v):
        """is the cell at offset v relaxed before the cell at the origin
        (lexicographic order, x_1 fastest)?"""
        for a in reversed(range(len(v))):
            if v[a] != 0:
                return v[a] < 0
        return False

    def _amp(self, f, i):
        d = self.d
        if f == d:
            return ("z", 2 * d) if self._before(i) else ("o", d)
        if self._before(i):
            return ("z", f)
        lo = i.copy()
        lo[f] -= 1
        if self._before(lo):
            return ("z", d + f)
        return ("o", f)

    def symbol(self, theta):
        """the (d+1)x(d+1) symbol at theta (a d-vector), or an (m, d+1, d+1)
        stack at the rows of an (m, d) array"""
        th = np.asarray(theta, dtype=float)
        one = th.ndim == 1
        th = np.atleast_2d(th)
        m, d = th.shape[0], self.d
        nz = 2 * d + 1
        Rz = np.zeros((m, nz, nz), dtype=complex)
        Ro = np.zeros((m, nz, d + 1), dtype=complex)
        for s, where, idx, a, x in self.terms:
            ph = np.exp(1j * (th @ x))
            if where == "z":
                Rz[:, s, idx] -= a * ph
            else:
                Ro[:, s, idx] -= a * ph
        E = np.zeros((m, nz, nz), dtype=complex)
        F = np.zeros((m, nz, d + 1), dtype=complex)
        for k in range(d):
            pl = np.exp(-0.5j * th[:, k])   # L_k sits at -e_k/2
            pr = np.exp(0.5j * th[:, k])    # R_k at +e_k/2
            E[:, 2 * k, k] = pl
            E[:, 2 * k, d + k] = -pl
            E[:, 2 * k + 1, d + k] = pr
            F[:, 2 * k + 1, k] = pr
        E[:, 2 * d, 2 * d] = 1.0
        F[:, 2 * d, d] = 1.0
        z = np.linalg.solve(E - self.w * self.Binv @ Rz, F + self.w * self.Binv @ Ro)
        out = z[:, list(range(d)) + [2 * d], :]
        return out[0] if one else out
