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
  * S: the smoother.  The paper analyses lexicographic (economic) Vanka,
    whose symbol it does not print; the build's production smoother is
    red-black full Vanka, whose symbol is derived here.  One colour's
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
    def __init__(self, dim, h, omega, gamma, beta, lam, mu, rho, alpha, w, nu1=1, nu2=1, cell_block=None):
        self.d = dim
        self.h, self.omega, self.gamma, self.beta = h, omega, gamma, beta
        self.lam, self.mu, self.rho = lam, mu, rho
        self.alpha, self.w, self.nu1, self.nu2 = alpha, w, nu1, nu2
        if cell_block is None:
            prob = PeriodicProblem(4, dim, h, omega, gamma, beta, lam, mu, rho)
            cell_block = vanka_cell_block(prob, alpha)
        self.Acell_inv = np.linalg.inv(cell_block)
        self.H = _harmonics(dim)

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
        return self.half_sweep(theta, 1) @ self.half_sweep(theta, 0)

    def two_grid(self, theta):
        theta = np.asarray(theta, dtype=float)
        Ah = self.fine(theta)
        Ac = self.A_sym(2 * theta, coarse=True)
        K = np.eye(Ah.shape[0]) - self.prolongation(theta) @ np.linalg.solve(Ac, self.restriction(theta) @ Ah)
        Sm = self.smoother(theta)
        return np.linalg.matrix_power(Sm, self.nu2) @ K @ np.linalg.matrix_power(Sm, self.nu1)

    def rho_loc(self, step=None, thetas=None):
        """max spectral radius of TG(theta) over theta in T_low (a grid with
        spacing `step`, or the given list)."""
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
        nf = self.d + 1
        Q = np.eye(len(self.H) * nf)
        Q[:nf, :nf] = 0.0                      # projector onto the high harmonics
        best = 0.0
        for th in itertools.product(g, repeat=self.d):
            Sm = self.smoother(np.asarray(th, dtype=float))
            ev = np.linalg.eigvals(Q @ Sm)
            best = max(best, float(np.abs(ev).max()))
        return best
