"""Coarse hierarchy, two-grid / V-cycle and coarsest-grid solves.

Test infrastructure (see the package header).

* Hierarchy (Section 3.2, Remark in Section 2.2): coarse operators are the
  same beta-stencil re-discretised on the 2h grid, shifted on every level
  (Section 2.2: the shift alpha is added to gamma).  Coarse media are not
  specified by the paper; reading: arithmetic mean of the 2^d child cells
  of lam, mu, rho; the absorbing layer keeps its physical width.
* Cycle: Algorithm 1 (two-grid cycle) applied recursively with one
  recursive call (V-cycle) or two (W-cycle: the second call solves for the
  residual left by the first, Section 2.2; on every level, so above the
  coarsest level the coarse problem gets two coarsest solves, the second on
  the residual of the first -- with an inexact coarsest solve that second
  solve is not a no-op), or two calls used as the
  preconditioners of two steps of a Krylov method on the coarse system
  (K-cycle, Section 2.2; reading: flexible GCR, i.e. the coarse correction
  minimises the coarse residual over the span of the two preconditioned
  directions), nu1 pre- and nu2
  post-relaxations with
  red-black full Vanka, per-level damping w_l (Section 5.2 uses 0.55 /
  0.35 / 0.25 for finest/second/third levels).  The cycle preconditions
  with a zero initial guess on every level.
* Coarsest solve (Section 3.2 "Coarsest grid solution"): 'direct' (sparse
  LU, the paper's 2D choice), 'relax' (a fixed number of red-black Vanka
  sweeps from zero), or 'krylov' (restarted GMRES preconditioned by a
  fixed number of red-black Vanka sweeps, with a fixed iteration budget
  and an optional residual-drop stop), or 'kaczmarz' (the paper's 3D
  choice: FGMRES on the Schur complement of the pressure preconditioned by
  hybrid Kaczmarz sweeps, `oracle.kaczmarz`).
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import grid as G
from . import operator as O
from . import transfer as T
from .smoother import Vanka
from .krylov import fgmres
from .kaczmarz import SchurKaczmarzSolver


def coarsen_media(a, dim):
    """mean of the 2^d children (numpy array of shape (n_d..n_1))."""
    out = a
    for ax in range(dim):
        sl0 = [slice(None)] * dim
        sl1 = [slice(None)] * dim
        sl0[ax] = slice(0, None, 2)
        sl1[ax] = slice(1, None, 2)
        out = 0.5 * (out[tuple(sl0)] + out[tuple(sl1)])
    return out


def coarsen_level(lv):
    for n in lv.n:
        if n % 2:
            raise ValueError("grid not divisible by 2")
    nc = tuple(n // 2 for n in lv.n)
    return G.Level(nc, 2 * lv.h, lv.omega, lv.gamma, lv.beta,
                   coarsen_media(lv.lam, lv.dim), coarsen_media(lv.mu, lv.dim),
                   coarsen_media(lv.rho, lv.dim), lv.abl_width, lv.abl_amp)


class CycleParams:
    def __init__(self, levels=2, alpha=0.1, damping=(0.55, 0.35, 0.25, 0.25),
                 nu1=1, nu2=1, coarse="direct", coarse_sweeps=2,
                 coarse_restart=5, coarse_maxit=10, coarse_rtol=0.0,
                 coarse_damping=None, calls=1, kacz_box=4):
        # calls: 1 V-cycle, 2 W-cycle, 3 K-cycle (two Krylov-accelerated calls)
        self.levels = levels
        self.calls = calls
        self.alpha = alpha
        self.damping = tuple(damping)
        self.nu1, self.nu2 = nu1, nu2
        self.coarse = coarse
        self.coarse_sweeps = coarse_sweeps
        self.coarse_restart = coarse_restart
        self.coarse_maxit = coarse_maxit
        self.coarse_rtol = coarse_rtol
        self.coarse_damping = coarse_damping
        self.kacz_box = kacz_box

    def w(self, l):
        return self.damping[min(l, len(self.damping) - 1)]

    def wc(self):
        if self.coarse_damping is not None:
            return self.coarse_damping
        if self.coarse == "kaczmarz":
            return 0.8  # the paper's Kaczmarz relaxation (Section 5.3)
        return self.w(self.levels - 1)


class Hierarchy:
    """Levels, shifted operators, transfers and smoothers of one problem.

    adjoint=True builds the cycle for H_s^H (conjugate-transposed operators
    and Vanka blocks, same transfers)."""

    def __init__(self, lv0, params, adjoint=False):
        self.p = params
        self.adjoint = adjoint
        self.levels = [lv0]
        for _ in range(params.levels - 1):
            self.levels.append(coarsen_level(self.levels[-1]))
        self.A = []
        for lv in self.levels:
            A = O.assemble(lv, shift=params.alpha)
            if adjoint:
                A = A.conj().T.tocsr()
            self.A.append(A)
        self.R = [T.restriction_matrix(lv) for lv in self.levels[:-1]]
        self.P = [T.prolongation_matrix(lv) for lv in self.levels[:-1]]
        self.smoothers = [Vanka(lv, A) for lv, A in zip(self.levels, self.A)]
        self._lu = None
        self._kz = None

    # -- coarsest-level solve -------------------------------------------------
    def _relax_from_zero(self, l, b, sweeps, w):
        x = np.zeros_like(b)
        for _ in range(sweeps):
            x = self.smoothers[l].sweep_rb(x, b, w)
        return x

    def coarse_solve(self, b):
        l = len(self.levels) - 1
        p = self.p
        if p.coarse == "direct":
            if self._lu is None:
                self._lu = spla.splu(self.A[l].tocsc())
            return self._lu.solve(b)
        if p.coarse == "relax":
            return self._relax_from_zero(l, b, p.coarse_sweeps, p.wc())
        if p.coarse == "krylov":
            A = self.A[l]
            x, _ = fgmres(lambda v: A @ v, b,
                          precond=lambda v: self._relax_from_zero(l, v, p.coarse_sweeps, p.wc()),
                          restart=p.coarse_restart, tol=p.coarse_rtol,
                          maxit=p.coarse_maxit)
            return x
        if p.coarse == "kaczmarz":
            if self._kz is None:
                self._kz = SchurKaczmarzSolver(self.levels[l], self.A[l], box=p.kacz_box, omega=p.wc(),
                                               sweeps=p.coarse_sweeps, restart=p.coarse_restart,
                                               rtol=p.coarse_rtol, maxit=p.coarse_maxit,
                                               adjoint=self.adjoint)
            return self._kz.solve(b)
        raise ValueError(p.coarse)

    # -- cycle ------------------------------------------------------------------
    def vcycle(self, b, l=0):
        """approximate solve of A_l x = b from x = 0 (compact vectors)."""
        if l == len(self.levels) - 1:
            return self.coarse_solve(b)
        w = self.p.w(l)
        sm = self.smoothers[l]
        x = np.zeros_like(b, dtype=np.complex128)
        for _ in range(self.p.nu1):
            x = sm.sweep_rb(x, b, w)
        r = b - self.A[l] @ x
        rc = self.R[l] @ r
        e = self.vcycle(rc, l + 1)
        if self.p.calls == 2:
            # second recursive call on the residual the first one leaves;
            # above the coarsest level both calls are coarsest solves
            e = e + self.vcycle(rc - self.A[l + 1] @ e, l + 1)
        elif self.p.calls == 3:
            e = self.krylov_correction(rc, e, l + 1)
        x = x + self.P[l] @ e
        for _ in range(self.p.nu2):
            x = sm.sweep_rb(x, b, w)
        return x

    def krylov_correction(self, rc, e1, l):
        """K-cycle coarse correction on level l: two steps of flexible GCR on
        A_l e = rc with the level-l cycle as preconditioner, e1 the first
        preconditioned direction.  Step 1: v1 = A e1, a1 = <v1, rc>/<v1, v1>,
        r1 = rc - a1 v1.  Step 2: e2 = cycle(r1), v2 = A e2 made orthogonal
        to v1 (b = <v1, v2>/<v1, v1>), a2 = <v2, r1>/<v2, v2>.  The result
        a1 e1 + a2 (e2 - b e1) minimises ||rc - A e|| over span{e1, e2}."""
        A = self.A[l]
        v1 = A @ e1
        d11 = np.vdot(v1, v1)
        a1 = np.vdot(v1, rc) / d11 if d11 != 0 else 0.0
        r1 = rc - a1 * v1
        e2 = self.vcycle(r1, l)
        v2 = A @ e2
        b = np.vdot(v1, v2) / d11 if d11 != 0 else 0.0
        v2 = v2 - b * v1
        e2 = e2 - b * e1
        d22 = np.vdot(v2, v2)
        a2 = np.vdot(v2, r1) / d22 if d22 != 0 else 0.0
        return a1 * e1 + a2 * e2

    def vcycle_storage(self, b):
        lv = self.levels[0]
        return G.unpack(lv, self.vcycle(G.pack(lv, b)))

    def two_grid_error_matrix_action(self, e, l=0):
        """error propagation of the two-grid cycle (exact coarse solve) on
        level l: e -> S^nu2 (I - P A_c^{-1} R A) S^nu1 e."""
        w = self.p.w(l)
        sm = self.smoothers[l]
        zero = np.zeros_like(e)
        for _ in range(self.p.nu1):
            e = sm.sweep_rb(e, zero, w)
        rc = self.R[l] @ (self.A[l] @ e)
        if self._lu is None or l + 1 != len(self.levels) - 1:
            lu = spla.splu(self.A[l + 1].tocsc())
        else:
            lu = self._lu
        e = e - self.P[l] @ lu.solve(rc)
        for _ in range(self.p.nu2):
            e = sm.sweep_rb(e, zero, w)
        return e


def solve(lv0, q, params, tol=1e-6, restart=5, maxit=500, adjoint=False,
          history=None, hierarchy=None):
    """FGMRES(restart) on H^beta (or its adjoint) right-preconditioned by
    V-cycles on the shifted operator; q and the result in storage layout."""
    hier = hierarchy or Hierarchy(lv0, params, adjoint=adjoint)
    A = O.assemble(lv0, shift=0.0)
    if adjoint:
        A = A.conj().T.tocsr()
    b = G.pack(lv0, q)
    x, info = fgmres(lambda v: A @ v, b, precond=hier.vcycle, restart=restart,
                     tol=tol, maxit=maxit, history=history)
    return G.unpack(lv0, x), info
