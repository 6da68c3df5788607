"""Python binding of libelh: argument marshalling only.

Every numerical step runs in the HIP library; torch supplies device memory
and the current stream.  Vectors are torch complex tensors on the GPU with
shape (d+1, n_d, ..., n_1) or (nrhs, d+1, n_d, ..., n_1) (fields u_1..u_d,
p; x_1 fastest; index 0 of u_k along x_k is the boundary face, held at 0).
"""
import ctypes

import torch

from . import _lib as L


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dtype_code(t):
    if t.dtype == torch.complex128:
        return L.ELH_C128
    if t.dtype == torch.complex64:
        return L.ELH_C64
    raise TypeError("vectors must be complex64 or complex128, got %s" % t.dtype)


def _info(s):
    """one solve-stats record as a dict (history: the per-iteration FGMRES
    residual estimates; times in ms)"""
    return dict(iters=s.iters, restarts=s.restarts, status=s.status, relres=s.relres,
                history=[s.history[i] for i in range(s.history_len)] if s.history else [],
                t_total_ms=s.t_total_ms, t_precond_ms=s.t_precond_ms, t_apply_ms=s.t_apply_ms,
                t_orth_ms=s.t_orth_ms, kernels=s.kernels)


def _media(lam, mu, rho, device):
    lam = torch.as_tensor(lam, dtype=torch.float64).to(device).contiguous()
    mu = torch.as_tensor(mu, dtype=torch.float64).to(device).contiguous()
    rho = torch.as_tensor(rho, dtype=torch.float64).to(device).contiguous()
    if not (lam.shape == mu.shape == rho.shape):
        raise ValueError("lam, mu, rho must have the same shape")
    if lam.dim() not in (2, 3):
        raise ValueError("media must be 2D or 3D")
    return lam, mu, rho


def _desc(shape, h=1.0, omega=1.0, gamma=0.01, alpha=0.3, beta=2.0 / 3.0, abl_width=0.0, abl_amp=2.0, levels=3,
          nu1=1, nu2=1, cycle='V', damping=(0.55, 0.35, 0.25), coarse_mode="krylov", coarse_sweeps=2,
          coarse_restart=5, coarse_maxit=10, coarse_rtol=0.0, coarse_damping=0.0, precond_dtype=torch.complex128,
          kacz_box=4):
    """the elh_desc of a problem on a grid of numpy shape `shape`"""
    dim = len(shape)
    d = L.Desc()
    d.dim = dim
    n = list(reversed(shape)) + [1] * (3 - dim)
    for a in range(3):
        d.n[a] = n[a]
    d.h, d.omega, d.gamma, d.alpha, d.beta = h, omega, gamma, alpha, beta
    d.abl_width, d.abl_amp = abl_width, abl_amp
    d.levels, d.nu1, d.nu2 = levels, nu1, nu2
    d.cycle_calls = {'V': 1, 'W': 2, 'K': 3}[cycle]
    damping = list(damping)
    while len(damping) < 8:
        damping.append(damping[-1])
    for i in range(8):
        d.damping[i] = damping[i]
    modes = {"krylov": L.ELH_COARSE_KRYLOV, "dense": L.ELH_COARSE_DENSE, "relax": L.ELH_COARSE_RELAX,
             "kaczmarz": L.ELH_COARSE_KACZMARZ}
    d.coarse_mode = modes[coarse_mode]
    d.coarse_sweeps, d.coarse_restart, d.coarse_maxit = coarse_sweeps, coarse_restart, coarse_maxit
    d.coarse_rtol, d.coarse_damping = coarse_rtol, coarse_damping
    d.precond_dtype = L.ELH_C64 if precond_dtype == torch.complex64 else L.ELH_C128
    d.kacz_box = kacz_box
    return d


class Problem:
    """One elastic Helmholtz problem (media + discretisation + solver
    parameters) living on one GPU.

    lam, mu, rho: float64 tensors of numpy shape (n_d, ..., n_1), any
    device (copied to the current GPU).  Lengths (h, abl_width) are in
    physical units.  cycle: 'V', 'W' or 'K' (the two coarse calls of every
    level precondition two flexible-GCR steps on the coarse system).
    coarse_mode: 'krylov' (GMRES preconditioned by Vanka sweeps), 'dense',
    'relax', or 'kaczmarz' (the paper's 3D solver: FGMRES on the Schur
    complement of the pressure preconditioned by hybrid Kaczmarz sweeps over
    sub-regions of kacz_box^d cells; the paper uses coarse_sweeps=10,
    coarse_restart=5, coarse_maxit=25, coarse_rtol=0.1 and relaxation
    coarse_damping=0.8, the default when coarse_damping <= 0).
    """

    def __init__(self, lam, mu, rho, device=None, **params):
        self.lib = L.load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        lam, mu, rho = _media(lam, mu, rho, self.device)
        self.shape = tuple(lam.shape)
        self.dim = len(self.shape)
        self.desc = _desc(self.shape, **params)
        self.levels = self.desc.levels
        self._media = (lam, mu, rho)
        self._owner = None
        self.handle = ctypes.c_void_p(0)
        with torch.cuda.device(self.device):
            st = torch.cuda.current_stream(self.device).cuda_stream
            L.check(self.lib.elh_create(ctypes.byref(self.desc), _ptr(lam), _ptr(mu), _ptr(rho),
                                        ctypes.c_void_p(st), ctypes.byref(self.handle)))

    # -- housekeeping ---------------------------------------------------------
    def close(self):
        if self._owner is None and self.handle and self.handle.value:
            self.lib.elh_destroy(self.handle)
        self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_media(self, lam, mu, rho):
        lam = torch.as_tensor(lam, dtype=torch.float64).to(self.device).contiguous()
        mu = torch.as_tensor(mu, dtype=torch.float64).to(self.device).contiguous()
        rho = torch.as_tensor(rho, dtype=torch.float64).to(self.device).contiguous()
        L.check(self.lib.elh_set_media(self.handle, _ptr(lam), _ptr(mu), _ptr(rho)))
        self._media = (lam, mu, rho)

    def level_shape(self, level):
        n3 = (ctypes.c_int * 3)()
        hl = ctypes.c_double()
        L.check(self.lib.elh_level_info(self.handle, level, n3, ctypes.byref(hl)))
        return tuple(reversed([n3[a] for a in range(self.dim)])), hl.value

    def stencil_choice(self, level=0, dtype=torch.complex128, residual=False, adjoint=False, nrhs=1):
        """x_3 chunk the stencil autotuner chose for one kind of 3D apply /
        residual (> 0), -1 when none was made."""
        c = ctypes.c_int()
        L.check(self.lib.elh_stencil_choice(self.handle, level, L.ELH_C64 if dtype == torch.complex64 else L.ELH_C128,
                                            self._flags(False, adjoint), 1 if residual else 0, nrhs,
                                            ctypes.byref(c)))
        return c.value

    def _vec(self, t, level):
        shp, _ = self.level_shape(level)
        if not t.is_cuda or t.device != self.device:
            raise ValueError("vectors must live on %s" % self.device)
        if not t.is_contiguous():
            raise ValueError("vectors must be contiguous")
        full = (self.dim + 1,) + shp
        if tuple(t.shape) == full:
            return 1
        if t.dim() == len(full) + 1 and tuple(t.shape[1:]) == full:
            return t.shape[0]
        raise ValueError("vector shape %s does not match level %d layout %s" % (tuple(t.shape), level, full))

    def _same(self, t, ref, name):
        """t must match ref (shape, dtype, device) and be contiguous: the
        library reads and writes it with ref's layout."""
        if (t is None or tuple(t.shape) != tuple(ref.shape) or t.dtype != ref.dtype or t.device != ref.device
                or not t.is_contiguous()):
            raise ValueError("%s must be a contiguous %s tensor of shape %s on %s"
                             % (name, ref.dtype, tuple(ref.shape), ref.device))
        return t

    @staticmethod
    def _flags(shifted, adjoint):
        return (L.ELH_SHIFTED if shifted else 0) | (L.ELH_ADJOINT if adjoint else 0)

    # -- level operations -----------------------------------------------------
    def apply(self, x, level=0, shifted=False, adjoint=False, out=None):
        nrhs = self._vec(x, level)
        y = torch.empty_like(x) if out is None else self._same(out, x, "out")
        L.check(self.lib.elh_apply(self.handle, level, self._flags(shifted, adjoint), _dtype_code(x), nrhs,
                                   _ptr(x), _ptr(y)))
        return y

    def apply_f32_input(self, x, adjoint=False, out=None):
        """y = H x (level 0, complex128) from complex64 x with float64
        arithmetic: the outer operator of the mixed-precision solve."""
        if x.dtype != torch.complex64:
            raise TypeError("x must be complex64")
        nrhs = self._vec(x, 0)
        y = torch.empty(x.shape, dtype=torch.complex128, device=x.device) if out is None else out
        if y.dtype != torch.complex128 or y.shape != x.shape or not y.is_contiguous():
            raise ValueError("out must be a contiguous complex128 tensor of x's shape")
        L.check(self.lib.elh_apply_f32in(self.handle, self._flags(False, adjoint), nrhs, _ptr(x), _ptr(y)))
        return y

    def residual(self, b, x, level=0, shifted=False, adjoint=False, out=None):
        nrhs = self._vec(x, level)
        self._same(b, x, "b")
        r = torch.empty_like(x) if out is None else self._same(out, x, "out")
        L.check(self.lib.elh_residual(self.handle, level, self._flags(shifted, adjoint), _dtype_code(x), nrhs,
                                      _ptr(b), _ptr(x), _ptr(r)))
        return r

    def restrict_residual(self, b, x=None, level=0, adjoint=False):
        nrhs = self._vec(b, level)
        if x is not None:
            self._same(x, b, "x")
        cshape, _ = self.level_shape(level + 1)
        full = (self.dim + 1,) + cshape
        out = torch.empty(((nrhs,) if b.dim() == len(full) + 1 else ()) + full, dtype=b.dtype, device=b.device)
        L.check(self.lib.elh_restrict_residual(self.handle, level, self._flags(False, adjoint), _dtype_code(b),
                                               nrhs, _ptr(b), _ptr(x), _ptr(out)))
        return out

    def prolong_add(self, e, x, level=0):
        nrhs = self._vec(x, level)
        if self._vec(e, level + 1) != nrhs or e.dtype != x.dtype:
            raise ValueError("e must hold %s vectors on level %d for every right-hand side" % (x.dtype, level + 1))
        L.check(self.lib.elh_prolong_add(self.handle, level, _dtype_code(x), nrhs, _ptr(e), _ptr(x)))
        return x

    def relax(self, b, x, colour, level=0, adjoint=False):
        nrhs = self._vec(x, level)
        self._same(b, x, "b")
        L.check(self.lib.elh_relax(self.handle, level, self._flags(False, adjoint), _dtype_code(x), nrhs,
                                   colour, _ptr(b), _ptr(x)))
        return x

    def relax_noalloc(self, b, x, colour, level=0, adjoint=False):
        """relax() through the allocation-free entry point (residual work in
        the library's static per-GPU array; for callers that cannot allocate)"""
        nrhs = self._vec(x, level)
        self._same(b, x, "b")
        L.check(self.lib.elh_relax_noalloc(self.handle, level, self._flags(False, adjoint), _dtype_code(x), nrhs,
                                           colour, _ptr(b), _ptr(x)))
        return x

    def coarse_solve(self, b, adjoint=False):
        nrhs = self._vec(b, self.levels - 1)
        x = torch.empty_like(b)
        L.check(self.lib.elh_coarse_solve(self.handle, self._flags(False, adjoint), _dtype_code(b), nrhs,
                                          _ptr(b), _ptr(x)))
        return x

    def kaczmarz(self, b, sweeps, adjoint=False):
        """`sweeps` hybrid Kaczmarz sweeps from zero on the coarsest level's
        Schur complement system (the preconditioner of coarse_mode
        'kaczmarz'); pressure entries of b are ignored, of the result zero."""
        nrhs = self._vec(b, self.levels - 1)
        x = torch.empty_like(b)
        L.check(self.lib.elh_kaczmarz(self.handle, self._flags(False, adjoint), _dtype_code(b), nrhs, sweeps,
                                      _ptr(b), _ptr(x)))
        return x

    def vcycle(self, b, adjoint=False):
        nrhs = self._vec(b, 0)
        x = torch.empty_like(b)
        L.check(self.lib.elh_vcycle(self.handle, self._flags(False, adjoint), _dtype_code(b), nrhs,
                                    _ptr(b), _ptr(x)))
        return x

    # -- solves ---------------------------------------------------------------
    def _opts(self, restart, maxit, rtol, x0, store_z_fp32):
        if store_z_fp32 is None:
            store_z_fp32 = self.desc.precond_dtype == L.ELH_C64
        return L.SolveOpts(restart, maxit, rtol, 0 if x0 else 1, 1 if store_z_fp32 else 0)

    def _solve(self, fn, q, restart, maxit, rtol, out, x0=None, store_z_fp32=None):
        if q.dtype != torch.complex128:
            raise TypeError("right-hand sides must be complex128")
        nrhs = self._vec(q, 0)
        u = torch.empty_like(q) if out is None else self._same(out, q, "out")
        if x0 is not None:
            self._same(x0, q, "x0")
            if x0.data_ptr() != u.data_ptr():
                u.copy_(x0)
        opts = self._opts(restart, maxit, rtol, x0 is not None, store_z_fp32)
        stats = (L.SolveStats * nrhs)()
        hist = [(ctypes.c_double * maxit)() for _ in range(nrhs)]
        for s, h in zip(stats, hist):
            s.history = ctypes.cast(h, ctypes.POINTER(ctypes.c_double))
            s.history_cap = maxit
        code = L.check(fn(self.handle, nrhs, _ptr(q), _ptr(u), ctypes.byref(opts), stats))
        return u, [_info(s) for s in stats], code

    def solve(self, q, restart=5, maxit=500, rtol=1e-6, out=None, x0=None, store_z_fp32=None):
        """u = H^{-1} q by preconditioned FGMRES; returns (u, info, code).
        x0: initial guess (default zero; e.g. the u of an earlier call that
        returned code 1 to resume it; may be `out` itself).  store_z_fp32:
        keep the preconditioned vectors in complex64 (default: with the
        float32 cycle)."""
        return self._solve(self.lib.elh_solve, q, restart, maxit, rtol, out, x0, store_z_fp32)

    def solve_adjoint(self, r, restart=5, maxit=500, rtol=1e-6, out=None, x0=None, store_z_fp32=None):
        return self._solve(self.lib.elh_solve_adjoint, r, restart, maxit, rtol, out, x0, store_z_fp32)

    @staticmethod
    def solve_batch(problems, qs, restart=5, maxit=500, rtol=1e-6):
        """Solve independent problems together: the library drives them from
        the calling thread, one iteration of each in flight (create the
        problems on different streams so their kernels overlap).  Returns
        (list of u, list of info lists, code)."""
        if len(problems) != len(qs) or not problems:
            raise ValueError("one right-hand-side batch per problem")
        lib = problems[0].lib
        n = len(problems)
        us, nr = [], []
        for p, q in zip(problems, qs):
            if q.dtype != torch.complex128:
                raise TypeError("right-hand sides must be complex128")
            nr.append(p._vec(q, 0))
            us.append(torch.empty_like(q))
        hs = (ctypes.c_void_p * n)(*[p.handle.value for p in problems])
        nrh = (ctypes.c_int * n)(*nr)
        qp = (ctypes.c_void_p * n)(*[q.data_ptr() for q in qs])
        up = (ctypes.c_void_p * n)(*[u.data_ptr() for u in us])
        z32 = all(p.desc.precond_dtype == L.ELH_C64 for p in problems)
        opts = L.SolveOpts(restart, maxit, rtol, 1, 1 if z32 else 0)
        stats = (L.SolveStats * sum(nr))()
        hist = [(ctypes.c_double * maxit)() for _ in range(sum(nr))]
        for s, h in zip(stats, hist):
            s.history = ctypes.cast(h, ctypes.POINTER(ctypes.c_double))
            s.history_cap = maxit
        code = L.check(lib.elh_solve_batch(n, hs, nrh, qp, up, ctypes.byref(opts), stats))
        infos, k = [], 0
        for r in nr:
            infos.append([_info(s) for s in stats[k:k + r]])
            k += r
        return us, infos, code

    # -- receivers (misfit and adjoint source) --------------------------------
    def receiver_indices(self, mask):
        """int64 storage indices (into one level-0 vector) of the True
        entries of a boolean receiver mask of the vector's shape."""
        full = (self.dim + 1,) + self.shape
        if mask.dtype != torch.bool or tuple(mask.shape) != full:
            raise ValueError("receiver mask must be a bool tensor of shape %s" % (full,))
        return torch.nonzero(mask.reshape(-1)).reshape(-1).to(device=self.device, dtype=torch.int64)

    def _idx(self, idx):
        if (idx.dtype != torch.int64 or idx.dim() != 1 or idx.numel() < 1 or not idx.is_cuda
                or idx.device != self.device or not idx.is_contiguous()):
            raise ValueError("receiver indices must be a non-empty contiguous int64 vector on %s" % self.device)
        return idx

    def receivers(self, u, idx, d_obs=None, misfit=False):
        """d = P_r u - d_obs (d_obs optional), shape (nrhs, nrec); with
        misfit=True also phi (nrhs + 1 float64: 1/2 |d_s|^2 per source,
        then their total)."""
        if u.dtype != torch.complex128:
            raise TypeError("wavefields must be complex128")
        nrhs = self._vec(u, 0)
        idx = self._idx(idx)
        d = torch.empty((nrhs, idx.numel()), dtype=torch.complex128, device=self.device)
        if d_obs is not None:
            if d_obs.dim() == 1 and u.dim() == self.dim + 1:
                d_obs = d_obs.reshape(1, -1)
            self._same(d_obs, d, "d_obs")
        phi = torch.empty(nrhs + 1, dtype=torch.float64, device=self.device) if misfit else None
        L.check(self.lib.elh_receivers(self.handle, nrhs, _ptr(u), idx.numel(), _ptr(idx), _ptr(d_obs), _ptr(d),
                                       _ptr(phi)))
        if u.dim() == self.dim + 1:
            d = d[0]
        return (d, phi) if misfit else d

    def inject(self, r, idx, scale=1.0):
        """v = scale P_r^T r: zero vectors with r at the receivers; r has
        shape (nrhs, nrec) (or (nrec,) for one vector)."""
        idx = self._idx(idx)
        if r.dtype != torch.complex128 or not r.is_cuda or r.device != self.device or not r.is_contiguous():
            raise ValueError("receiver values must be a contiguous complex128 tensor on %s" % self.device)
        one = r.dim() == 1
        if r.shape[-1] != idx.numel() or r.dim() not in (1, 2):
            raise ValueError("receiver values must have shape (nrhs, %d)" % idx.numel())
        nrhs = 1 if one else r.shape[0]
        full = (self.dim + 1,) + self.shape
        v = torch.empty(full if one else (nrhs,) + full, dtype=torch.complex128, device=self.device)
        L.check(self.lib.elh_inject(self.handle, nrhs, idx.numel(), _ptr(idx), _ptr(r), float(scale), _ptr(v)))
        return v

    def gradient(self, u, v):
        if u.dtype != torch.complex128:
            raise TypeError("forward fields must be complex128")
        nrhs = self._vec(u, 0)
        self._same(v, u, "v")
        g = [torch.empty(self.shape, dtype=torch.float64, device=self.device) for _ in range(3)]
        L.check(self.lib.elh_gradient(self.handle, nrhs, _ptr(u), _ptr(v), _ptr(g[0]), _ptr(g[1]), _ptr(g[2])))
        return tuple(g)


class Batch:
    """Problems of uneven grid sizes solved together (elh_batch_*): each
    problem gets a library-owned stream, and solve() drives all of them from
    the calling thread, one iteration of each in flight, so their kernels
    overlap on the GPU.

    problems: list of dicts with keys lam, mu, rho (float64 tensors, numpy
    grid shape) and the Problem keyword parameters.  problem(i) returns a
    Problem view of problem i (owned by the batch) for the other entry
    points."""

    def __init__(self, problems, device=None):
        self.lib = L.load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if not problems:
            raise ValueError("a batch needs at least one problem")
        n = len(problems)
        self._media, descs, self._shapes = [], (L.Desc * n)(), []
        for i, pr in enumerate(problems):
            pr = dict(pr)
            media = _media(pr.pop("lam"), pr.pop("mu"), pr.pop("rho"), self.device)
            self._media.append(media)
            self._shapes.append(tuple(media[0].shape))
            descs[i] = _desc(self._shapes[-1], **pr)
        self._descs = descs
        ptrs = [(ctypes.c_void_p * n)(*[m[k].data_ptr() for m in self._media]) for k in range(3)]
        self.handle = ctypes.c_void_p(0)
        with torch.cuda.device(self.device):
            st = torch.cuda.current_stream(self.device).cuda_stream
            L.check(self.lib.elh_batch_create(n, descs, ptrs[0], ptrs[1], ptrs[2], ctypes.c_void_p(st),
                                              ctypes.byref(self.handle)))
        self._views = [None] * n

    def __len__(self):
        return len(self._shapes)

    def problem(self, i):
        if self._views[i] is None:
            h = ctypes.c_void_p(0)
            L.check(self.lib.elh_batch_handle(self.handle, i, ctypes.byref(h)))
            p = object.__new__(Problem)
            p.lib, p.device, p.shape = self.lib, self.device, self._shapes[i]
            p.dim, p.desc, p.levels = len(p.shape), self._descs[i], self._descs[i].levels
            p._media, p._owner, p.handle = self._media[i], self, h
            self._views[i] = p
        return self._views[i]

    def solve(self, qs, restart=5, maxit=500, rtol=1e-6, store_z_fp32=None):
        """u_i = H_i^{-1} q_i for every problem; returns (list of u, list of
        info lists, code)."""
        n = len(self)
        if len(qs) != n:
            raise ValueError("one right-hand-side batch per problem")
        us, nr = [], []
        for i, q in enumerate(qs):
            if q.dtype != torch.complex128:
                raise TypeError("right-hand sides must be complex128")
            nr.append(self.problem(i)._vec(q, 0))
            us.append(torch.empty_like(q))
        if store_z_fp32 is None:
            store_z_fp32 = all(d.precond_dtype == L.ELH_C64 for d in self._descs)
        opts = L.SolveOpts(restart, maxit, rtol, 1, 1 if store_z_fp32 else 0)
        stats = (L.SolveStats * sum(nr))()
        hist = [(ctypes.c_double * maxit)() for _ in range(sum(nr))]
        for s, h in zip(stats, hist):
            s.history = ctypes.cast(h, ctypes.POINTER(ctypes.c_double))
            s.history_cap = maxit
        qp = (ctypes.c_void_p * n)(*[q.data_ptr() for q in qs])
        up = (ctypes.c_void_p * n)(*[u.data_ptr() for u in us])
        code = L.check(self.lib.elh_batch_solve(self.handle, (ctypes.c_int * n)(*nr), qp, up, ctypes.byref(opts),
                                                stats))
        infos, k = [], 0
        for r in nr:
            infos.append([_info(s) for s in stats[k:k + r]])
            k += r
        return us, infos, code

    def close(self):
        if self.handle and self.handle.value:
            for v in self._views:
                if v is not None:
                    v.handle = ctypes.c_void_p(0)
            self.lib.elh_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
