"""Grid, 1D operators and Kronecker helpers of the MAC discretization.

Test infrastructure (see the package header).

MAC staggered grid (Section 2.3, Figure 1a): n_k cells of width h along
each axis x_k; the pressure p sits at cell centres, displacement u_k on the
faces normal to x_k.  Faces along x_k are numbered 0..n_k; faces 0 and n_k
lie on the domain boundary.  Boundary conditions are not stated in the
paper; the reading used here (and by the GPU library) is:
  * normal displacement is zero on boundary faces (they are not unknowns);
  * any value outside the arrays (tangential neighbours, pressure, averaged
    neighbours) reads as zero;
  * media are replicated (clamped) outward when averaged onto boundary
    edges.

Vectors: "storage" layout is numpy shape (d+1, n_d, ..., n_1) with the x_k
axis of field u_k holding faces 0..n_k-1 (face 0 stored as zero).  The
sparse operators act on the "compact" vector: for each field the interior
unknowns only (faces 1..n_k-1 along x_k), fields concatenated u_1..u_d, p,
each flattened in C order (x_1 fastest).

Numpy axis of coordinate x_k (k = 1..d) is  dim - k.
"""
import numpy as np
import scipy.sparse as sp


# ----------------------------------------------------------------------------
# problem description
# ----------------------------------------------------------------------------
class Level:
    """Parameters and media of one grid level.

    n      : cells per axis in x-order (n_1, ..., n_d)
    h      : grid spacing
    omega  : angular frequency; gamma: physical attenuation (eq. 2.1-2.3)
    beta   : spread weight of the compact stencils (eq. dxSpread, 3D form)
    abl_width : absorbing-layer width in physical units; abl_amp: its peak
    lam, mu, rho : cell-centred media, numpy shape (n_d, ..., n_1)
    """

    def __init__(self, n, h, omega, gamma, beta, lam, mu, rho,
                 abl_width=0.0, abl_amp=0.0):
        self.n = tuple(int(v) for v in n)
        self.dim = len(self.n)
        self.h = float(h)
        self.omega = float(omega)
        self.gamma = float(gamma)
        self.beta = float(beta)
        self.abl_width = float(abl_width)
        self.abl_amp = float(abl_amp)
        shp = self.np_shape
        self.lam = np.asarray(lam, dtype=np.float64).reshape(shp)
        self.mu = np.asarray(mu, dtype=np.float64).reshape(shp)
        self.rho = np.asarray(rho, dtype=np.float64).reshape(shp)

    @property
    def np_shape(self):
        return tuple(reversed(self.n))

    def axis(self, k):
        """numpy axis of coordinate x_k (1-based k)."""
        return self.dim - k

    def field_shape(self, f):
        """compact numpy shape of field f (0..d-1: u_{f+1}; d: p)."""
        shp = list(self.np_shape)
        if f < self.dim:
            shp[self.axis(f + 1)] -= 1
        return tuple(shp)

    def field_sizes(self):
        return [int(np.prod(self.field_shape(f))) for f in range(self.dim + 1)]

    def nunknowns(self):
        return int(sum(self.field_sizes()))


# ----------------------------------------------------------------------------
# storage <-> compact
# ----------------------------------------------------------------------------
def pack(lv, x):
    """storage (d+1, n_d..n_1) -> compact 1D vector (interior unknowns)."""
    parts = []
    for f in range(lv.dim + 1):
        a = x[f]
        if f < lv.dim:
            idx = [slice(None)] * lv.dim
            idx[lv.axis(f + 1)] = slice(1, None)
            a = a[tuple(idx)]
        parts.append(np.ascontiguousarray(a).ravel())
    return np.concatenate(parts)


def unpack(lv, v):
    """compact 1D vector -> storage array with zero boundary faces."""
    out = np.zeros((lv.dim + 1,) + lv.np_shape, dtype=np.result_type(v, np.complex128))
    off = 0
    for f in range(lv.dim + 1):
        shp = lv.field_shape(f)
        sz = int(np.prod(shp))
        a = v[off:off + sz].reshape(shp)
        off += sz
        if f < lv.dim:
            idx = [slice(None)] * lv.dim
            idx[lv.axis(f + 1)] = slice(1, None)
            out[f][tuple(idx)] = a
        else:
            out[f] = a
    return out


def field_views(lv, v):
    """split a compact vector into per-field arrays of compact shape."""
    out, off = [], 0
    for f in range(lv.dim + 1):
        shp = lv.field_shape(f)
        sz = int(np.prod(shp))
        out.append(v[off:off + sz].reshape(shp))
        off += sz
    return out


# ----------------------------------------------------------------------------
# 1D matrices (n = number of cells along the axis)
# ----------------------------------------------------------------------------
def d_int(n, h):
    """Standard staggered derivative (1/h)[-1 * 1] (eq. dxdyStandard) from
    the interior faces 1..n-1 to the n cells; boundary faces are zero.
    Cell c sits between faces c and c+1."""
    m = sp.lil_matrix((n, n - 1))
    for c in range(n):
        if c + 1 <= n - 1:
            m[c, c] = 1.0 / h          # face c+1 -> column c
        if c >= 1:
            m[c, c - 1] = -1.0 / h     # face c   -> column c-1
    return m.tocsr()


def g_full(n, h):
    """Standard staggered derivative from the n cells to all n+1 faces,
    with zero values outside the domain: (g p)_f = (p_f - p_{f-1})/h."""
    m = sp.lil_matrix((n + 1, n))
    for f in range(n + 1):
        if f <= n - 1:
            m[f, f] = 1.0 / h
        if f >= 1:
            m[f, f - 1] = -1.0 / h
    return m.tocsr()


def g_int(n, h):
    """Rows 1..n-1 of g_full: cell -> interior-face derivative."""
    return g_full(n, h)[1:n, :]


def avg121(m):
    """(1/4)[1 2 1] averaging on m points, zero outside (the transverse
    weights of the beta-spread derivative, eq. dxSpread and its 3D form)."""
    return sp.diags([np.full(m - 1, 0.25), np.full(m, 0.5), np.full(m - 1, 0.25)],
                    [-1, 0, 1], shape=(m, m), format="csr")


def nbr_sum(m):
    """sum of the two neighbours on m points, zero outside."""
    return sp.diags([np.ones(m - 1), np.ones(m - 1)], [-1, 1], shape=(m, m),
                    format="csr")


def face_mean(n):
    """interior face f (1..n-1) <- mean of the two adjacent cells f-1, f."""
    m = sp.lil_matrix((n - 1, n))
    for f in range(1, n):
        m[f - 1, f - 1] = 0.5
        m[f - 1, f] = 0.5
    return m.tocsr()


def face_mean_clamped(n):
    """every face f (0..n) <- mean of cells clamp(f-1), clamp(f)."""
    m = sp.lil_matrix((n + 1, n))
    for f in range(n + 1):
        a = min(max(f - 1, 0), n - 1)
        b = min(max(f, 0), n - 1)
        m[f, a] += 0.5
        m[f, b] += 0.5
    return m.tocsr()


def eye(m):
    return sp.identity(m, format="csr")


# ----------------------------------------------------------------------------
# Kronecker helpers
# ----------------------------------------------------------------------------
def kron_axes(lv, mats, sizes):
    """Full sparse operator acting with mats[k] along coordinate x_k and the
    identity of size sizes[k] along the others.  C-order flattening with x_1
    fastest means the product is  M_d (x) ... (x) M_1."""
    out = None
    for k in range(lv.dim, 0, -1):
        m = mats.get(k)
        if m is None:
            m = eye(sizes[k])
        out = m if out is None else sp.kron(out, m, format="csr")
    return out.tocsr()


def apply_axes(lv, arr, mats):
    """Apply mats[k] along coordinate x_k of a numpy array, one axis at a
    time (the same product as kron_axes, without forming it)."""
    out = arr
    for k, m in mats.items():
        ax = lv.axis(k)
        moved = np.moveaxis(out, ax, 0)
        shp = moved.shape
        res = m @ moved.reshape(shp[0], -1)
        res = np.asarray(res).reshape((m.shape[0],) + shp[1:])
        out = np.moveaxis(res, 0, ax)
    return out


# ----------------------------------------------------------------------------
# DOF positions and absorbing layer
# ----------------------------------------------------------------------------
def dof_coords(lv, f):
    """Physical coordinates of the compact DOFs of field f, as a list of d
    arrays (x-order), each broadcastable to the compact field shape."""
    shp = lv.field_shape(f)
    coords = []
    for k in range(1, lv.dim + 1):
        ax = lv.axis(k)
        if f == k - 1:
            pos = np.arange(1, lv.n[k - 1]) * lv.h          # interior faces
        else:
            pos = (np.arange(lv.n[k - 1]) + 0.5) * lv.h      # cell centres
        sh = [1] * lv.dim
        sh[ax] = shp[ax]
        coords.append(pos.reshape(sh))
    return coords


def abl_profile(lv, coords):
    """Attenuation added by the absorbing layer at the given coordinates.

    The paper uses an absorbing layer of a fixed number of cells (Section 5)
    without giving its profile.  Reading used here: quadratic ramp
        gamma_abl(x) = A * sum_k (delta_k(x)/W)^2,
    delta_k = distance (physical) into the layer along x_k, W = layer width
    (physical), A = abl_amp; zero in the interior.
    """
    total = 0.0
    W = lv.abl_width
    if W <= 0 or lv.abl_amp == 0:
        return np.zeros(np.broadcast_shapes(*[c.shape for c in coords]))
    for k in range(1, lv.dim + 1):
        L = lv.n[k - 1] * lv.h
        x = coords[k - 1]
        dlt = np.maximum(0.0, W - x) + np.maximum(0.0, x - (L - W))
        total = total + lv.abl_amp * (dlt / W) ** 2
    return total + np.zeros(np.broadcast_shapes(*[c.shape for c in coords]))
