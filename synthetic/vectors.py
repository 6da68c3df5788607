"""Seeded vectors in the MAC storage layout.

Storage layout of one vector (one right-hand side): complex array of numpy
shape (d+1, n_d, ..., n_1) holding fields u_1..u_d, p.  Field u_k lives on
the faces normal to x_k; its entry with index 0 along x_k is the domain
boundary face, which is not an unknown and is held at zero.  A batch adds a
leading axis: (nrhs, d+1, n_d, ..., n_1).
"""
import numpy as np


def zero_boundary_faces(x):
    """Zero the boundary-face entries (index 0 along x_k for field u_k).

    Works on (d+1, ...) or (nrhs, d+1, ...) arrays; returns x (modified).
    """
    for dim in (2, 3):
        if x.ndim in (dim + 1, dim + 2) and x.shape[x.ndim - dim - 1] == dim + 1:
            break
    else:
        raise ValueError("cannot infer dimension from shape %s" % (x.shape,))
    fax = x.ndim - dim - 1
    for k in range(1, dim + 1):
        idx = [slice(None)] * x.ndim
        idx[fax] = k - 1
        idx[x.ndim - k] = 0          # x_k is the k-th numpy axis from the end
        x[tuple(idx)] = 0
    return x


def random_field(shape, seed, nrhs=None, dtype=np.complex128):
    """Standard complex normal vector in storage layout, boundary faces zero.

    shape: spatial numpy shape (n_d, ..., n_1).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    dim = len(shape)
    full = (dim + 1,) + tuple(shape)
    if nrhs is not None:
        full = (nrhs,) + full
    x = rng.standard_normal(full) + 1j * rng.standard_normal(full)
    x = x.astype(dtype)
    return zero_boundary_faces(x)


def point_source(shape, component=None, position=None, dtype=np.complex128):
    """Unit impulse on one displacement component at one face.

    Default: the last-axis component u_d at the face nearest the domain
    centre (face index n_k//2 along x_k, cell n//2 along the others).
    position is given in numpy order (i_d, ..., i_1).
    """
    dim = len(shape)
    if component is None:
        component = dim
    if position is None:
        position = tuple(s // 2 for s in shape)
    q = np.zeros((dim + 1,) + tuple(shape), dtype=dtype)
    q[(component - 1,) + tuple(position)] = 1.0
    return q


def lattice_sources(shape, rows, cols, depth_index, component=None,
                    margin=0, dtype=np.complex128):
    """rows x cols point sources on the x_1-x_2 plane at depth index
    `depth_index` (3D), evenly spaced over the interior [margin, n-margin).
    Returns (rows*cols, 4, n3, n2, n1)."""
    assert len(shape) == 3
    n3, n2, n1 = shape
    if component is None:
        component = 3
    i2s = np.linspace(margin, n2 - margin, rows + 2)[1:-1].round().astype(int)
    i1s = np.linspace(margin, n1 - margin, cols + 2)[1:-1].round().astype(int)
    out = np.zeros((rows * cols, 4, n3, n2, n1), dtype=dtype)
    s = 0
    for a in i2s:
        for b in i1s:
            out[s, component - 1, depth_index, a, b] = 1.0
            s += 1
    return out


def receiver_plane_mask(shape, depth_index):
    """Boolean mask (4, n3, n2, n1) selecting every interior u-face on the
    x_1-x_2 plane at depth index `depth_index` (receivers record u_1..u_3)."""
    assert len(shape) == 3
    m = np.zeros((4,) + tuple(shape), dtype=bool)
    m[0:3, depth_index] = True
    zero = np.ones((4,) + tuple(shape))
    zero_boundary_faces(zero)
    return m & (zero != 0)


def plane_wave_field(shape, theta, amp, h=1.0, dtype=np.complex128):
    """Plane wave exp(i theta . x / h) sampled at each DOF's physical
    position, with per-field amplitudes `amp` (length d+1).

    theta is given in x-order (theta_1, ..., theta_d).  u_k sits at the face
    position i_k*h along x_k and at cell centres (i+1/2)h along the others;
    p at cell centres.  Boundary faces are zeroed.
    """
    dim = len(shape)
    out = np.zeros((dim + 1,) + tuple(shape), dtype=dtype)
    for f in range(dim + 1):
        phase = 0.0
        for k in range(1, dim + 1):
            n = shape[dim - k]
            pos = np.arange(n) + (0.0 if f == k - 1 else 0.5)
            sh = [1] * dim
            sh[dim - k] = n
            phase = phase + theta[k - 1] * pos.reshape(sh)
        out[f] = amp[f] * np.exp(1j * phase)
    return zero_boundary_faces(out)
