"""The discrete mixed elastic Helmholtz operator H^beta.

Test infrastructure (see the package header).

Follows eq. (mixed-discretized) in Section 3.1, its 3D extension in
Section 5.3 (eq. dxSkew3D, massHO3D) and the shift of Section 2.2:

    H^beta = [ grad_h^T A_e(mu) grad^beta_h - M^beta A_f(rho)   C      ]
             [ (div)^beta_h                              diag(1/(lam+mu)) ]

per displacement component u_k (block diagonal in k), with
  * grad^beta_h: the beta-spread first derivatives; along x_l the standard
    two-point difference (1/h)[-1 * 1] mixed with weight (1-beta) with the
    same difference averaged over every other axis by (1/4)[1 2 1]
    (eq. dxSpread in 2D; the 1/16 [1 2 1]x[1 2 1] weights of eq. dxSkew3D
    in 3D, with the 1/h the 3D formula omits);
  * grad_h^T: the transpose of the standard derivative (so grad^T grad^beta
    = -Laplacian^beta, eq. LapHO);
  * A_e(mu): mu averaged onto the flux location -- the cell itself for the
    derivative of u_k along x_k, the mean of the four cells around the edge
    otherwise (arithmetic mean; the paper states no formula);
  * M^beta A_f(rho): rho averaged onto faces (mean of the two cells), then
    the spread mass beta*I + (1-beta)/(2d) * (sum of the 2d face
    neighbours) (eq. massHO, massHO3D), then the factor
    omega^2 (1 - i gamma~) taken at the output face, gamma~ = gamma + alpha
    (shifted operator) + absorbing-layer profile;
  * C: coupling of u_k to p.  The paper writes (div)_h^T in eq.
    mixed-discretized and (d/dx_k)_{h/2} in the constant-coefficient form
    (eq. mixed-discretized-homogeneous); the latter -- the standard
    cell-to-face difference (p_right - p_left)/h -- is the reading used
    (it is the sign for which eliminating p yields
    -div mu grad - grad (lam+mu) div - rho omega^2, i.e. eq. 2.3 negated,
    consistently with the negated Laplacian block);
  * (div)^beta_h: the beta-spread divergence (standard difference along
    x_k spread over the other axes), rows at cell centres.

Two evaluations of the same term list are provided:
  assemble(lv, ...)  -- explicit scipy.sparse matrix (Kronecker products),
  apply(lv, x, ...)  -- the same 1D factors applied axis by axis.
"""
import numpy as np
import scipy.sparse as sp

from . import grid as G


def _sizes_u(lv, k):
    """grid sizes (x-order dict) of field u_k: interior faces along x_k."""
    return {a: (lv.n[a - 1] - 1 if a == k else lv.n[a - 1]) for a in range(1, lv.dim + 1)}


def _sizes_c(lv):
    return {a: lv.n[a - 1] for a in range(1, lv.dim + 1)}


def _spread_deriv_mats(lv, k, l):
    """1D factor lists of the beta-spread derivative of u_k along x_l:
    returns (D_l, [(coef, mats), ...])."""
    su = _sizes_u(lv, k)
    Dl = G.d_int(lv.n[l - 1], lv.h) if l == k else G.g_full(lv.n[l - 1], lv.h)
    t1 = (lv.beta, {l: Dl})
    m2 = {l: Dl}
    for a in range(1, lv.dim + 1):
        if a != l:
            m2[a] = G.avg121(su[a])
    t2 = (1.0 - lv.beta, m2)
    return Dl, [t1, t2]


def _flux_shape(lv, k, l):
    su = _sizes_u(lv, k)
    shp = {a: su[a] for a in su}
    shp[l] = lv.n[l - 1] if l == k else lv.n[l - 1] + 1
    return tuple(shp[a] for a in range(lv.dim, 0, -1))


def edge_mu(lv, k, l):
    """A_e(mu) on the flux grid of (u_k, d/dx_l): cell mu for l == k,
    the clamped four-cell mean on edges otherwise (numpy array)."""
    if l == k:
        return lv.mu
    mats = {k: G.face_mean(lv.n[k - 1]), l: G.face_mean_clamped(lv.n[l - 1])}
    return G.apply_axes(lv, lv.mu, mats)


def face_rho(lv, k):
    """A_f(rho) on the interior k-faces (numpy array, compact u_k shape)."""
    return G.apply_axes(lv, lv.rho, {k: G.face_mean(lv.n[k - 1])})


def mass_factor(lv, f, shift):
    """omega^2 (1 - i (gamma + shift + gamma_abl)) at the DOFs of field f."""
    coords = G.dof_coords(lv, f)
    gt = lv.gamma + shift + G.abl_profile(lv, coords)
    return (lv.omega ** 2) * (1.0 - 1j * gt) * np.ones(lv.field_shape(f))


def kappa(lv):
    return 1.0 / (lv.lam + lv.mu)


# ----------------------------------------------------------------------------
# sparse assembly (tiny grids)
# ----------------------------------------------------------------------------
def assemble(lv, shift=0.0):
    """H^beta (shift = 0) or H^beta_s (shift = alpha) as a CSR matrix on the
    compact unknown vector."""
    d = lv.dim
    sc = _sizes_c(lv)
    blocks = [[None] * (d + 1) for _ in range(d + 1)]
    for k in range(1, d + 1):
        su = _sizes_u(lv, k)
        lap = None
        for l in range(1, d + 1):
            Dl, terms = _spread_deriv_mats(lv, k, l)
            sd = sum(c * G.kron_axes(lv, m, su) for c, m in terms)
            mu_e = sp.diags(np.ravel(edge_mu(lv, k, l)))
            DlT = G.kron_axes(lv, {l: Dl.T.tocsr()}, su)
            term = DlT @ mu_e @ sd
            lap = term if lap is None else lap + term
        nsum = sum(G.kron_axes(lv, {a: G.nbr_sum(su[a])}, su) for a in range(1, d + 1))
        spread_mass = lv.beta * sp.identity(nsum.shape[0]) + (1.0 - lv.beta) / (2 * d) * nsum
        mass = (sp.diags(np.ravel(mass_factor(lv, k - 1, shift))) @ spread_mass
                @ sp.diags(np.ravel(face_rho(lv, k))))
        blocks[k - 1][k - 1] = (lap - mass).tocsr()
        blocks[k - 1][d] = G.kron_axes(lv, {k: G.g_int(lv.n[k - 1], lv.h)}, sc)
        _, terms = _spread_deriv_mats(lv, k, k)
        blocks[d][k - 1] = sum(c * G.kron_axes(lv, m, su) for c, m in terms)
    blocks[d][d] = sp.diags(np.ravel(kappa(lv)))
    return sp.bmat(blocks, format="csr").astype(np.complex128)


# ----------------------------------------------------------------------------
# matrix-free evaluation of the same terms
# ----------------------------------------------------------------------------
def apply_fields(lv, u, shift=0.0, adjoint=False):
    """y = H u (or H^H u) on compact per-field arrays (list of d+1)."""
    d = lv.dim
    y = [None] * (d + 1)
    p = u[d]
    kap = kappa(lv)
    for k in range(1, d + 1):
        uk = u[k - 1]
        acc = np.zeros(lv.field_shape(k - 1), dtype=np.complex128)
        for l in range(1, d + 1):
            Dl, terms = _spread_deriv_mats(lv, k, l)
            mu_e = edge_mu(lv, k, l)
            if not adjoint:
                sd = sum(c * G.apply_axes(lv, uk, m) for c, m in terms)
                acc = acc + G.apply_axes(lv, mu_e * sd, {l: Dl.T.tocsr()})
            else:
                # (Dl^T mu S)^H = S^T mu Dl   (all factors real)
                g = mu_e * G.apply_axes(lv, uk, {l: Dl})
                acc = acc + sum(c * G.apply_axes(lv, g, {a: mm.T.tocsr() for a, mm in m.items()})
                                for c, m in terms)
        su = _sizes_u(lv, k)
        mf = mass_factor(lv, k - 1, shift)
        rf = face_rho(lv, k)

        def spread_mass(v):
            nb = sum(G.apply_axes(lv, v, {a: G.nbr_sum(su[a])}) for a in range(1, d + 1))
            return lv.beta * v + (1.0 - lv.beta) / (2 * d) * nb

        if not adjoint:
            acc = acc - mf * spread_mass(rf * uk)
            acc = acc + G.apply_axes(lv, p, {k: G.g_int(lv.n[k - 1], lv.h)})
        else:
            acc = acc - rf * spread_mass(np.conj(mf) * uk)   # nbr_sum symmetric
            _, terms = _spread_deriv_mats(lv, k, k)
            # coupling of u_k into the p-row transposes into the u_k row
            # (handled in the p loop below); here the p column of row u_k:
        y[k - 1] = acc
    if not adjoint:
        acc = kap * p
        for k in range(1, d + 1):
            _, terms = _spread_deriv_mats(lv, k, k)
            acc = acc + sum(c * G.apply_axes(lv, u[k - 1], m) for c, m in terms)
        y[d] = acc
    else:
        # row u_k of H^H gets (div^beta_k)^T p ; row p gets G_k^T u_k + kappa p
        acc = kap * p
        for k in range(1, d + 1):
            _, terms = _spread_deriv_mats(lv, k, k)
            y[k - 1] = y[k - 1] + sum(c * G.apply_axes(lv, p, {a: mm.T.tocsr() for a, mm in m.items()})
                                      for c, m in terms)
            acc = acc + G.apply_axes(lv, u[k - 1], {k: G.g_int(lv.n[k - 1], lv.h).T.tocsr()})
        y[d] = acc
    return y


def apply(lv, x, shift=0.0, adjoint=False):
    """Matrix-free y = H^beta_(s) x on storage-layout arrays (d+1, n_d..n_1),
    or a batch (nrhs, d+1, ...).  Boundary-face entries of x are ignored;
    those of y are zero."""
    if x.ndim == lv.dim + 2:
        return np.stack([apply(lv, xi, shift, adjoint) for xi in x])
    comp = G.field_views(lv, G.pack(lv, x))
    y = apply_fields(lv, comp, shift, adjoint)
    return G.unpack(lv, np.concatenate([np.ravel(a) for a in y]))
