"""Adjoint solve, FWI-style misfit and parameter gradient.

Test infrastructure (see the package header).

The paper motivates the solver as the forward engine of frequency-domain
full waveform inversion (Section 1; the jInv implementation of Section 5)
but does not state the gradient.  The standard adjoint-state form for the
discrete model H(m) u_s = q_s (eq. mixed-discretized, for every medium) is
used:
    Phi(m)      = 1/2 sum_s || P_r u_s - d_s ||^2
    H^H v_s     = P_r^T (P_r u_s - d_s)
    dPhi/dm_c   = - Re sum_s v_s^H (dH/dm_c) u_s ,   m in {lam, mu, rho}.
H depends on mu through A_e(mu) (cell value or edge mean) and through
kappa = 1/(lam+mu); on lam through kappa only; on rho through A_f(rho)
(face mean).  The matrix-free gradient below contracts the products of
the same flux/mass factors with the transposed averaging maps.
"""
import numpy as np

from . import grid as G
from . import operator as O


def misfit(u, d, mask):
    """Phi for a batch u, d of storage arrays (nsrc, d+1, ...) and a
    boolean receiver mask of shape (d+1, ...)."""
    r = np.where(mask[None], u - d, 0.0)
    return 0.5 * float(np.sum(np.abs(r) ** 2))


def adjoint_source(u, d, mask):
    """P_r^T (P_r u - d) (storage layout)."""
    return np.where(mask[None], u - d, 0.0)


def gradient(lv, u, v):
    """(g_lam, g_mu, g_rho), each numpy shape (n_d..n_1), for forward
    fields u and adjoint fields v (storage layout, batch or single)."""
    if u.ndim == lv.dim + 1:
        u, v = u[None], v[None]
    d = lv.dim
    kap = O.kappa(lv)
    g_lam = np.zeros(lv.np_shape)
    g_mu = np.zeros(lv.np_shape)
    g_rho = np.zeros(lv.np_shape)
    for s in range(u.shape[0]):
        uc = G.field_views(lv, G.pack(lv, u[s]))
        vc = G.field_views(lv, G.pack(lv, v[s]))
        # kappa block: dkappa/dlam = dkappa/dmu = -kappa^2
        kterm = -np.real(np.conj(vc[d]) * (-kap ** 2) * uc[d])
        g_lam += kterm
        g_mu += kterm
        for k in range(1, d + 1):
            for l in range(1, d + 1):
                Dl, terms = O._spread_deriv_mats(lv, k, l)
                sd = sum(c * G.apply_axes(lv, uc[k - 1], m) for c, m in terms)
                prod = np.conj(G.apply_axes(lv, vc[k - 1], {l: Dl})) * sd
                if l == k:
                    back = prod
                else:
                    E = {k: G.face_mean(lv.n[k - 1]), l: G.face_mean_clamped(lv.n[l - 1])}
                    back = G.apply_axes(lv, prod, {a: m.T.tocsr() for a, m in E.items()})
                g_mu += -np.real(back)
            # mass: - diag(mf) S diag(F rho);  w = S (conj(mf) v)
            su = O._sizes_u(lv, k)
            mf = O.mass_factor(lv, k - 1, 0.0)
            t = np.conj(mf) * vc[k - 1]
            nb = sum(G.apply_axes(lv, t, {a: G.nbr_sum(su[a])}) for a in range(1, d + 1))
            w = lv.beta * t + (1 - lv.beta) / (2 * d) * nb
            prod = np.conj(w) * uc[k - 1]
            back = G.apply_axes(lv, prod, {k: G.face_mean(lv.n[k - 1]).T.tocsr()})
            g_rho += np.real(back)
    return g_lam, g_mu, g_rho
