"""Closed-form Fourier symbols of the constant-coefficient operators.

Test infrastructure (see the package header).

For constant media and no absorbing layer, eq. (mixed-discretized-homogeneous)
(and its 3D analogue) acts on a plane wave exp(i theta.x/h), sampled at each
DOF's own physical position, as multiplication by a (d+1)x(d+1) matrix.
Each entry follows directly from the printed stencils:
  * standard staggered difference (1/h)[-1 * 1]:     g_k = (2i/h) sin(theta_k/2)
  * beta-spread difference (eq. dxSpread / dxSkew3D): g_k * s_k,
      s_k = beta + (1-beta) * prod_{m != k} (1 + cos theta_m)/2
  * Laplacian grad^T grad^beta (eq. LapHO):  sum_k (4/h^2) sin^2(theta_k/2) s_k
  * spread mass (eq. massHO / massHO3D):
      omega^2 (1 - i gamma) (beta + (1-beta)/d * sum_k cos theta_k)
  * rows u_k: mu*Lap - rho*mass on the diagonal, g_k in the p column
    (coupling reading: the standard cell-to-face difference);
    row p: g_k s_k in the u_k columns, 1/(lam+mu) on the diagonal.
Transfers (Section 2.3 stencils; symbol of a restriction stencil is the sum
of weight*exp(i theta.offset/h); prolongation uses the transposed stencil):
  R_{u_k} = (1+cos theta_k)/2 * prod_{m != k} cos(theta_m/2)
  R_p     = prod_m cos(theta_m/2)
  P_{u_k} = (1+cos theta_k) * prod_{m != k} (3 cos(theta_m/2) + cos(3 theta_m/2))/2
  P_p     = prod_m (3 cos(theta_m/2) + cos(3 theta_m/2))/2
(eq. Ru1Symbol prints R_{u_1} without its 1/8 factor and with a dropped
'+'; its value times 1/8 equals the formula above.)
theta is a d-vector, or a (d, m) array of m frequencies; the results then
carry a trailing axis of length m.
"""
import numpy as np


def spread_factors(theta, beta):
    th = np.asarray(theta, dtype=np.float64)
    d = th.shape[0]
    s = []
    for k in range(d):
        prod = 1.0
        for m in range(d):
            if m != k:
                prod = prod * (1.0 + np.cos(th[m])) / 2.0
        s.append(beta + (1.0 - beta) * prod)
    return s


def operator_symbol(theta, h, omega, gamma, beta, lam, mu, rho):
    """(d+1)x(d+1) symbol of H^beta (gamma includes any shift)."""
    th = np.asarray(theta, dtype=np.float64)
    d = th.shape[0]
    s = spread_factors(th, beta)
    g = [2j / h * np.sin(th[k] / 2.0) for k in range(d)]
    lap = sum(4.0 / h ** 2 * np.sin(th[k] / 2.0) ** 2 * s[k] for k in range(d))
    mass = omega ** 2 * (1 - 1j * gamma) * (beta + (1 - beta) / d * sum(np.cos(th[k]) for k in range(d)))
    H = np.zeros((d + 1, d + 1) + th.shape[1:], dtype=np.complex128)
    for k in range(d):
        H[k, k] = mu * lap - rho * mass
        H[k, d] = g[k]
        H[d, k] = g[k] * s[k]
    H[d, d] = 1.0 / (lam + mu)
    return H


def restriction_symbol(theta):
    th = np.asarray(theta, dtype=np.float64)
    d = th.shape[0]
    out = np.zeros((d + 1,) + th.shape[1:])
    for f in range(d + 1):
        v = 1.0
        for m in range(d):
            v *= (1.0 + np.cos(th[m])) / 2.0 if m == f else np.cos(th[m] / 2.0)
        out[f] = v
    return out


def prolongation_symbol(theta):
    th = np.asarray(theta, dtype=np.float64)
    d = th.shape[0]
    out = np.zeros((d + 1,) + th.shape[1:])
    for f in range(d + 1):
        v = 1.0
        for m in range(d):
            if m == f:
                v *= 1.0 + np.cos(th[m])
            else:
                v *= (3.0 * np.cos(th[m] / 2.0) + np.cos(1.5 * th[m])) / 2.0
        out[f] = v
    return out
