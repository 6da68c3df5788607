"""Seeded synthetic elastic media.

Layered earth with smooth Gaussian perturbations, the stand-in for the
geophysical models of the paper's numerical results (Marmousi-2, SEG
Overthrust), which are not available.  Shear velocity and density are tied
to the compressional velocity as in the 3D experiments section
(Vs proportional to Vp, density affine in Vp).  Lame parameters follow from
Vp = sqrt((lam + 2 mu)/rho) and Vs = sqrt(mu/rho) (Section 2.1).

Arrays are returned with numpy shape (n_d, ..., n_1): the first spatial
coordinate x_1 is the fastest-varying (last) numpy axis, x_d (depth) the
slowest.
"""
import numpy as np


def velocities_to_lame(vp, vs, rho):
    """Lame parameters from velocities and density (Section 2.1 relations)."""
    mu = rho * vs * vs
    lam = rho * vp * vp - 2.0 * mu
    return lam, mu


def omega_for_ppw(vs_min, h, ppw):
    """Angular frequency giving `ppw` grid points per minimal shear wavelength.

    The shear wavelength is 2*pi*Vs/omega; asking for ppw*h of it gives
    omega = 2*pi*Vs_min/(ppw*h)  (e.g. pi/(5h) for ppw=10 and Vs=1).
    """
    return 2.0 * np.pi * vs_min / (ppw * h)


def make_media(shape, seed, vp_range=(1.5, 4.5), vs_ratio=1.73,
               n_layers=6, n_blobs=8):
    """Layered + Gaussian-perturbed medium.

    shape: (n_d, ..., n_1) numpy shape (2D or 3D).
    Returns dict(lam, mu, rho, vp, vs) of float64 arrays with that shape.
    Recipe: `n_layers` layers along the depth axis (first numpy axis) with
    interfaces at sorted U(0.1, 0.9)*n_d and base Vp = linspace(1.8, 4.2) +
    U(-0.1, 0.1); `n_blobs` Gaussian blobs with centres uniform in the
    domain, width U(n/16, n/6) cells and relative amplitude U(-0.15, 0.15);
    Vp clipped to vp_range; Vs = Vp/vs_ratio; rho = 0.25 + 0.5 Vp.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    nd = shape[0]
    interfaces = np.sort(rng.uniform(0.1, 0.9, n_layers - 1) * nd)
    base = np.linspace(1.8, 4.2, n_layers) + rng.uniform(-0.1, 0.1, n_layers)
    depth = np.arange(nd) + 0.5
    layer_id = np.searchsorted(interfaces, depth)
    vp_depth = base[layer_id]
    bshape = [nd] + [1] * (dim - 1)
    vp = np.broadcast_to(vp_depth.reshape(bshape), shape).astype(np.float64).copy()
    nmean = float(np.mean(shape))
    pert = np.zeros(shape)
    for _ in range(n_blobs):
        centre = [rng.uniform(0, s) for s in shape]
        sigma = rng.uniform(nmean / 16.0, nmean / 6.0)
        amp = rng.uniform(-0.15, 0.15)
        g = amp
        for ax, s in enumerate(shape):
            x = np.arange(s) + 0.5
            prof = np.exp(-((x - centre[ax]) ** 2) / (2.0 * sigma * sigma))
            sh = [1] * dim
            sh[ax] = s
            g = g * prof.reshape(sh)
        pert = pert + g
    vp = vp * (1.0 + pert)
    vp = np.clip(vp, vp_range[0], vp_range[1])
    vs = vp / vs_ratio
    rho = 0.25 + 0.5 * vp
    lam, mu = velocities_to_lame(vp, vs, rho)
    return dict(lam=lam, mu=mu, rho=rho, vp=vp, vs=vs)


def constant_media(shape, lam, mu, rho):
    """Homogeneous medium with the given Lame parameters and density."""
    shape = tuple(int(s) for s in shape)
    return dict(lam=np.full(shape, float(lam)), mu=np.full(shape, float(mu)),
                rho=np.full(shape, float(rho)))


def linear_media(shape, lam_range, mu_range, rho_range):
    """Media varying linearly along x_1 (numpy last axis), as in the paper's
    linear model of Table 3 (rho in [2,3], lam in [4,20], mu in [1,15])."""
    shape = tuple(int(s) for s in shape)
    n1 = shape[-1]
    t = (np.arange(n1) + 0.5) / n1
    out = {}
    for name, (a, b) in (("lam", lam_range), ("mu", mu_range), ("rho", rho_range)):
        prof = a + (b - a) * t
        out[name] = np.broadcast_to(prof, shape).astype(np.float64).copy()
    return out
