"""GPU tests of the receiver kernels (elh_receivers, elh_inject) through the
C ABI: sampling, misfit and injection against numpy gathers/scatters and the
oracle's misfit, their edge cases, and the autograd paths built on them."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import adjoint as AD
from synthetic import make_media, random_field, omega_for_ppw, lattice_sources

pytestmark = pytest.mark.gpu


def _problem(shape, levels=2):
    from paper_2307_03242_amd import Problem
    m = make_media(shape, 31)
    return Problem(torch.from_numpy(m["lam"]), torch.from_numpy(m["mu"]), torch.from_numpy(m["rho"]),
                   h=1.0, omega=omega_for_ppw(m["vs"].min(), 1.0, 10), gamma=0.01, alpha=0.5,
                   abl_width=0.25 * min(shape), abl_amp=2.0, levels=levels, cycle="W",
                   damping=(0.55, 0.35, 0.25), coarse_mode="krylov", coarse_sweeps=2, coarse_maxit=6)


def _mask(shape, seed):
    """random receivers, about 400 of them (several 256-thread blocks and a
    ragged tail)"""
    rng = np.random.default_rng(seed)
    full = (len(shape) + 1,) + shape
    return rng.random(full) < min(0.6, 400.0 / np.prod(full))


@pytest.mark.parametrize("shape", [(8, 12, 16), (12, 20), (20, 16, 24)])
def test_sampling_and_misfit_match_numpy_and_oracle(shape):
    prob = _problem(shape)
    mask = _mask(shape, 1)
    idx_np = np.flatnonzero(mask)
    assert idx_np.size > 256          # several blocks and a ragged tail
    u = random_field(shape, 2, nrhs=3)
    d_obs_full = random_field(shape, 3, nrhs=3)
    ud = torch.from_numpy(u).cuda()
    idx = prob.receiver_indices(torch.from_numpy(mask).cuda())
    assert np.array_equal(idx.cpu().numpy(), idx_np)
    d = prob.receivers(ud, idx)
    ref = u.reshape(3, -1)[:, idx_np]
    assert np.array_equal(d.cpu().numpy(), ref)
    dobs = torch.from_numpy(d_obs_full.reshape(3, -1)[:, idx_np].copy()).cuda()
    r, phi = prob.receivers(ud, idx, dobs, misfit=True)
    assert np.array_equal(r.cpu().numpy(), ref - d_obs_full.reshape(3, -1)[:, idx_np])
    phi = phi.cpu().numpy()
    for s in range(3):
        want = AD.misfit(u[s:s + 1], d_obs_full[s:s + 1], mask)
        assert abs(phi[s] - want) <= 1e-13 * want
    want = AD.misfit(u, d_obs_full, mask)
    assert abs(phi[3] - want) <= 1e-13 * want
    assert phi[3] == phi[0] + phi[1] + phi[2]
    # one vector without the rhs axis
    d1 = prob.receivers(ud[1].contiguous(), idx)
    assert d1.shape == (idx_np.size,) and torch.equal(d1, d[1])
    prob.close()


@pytest.mark.parametrize("shape", [(8, 12, 16), (12, 20)])
def test_injection_is_the_transpose(shape):
    prob = _problem(shape)
    mask = _mask(shape, 4)
    idx_np = np.flatnonzero(mask)
    idx = torch.from_numpy(idx_np).cuda()
    rng = np.random.default_rng(5)
    r = rng.standard_normal((2, idx_np.size)) + 1j * rng.standard_normal((2, idx_np.size))
    v = prob.inject(torch.from_numpy(r).cuda(), idx).cpu().numpy()
    ref = np.zeros((2, mask.size), dtype=np.complex128)
    ref[:, idx_np] = r
    assert np.array_equal(v.reshape(2, -1), ref)
    # the injection overwrites its output (no stale values) and scales exactly by 2
    v2 = prob.inject(torch.from_numpy(r).cuda(), idx, scale=2.0).cpu().numpy()
    assert np.array_equal(v2.reshape(2, -1), 2.0 * ref)
    # <P u, r> = <u, P^T r> exactly (a gather against a scatter)
    u = random_field(shape, 6, nrhs=2)
    pu = prob.receivers(torch.from_numpy(u).cuda(), idx).cpu().numpy()
    for s in range(2):
        a = np.vdot(pu[s], r[s])
        b = np.vdot(u[s].reshape(-1), v[s].reshape(-1))
        assert abs(a - b) <= 1e-14 * abs(a)
    prob.close()


def test_indices_outside_the_vector_and_repeats():
    """an index outside the vector samples 0 and is skipped by the
    injection; a repeated index samples the same value twice"""
    shape = (8, 8, 8)
    prob = _problem(shape)
    n = 4 * 8 * 8 * 8
    idx_np = np.array([0, n - 1, n, -1, 17, 17, 2 ** 40], dtype=np.int64)
    u = random_field(shape, 7, nrhs=2)
    d = prob.receivers(torch.from_numpy(u).cuda(), torch.from_numpy(idx_np).cuda()).cpu().numpy()
    flat = u.reshape(2, -1)
    want = np.stack([[flat[s, j] if 0 <= j < n else 0 for j in idx_np] for s in range(2)])
    assert np.array_equal(d, want)
    r = np.arange(3, dtype=np.complex128) + 1.0
    v = prob.inject(torch.from_numpy(r).cuda(), torch.from_numpy(idx_np[:3]).cuda()).cpu().numpy().reshape(-1)
    ref = np.zeros(n, dtype=np.complex128)
    ref[0], ref[n - 1] = 1.0, 2.0
    assert np.array_equal(v, ref)
    prob.close()


def test_receiver_entry_points_reject_bad_arguments():
    from paper_2307_03242_amd import _lib as L
    shape = (8, 8, 8)
    prob = _problem(shape)
    u = torch.zeros((1, 4) + shape, dtype=torch.complex128, device="cuda")
    idx = torch.arange(4, dtype=torch.int64, device="cuda")
    d = torch.empty((1, 4), dtype=torch.complex128, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    lib = prob.lib
    assert lib.elh_receivers(prob.handle, 1, p(u), 0, p(idx), None, p(d), None) == L.ELH_ERR_ARG
    assert lib.elh_receivers(prob.handle, 0, p(u), 4, p(idx), None, p(d), None) == L.ELH_ERR_ARG
    assert lib.elh_receivers(prob.handle, 1, None, 4, p(idx), None, p(d), None) == L.ELH_ERR_ARG
    assert lib.elh_inject(prob.handle, 1, 4, p(idx), p(d), float("nan"), p(u)) == L.ELH_ERR_ARG
    assert lib.elh_inject(prob.handle, 1, 4, None, p(d), 1.0, p(u)) == L.ELH_ERR_ARG
    assert lib.elh_receivers(prob.handle, 1, p(u), 4, p(idx), None, p(u), None) == L.ELH_ERR_ARG
    assert lib.elh_inject(prob.handle, 1, 4, p(idx), p(u), 1.0, p(u)) == L.ELH_ERR_ARG
    with pytest.raises(ValueError):
        prob.receivers(u, idx.to(torch.int32))
    with pytest.raises(ValueError):
        prob.receivers(u, idx, torch.empty((1, 5), dtype=torch.complex128, device="cuda"))
    with pytest.raises(ValueError):
        prob.inject(torch.zeros((1, 5), dtype=torch.complex128, device="cuda"), idx)
    prob.close()


def test_data_and_misfit_functions_give_the_same_gradient():
    """the gradient of 1/2 |d - d_obs|^2 taken through ElasticFWI's data
    (torch differentiates the norm, the library injects its gradient) equals
    the one through ElasticMisfit (the library forms the residual and the
    adjoint source).  Both adjoint sources are d - d_obs up to torch's
    rounding in the backward of the norm; the adjoint solves to 1e-12 then
    agree to about that relative accuracy."""
    from paper_2307_03242_amd.autograd import ElasticFWI, misfit
    shape = (16, 16, 16)
    prob = _problem(shape, levels=3)
    m0 = make_media(shape, 501)
    q = torch.from_numpy(lattice_sources(shape, 1, 2, depth_index=5)).cuda()
    mask = np.zeros((4,) + shape, dtype=bool)
    mask[:3, 5, 2:-2, 2:-2] = True
    idx = prob.receiver_indices(torch.from_numpy(mask).cuda())
    rng = np.random.default_rng(8)
    d_obs = torch.from_numpy(rng.standard_normal((2, idx.numel())) * 1e-3 + 0j).cuda()
    grads = []
    for path in ("data", "misfit"):
        params = [torch.from_numpy(m0[k]).cuda().requires_grad_(True) for k in ("lam", "mu", "rho")]
        if path == "data":
            d = ElasticFWI.apply(*params, prob, q, idx, 1e-12, 2000)
            r = d - d_obs
            phi = 0.5 * (r.real ** 2 + r.imag ** 2).sum()
        else:
            phi = misfit(prob, *params, q, idx, d_obs, rtol=1e-12, maxit=2000)
        phi.backward()
        grads.append([t.grad.clone() for t in params])
        if path == "data":
            phi_data = phi.item()
        else:
            assert abs(phi.item() - phi_data) <= 1e-14 * phi_data
    for a, b in zip(*grads):
        assert float(torch.linalg.vector_norm(a - b)) <= 1e-10 * float(torch.linalg.vector_norm(b))
    prob.close()
