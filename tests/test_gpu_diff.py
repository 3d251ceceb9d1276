"""GPU forward/backward of F_U[g(omega)] against the oracle, finite differences and Delta."""
import numpy as np
import pytest
import torch

import oracle
from paper_1210_8018_amd import gf
from paper_1210_8018_amd.api import GaugeFixer, GaugeFunctional
from paper_1210_8018_amd.inputs import gell_mann, random_links, random_omega

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().to("cpu").numpy()


@pytest.mark.parametrize("dims,sigma", [((4, 4, 4, 4), 0.1), ((6, 4, 4, 8), 0.5), ((12, 8, 6, 4), 1.5)])
def test_forward_and_backward_match_oracle(dims, sigma):
    V = int(np.prod(dims))
    U = random_links(dims, 0.3, 51)
    om = random_omega(dims, sigma, 52)
    Ud, omd = dev(U), dev(om)
    F = GaugeFunctional.apply(Ud, omd)
    assert abs(float(F) - oracle.functional_g(dims, U, om)) < 1e-14
    Ud.requires_grad_(True)
    omd.requires_grad_(True)
    F = GaugeFunctional.apply(Ud, omd)
    F.backward()
    g_om = host(omd.grad)
    ref = oracle.grad_omega_sites(dims, U, om, np.arange(V)).T  # (8, V)
    assert np.max(np.abs(g_om - ref)) < 1e-13 * np.max(np.abs(ref))
    g_U = host(Ud.grad).reshape(4, 3, 3, V)
    refU = oracle.grad_links(dims, om)
    assert np.max(np.abs(g_U - refU)) < 1e-13 / (12 * V)


def test_gradient_at_zero_is_delta():
    dims = (8, 8, 8, 8)
    V = int(np.prod(dims))
    U = random_links(dims, 0.3, 53)
    Ud = dev(U)
    om = torch.zeros((8, V), dtype=torch.float64, device="cuda", requires_grad=True)
    GaugeFunctional.apply(Ud, om).backward()
    D = oracle.delta(dims, U)
    lam = gell_mann()
    da = np.stack([(-0.5j * np.einsum("ij,jiv->v", lam[a], D)).real for a in range(8)])
    assert np.max(np.abs(host(om.grad) * 12 * V - da)) < 1e-12


def test_gradcheck_2x4():
    dims = (2, 2, 2, 2)
    U = dev(random_links(dims, 0.5, 54)).requires_grad_(True)
    om = dev(random_omega(dims, 0.3, 55)).requires_grad_(True)
    assert torch.autograd.gradcheck(GaugeFunctional.apply, (U, om), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_central_differences_24x4():
    """24^4, links eps 0.3 seed 5, omega ~ N(0, 0.1^2) seed 6, 64 sites drawn with seed 7."""
    dims = (24, 24, 24, 24)
    V = int(np.prod(dims))
    U = random_links(dims, 0.3, 5)
    om = random_omega(dims, 0.1, 6)
    sites = np.random.default_rng(7).choice(V, 64, replace=False)
    Ud = dev(U)
    omd = dev(om)
    fx = GaugeFixer(Ud)
    F = gf.gf_functional_g(fx.ctx, omd)
    assert abs(F - oracle.functional_g(dims, U, om)) < 1e-13
    d_om = torch.empty_like(omd)
    gf.gf_functional_g_backward(fx.ctx, omd, 1.0, d_om, None)
    got = host(d_om)[:, sites].T * 12 * V  # site-local scale
    ref = oracle.grad_omega_sites(dims, U, om, sites) * 12 * V
    assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))
    h = 1e-6
    for k, s in enumerate(sites):
        w0 = om[:, s].copy()
        for a in range(8):
            wp, wm = w0.copy(), w0.copy()
            wp[a] += h
            wm[a] -= h
            fd = (oracle.local_functional_g(dims, U, om, s, wp) - oracle.local_functional_g(dims, U, om, s, wm)) / (2 * h)
            assert abs(fd - got[k, a]) < 1e-7 * max(1.0, abs(fd)), (s, a, fd, got[k, a])


def test_functional_context_is_light_reused_and_checks_omega():
    """Forward and backward share one functional-only context (g and block
    partials, no iteration workspace, no measurement); the iteration calls are
    refused on it; omega of the wrong type, shape or device is rejected before
    any kernel reads it."""
    from paper_1210_8018_amd import api

    dims = (6, 4, 4, 8)
    V = int(np.prod(dims))
    p = gf.make_params(dims)
    assert gf.gf_workspace_bytes_functional(p) < 160 * V + 65536 < gf.gf_workspace_bytes(p)
    U = random_links(dims, 0.3, 54)
    om = random_omega(dims, 0.2, 55)
    Ud, omd = dev(U), dev(om)
    omd.requires_grad_(True)
    api._fn_contexts.clear()
    F = GaugeFunctional.apply(Ud, omd)
    F.backward()
    assert len(api._fn_contexts) == 1
    ctx = next(iter(api._fn_contexts.values()))[0]
    assert gf.lib().gf_step(ctx, 1, None, None) == gf.GF_ERR_STATE
    assert gf.lib().gf_functional(ctx, None, None) == gf.GF_ERR_STATE
    assert abs(float(F) - oracle.functional_g(dims, U, om)) < 1e-14
    # the context reads the links as they are at each call
    U2 = random_links(dims, 0.3, 56)
    Ud.copy_(dev(U2))
    F2 = GaugeFunctional.apply(Ud, omd.detach())
    assert abs(float(F2) - oracle.functional_g(dims, U2, om)) < 1e-14
    assert len(api._fn_contexts) == 1
    for bad in (omd.detach().float(), omd.detach()[:, : V - 1], omd.detach().cpu(), omd.detach().reshape(-1)):
        with pytest.raises(ValueError):
            GaugeFunctional.apply(Ud, bad)
