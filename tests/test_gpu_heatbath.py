"""GPU input generator (Wilson-action heatbath, overrelaxation, plaquette)
against the CPU oracle with the same Philox counters.

Both sides draw the same random numbers and take the same accept/reject
decisions; the links differ only by FP64 rounding (the device's log, cos,
sin and sqrt against the host's, and the order of operations). A link
updated once from untouched neighbours (U_x at even sites in the first pass
of a sweep) agrees to a few ulps; later updates take neighbours that already
differ, and a Monte Carlo chain amplifies such differences (1e-10 to 1e-9
after a few sweeps with overrelaxation), which stays far below what a wrong
staple, draw or counter would give (order one). An acceptance flipped by
rounding has probability of order 1e-16 per draw.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1210_8018_amd import gf
from paper_1210_8018_amd.api import GaugeFixer
from paper_1210_8018_amd.inputs import haar_su3

pytestmark = pytest.mark.gpu


def hot_links(dims, seed):
    V = int(np.prod(dims))
    h = haar_su3(np.random.default_rng(seed), 4 * V).reshape(4, V, 3, 3)
    return np.ascontiguousarray(np.moveaxis(h, 1, 3)).reshape(4, 3, 3, *dims[::-1])


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("dims,beta,sweeps,n_or,seed,sweep0", [((4, 4, 4, 4), 6.0, 2, 2, 7, 3),
                                                                 ((6, 4, 4, 8), 5.7, 1, 1, 11, 0),
                                                                 ((4, 6, 2, 4), 0.8, 1, 0, 2, 100)])
def test_heatbath_matches_oracle(dims, beta, sweeps, n_or, seed, sweep0):
    U = hot_links(dims, seed)
    ref = oracle.heatbath(dims, U, beta, sweeps, n_or, seed=seed, sweep0=sweep0)
    Ud = dev(U)
    fx = GaugeFixer(Ud)
    fx.heatbath(beta, sweeps, n_or, seed=seed, sweep0=sweep0)
    got = Ud.cpu().numpy()
    assert np.max(np.abs(got - ref)) < 1e-7
    assert abs(fx.plaquette() - oracle.plaquette(dims, ref)) < 1e-9


@pytest.mark.parametrize("dims,beta", [((4, 4, 4, 4), 6.0), ((6, 4, 4, 8), 2.0)])
def test_single_heatbath_pass_matches_oracle(dims, beta):
    """One sweep without overrelaxation: the first pass (U_x, even sites) is
    computed from the untouched input on both sides and agrees to a few ulps."""
    U = hot_links(dims, 5)
    ref = oracle.heatbath(dims, U, beta, 1, 0, seed=3, sweep0=17)
    Ud = dev(U)
    fx = GaugeFixer(Ud)
    fx.heatbath(beta, 1, 0, seed=3, sweep0=17)
    got = Ud.cpu().numpy()
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(range(Lt), range(Lz), range(Ly), range(Lx), indexing="ij")
    even = (x + y + z + t) % 2 == 0
    d0 = np.abs(got[0] - ref[0])[:, :, even]
    assert np.max(d0) < 1e-13
    assert np.max(np.abs(got - ref)) < 1e-10
    assert not np.allclose(got[0][:, :, even], U[0][:, :, even])  # the pass did update them
    # the context measured the new links
    F, th = fx.functional()
    Fr, thr = oracle.measure(dims, ref)
    assert abs(F - Fr) < 1e-13 and abs(th - thr) < 1e-12 * thr


def test_plaquette_of_generated_links():
    from paper_1210_8018_amd.inputs import random_links

    dims = (8, 6, 4, 4)
    U = random_links(dims, 0.4, 3)
    fx = GaugeFixer(dev(U))
    assert abs(fx.plaquette() - oracle.plaquette(dims, U)) < 1e-13


def test_heatbath_rejects_odd_extents():
    fx = GaugeFixer(dev(hot_links((6, 6, 6, 3), 1)))
    with pytest.raises(gf.GFError):
        fx.heatbath(6.0, 1)


def test_thermalised_input_is_fixed_like_the_oracle():
    """A short thermalisation on the GPU, then gauge fixing on both sides from
    the same (GPU-generated) links."""
    dims = (8, 8, 8, 8)
    V = int(np.prod(dims))
    one = np.zeros((4, 3, 3, V), dtype=np.complex128)
    for i in range(3):
        one[:, i, i, :] = 1
    Ud = dev(one.reshape(4, 3, 3, 8, 8, 8, 8))
    fx = GaugeFixer(Ud)
    fx.heatbath(6.0, 20, 2, seed=1)
    P = fx.plaquette()
    assert 0.55 < P < 0.65
    U = Ud.cpu().numpy()
    n_ref, _, Fr, Tr = oracle.fix(dims, U, eps=1e-15, max_iter=20000)
    fx2 = GaugeFixer(Ud)
    it, F, th = fx2.fix_until(1e-15, 20000)
    assert abs(it - n_ref) <= max(1, int(0.01 * n_ref))
    assert abs(F - Fr[-1]) < 1e-10 and th <= 1e-15
