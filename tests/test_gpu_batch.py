"""Batched gauge fixing against the CPU oracle, member by member.

A batch context fixes several configurations of uneven shapes in shared
launches, each with its own stopping rule theta <= eps (Alg. 1). Each
member's (F, theta) history, iteration count and final links are compared
with the oracle's run of that configuration alone, at the library's default
decomposition (no t-chunk override), with the FP64 transform (same bounds as
the single-configuration trajectories) and with the FP32 transform (its
bounds: same fixed point, theta within 1e-4 relative while theta > 1e-10).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1210_8018_amd import gf
from paper_1210_8018_amd.api import BatchGaugeFixer, GaugeFixer
from paper_1210_8018_amd.inputs import random_links
from test_gpu_parity import compare_trajectory, oracle_reference

pytestmark = pytest.mark.gpu

ALPHA = 0.08
EPS = 1e-15

# uneven shapes: power-of-two and radix-3 extents, a ragged last site block
# (6^4 = 1296 sites), xy- and zt-planes of different sizes
MEMBERS = [((12, 12, 12, 12), 0.3, 201), ((8, 8, 8, 16), 0.25, 202), ((6, 6, 6, 6), 0.35, 203),
           ((12, 8, 6, 4), 0.3, 204), ((4, 4, 4, 4), 0.2, 205)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().to("cpu").numpy()


@pytest.fixture(scope="module")
def oracle_runs():
    out = []
    for dims, eps, seed in MEMBERS:
        U = random_links(dims, eps, seed)
        out.append((U,) + oracle_reference(dims, U, max_iter=5000))
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_members_match_oracle(oracle_runs, prec):
    Ubs = [dev(r[0]) for r in oracle_runs]
    print(f"batch of {len(Ubs)} vs oracle, fft_prec {prec}", flush=True)
    bx = BatchGaugeFixer(Ubs, fft_prec=prec)
    its, Fs, ths = bx.fix_until(EPS, 5000)
    for k, (dims, eps, seed) in enumerate(MEMBERS):
        U, n_ref, U_ref, Fr, Tr, spread = oracle_runs[k]
        V = int(np.prod(dims))
        Fh, Th = bx.history(k)
        assert len(Fh) == its[k] + 1 and Fh[-1] == Fs[k] and Th[-1] == ths[k]
        assert ths[k] <= EPS
        Uf = host(Ubs[k])
        if prec == 0:
            assert abs(its[k] - n_ref) <= max(0, int(0.01 * n_ref)), (dims, its[k], n_ref)
            compare_trajectory(Fh, Th, Fr, Tr, spread, dims, f"batch member {dims}")
            assert abs(Fs[k] - Fr[-1]) <= 1e-10 * Fr[-1]
            assert np.max(np.abs(Uf.reshape(U_ref.shape) - U_ref)) < 1e-11
        else:
            assert abs(its[k] - n_ref) <= max(1, int(0.05 * n_ref)), (dims, its[k], n_ref)
            assert abs(Fs[k] - Fr[-1]) <= 1e-12 * Fr[-1]
            n = min(len(Th), len(Tr))
            T, R = np.asarray(Th[:n]), np.asarray(Tr[:n])
            big = R > 1e-10
            assert np.max(np.abs(T[big] - R[big]) / R[big]) < 1e-4
            # F per iteration: the FP32 rounding of the filtered field moves g,
            # hence F, by a few binary32 ulps of an O(1) value
            assert np.max(np.abs(np.asarray(Fh[:n]) - Fr[:n])) < 2e-7
        assert abs(oracle.plaquette(dims, Uf) - oracle.plaquette(dims, U)) < 1e-13


def test_history_batch_arguments():
    dims = (4, 4, 4, 4)
    Ubs = [dev(random_links(dims, 0.2, 206)), dev(random_links(dims, 0.3, 207))]
    bx = BatchGaugeFixer(Ubs)
    F0, T0 = bx.history(1)
    assert len(F0) == 1  # the initial measurement
    with pytest.raises(gf.GFError):
        bx.history(2)
    with pytest.raises(gf.GFError):
        bx.history(-1)
    fx = GaugeFixer(dev(random_links(dims, 0.2, 208)))
    fx.step(3)
    assert gf.gf_history_batch(fx.ctx, 0) == fx.history()


def test_single_precision_batch_refines_members_that_reached_refine_theta(monkeypatch):
    """link_prec 1: a member that stops at the iteration cap in the
    single-precision phase does not keep the others from their FP64-storage
    refinement; those reach theta_eps as in their own contexts (bitwise, at
    the same t-chunk), each within its own budget."""
    monkeypatch.setenv("GF_TCHUNK", "2")
    monkeypatch.setenv("GF_TCHUNK_BATCH", "2")
    cases = [((8, 8, 8, 8), 0.3, 1), ((6, 4, 8, 4), 0.6, 2), ((12, 8, 6, 4), 0.3, 3)]
    cap = 150
    Us = [random_links(d, e, s) for d, e, s in cases]
    single = []
    for U in Us:
        Ud = dev(U)
        fx = GaugeFixer(Ud, link_prec=1, fft_prec=1, fft_schedule=3)
        it, F, th, st = gf.gf_fix_until(fx.ctx, EPS, cap, allow_maxiter=True)
        single.append((it, F, th, st, host(Ud)))
    # the eps = 0.6 member needs thousands of updates; the others well under the cap
    assert single[1][3] == gf.GF_ERR_MAXITER and single[1][2] > 1e-10
    assert single[0][3] == gf.GF_OK and single[2][3] == gf.GF_OK
    Ubs = [dev(U) for U in Us]
    bx = BatchGaugeFixer(Ubs, link_prec=1, fft_prec=1, fft_schedule=3)
    its, Fs, ths, st = gf.gf_fix_until_batch(bx.ctx, len(cases), EPS, cap, allow_maxiter=True)
    assert st == gf.GF_ERR_MAXITER
    for k in range(len(cases)):
        it, F, th, _, Uf = single[k]
        assert its[k] == it and Fs[k] == F and ths[k] == th, (k, its[k], it, ths[k], th)
        assert np.array_equal(host(Ubs[k]), Uf)
    assert ths[0] <= EPS and ths[2] <= EPS and its[1] == cap
