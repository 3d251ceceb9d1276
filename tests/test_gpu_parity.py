"""GPU (HIP, gfx950) path against the CPU oracle, stage by stage and per iteration.

Every case draws its inputs from the seeded generator; the oracle computes the
expected values on the CPU (or, for the 32^4 trajectory, a stored oracle run
written by tests/golden/make_golden.py). Tolerances: stages 1e-13 absolute on
O(1) values (FP64 rounding of a few hundred operations); per-iteration F 1e-11
relative; theta 1e-11 relative, or, where larger, near theta's rounding floor,
10 times the spread between the oracle and two other correct FP64 runs
(reversed transform axis order; 12-real link storage) or 100 u / sqrt(V theta)
(theta_tolerance);
iteration count within 1 %; final F 1e-10.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1210_8018_amd import gf
from paper_1210_8018_amd.api import BatchGaugeFixer, GaugeFixer
from paper_1210_8018_amd.inputs import haar_su3, random_links

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ALPHA = 0.08
EPS = 1e-15

# several tiles, ragged site blocks (V not a multiple of 256), radix-3 lengths
# (27 = three radix-3 stages, odd extents 3 and 9), L = 2, the longest axis
# (256); t extents 2, 4, 16, 256 (last radix 2 or 4: the t-axis centre stage
# with 1, 2 or 3 stages) and 8 (last radix 8: separate scaling step); 48 x 48
# planes (a general-extent tile filling 56 % of its 4096-element capacity) in
# the xy and in the zt pass; 64 x 64 planes (the 64^4 workload's, filling
# the 4096-element tile exactly); Lz = Lt = 64 with Lx Ly a multiple of 16
# (the z and t lines of schedules 1 and 2 in registers, k_fft_line; 4 x 4
# and 6 x 8 xy-planes, the latter with general extents in the xy pass)
SHAPES = [(8, 8, 8, 8), (12, 8, 6, 4), (6, 6, 6, 2), (2, 2, 2, 2), (24, 4, 2, 6), (4, 12, 4, 8),
          (27, 2, 4, 6), (3, 9, 2, 4), (256, 4, 2, 2), (2, 2, 2, 256), (4, 4, 4, 4), (4, 2, 4, 16),
          (48, 48, 2, 2), (2, 2, 48, 48), (64, 64, 2, 2), (2, 2, 64, 64), (4, 4, 64, 64), (6, 8, 64, 64)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().to("cpu").numpy()


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.mark.parametrize("dims", SHAPES)
def test_delta_and_functional(dims):
    U = random_links(dims, 0.4, 41)
    fx = GaugeFixer(dev(U))
    D = host(fx.delta())
    Dref = oracle.delta(dims, U)
    assert np.max(np.abs(D - Dref)) < 1e-13
    F, th = fx.functional()
    Fr, thr = oracle.measure(dims, U)
    assert rel(F, Fr) < 1e-14 and rel(th, thr) < 1e-14


SCHEDULES = [1, 2, 3]  # 1D passes; (x,y) + 1D z, t; (x,y) + (z,t)


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("sched", SCHEDULES)
def test_fft_matches_oracle(dims, prec, sched):
    V = int(np.prod(dims))
    rng = np.random.default_rng(42)
    f = rng.standard_normal((3, V)) + 1j * rng.standard_normal((3, V))
    fx = GaugeFixer(dev(random_links(dims, 0.3, 1)), fft_prec=prec, fft_schedule=sched)
    assert gf.gf_fft_schedule(fx.ctx) == sched
    ct = torch.complex64 if prec else torch.complex128
    tol = 3e-6 if prec else 1e-13
    for sign in (-1, +1):
        t = torch.from_numpy(f).to(ct).to("cuda").contiguous()
        got = host(fx.fft(t, sign)).astype(np.complex128)
        for k in range(3):
            ref = oracle.fft4d(dims, f[k], sign)
            assert np.max(np.abs(got[k] - ref)) < tol * np.max(np.abs(ref)), (sign, k)


def fp32_gauge_tolerance(dims):
    """Bound on |g_fp32 - g_oracle|: the FP32 transform's rounding (a few
    1e-7 of the field) is multiplied by K(p), whose range is
    p2max / p2min = p2max / (4 sin^2(pi / Lmax)); 2e-6 up to a range of 1000
    (every extent <= 48), growing in proportion beyond (256: 2.6e4)."""
    p2max = sum(4 * np.sin(np.pi * (L // 2) / L) ** 2 for L in dims)
    p2min = 4 * np.sin(np.pi / max(dims)) ** 2
    return 2e-6 * max(1.0, p2max / p2min / 1000)


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("sched", SCHEDULES)
def test_gauge_vector_matches_oracle(dims, prec, sched):
    U = random_links(dims, 0.4, 43)
    fx = GaugeFixer(dev(U), fft_prec=prec, fft_schedule=sched)
    g = host(fx.gauge())
    gref = oracle.gauge_from_delta(dims, oracle.delta(dims, U), ALPHA)
    assert np.max(np.abs(g - gref)) < (fp32_gauge_tolerance(dims) if prec else 1e-13)
    M = np.moveaxis(g, 2, 0)
    assert np.max(np.abs(M @ np.conj(np.swapaxes(M, -1, -2)) - np.eye(3))) < 1e-13
    assert np.max(np.abs(np.linalg.det(M) - 1)) < 1e-13


TILE_VARIANTS = [  # (xy target, xy elements per work-item, zt target, zt elements per work-item)
    (1024, 8, 2048, 4), (4096, 4, 2048, 8), (4096, 8, 4096, 4), (2048, 4, 1024, 8), (1024, 4, 4096, 8)]


def check_2d_passes(dims, prec):
    """Gauge vector and forward/backward transform of the xy + zt schedule against the oracle."""
    V = int(np.prod(dims))
    U = random_links(dims, 0.4, 43)
    fx = GaugeFixer(dev(U), fft_prec=prec, fft_schedule=3)
    g = host(fx.gauge())
    gref = oracle.gauge_from_delta(dims, oracle.delta(dims, U), ALPHA)
    assert np.max(np.abs(g - gref)) < (fp32_gauge_tolerance(dims) if prec else 1e-13)
    # five fields: work-groups of the 2D passes take four fields of a tile
    # each, the next one prefetched while the current one is transformed, so
    # the last group has one
    rng = np.random.default_rng(7)
    nf = 5
    f = rng.standard_normal((nf, V)) + 1j * rng.standard_normal((nf, V))
    ct = torch.complex64 if prec else torch.complex128
    tol = 3e-6 if prec else 1e-13
    for sign in (-1, +1):
        got = host(fx.fft(torch.from_numpy(f).to(ct).to("cuda").contiguous(), sign)).astype(np.complex128)
        for k in range(nf):
            ref = oracle.fft4d(dims, f[k], sign)
            assert np.max(np.abs(got[k] - ref)) < tol * np.max(np.abs(ref)), (sign, k)


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (12, 8, 6, 4), (24, 4, 2, 6), (4, 12, 4, 8), (16, 8, 4, 32),
                                  (64, 64, 2, 2), (2, 2, 64, 64)])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("tiles", TILE_VARIANTS)
def test_2d_tile_variants_match_oracle(monkeypatch, dims, prec, tiles):
    """Every (tile size, work-group size) instance of the 2D passes: transform and gauge vector."""
    for name, v in zip(("GF_XY_TARGET", "GF_XY_EPT", "GF_ZT_TARGET", "GF_ZT_EPT"), tiles):
        monkeypatch.setenv(name, str(v))
    check_2d_passes(dims, prec)


@pytest.mark.parametrize("dims", SHAPES)
def test_link_update_matches_oracle(dims):
    V = int(np.prod(dims))
    U = random_links(dims, 0.4, 44)
    g = np.ascontiguousarray(np.moveaxis(haar_su3(np.random.default_rng(5), V), 0, 2))
    Ud = dev(U)
    fx = GaugeFixer(Ud)
    fx.apply_gauge(dev(g))
    got = host(Ud).reshape(4, 3, 3, V)
    ref = oracle.apply_gauge(dims, U, g).reshape(4, 3, 3, V)
    assert np.max(np.abs(got - ref)) < 1e-14
    assert abs(oracle.plaquette(dims, host(Ud)) - oracle.plaquette(dims, U)) < 1e-13


def theta_tolerance(theta, spread, V):
    """Relative bound on |theta_gpu - theta_oracle| per iteration: the largest
    of 1e-11; 10 times the largest relative spread up to that iteration
    between the oracle and two other correct FP64 runs (`spread`, the sum of
    the two differences: the GPU departs from the oracle in both ways at
    once; oracle_reference); and 100 u / sqrt(V theta) (u = 2^-53).

    theta is a sum of squares of Delta, itself a difference of O(1) link
    entries, so two correct FP64 codes agree on it only to about
    u / sqrt(V theta) relative (V terms, each |Delta|^2 ~ theta, each Delta
    carrying an absolute rounding of a few u): near its floor (theta below
    ~1e-12, or above it on small lattices) they differ by more than 1e-11.
    The measured spread of the two oracle variants sets the bound there; the
    last term covers orders of rounding the two variants do not sample (their
    own spread is 1.7 to 6 times u / sqrt(V theta) in the median below
    theta = 1e-12 on the lattices of these tests). On a 32^4 lattice both
    stay far below 1e-11 while theta >= 1e-12.
    """
    theta = np.asarray(theta)
    spread = np.asarray(spread)
    if len(spread) < len(theta):
        spread = np.concatenate([spread, np.full(len(theta) - len(spread), spread.max())])
    floor = 100 * 2.0 ** -53 / np.sqrt(V * theta)
    return np.maximum(np.maximum(1e-11, 10 * np.maximum.accumulate(spread[: len(theta)])), floor)


def oracle_reference(dims, U, **kw):
    """The oracle's run of Alg. 1 and the per-iteration relative theta spread
    between it and two runs that differ only in rounding (the sum of both
    differences): the transform's axes taken in reverse order, and the links
    and g kept in the 12-real form of section 2.2 (two rows in FP64, the
    third rebuilt), the form the GPU stores."""
    n, Uf, Fr, Tr = oracle.fix(dims, U, alpha=ALPHA, eps=EPS, **kw)
    _, _, _, T1 = oracle.fix(dims, U, alpha=ALPHA, eps=EPS, fft_axis_order=(3, 2, 1, 0), **kw)
    _, _, _, T2 = oracle.fix(dims, U, alpha=ALPHA, eps=EPS, two_row=True, **kw)
    k = min(len(Tr), len(T1), len(T2))
    spread = (np.abs(T1[:k] - Tr[:k]) + np.abs(T2[:k] - Tr[:k])) / Tr[:k]
    return n, Uf, Fr, Tr, spread


def compare_trajectory(F, T, Fr, Tr, spread, dims, label=""):
    """Per-iteration F (1e-11 relative) and theta (theta_tolerance) over the
    first 100 updates on a lattice of extents dims; prints the largest errors
    seen."""
    F, T, Fr, Tr = map(np.asarray, (F, T, Fr, Tr))
    n = min(len(F), len(Fr), 101)
    eF = np.abs(F[:n] - Fr[:n]) / np.abs(Fr[:n]).clip(1e-300)
    assert np.max(eF) < 1e-11
    err = np.abs(T[:n] - Tr[:n]) / Tr[:n]
    tol = theta_tolerance(Tr[:n], spread, int(np.prod(dims)))
    tail = Tr[:n] < 1e-12
    print(f"trajectory {label}: max F err {eF.max():.2e}; theta err {err[~tail].max():.2e} above 1e-12, "
          f"{err[tail].max() if tail.any() else 0.0:.2e} below (largest err/tol {np.max(err / tol):.3f}, "
          f"tol {tol[~tail].max():.1e} above 1e-12)", flush=True)
    assert np.all(err < tol), (err, tol, Tr[:n])


@pytest.mark.parametrize("dims,eps,seed", [((8, 8, 8, 8), 0.3, 1), ((12, 8, 6, 4), 0.3, 3), ((6, 6, 6, 2), 0.35, 4),
                                           ((27, 2, 4, 6), 0.3, 5), ((3, 9, 2, 4), 0.3, 6),
                                           ((4, 4, 64, 64), 0.3, 7), ((4, 4, 48, 48), 0.3, 8)])
@pytest.mark.parametrize("sched", [0] + SCHEDULES)
def test_trajectory_matches_oracle(dims, eps, seed, sched):
    U = random_links(dims, eps, seed)
    n_ref, U_ref, Fr, Tr, spread = oracle_reference(dims, U, max_iter=5000)
    Ud = dev(U)
    fx = GaugeFixer(Ud, fft_schedule=sched)
    it, F, th = fx.fix_until(EPS, 5000)
    Fh, Th = fx.history()
    assert abs(it - n_ref) <= max(0, int(0.01 * n_ref)), (it, n_ref)
    compare_trajectory(Fh, Th, Fr, Tr, spread, dims, f"{dims} schedule {sched}")
    assert th <= EPS
    assert rel(F, Fr[-1]) < 1e-10
    Uf = host(Ud)
    assert abs(oracle.plaquette(dims, Uf) - oracle.plaquette(dims, U)) < 1e-13
    M = np.moveaxis(Uf.reshape(4, 3, 3, -1), 3, 1).reshape(-1, 3, 3)
    assert np.max(np.abs(M @ np.conj(np.swapaxes(M, -1, -2)) - np.eye(3))) < 1e-13
    assert np.max(np.abs(np.linalg.det(M) - 1)) < 1e-13
    Fh = np.asarray(Fh)
    assert np.all(np.diff(Fh) >= -4 * np.spacing(np.abs(Fh[:-1])))


def test_unfused_full_storage_path_matches_oracle(monkeypatch):
    """The separate update and divergence kernels on full 18-real links (GF_NOFUSE)."""
    monkeypatch.setenv("GF_NOFUSE", "1")
    dims = (8, 8, 8, 8)
    U = random_links(dims, 0.3, 1)
    n_ref, _, Fr, Tr, spread = oracle_reference(dims, U, max_iter=5000)
    Ud = dev(U)
    fx = GaugeFixer(Ud)
    it, F, th = fx.fix_until(EPS, 5000)
    Fh, Th = fx.history()
    assert it == n_ref
    compare_trajectory(Fh, Th, Fr, Tr, spread, dims, "18-real storage")
    assert abs(oracle.plaquette(dims, host(Ud)) - oracle.plaquette(dims, U)) < 1e-13


@pytest.mark.parametrize("dims,tile,fuse", [((8, 8, 8, 8), "4,4,4", True), ((12, 8, 6, 4), "8,4,4", True),
                                            ((12, 8, 6, 4), "8,4,4", False), ((6, 6, 6, 2), "4,4,6", True)])
def test_box_tiles_match_oracle(monkeypatch, dims, tile, fuse):
    """Marching kernels with box-shaped site sets (GF_TILE), ragged boxes included."""
    monkeypatch.setenv("GF_TILE", tile)
    if not fuse:
        monkeypatch.setenv("GF_NOFUSE", "1")
    U = random_links(dims, 0.3, 1)
    n_ref, _, Fr, Tr, spread = oracle_reference(dims, U, max_iter=5000)
    Ud = dev(U)
    fx = GaugeFixer(Ud)
    it, F, th = fx.fix_until(EPS, 5000)
    Fh, Th = fx.history()
    assert it == n_ref
    compare_trajectory(Fh, Th, Fr, Tr, spread, dims, f"{dims} box {tile}")


@pytest.mark.parametrize("dims,tiles,kw", [((8, 8, 8, 8), ["4,4,4", "8,8,4", "8,4,8"], {}),
                                           ((12, 8, 6, 4), ["8,4,4", "4,8,2", "12,8,2"], {}),
                                           ((6, 6, 6, 2), ["4,4,6", "6,6,6"], {}),
                                           ((8, 8, 8, 8), ["8,8,4"], {"reunit_every": 2}),
                                           ((12, 8, 6, 4), ["8,4,4"], {"link_prec": 1, "fft_prec": 1})])
def test_site_sets_give_bitwise_equal_links(monkeypatch, dims, tiles, kw):
    """In the exchange pass a site's divergence is accumulated in one fixed
    order whether a neighbour's link comes through LDS or is recomputed from
    the old links, and the transform does not depend on the marching blocks, so
    the links after a fixed number of updates are bitwise equal for linear site
    sets and boxes (ragged ones included). (The pass without exchange sums the
    divergence as full matrices and is compared with the oracle instead.)"""
    U = random_links(dims, 0.3, 1)

    def run(env):
        monkeypatch.delenv("GF_TILE", raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        Ud = dev(U)
        fx = GaugeFixer(Ud, **kw)
        fx.step(6)
        del fx
        return host(Ud)

    ref = run({})
    for env in [{"GF_TILE": t} for t in tiles]:
        assert np.array_equal(run(env), ref), env


@pytest.mark.parametrize("kw", [dict(), dict(fft_prec=1, link_prec=1)])
def test_walk_lengths_give_bitwise_equal_links(monkeypatch, kw):
    """The walk length of the marching blocks (t-slices per block, chosen by
    the planner from the lattice shape) changes only the order of the partial
    sums of F and theta: the links after a fixed number of updates are
    bitwise equal for every walk length that divides Lt, and F after them
    agrees to rounding."""
    dims = (8, 8, 4, 24)
    U = random_links(dims, 0.3, 5)

    def run(t):
        monkeypatch.setenv("GF_TCHUNK", str(t))
        Ud = dev(U)
        fx = GaugeFixer(Ud, **kw)
        fx.step(6)
        F, _ = fx.functional()
        del fx
        return host(Ud), F

    ref, Fref = run(1)
    for t in (2, 3, 4, 6, 8):
        Ut, Ft = run(t)
        assert np.array_equal(Ut, ref), t
        assert abs(Ft - Fref) < 1e-14, t


@pytest.mark.parametrize("dims", [(24, 24, 8, 8), (32, 32, 8, 8), (48, 48, 4, 4), (64, 64, 2, 4), (24, 24, 6, 4)])
@pytest.mark.parametrize("kw", [dict(), dict(fft_prec=1), dict(fft_prec=1, link_prec=1)])
def test_paired_site_sets_give_bitwise_equal_results(monkeypatch, dims, kw):
    """The fused pass with two site sets per block (GF_PAIR=1; the default
    for Lx = 24, 48 and 64) against one set per block (GF_PAIR=0): the links
    and the per-iteration F and theta after a fixed number of updates are
    bitwise equal (each set keeps its own partial sums, reduced in the same
    order). 24 x 24 x 6 x 4: 3456 sites per slice, so the last set of each
    walk is ragged (128 of its 256 work-items hold a site)."""
    U = random_links(dims, 0.3, 9)
    out = []
    for p in ("0", "1"):
        monkeypatch.setenv("GF_PAIR", p)
        Ud = dev(U)
        fx = GaugeFixer(Ud, **kw)
        fx.step(7)
        F, T = fx.history()
        out.append((host(Ud), np.asarray(F), np.asarray(T)))
        del fx
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", [0, 1])
def test_paired_batch_equals_single_runs(monkeypatch, prec):
    """A batch whose members all take two site sets per fused-pass block
    (Lx = 24, 48, 64; one with a ragged last set per walk), finishing at
    different iterations, so the map is compacted while paired: every member
    bitwise equal to its own context's run."""
    monkeypatch.setenv("GF_TCHUNK", "2")
    monkeypatch.setenv("GF_TCHUNK_BATCH", "2")
    cases = [((24, 24, 8, 8), 0.3, 89), ((48, 48, 4, 4), 0.35, 90), ((64, 64, 2, 4), 0.3, 91),
             ((24, 24, 6, 4), 0.4, 92)]
    Us = [random_links(d, e, s) for d, e, s in cases]
    single = []
    for U in Us:
        Ud = dev(U)
        fx = GaugeFixer(Ud, fft_prec=prec, fft_schedule=2)
        single.append((fx.fix_until(EPS, 5000), host(Ud)))
    Ubs = [dev(U) for U in Us]
    bx = BatchGaugeFixer(Ubs, fft_prec=prec, fft_schedule=2)
    its, Fs, ths = bx.fix_until(EPS, 5000)
    for k in range(len(cases)):
        (it, F, th), Uf = single[k]
        assert its[k] == it and Fs[k] == F and ths[k] == th, (k, its[k], it)
        assert np.array_equal(host(Ubs[k]), Uf)


def test_step_equals_fix_prefix():
    """Calls of every length give the trajectory of one uninterrupted run,
    bitwise: the first update of a call reads the caller's links, the last of
    a gf_step call writes them, and one-update calls and chunk remainders go
    through the two-row buffers."""
    dims = (8, 8, 8, 8)
    U = random_links(dims, 0.3, 1)
    Ua = dev(U)
    a = GaugeFixer(Ua)
    a.fix_until(EPS, 5000)
    Fa, Ta = a.history()
    b = GaugeFixer(dev(U), chunk=3)
    for _ in range(5):
        b.step(2)
    Fb, Tb = b.history()
    assert len(Fb) == 11
    assert Fb == Fa[:11] and Tb == Ta[:11]  # deterministic: bitwise equal
    Uc = dev(U)
    c = GaugeFixer(Uc)
    for n in (1, 9, 3, 1, 16):
        c.step(n)
    Fc, Tc = c.history()
    assert len(Fc) == 31 and Fc == Fa[:31] and Tc == Ta[:31]
    c.fix_until(EPS, 5000)
    Fc, Tc = c.history()
    assert Fc == Fa and Tc == Ta
    assert torch.equal(Uc, Ua)  # the links each call leaves in the caller's array


def test_resume_from_saved_links():
    """The links a call leaves behind are the whole state: a run stopped after 4
    updates and resumed in a new context from a copy of its links follows the
    uninterrupted run. Not bitwise: the first measurement of a call computes the
    divergence with the separate kernel, whose summation order differs from the
    fused pass's, so the two paths differ by rounding from there on."""
    dims = (8, 8, 8, 8)
    U = random_links(dims, 0.3, 1)
    Ua = dev(U)
    a = GaugeFixer(Ua)
    a.step(10)
    Fa, Ta = a.history()
    Ub = dev(U)
    b = GaugeFixer(Ub)
    b.step(4)
    saved = Ub.clone()  # the checkpoint
    del b
    c = GaugeFixer(saved)
    c.step(6)
    Fc, Tc = c.history()
    assert len(Fc) == 7
    assert np.max(np.abs(np.array(Fc) - np.array(Fa[4:11]))) < 1e-14
    assert np.max(np.abs(np.array(Tc) / np.array(Ta[4:11]) - 1)) < 1e-9
    assert np.max(np.abs(host(saved) - host(Ua))) < 1e-13


def test_trajectory_32x4_matches_stored_oracle():
    """Plain FP64 at 32^4 (eps 0.3, seed 2) against the stored oracle run."""
    ref = json.load(open(os.path.join(HERE, "golden", "oracle_32x32x32x32_eps0.3_seed2.json")))
    dims = tuple(ref["dims"])
    U = random_links(dims, ref["eps_generator"], ref["seed"])
    Ud = dev(U)
    del U
    fx = GaugeFixer(Ud)
    it, F, th = fx.fix_until(EPS, 5000)
    Fh, Th = fx.history()
    n_ref = ref["iterations"]
    assert abs(it - n_ref) <= max(0, int(0.01 * n_ref)), (it, n_ref)
    compare_trajectory(Fh, Th, ref["F"], ref["theta"], ref["theta_spread"], dims, "32^4 stored")
    assert rel(F, ref["F"][-1]) < 1e-10 and th <= EPS
    Uf = host(Ud)
    assert abs(oracle.plaquette(dims, Uf) - ref["plaquette_initial"]) < 1e-13


@pytest.mark.parametrize("dims,seed", [((8, 8, 8, 8), 1), ((12, 8, 6, 4), 3)])
def test_fp32_fft_against_fp64_oracle(dims, seed):
    """FFT, scaling and inverse FFT in complex64; the rest FP64. Same fixed point."""
    U = random_links(dims, 0.3, seed)
    n_ref, U_ref, Fr, Tr = oracle.fix(dims, U, alpha=ALPHA, eps=EPS, max_iter=5000)
    Ud = dev(U)
    fx = GaugeFixer(Ud, fft_prec=1)
    it, F, th = fx.fix_until(EPS, 5000)
    Fh, Th = fx.history()
    assert abs(it - n_ref) <= max(1, int(0.05 * n_ref)), (it, n_ref)
    assert th <= EPS
    assert rel(F, Fr[-1]) < 1e-12
    n = min(len(Th), len(Tr))
    big = np.asarray(Tr[:n]) > 1e-10
    assert np.max(np.abs(np.asarray(Th[:n])[big] - np.asarray(Tr[:n])[big]) / np.asarray(Tr[:n])[big]) < 1e-4
    assert abs(oracle.plaquette(dims, host(Ud)) - oracle.plaquette(dims, U)) < 1e-13


def test_reunit_every_matches_oracle():
    dims = (6, 6, 6, 2)
    U = random_links(dims, 0.35, 4)
    n_ref, _, Fr, Tr, spread = oracle_reference(dims, U, reunit_every=4)
    fx = GaugeFixer(dev(U), reunit_every=4)
    it, F, th = fx.fix_until(EPS, 5000)
    Fh, Th = fx.history()
    assert it == n_ref
    compare_trajectory(Fh, Th, Fr, Tr, spread, dims, "reunit every 4")


def test_unit_links_need_no_iteration():
    dims = (4, 4, 4, 4)
    U = np.zeros((4, 3, 3, 4, 4, 4, 4), dtype=np.complex128)
    for i in range(3):
        U[:, i, i] = 1
    fx = GaugeFixer(dev(U))
    assert fx.functional() == (1.0, 0.0)
    it, F, th = fx.fix_until(EPS, 100)
    assert it == 0 and F == 1.0 and th == 0.0


def test_nonfinite_and_maxiter_statuses():
    dims = (8, 8, 8, 8)
    U = random_links(dims, 0.3, 1)
    fx = GaugeFixer(dev(U))
    it, F, th, st = gf.gf_fix_until(fx.ctx, EPS, 3, allow_maxiter=True)
    assert st == gf.GF_ERR_MAXITER and it == 3
    bad = U.copy()
    bad[1, 0, 2, 3, 2, 1, 0] = np.nan
    fb = GaugeFixer(dev(bad))
    with pytest.raises(gf.GFError) as e:
        fb.fix_until(EPS, 10)
    assert e.value.status == gf.GF_ERR_NONFINITE


def test_wide_planes_fall_back_to_1d_passes():
    """Lx*Ly > 4096: the 2D (x, y) pass does not fit; the autotuner keeps 1D passes."""
    dims = (96, 48, 2, 2)
    assert gf.gf_workspace_bytes(gf.make_params(dims, fft_schedule=2)) == 0
    U = random_links(dims, 0.3, 45)
    fx = GaugeFixer(dev(U))
    assert gf.gf_fft_schedule(fx.ctx) == 1
    g = host(fx.gauge())
    gref = oracle.gauge_from_delta(dims, oracle.delta(dims, U), ALPHA)
    assert np.max(np.abs(g - gref)) < 1e-13


def test_invalid_shapes_rejected():
    assert gf.gf_workspace_bytes(gf.make_params((5, 8, 8, 8))) == 0
    assert gf.gf_workspace_bytes(gf.make_params((1, 8, 8, 8))) == 0
    assert gf.gf_workspace_bytes(gf.make_params((512, 8, 8, 8))) == 0
    assert gf.gf_workspace_bytes(gf.make_params((8, 8, 8, 8), alpha=-1)) == 0


@pytest.mark.parametrize("prec,sched", [(0, 1), (0, 3), (1, 2), (1, 3)])
def test_batch_equals_single_runs(monkeypatch, prec, sched):
    """Each configuration of a batch evolves bitwise as in its own context.

    Bitwise equality needs the same decomposition into blocks (the t-slices a
    marching block walks set where the carried U'_t is recomputed and how the
    block sums group), so both contexts are given the same t-chunk.
    """
    monkeypatch.setenv("GF_TCHUNK", "2")
    monkeypatch.setenv("GF_TCHUNK_BATCH", "2")
    cases = [((8, 8, 8, 8), 0.3, 1), ((6, 4, 8, 4), 0.25, 2), ((12, 8, 6, 4), 0.45, 3), ((4, 4, 4, 4), 0.2, 4)]
    Us = [random_links(d, e, s) for d, e, s in cases]
    single = []
    for U in Us:
        Ud = dev(U)
        fx = GaugeFixer(Ud, fft_prec=prec, fft_schedule=sched)
        single.append((fx.fix_until(EPS, 20000), host(Ud)))
    Ubs = [dev(U) for U in Us]
    bx = BatchGaugeFixer(Ubs, fft_prec=prec, fft_schedule=sched)
    its, Fs, ths = bx.fix_until(EPS, 20000)
    for k in range(len(cases)):
        (it, F, th), Uf = single[k]
        assert its[k] == it and Fs[k] == F and ths[k] == th
        assert np.array_equal(host(Ubs[k]), Uf)


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_mixed_general_and_power_of_two(monkeypatch, prec):
    """48 x 48 planes (general-extent instances of the 2D passes) batched with a
    power-of-two lattice (the other instances, same launches): each evolves
    bitwise as in its own context."""
    monkeypatch.setenv("GF_TCHUNK", "2")
    monkeypatch.setenv("GF_TCHUNK_BATCH", "2")
    cases = [((48, 48, 2, 2), 0.3, 7), ((2, 2, 48, 48), 0.3, 8), ((8, 8, 8, 8), 0.3, 9)]
    Us = [random_links(d, e, s) for d, e, s in cases]
    single = []
    for U in Us:
        Ud = dev(U)
        fx = GaugeFixer(Ud, fft_prec=prec, fft_schedule=3)
        single.append((fx.fix_until(EPS, 20000), host(Ud)))
    Ubs = [dev(U) for U in Us]
    bx = BatchGaugeFixer(Ubs, fft_prec=prec, fft_schedule=3)
    its, Fs, ths = bx.fix_until(EPS, 20000)
    for k in range(len(cases)):
        (it, F, th), Uf = single[k]
        assert its[k] == it and Fs[k] == F and ths[k] == th
        assert np.array_equal(host(Ubs[k]), Uf)


# ---------------------------------------------------------------- single-precision link storage

def test_single_precision_storage_matches_oracle():
    """link_prec 1, FP64 transform: per-iteration F and theta against the oracle
    run with the same storage (binary32 two-row links and g, FP64 arithmetic).
    Both round the same FP64 values, so they agree far below the storage
    rounding unless an FP64 difference straddles a binary32 rounding boundary
    (then one entry differs by one binary32 ulp)."""
    dims = (8, 8, 8, 8)
    U = random_links(dims, 0.3, 1)
    n = 25
    _, Uo, Fr, Tr = oracle.fix(dims, U, alpha=ALPHA, eps=-1.0, max_iter=n, f32_storage=True)
    Ud = dev(U)
    fx = GaugeFixer(Ud, link_prec=1)
    fx.step(n)
    Fh, Th = fx.history()
    assert len(Fh) == n + 1
    Fh, Th = np.asarray(Fh), np.asarray(Th)
    assert np.max(np.abs(Fh - Fr)) < 1e-10
    assert np.max(np.abs(Th - Tr) / Tr) < 1e-6
    # the caller's links hold the stored links (binary32 rows)
    got = host(Ud)
    assert np.max(np.abs(got - Uo)) < 1e-6
    rows = got[:, :2]
    assert np.array_equal(rows.real.astype(np.float32).astype(np.float64), rows.real)


@pytest.mark.parametrize("prec", [0, 1])
def test_single_precision_storage_then_fp64_refinement(prec):
    """gf_fix_until with link_prec 1: single-precision storage down to
    refine_theta, FP64 storage down to 1e-15; compared with the oracle doing
    the same two phases (FP64 transform) and with the plain FP64 run."""
    dims = (8, 8, 8, 8)
    U = random_links(dims, 0.3, 1)
    n1, U1, F1, T1 = oracle.fix(dims, U, alpha=ALPHA, eps=1e-10, max_iter=5000, f32_storage=True)
    n2, U2, F2, T2 = oracle.fix(dims, U1, alpha=ALPHA, eps=EPS, max_iter=5000)
    n64, _, F64, _ = oracle.fix(dims, U, alpha=ALPHA, eps=EPS, max_iter=5000)
    Ud = dev(U)
    fx = GaugeFixer(Ud, link_prec=1, refine_theta=1e-10, fft_prec=prec)
    it, F, th = fx.fix_until(EPS, 5000)
    assert th <= EPS
    if prec == 0:
        assert abs(it - (n1 + n2)) <= 1, (it, n1, n2)
        assert abs(F - F2[-1]) < 1e-11
    assert abs(F - F64[-1]) < 1e-6
    Uf = host(Ud)
    assert abs(oracle.plaquette(dims, Uf) - oracle.plaquette(dims, U)) < 1e-6
    M = np.moveaxis(Uf.reshape(4, 3, 3, -1), 3, 1).reshape(-1, 3, 3)
    assert np.max(np.abs(M @ np.conj(np.swapaxes(M, -1, -2)) - np.eye(3))) < 1e-5


def test_single_precision_storage_batch_equals_single(monkeypatch):
    monkeypatch.setenv("GF_TCHUNK", "2")
    monkeypatch.setenv("GF_TCHUNK_BATCH", "2")
    cases = [((8, 8, 8, 8), 0.3, 1), ((12, 8, 6, 4), 0.35, 3)]
    Us = [random_links(d, e, s) for d, e, s in cases]
    single = []
    for U in Us:
        Ud = dev(U)
        fx = GaugeFixer(Ud, link_prec=1, fft_prec=1, fft_schedule=3)
        single.append((fx.fix_until(EPS, 5000), host(Ud)))
    Ubs = [dev(U) for U in Us]
    bx = BatchGaugeFixer(Ubs, link_prec=1, fft_prec=1, fft_schedule=3)
    its, Fs, ths = bx.fix_until(EPS, 5000)
    for k in range(len(cases)):
        (it, F, th), Uf = single[k]
        assert its[k] == it and Fs[k] == F and ths[k] == th
        assert np.array_equal(host(Ubs[k]), Uf)


@pytest.mark.parametrize("dims", [(16, 16, 2, 4), (24, 24, 2, 2), (32, 32, 2, 4), (48, 48, 2, 2), (64, 64, 2, 2)])
@pytest.mark.parametrize("reg", ["1", "0"])
def test_single_precision_storage_register_xy_passes(monkeypatch, dims, reg):
    """Single-precision storage with the FP32 transform on 16 x 16 to 64 x 64
    xy-planes, whose inverse (x, y) pass (GF_XY_REG=1) forms the
    binary32 two-row g from the four fields in registers (0: the LDS-staged
    pass): per-iteration F and theta against the oracle's run with the same
    storage (FP64 transform), then the refinement down to 1e-15."""
    monkeypatch.setenv("GF_XY_REG", reg)
    U = random_links(dims, 0.3, 75)
    n = 20
    _, _, Fr, Tr = oracle.fix(dims, U, alpha=ALPHA, eps=-1.0, max_iter=n, f32_storage=True)
    fx = GaugeFixer(dev(U), link_prec=1, fft_prec=1, fft_schedule=3)
    fx.step(n)
    Fh, Th = map(np.asarray, fx.history())
    assert np.max(np.abs(Fh - Fr)) < 1e-6
    assert np.max(np.abs(Th - Tr) / Tr) < 1e-3
    Ud = dev(U)
    fx = GaugeFixer(Ud, link_prec=1, fft_prec=1, refine_theta=1e-10, fft_schedule=3)
    it, F, th = fx.fix_until(EPS, 5000)
    assert th <= EPS
    _, _, F64, _ = oracle.fix(dims, U, alpha=ALPHA, eps=EPS, max_iter=5000)
    assert abs(F - F64[-1]) < 1e-6
    Uf = host(Ud)
    assert abs(oracle.plaquette(dims, Uf) - oracle.plaquette(dims, U)) < 1e-6


def test_single_precision_storage_register_xy_batch_equals_single(monkeypatch):
    monkeypatch.setenv("GF_TCHUNK", "2")
    monkeypatch.setenv("GF_TCHUNK_BATCH", "2")
    cases = [((32, 32, 2, 4), 0.3, 76), ((48, 48, 2, 2), 0.3, 77), ((8, 8, 8, 8), 0.3, 78),
             ((16, 16, 2, 4), 0.3, 87), ((24, 24, 2, 2), 0.3, 88)]
    Us = [random_links(d, e, s) for d, e, s in cases]
    single = []
    for U in Us:
        Ud = dev(U)
        fx = GaugeFixer(Ud, link_prec=1, fft_prec=1, fft_schedule=3)
        single.append((fx.fix_until(EPS, 5000), host(Ud)))
    Ubs = [dev(U) for U in Us]
    bx = BatchGaugeFixer(Ubs, link_prec=1, fft_prec=1, fft_schedule=3)
    its, Fs, ths = bx.fix_until(EPS, 5000)
    for k in range(len(cases)):
        (it, F, th), Uf = single[k]
        assert its[k] == it and Fs[k] == F and ths[k] == th, (k, its[k], it)
        assert np.array_equal(host(Ubs[k]), Uf)


# ---------------------------------------------------------------- z and t lines of 16 to 64 points

# both axes in registers (64, 48 and 32 points over four lanes: 4 x 4,
# 16 x 2, 6 x 8, 8 x 2 xy-planes; 24 and 16 points over two lanes: 8 x 4,
# 16 x 2); lines of different lengths and lane counts in one configuration;
# only the t lines (z = 12; z = 16 on 4 x 4 xy-planes, fewer than the 32
# xy-sites a two-lane row needs) or only the z lines (t = 8)
LINE_SHAPES = [(4, 4, 64, 64), (16, 2, 64, 64), (6, 8, 64, 64), (4, 4, 48, 48), (8, 2, 32, 32),
               (4, 4, 32, 64), (8, 2, 12, 48), (4, 4, 64, 8), (8, 4, 24, 24), (16, 2, 16, 16),
               (4, 8, 16, 32), (4, 4, 16, 32), (8, 4, 24, 8)]


@pytest.mark.parametrize("dims", LINE_SHAPES)
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("sched,line", [(1, "1"), (2, "1"), (2, "0")])
def test_line_register_passes_match_oracle(monkeypatch, dims, prec, sched, line):
    """The 1D z and t passes with their lines in registers (GF_LINE_REG=1,
    k_fft_line: forward z, forward t + K(p) + backward t, backward z) and
    LDS-staged (0), in schedules 1 and 2: the plain transform of three fields
    (an odd field count) both ways and the gauge vector against the oracle."""
    monkeypatch.setenv("GF_LINE_REG", line)
    U = random_links(dims, 0.4, 61)
    fx = GaugeFixer(dev(U), fft_prec=prec, fft_schedule=sched)
    g = host(fx.gauge())
    gref = oracle.gauge_from_delta(dims, oracle.delta(dims, U), ALPHA)
    assert np.max(np.abs(g - gref)) < (fp32_gauge_tolerance(dims) if prec else 1e-13)
    V = int(np.prod(dims))
    rng = np.random.default_rng(62)
    f = rng.standard_normal((3, V)) + 1j * rng.standard_normal((3, V))
    ct = torch.complex64 if prec else torch.complex128
    tol = 3e-6 if prec else 1e-13
    for sign in (-1, +1):
        got = host(fx.fft(torch.from_numpy(f).to(ct).to("cuda").contiguous(), sign)).astype(np.complex128)
        for k in range(3):
            ref = oracle.fft4d(dims, f[k], sign)
            assert np.max(np.abs(got[k] - ref)) < tol * np.max(np.abs(ref)), (sign, k)


def test_line_batch_equals_single_runs(monkeypatch):
    """A batch mixing configurations whose z and t lines run in registers
    (64 and 48 points, so two instances per pass) with one that takes the
    LDS-staged 1D passes (schedule 2, all in one launch per pass): every
    member bitwise equal to its own context's run."""
    monkeypatch.setenv("GF_TCHUNK", "2")
    monkeypatch.setenv("GF_TCHUNK_BATCH", "2")
    cases = [((4, 4, 64, 64), 0.3, 63), ((8, 8, 8, 8), 0.3, 64), ((16, 2, 64, 64), 0.35, 65),
             ((4, 4, 48, 48), 0.3, 66)]
    Us = [random_links(d, e, s) for d, e, s in cases]
    single = []
    for U in Us:
        Ud = dev(U)
        fx = GaugeFixer(Ud, fft_prec=1, fft_schedule=2)
        single.append((fx.fix_until(EPS, 5000), host(Ud)))
    Ubs = [dev(U) for U in Us]
    bx = BatchGaugeFixer(Ubs, fft_prec=1, fft_schedule=2)
    its, Fs, ths = bx.fix_until(EPS, 5000)
    for k in range(len(cases)):
        (it, F, th), Uf = single[k]
        assert its[k] == it and Fs[k] == F and ths[k] == th, (k, its[k], it)
        assert np.array_equal(host(Ubs[k]), Uf)


@pytest.mark.parametrize("sched", [2, 3])
@pytest.mark.parametrize("prec", [0, 1])
def test_register_plane_sizes_batch_equals_single_runs(monkeypatch, sched, prec):
    """A batch of 32 x 32, 48 x 48 and 64 x 64 xy-planes (three instances of
    each register (x, y) pass in one iteration; the final reduction folded
    into the 32- or 64-point instance, which the 48-point one, with 192
    work-items, cannot carry) beside an LDS-staged member: every member
    bitwise equal to its own context's run (where a lone 48-point member
    launches its own reduction)."""
    monkeypatch.setenv("GF_TCHUNK", "2")
    monkeypatch.setenv("GF_TCHUNK_BATCH", "2")
    cases = [((32, 32, 2, 4), 0.3, 71), ((48, 48, 2, 2), 0.3, 72), ((64, 64, 2, 2), 0.35, 73),
             ((8, 8, 8, 8), 0.3, 74)]
    Us = [random_links(d, e, s) for d, e, s in cases]
    single = []
    for U in Us:
        Ud = dev(U)
        fx = GaugeFixer(Ud, fft_prec=prec, fft_schedule=sched)
        single.append((fx.fix_until(EPS, 5000), host(Ud)))
    Ubs = [dev(U) for U in Us]
    bx = BatchGaugeFixer(Ubs, fft_prec=prec, fft_schedule=sched)
    its, Fs, ths = bx.fix_until(EPS, 5000)
    for k in range(len(cases)):
        (it, F, th), Uf = single[k]
        assert its[k] == it and Fs[k] == F and ths[k] == th, (k, its[k], it)
        assert np.array_equal(host(Ubs[k]), Uf)


@pytest.mark.parametrize("sched", [2, 3])
@pytest.mark.parametrize("prec", [0, 1])
def test_two_lane_lines_batch_equals_single_runs(monkeypatch, sched, prec):
    """A batch of members whose register lines span two lanes (16 x 16 and
    24 x 24 xy-planes; 16- and 24-point z and t lines) beside four-lane ones
    (32-point t lines, 32 x 32 planes) and an LDS-staged member: the register
    (x, y) passes run their 16-, 24- and 32-point instances in one iteration,
    the 16-point one carrying the folded reduction; every member bitwise
    equal to its own context's run."""
    monkeypatch.setenv("GF_TCHUNK", "2")
    monkeypatch.setenv("GF_TCHUNK_BATCH", "2")
    cases = [((16, 16, 2, 4), 0.3, 81), ((24, 24, 4, 4), 0.3, 82), ((8, 4, 24, 24), 0.3, 83),
             ((4, 8, 16, 32), 0.35, 84), ((32, 32, 2, 2), 0.3, 85), ((8, 8, 8, 8), 0.3, 86)]
    Us = [random_links(d, e, s) for d, e, s in cases]
    single = []
    for U in Us:
        Ud = dev(U)
        fx = GaugeFixer(Ud, fft_prec=prec, fft_schedule=sched)
        single.append((fx.fix_until(EPS, 5000), host(Ud)))
    Ubs = [dev(U) for U in Us]
    bx = BatchGaugeFixer(Ubs, fft_prec=prec, fft_schedule=sched)
    its, Fs, ths = bx.fix_until(EPS, 5000)
    for k in range(len(cases)):
        (it, F, th), Uf = single[k]
        assert its[k] == it and Fs[k] == F and ths[k] == th, (k, its[k], it)
        assert np.array_equal(host(Ubs[k]), Uf)


# ---------------------------------------------------------------- 32 x 32 (z, t) planes

# 32 x 32 (z, t) planes (k_fft_zt_reg) and 24 x 24, 16 x 16, 16 x 32, 48 x 48
# ones (k_fft_zt_lines; 24-point planes need 4 or 8 xy-sites per tile and
# 48-point planes 2, other widths take the LDS-staged pass)
ZT32_SHAPES = [(2, 2, 32, 32), (4, 2, 32, 32), (6, 4, 32, 32), (8, 8, 32, 32), (16, 2, 32, 32), (4, 2, 24, 24),
               (4, 4, 24, 24), (2, 2, 16, 16), (4, 4, 16, 16), (6, 4, 24, 24), (2, 2, 16, 32), (4, 4, 16, 32),
               (6, 2, 16, 32), (2, 2, 48, 48), (6, 2, 48, 48)]


@pytest.mark.parametrize("dims", ZT32_SHAPES)
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("reg", ["1", "2", "4", "0", "1/4", "2/8", "4/8", "2/2"])
def test_zt_register_pass_matches_oracle(monkeypatch, dims, prec, reg):
    """The scaled (z, t) pass of 32 x 32, 24 x 24, 16 x 16 and 16 x 32 planes
    with its radix stages in registers (GF_ZT_REG = work-groups per tile, 1, 2 or 4; after the slash
    GF_ZT_REG_P = xy-sites per tile, 2, 4 or 8, where it divides Lx Ly) and
    LDS-staged (GF_ZT_REG=0): the
    gauge vector of the xy + zt schedule against the oracle; 6 x 4 xy-planes
    take the general-extent xy instances beside it."""
    g, _, P = reg.partition("/")
    monkeypatch.setenv("GF_ZT_REG", g)
    if P:
        monkeypatch.setenv("GF_ZT_REG_P", P)
    U = random_links(dims, 0.4, 47)
    fx = GaugeFixer(dev(U), fft_prec=prec, fft_schedule=3)
    g = host(fx.gauge())
    gref = oracle.gauge_from_delta(dims, oracle.delta(dims, U), ALPHA)
    assert np.max(np.abs(g - gref)) < (fp32_gauge_tolerance(dims) if prec else 1e-13)


@pytest.mark.parametrize("dims,seed,P", [((4, 2, 32, 32), 48, "2"), ((6, 4, 32, 32), 49, "4"),
                                         ((16, 2, 32, 32), 50, "8"), ((4, 2, 24, 24), 93, "4"),
                                         ((4, 4, 24, 24), 94, "8"), ((2, 4, 16, 16), 95, "2"),
                                         ((4, 2, 16, 32), 96, "4"), ((2, 2, 48, 48), 97, "2")])
def test_zt_register_pass_trajectory(monkeypatch, dims, seed, P):
    monkeypatch.setenv("GF_ZT_REG_P", P)
    U = random_links(dims, 0.3, seed)
    n_ref, _, Fr, Tr, spread = oracle_reference(dims, U, max_iter=5000)
    fx = GaugeFixer(dev(U), fft_schedule=3)
    it, F, th = fx.fix_until(EPS, 5000)
    Fh, Th = fx.history()
    assert it == n_ref
    compare_trajectory(Fh, Th, Fr, Tr, spread, dims, f"{dims} register zt pass")


# 32 x 32 planes (two per tile; 32 x 32 x 3 x 3 has an odd plane count and
# takes the LDS-staged passes), 48 x 48 and 64 x 64 planes (one per tile),
# 16 x 16 (eight per tile) and 24 x 24 planes (four per tile; 3 x 3 planes
# of either take the LDS-staged passes)
XY32_SHAPES = [(32, 32, 2, 2), (32, 32, 4, 2), (32, 32, 6, 4), (32, 32, 3, 2), (32, 32, 3, 3), (48, 48, 2, 2),
               (48, 48, 3, 3), (64, 64, 2, 2), (64, 64, 3, 3), (16, 16, 2, 4), (16, 16, 4, 6), (16, 16, 3, 3),
               (24, 24, 2, 2), (24, 24, 4, 3), (24, 24, 3, 3)]


@pytest.mark.parametrize("dims", XY32_SHAPES)
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("sched,reg", [(3, "1"), (3, "2"), (3, "4"), (2, "1"), (3, "0")])
def test_xy_register_pass_matches_oracle(monkeypatch, dims, prec, sched, reg):
    """The forward (x, y) pass of 16 x 16 to 64 x 64 planes with its
    radix stages in registers (GF_XY_REG = work-groups per tile) or
    LDS-staged (0), beside
    the (z, t) passes of schedule 3 or the 1D z and t passes of schedule 2:
    the gauge vector against the oracle (the inverse pass then forms g in the
    LDS-staged kernel)."""
    monkeypatch.setenv("GF_XY_REG", reg)
    U = random_links(dims, 0.4, 57)
    fx = GaugeFixer(dev(U), fft_prec=prec, fft_schedule=sched)
    g = host(fx.gauge())
    gref = oracle.gauge_from_delta(dims, oracle.delta(dims, U), ALPHA)
    assert np.max(np.abs(g - gref)) < (fp32_gauge_tolerance(dims) if prec else 1e-13)


@pytest.mark.parametrize("dims,seed,reg", [((32, 32, 4, 2), 58, "1"), ((32, 32, 3, 2), 59, "2"),
                                           ((32, 32, 6, 4), 60, "1"), ((48, 48, 2, 2), 67, "1"),
                                           ((64, 64, 3, 2), 68, "2"), ((16, 16, 2, 4), 79, "1"),
                                           ((24, 24, 4, 3), 80, "2")])
def test_xy_register_pass_trajectory(monkeypatch, dims, seed, reg):
    """Both register (x, y) passes in the iteration (the inverse one writes the
    filtered fields the fused pass forms g from) against the oracle."""
    monkeypatch.setenv("GF_XY_REG", reg)
    U = random_links(dims, 0.3, seed)
    n_ref, _, Fr, Tr, spread = oracle_reference(dims, U, max_iter=5000)
    fx = GaugeFixer(dev(U), fft_schedule=3)
    it, F, th = fx.fix_until(EPS, 5000)
    Fh, Th = fx.history()
    assert it == n_ref
    compare_trajectory(Fh, Th, Fr, Tr, spread, dims, f"{dims} register xy passes")
