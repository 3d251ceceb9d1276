"""Pins of the oracle's 4D Fourier transform (Alg. 1, "apply FFT forward/backward").

The transform is checked against a brute-force DFT written as an explicit sum
(a V x V matrix of phases exp(-i p.x) built from the site coordinates), on 4^4
as the method statement asks and on shapes with factors 3 and 5 (the workloads
need lengths 12, 24 and 48).
"""
import numpy as np
import pytest


def coords(dims):
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel(), t.ravel()], axis=1)  # (V, 4), site order


def brute_dft(dims, f, sign):
    c = coords(dims).astype(np.float64)
    L = np.asarray(dims, dtype=np.float64)
    phase = (c / L) @ c.T  # sum_mu k_mu x_mu / L_mu, rows k, columns x
    E = np.exp(sign * 2j * np.pi * phase)
    return E @ f


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 3, 2), (3, 3, 3, 3), (5, 2, 3, 4), (2, 2, 2, 2)])
@pytest.mark.parametrize("sign", [-1, +1])
def test_fft_matches_brute_force(orc, dims, sign):
    rng = np.random.default_rng(11)
    V = int(np.prod(dims))
    f = rng.standard_normal(V) + 1j * rng.standard_normal(V)
    got = orc.fft4d(dims, f, sign)
    ref = brute_dft(dims, f, sign)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_fft_roundtrip_and_parseval(orc):
    dims = (12, 8, 6, 4)
    rng = np.random.default_rng(3)
    V = int(np.prod(dims))
    f = rng.standard_normal(V) + 1j * rng.standard_normal(V)
    F = orc.fft4d(dims, f, -1)
    back = orc.fft4d(dims, F, +1) / V
    assert np.max(np.abs(back - f)) < 1e-13
    assert abs(np.sum(np.abs(F) ** 2) - V * np.sum(np.abs(f) ** 2)) < 1e-11 * V * np.sum(np.abs(f) ** 2)


def test_fft_impulse_and_constant(orc):
    dims = (4, 6, 2, 8)
    V = int(np.prod(dims))
    imp = np.zeros(V, dtype=np.complex128)
    imp[0] = 1.0
    assert np.allclose(orc.fft4d(dims, imp, -1), np.ones(V), atol=1e-15)
    const = np.ones(V, dtype=np.complex128)
    out = orc.fft4d(dims, const, -1)
    assert abs(out[0] - V) < 1e-12 and np.max(np.abs(out[1:])) < 1e-12


def test_fft_single_mode(orc):
    # exp(+i p.x) for a chosen momentum n transforms to V at that momentum only.
    dims = (8, 12, 6, 4)
    n = np.array([3, 5, 1, 2])
    c = coords(dims)
    f = np.exp(2j * np.pi * np.sum(c * n / np.asarray(dims), axis=1))
    out = orc.fft4d(dims, f, -1)
    k = n[0] + dims[0] * (n[1] + dims[1] * (n[2] + dims[2] * n[3]))
    V = int(np.prod(dims))
    assert abs(out[k] - V) < 1e-10
    out[k] = 0
    assert np.max(np.abs(out)) < 1e-10


def test_fft_numpy_cross_check(orc):
    # numpy's FFT is an independent implementation (the oracle does not call it).
    dims = (12, 8, 6, 4)
    rng = np.random.default_rng(5)
    V = int(np.prod(dims))
    f = rng.standard_normal(V) + 1j * rng.standard_normal(V)
    ref = np.fft.fftn(f.reshape(dims[::-1])).ravel()
    got = orc.fft4d(dims, f, -1)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
