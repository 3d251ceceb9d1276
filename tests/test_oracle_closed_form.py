"""Closed-form pins of the oracle's normalisations (Eq. 1, Eq. 4, Eq. 5).

An abelian plane wave embedded in one SU(2) subgroup of SU(3),
    U_mu(x) = diag(exp(i phi(x)), exp(-i phi(x)), 1)   (or the same in the
    (0, 2) subgroup), phi(x) = a cos(2 pi x_nu / L_nu + c),
and unit links in the other three directions, has everything in closed form.

  F (Eq. 1 at g = 1, N_c = 3):
      F = [sum_x (2 cos phi(x) + 1) + 9 V] / (12 V).
  Delta (Eq. 5) with D = sum_rho [U_rho(x - rho) - U_rho(x)]: only rho = mu
  contributes, so D = U_mu(x - mu) - U_mu(x) and
      Delta = diag(2 i s(x), -2 i s(x), 0),  s(x) = sin phi(x - mu) - sin phi(x),
  which is already traceless.
  theta (Eq. 4): (1/(N_c V)) sum_x Tr[Delta Delta^dag] = (8 / (3 V)) sum_x s(x)^2.

A longitudinal wave (nu = mu) has theta > 0; a transverse one (nu != mu)
does not depend on x_mu, so D = 0 and theta = 0 exactly: the configuration is
already in Landau gauge while F < 1. A factor error in 1/(N_c V) or 1/(4 N_c V),
a dropped h.c. term, or the neighbour taken at x + mu instead of x - mu fails
one of these.
"""
import numpy as np
import pytest


def plane_wave(dims, mu, nu, a, c=0.0, sub=(0, 1)):
    """Links (4, 3, 3, V) and phi (V,) of the plane wave described above."""
    Lx, Ly, Lz, Lt = dims
    V = Lx * Ly * Lz * Lt
    coords = np.indices((Lt, Lz, Ly, Lx)).reshape(4, -1)[::-1]  # x, y, z, t of site s (x fastest)
    phi = a * np.cos(2 * np.pi * coords[nu] / dims[nu] + c)
    U = np.zeros((4, 3, 3, V), dtype=np.complex128)
    for r in range(4):
        for i in range(3):
            U[r, i, i] = 1.0
    i, j = sub
    U[mu, i, i] = np.exp(1j * phi)
    U[mu, j, j] = np.exp(-1j * phi)
    return U, phi, coords


def shift_back(field, coords, dims, mu):
    """field(x - mu) for a field over sites."""
    c = coords.copy()
    c[mu] = (c[mu] - 1) % dims[mu]
    s = c[0] + dims[0] * (c[1] + dims[1] * (c[2] + dims[2] * c[3]))
    return field[s]


CASES = [
    ((8, 4, 4, 6), 0, 0.7, 0.0, (0, 1)),
    ((4, 6, 4, 4), 1, 1.3, 0.4, (0, 2)),
    ((4, 4, 6, 2), 2, 0.25, 1.1, (1, 2)),
    ((2, 4, 4, 12), 3, 2.0, -0.3, (0, 1)),
]


@pytest.mark.parametrize("dims,mu,a,c,sub", CASES)
def test_longitudinal_plane_wave(orc, dims, mu, a, c, sub):
    U, phi, coords = plane_wave(dims, mu, mu, a, c, sub)
    V = int(np.prod(dims))
    s = np.sin(shift_back(phi, coords, dims, mu)) - np.sin(phi)
    F_cf = (np.sum(2 * np.cos(phi) + 1) + 9 * V) / (12 * V)
    th_cf = 8.0 / (3 * V) * np.sum(s * s)
    F, th = orc.measure(dims, U)
    assert th_cf > 1e-3
    assert abs(F - F_cf) <= 1e-14 * F_cf, (F, F_cf)
    assert abs(th - th_cf) <= 1e-14 * th_cf, (th, th_cf)
    # Delta element by element
    D = orc.delta(dims, U)
    want = np.zeros((3, 3, V), dtype=np.complex128)
    i, j = sub
    want[i, i] = 2j * s
    want[j, j] = -2j * s
    assert np.max(np.abs(D - want)) <= 1e-14


@pytest.mark.parametrize("dims,mu,nu", [((4, 6, 4, 4), 0, 1), ((6, 4, 4, 4), 3, 0), ((4, 4, 6, 4), 1, 2)])
def test_transverse_plane_wave_is_in_landau_gauge(orc, dims, mu, nu):
    U, phi, _ = plane_wave(dims, mu, nu, 0.9, 0.2)
    V = int(np.prod(dims))
    F, th = orc.measure(dims, U)
    F_cf = (np.sum(2 * np.cos(phi) + 1) + 9 * V) / (12 * V)
    assert th == 0.0
    assert abs(F - F_cf) <= 1e-14 * F_cf and F < 1 - 1e-3
    assert np.all(orc.delta(dims, U) == 0)
    # Alg. 1 stops before its first update (theta <= eps already)
    n, _, Fh, _ = orc.fix(dims, U, max_iter=10)
    assert n == 0 and Fh[0] == F
