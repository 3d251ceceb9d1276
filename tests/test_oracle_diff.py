"""Pins of the oracle's functional of Lie-algebra gauge parameters and its gradients.

F_U[g] is Eq. 1 with g(x) = exp(i sum_a lambda_a omega_a(x)). scipy's matrix
exponential and its Frechet derivative are independent implementations (the
oracle uses a Jacobi eigendecomposition and the Daleckii-Krein formula), and
central finite differences of the site-local part of Eq. 1 pin the gradient.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_1210_8018_amd.inputs import gell_mann, random_links, random_omega


def rand_herm(rng, scale=1.0):
    a = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    return scale * (a + a.conj().T) / 2


def test_eigh3_reconstructs(orc):
    rng = np.random.default_rng(0)
    for _ in range(50):
        Q = rand_herm(rng)
        lam, W = orc.eigh3(Q)
        nrm = np.linalg.norm(Q, 2)
        assert np.max(np.abs(W @ np.diag(lam) @ W.conj().T - Q)) < 1e-14 * nrm
        assert np.max(np.abs(W.conj().T @ W - np.eye(3))) < 5e-14
        assert np.allclose(np.sort(lam), np.linalg.eigvalsh(Q), atol=1e-14 * nrm)


def test_expi_on_many_algebra_elements(orc):
    """exp(i omega.lambda) for 20000 draws at the scales the workloads use, against scipy."""
    lam = gell_mann()
    rng = np.random.default_rng(12)
    for sigma in (1e-6, 0.1, 1.5):
        w = sigma * rng.standard_normal((20000 if sigma == 0.1 else 2000, 8))
        Q = np.einsum("na,aij->nij", w, lam)
        for k in range(len(w)):
            e = orc.expi(Q[k])
            assert np.max(np.abs(e - sla.expm(1j * Q[k]))) < 1e-14 * max(1.0, sigma * 8), (sigma, k)


def test_expi_matches_scipy_and_closed_forms(orc):
    rng = np.random.default_rng(1)
    for _ in range(50):
        Q = rand_herm(rng, 2.0)
        assert np.max(np.abs(orc.expi(Q) - sla.expm(1j * Q))) < 1e-13
    d = np.array([0.3, -1.1, 0.8])
    assert np.max(np.abs(orc.expi(np.diag(d)) - np.diag(np.exp(1j * d)))) < 1e-15
    assert np.max(np.abs(orc.expi(np.zeros((3, 3))) - np.eye(3))) == 0.0
    lam = gell_mann()
    # exp(i t lambda_1) on the 2x2 block is cos t + i sin t sigma_x
    t = 0.4
    e = orc.expi(t * lam[0])
    assert abs(e[0, 0] - np.cos(t)) < 1e-15 and abs(e[0, 1] - 1j * np.sin(t)) < 1e-15 and abs(e[2, 2] - 1) < 1e-15


def test_frechet_matches_scipy(orc):
    rng = np.random.default_rng(2)
    for scale in (1e-3, 0.3, 2.0):
        for _ in range(20):
            Q = rand_herm(rng, scale)
            E = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
            _, ref = sla.expm_frechet(1j * Q, E)
            assert np.max(np.abs(orc.expi_frechet(Q, E) - ref)) < 1e-13
    # degenerate spectra: Q = 0 gives L = E; Q = lambda_8 has a doubly degenerate eigenvalue
    E = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    assert np.max(np.abs(orc.expi_frechet(np.zeros((3, 3)), E) - E)) < 1e-15
    Q = 0.7 * gell_mann()[7]
    _, ref = sla.expm_frechet(1j * Q, E)
    assert np.max(np.abs(orc.expi_frechet(Q, E) - ref)) < 1e-13


def test_grad_omega_matches_central_differences(orc):
    dims = (4, 4, 4, 6)
    V = int(np.prod(dims))
    U = random_links(dims, 0.3, 31)
    omega = random_omega(dims, 0.1, 32)
    sites = np.random.default_rng(3).choice(V, 8, replace=False)
    grad = orc.grad_omega_sites(dims, U, omega, sites) * 12 * V  # drop 1/(4 N_c V)
    h = 1e-6
    for k, s in enumerate(sites):
        w0 = omega[:, s].copy()
        for a in range(8):
            wp = w0.copy()
            wm = w0.copy()
            wp[a] += h
            wm[a] -= h
            fd = (orc.local_functional_g(dims, U, omega, s, wp) - orc.local_functional_g(dims, U, omega, s, wm)) / (2 * h)
            assert abs(fd - grad[k, a]) < 1e-7 * max(1.0, abs(fd)), (s, a, fd, grad[k, a])


def test_grad_omega_at_zero_is_delta(orc):
    """At omega = 0 the gradient is the Lie-algebra components of Delta(x) over 4 N_c V."""
    dims = (4, 6, 4, 4)
    V = int(np.prod(dims))
    U = random_links(dims, 0.4, 33)
    D = orc.delta(dims, U)
    lam = gell_mann()
    sites = np.arange(0, V, 7)
    grad = orc.grad_omega_sites(dims, U, np.zeros((8, V)), sites)
    for k, s in enumerate(sites):
        da = np.array([(-0.5j * np.trace(lam[a] @ D[:, :, s])).real for a in range(8)])
        assert np.max(np.abs(grad[k] * 12 * V - da)) < 1e-13


def test_grad_links_closed_form_and_differences(orc):
    dims = (4, 4, 2, 4)
    V = int(np.prod(dims))
    U = random_links(dims, 0.3, 34)
    # omega = 0: dF/dU = 1/(4 N_c V) on the diagonal
    dU0 = orc.grad_links(dims, np.zeros((8, V)))
    eye = np.zeros_like(dU0)
    for i in range(3):
        eye[:, i, i, :] = 1 / (12 * V)
    assert np.max(np.abs(dU0 - eye)) < 1e-18
    omega = random_omega(dims, 0.3, 35)
    dU = orc.grad_links(dims, omega)
    rng = np.random.default_rng(4)
    h = 1e-3  # F is linear in each link, so central differences are exact up to roundoff
    for _ in range(10):
        mu, i, j, s = rng.integers(4), rng.integers(3), rng.integers(3), rng.integers(V)
        fd = []
        for d in (1.0, 1j):
            Up = U.copy()
            Um = U.copy()
            Up[mu, i, j].reshape(-1)[s] += h * d
            Um[mu, i, j].reshape(-1)[s] -= h * d
            fd.append((orc.functional_g(dims, Up, omega) - orc.functional_g(dims, Um, omega)) / (2 * h))
        got = dU[mu, i, j, s]
        assert abs(fd[0] - got.real) < 1e-10 and abs(fd[1] - got.imag) < 1e-10
