"""The seeded input generator: Haar SU(3) statistics, unitarity, determinism."""
import numpy as np

from paper_1210_8018_amd.inputs import batch_workload, gell_mann, haar_su3, random_links


def test_gell_mann_normalisation():
    lam = gell_mann()
    G = np.einsum("aij,bji->ab", lam, lam)
    assert np.allclose(G, 2 * np.eye(8), atol=1e-15)
    assert np.allclose(lam, np.conj(np.swapaxes(lam, -1, -2)))
    assert np.allclose(np.trace(lam, axis1=1, axis2=2), 0)


def test_haar_moments():
    # For Haar SU(3): E Tr h = 0 and E |Tr h|^2 = 1.
    h = haar_su3(np.random.default_rng(7), 100_000)
    tr = np.trace(h, axis1=1, axis2=2)
    assert abs(np.mean(tr)) < 0.02
    assert abs(np.mean(np.abs(tr) ** 2) - 1) < 0.02
    assert np.max(np.abs(np.linalg.det(h) - 1)) < 1e-13
    assert np.max(np.abs(h @ np.conj(np.swapaxes(h, -1, -2)) - np.eye(3))) < 1e-13


def test_links_su3_and_deterministic():
    dims = (4, 6, 2, 4)
    U = random_links(dims, 0.3, 5)
    assert U.shape == (4, 3, 3, 4, 2, 6, 4)
    M = np.moveaxis(U.reshape(4, 3, 3, -1), 3, 1).reshape(-1, 3, 3)
    assert np.max(np.abs(M @ np.conj(np.swapaxes(M, -1, -2)) - np.eye(3))) < 1e-13
    assert np.max(np.abs(np.linalg.det(M) - 1)) < 1e-13
    assert np.array_equal(U, random_links(dims, 0.3, 5))
    assert not np.array_equal(U, random_links(dims, 0.3, 6))


def test_batch_workload_eps_range():
    shapes = [(4, 4, 4, 4), (4, 4, 2, 6)]
    got = list(batch_workload(shapes, first_seed=100))
    assert [g[2] for g in got] == [100, 101]
    for dims, eps, seed, U in got:
        assert 0.2 <= eps < 0.6
        assert U.shape[3:] == tuple(dims[::-1])


def test_worker_pool_is_bitwise_serial_and_leaves_nothing(monkeypatch):
    """The per-matrix arithmetic spread over worker processes (used for large
    lattices) gives bitwise the serial result and leaves no process and no
    shared file behind."""
    import glob
    import os

    import psutil

    from paper_1210_8018_amd import inputs

    def draw():
        return inputs.random_links((6, 4, 4, 4), 0.3, 9)

    monkeypatch.setattr(inputs, "_POOL_MIN", 1 << 40)
    serial = draw()
    monkeypatch.setattr(inputs, "_POOL_MIN", 100)
    monkeypatch.setenv("GF_GEN_PROCS", "3")
    before = set(glob.glob(os.path.join(inputs._shm_dir(), "gf_gen_*")))
    pooled = draw()
    assert np.array_equal(pooled, serial)
    assert psutil.Process().children(recursive=True) == []
    assert set(glob.glob(os.path.join(inputs._shm_dir(), "gf_gen_*"))) == before
