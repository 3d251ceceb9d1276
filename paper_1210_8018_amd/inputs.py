"""Seeded synthetic SU(3) link fields.

This module only draws inputs. It holds none of the gauge-fixing arithmetic
(no divergence, no Fourier transform, no functional), so both the CPU oracle
and the HIP path can take their inputs from here.

Recipe (one definition for every workload):

* ``rng = numpy.random.Generator(numpy.random.PCG64(seed))``.
* In batch mode the amplitude ``eps`` is drawn first, ``eps ~ U[lo, hi)``.
* ``h(x)``: a Haar-random SU(3) matrix for every site, in lexicographic site
  order. Method of Mezzadri (Notices AMS 54, 2007): complex Ginibre matrix with
  entries ``(N(0,1) + i N(0,1))/sqrt(2)``, QR decomposition, columns of Q
  multiplied by the phases of diag(R) (this gives Haar U(3)), then division by
  the principal cube root of the determinant (Haar SU(3)).
* ``w``: shape ``(4, V, 8)``, i.i.d. ``N(0, 1)``.
* ``V_mu(x) = exp(i eps sum_a lambda_a w_{mu,x,a})`` with the Gell-Mann
  matrices ``lambda_a``; the exponential of the hermitian argument is taken
  from its eigendecomposition.
* ``U_mu(x) = h(x) V_mu(x) h^dagger(x + mu)``: a near-identity field hidden
  behind a random gauge rotation, so the gauge-fixed result is far from the
  input and the whole iteration is exercised.

Lattice conventions: ``dims = (Lx, Ly, Lz, Lt)``; site ``s = x + Lx*(y +
Ly*(z + Lz*t))``; direction ``mu = 0..3`` is x, y, z, t; periodic boundaries.
Links are returned in structure-of-arrays form, complex128 of shape
``(4, 3, 3, Lt, Lz, Ly, Lx)`` (that is ``U[mu][i][j][s]``).
"""
from __future__ import annotations

import os

import numpy as np

__all__ = [
    "gell_mann",
    "haar_su3",
    "random_links",
    "random_omega",
    "batch_workload",
    "volume",
    "aos_to_soa",
    "soa_to_aos",
]


def volume(dims) -> int:
    v = 1
    for L in dims:
        v *= int(L)
    return v


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, normalised Tr(l_a l_b) = 2 delta_ab."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0, 0, 1] = l[0, 1, 0] = 1
    l[1, 0, 1] = -1j
    l[1, 1, 0] = 1j
    l[2, 0, 0] = 1
    l[2, 1, 1] = -1
    l[3, 0, 2] = l[3, 2, 0] = 1
    l[4, 0, 2] = -1j
    l[4, 2, 0] = 1j
    l[5, 1, 2] = l[5, 2, 1] = 1
    l[6, 1, 2] = -1j
    l[6, 2, 1] = 1j
    l[7, 0, 0] = l[7, 1, 1] = 1 / np.sqrt(3)
    l[7, 2, 2] = -2 / np.sqrt(3)
    return l


def _workers() -> int:
    return max(1, min(16, int(os.environ.get("GF_GEN_PROCS", os.cpu_count() or 1))))


_POOL_MIN = 1 << 20  # sites from which the per-matrix arithmetic is spread over processes


# Shared blocks between the generator and its worker processes are plain
# files in /dev/shm (memory-backed), mapped by both sides: unlike
# multiprocessing.shared_memory this starts no resource-tracker process that
# could outlive the caller. The parent creates and removes every file.
def _shm_dir() -> str:
    return "/dev/shm" if os.path.isdir("/dev/shm") else __import__("tempfile").gettempdir()


def _shm_put(arr, owned):
    import mmap
    import tempfile

    fd, path = tempfile.mkstemp(prefix="gf_gen_", dir=_shm_dir())
    owned.append(path)
    try:
        os.ftruncate(fd, max(1, arr.nbytes))
        with mmap.mmap(fd, max(1, arr.nbytes)) as m:
            np.ndarray(arr.shape, arr.dtype, buffer=m)[...] = arr
    finally:
        os.close(fd)
    return (path, arr.shape, arr.dtype.str)


def _shm_get(desc, keep):
    import mmap

    path, shape, dt = desc
    shape = tuple(shape)
    nbytes = int(np.prod(shape, dtype=np.int64)) * np.dtype(dt).itemsize
    fd = os.open(path, os.O_RDWR)
    try:
        m = mmap.mmap(fd, max(1, nbytes))
    finally:
        os.close(fd)
    keep.append(m)
    return np.ndarray(shape, np.dtype(dt), buffer=m)


def _worker_main():
    """Entry of a generator worker process: one slice of one per-matrix job.

    Reads a JSON job from stdin: the shared-memory blocks of the inputs and
    the output, the slice [a, b) and eps.
    """
    import json
    import sys

    job = json.loads(sys.stdin.read())
    keep = []
    arrs = [_shm_get(tuple(d), keep) for d in job["descs"]]
    a, b = job["a"], job["b"]
    if job["kind"] == "haar":
        z, out = arrs
        out[a:b] = _haar_from_ginibre(z[a:b])
    else:
        h, w, fwd, out = arrs
        out[a:b] = _link_block(h[a:b], job["eps"] * w[a:b], h[fwd[a:b]])
    for m in keep:
        m.flush()


def _parallel(kind, n, inputs, out_shape, eps=0.0):
    """Per-matrix arithmetic of `kind` over n matrices in worker processes.

    Each worker is a fresh interpreter that reads its slice of the inputs and
    writes its slice of the output in shared memory, so the result is bitwise
    the serial one.
    """
    import json
    import subprocess
    import sys

    owned = []
    procs = []
    try:
        descs = [_shm_put(x, owned) for x in inputs]
        out_desc = _shm_put(np.zeros(out_shape, np.complex128), owned)
        nw = _workers()
        bounds = np.linspace(0, n, nw + 1).astype(int)
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        code = "from paper_1210_8018_amd.inputs import _worker_main; _worker_main()"
        for k in range(nw):
            job = json.dumps({"kind": kind, "a": int(bounds[k]), "b": int(bounds[k + 1]), "eps": float(eps),
                              "descs": [list(d) for d in descs + [out_desc]]})
            p = subprocess.Popen([sys.executable, "-c", code], stdin=subprocess.PIPE, cwd=root)
            p.stdin.write(job.encode())
            p.stdin.close()
            procs.append(p)
        for p in procs:
            if p.wait(timeout=1800) != 0:
                raise RuntimeError(f"input generator worker failed with status {p.returncode}")
        return np.fromfile(owned[-1], dtype=np.complex128).reshape(out_shape)
    finally:
        for p in procs:
            if p.poll() is None:
                p.kill()
                p.wait()
        for path in owned:
            try:
                os.unlink(path)
            except OSError:
                pass


def _haar_from_ginibre(z: np.ndarray) -> np.ndarray:
    g = (z[..., 0] + 1j * z[..., 1]) / np.sqrt(2.0)
    q, r = np.linalg.qr(g)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    ph = d / np.abs(d)
    q = q * ph[:, None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[:, None, None]


def haar_su3(rng: np.random.Generator, n: int) -> np.ndarray:
    """``n`` Haar-distributed SU(3) matrices, shape (n, 3, 3) (Mezzadri 2007)."""
    z = rng.standard_normal((n, 3, 3, 2))
    if n >= _POOL_MIN and _workers() > 1:
        return _parallel("haar", n, [z], (n, 3, 3))
    return _haar_from_ginibre(z)


def _expi_hermitian(h: np.ndarray) -> np.ndarray:
    """exp(i h) for a stack of hermitian matrices, via eigendecomposition."""
    w, v = np.linalg.eigh(h)
    return (v * np.exp(1j * w)[..., None, :]) @ np.conj(np.swapaxes(v, -1, -2))


def _link_block(hx, ew, hf):
    """h(x) exp(i sum_a lambda_a ew_a) h^dag(x + mu) for a block of sites."""
    herm = np.einsum("va,aij->vij", ew, gell_mann())
    return hx @ _expi_hermitian(herm) @ np.conj(np.swapaxes(hf, -1, -2))


def _neighbour_forward(dims, mu: int) -> np.ndarray:
    """Index array s -> s + mu-hat (periodic), lexicographic order."""
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    idx = np.arange(Lx * Ly * Lz * Lt).reshape(Lt, Lz, Ly, Lx)
    axis = 3 - mu
    return np.roll(idx, -1, axis=axis).reshape(-1)


def aos_to_soa(u_aos: np.ndarray, dims) -> np.ndarray:
    """(4, V, 3, 3) -> (4, 3, 3, Lt, Lz, Ly, Lx)."""
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    soa = np.ascontiguousarray(np.moveaxis(u_aos, 1, 3))
    return soa.reshape(u_aos.shape[0], 3, 3, Lt, Lz, Ly, Lx)


def soa_to_aos(u_soa: np.ndarray) -> np.ndarray:
    """(n, 3, 3, Lt, Lz, Ly, Lx) -> (n, V, 3, 3)."""
    n = u_soa.shape[0]
    flat = u_soa.reshape(n, 3, 3, -1)
    return np.ascontiguousarray(np.moveaxis(flat, 3, 1))


def random_links(dims, eps: float, seed: int, *, rng: np.random.Generator | None = None,
                 h_identity: bool = False) -> np.ndarray:
    """Link field ``U_mu(x) = h(x) exp(i eps lambda.w) h^dagger(x+mu)``.

    ``h_identity=True`` skips the gauge rotation draw and uses ``h = 1``
    (a field already close to the Landau gauge; used for linear-regime checks).
    Returns complex128 SoA of shape (4, 3, 3, Lt, Lz, Ly, Lx).
    """
    dims = tuple(int(d) for d in dims)
    V = volume(dims)
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(seed))
    if h_identity:
        h = np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 3, 3))
    else:
        h = haar_su3(rng, V)
    w = rng.standard_normal((4, V, 8))
    u = np.empty((4, V, 3, 3), dtype=np.complex128)
    hc = np.ascontiguousarray(h)
    for mu in range(4):
        fwd = _neighbour_forward(dims, mu)
        if V >= _POOL_MIN and _workers() > 1:
            u[mu] = _parallel("link", V, [hc, w[mu], fwd], (V, 3, 3), eps=eps)
        else:
            u[mu] = _link_block(hc, eps * w[mu], hc[fwd])
    return aos_to_soa(u, dims)


def random_omega(dims, sigma: float, seed: int) -> np.ndarray:
    """Lie-algebra gauge parameters ``omega[a][s] ~ N(0, sigma^2)``, shape (8, V) float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return sigma * rng.standard_normal((8, volume(dims)))


#: The batch workload: 8 x 12^4, 8 x 16^3x32, 6 x 24^4, 2 x 32^4, seeds 100..123 in that order.
BATCH_SHAPES = ([(12, 12, 12, 12)] * 8 + [(16, 16, 16, 32)] * 8 + [(24, 24, 24, 24)] * 6
                + [(32, 32, 32, 32)] * 2)


def batch_workload(shapes=None, first_seed: int = 100, eps_range=(0.2, 0.6)):
    """Yield ``(dims, eps, seed, links)`` for each configuration of a batch.

    Each configuration draws its own ``eps ~ U[eps_range)`` first from its own
    generator, then the field.
    """
    shapes = BATCH_SHAPES if shapes is None else shapes
    for k, dims in enumerate(shapes):
        seed = first_seed + k
        rng = np.random.Generator(np.random.PCG64(seed))
        eps = float(rng.uniform(eps_range[0], eps_range[1]))
        yield dims, eps, seed, random_links(dims, eps, seed, rng=rng)
