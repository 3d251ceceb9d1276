"""ctypes wrapper of the CPU oracle (``gf_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users. The product path never imports this
package. Arrays are numpy, complex128 / float64, in the lattice conventions of
``gf_oracle.c`` (SoA links of shape (4, 3, 3, Lt, Lz, Ly, Lx)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gf_oracle.c")
_LIB = os.path.join(_HERE, "libgforacle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu99", "-fopenmp", "-fcx-limited-range", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        sig = {
            "or_delta": (None, [P, P, P]),
            "or_measure": (None, [P, P, P, P]),
            "or_fft4d": (None, [P, P, ctypes.c_int]),
            "or_set_fft_axis_order": (None, [P]),
            "or_momentum_factor": (None, [P, D, P]),
            "or_reunit": (None, [P]),
            "or_gauge_from_delta": (None, [P, P, D, P]),
            "or_apply_gauge": (None, [P, P, P]),
            "or_reunit_links": (None, [P, P]),
            "or_fix": (I64, [P, P, D, D, I64, ctypes.c_int, P, P, I64]),
            "or_fix_f32_storage": (I64, [P, P, D, D, I64, ctypes.c_int, P, P, I64]),
            "or_fix_two_row": (I64, [P, P, D, D, I64, ctypes.c_int, P, P, I64]),
            "or_store_f32": (None, [P, P, ctypes.c_int]),
            "or_plaquette": (D, [P, P]),
            "or_polyakov": (None, [P, P, P, P]),
            "or_eigh3": (None, [P, P, P]),
            "or_expi": (None, [P, P]),
            "or_expi_frechet": (None, [P, P, P]),
            "or_gauge_from_omega": (None, [P, P, P]),
            "or_functional_g": (D, [P, P, P]),
            "or_local_functional_g": (D, [P, P, P, I64, P]),
            "or_grad_omega_sites": (None, [P, P, P, I64, P, P]),
            "or_grad_links": (None, [P, P, P]),
            "or_philox4x32_10": (None, [P, P, P]),
            "or_heatbath": (None, [P, P, D, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, I64]),
            "or_kp_samples": (I64, [D, I64, ctypes.c_uint64, P]),
            "or_overrelax": (None, [P, P, ctypes.c_int]),
            "or_num_threads": (ctypes.c_int, []),
            "or_set_num_threads": (None, [ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dims(dims):
    return np.ascontiguousarray(np.asarray(dims, dtype=np.int32))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _vol(dims):
    return int(np.prod(np.asarray(dims, dtype=np.int64)))


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(n: int) -> None:
    lib().or_set_num_threads(int(n))


def delta(dims, U):
    """Delta(x) (Eq. 5) as (3, 3, V) complex128."""
    U = _c128(U)
    V = _vol(dims)
    out = np.empty((3, 3, V), dtype=np.complex128)
    d = _dims(dims)
    lib().or_delta(_p(d), _p(U), _p(out))
    return out


def measure(dims, U):
    """(F, theta) of the current links (Eq. 1 at g = 1, Eq. 4)."""
    U = _c128(U)
    d = _dims(dims)
    F = ctypes.c_double()
    th = ctypes.c_double()
    lib().or_measure(_p(d), _p(U), ctypes.byref(F), ctypes.byref(th))
    return F.value, th.value


def fft4d(dims, f, sign: int):
    """Unnormalised 4D transform of one complex field (V,), sign -1 forward, +1 backward."""
    f = np.array(f, dtype=np.complex128, copy=True).reshape(-1)
    d = _dims(dims)
    lib().or_fft4d(_p(d), _p(f), int(sign))
    return f


def momentum_factor(dims, alpha: float):
    d = _dims(dims)
    K = np.empty(_vol(dims), dtype=np.float64)
    lib().or_momentum_factor(_p(d), float(alpha), _p(K))
    return K


def reunit(m):
    """Row Gram-Schmidt projection of one 3x3 matrix to SU(3)."""
    m = np.array(m, dtype=np.complex128, copy=True).reshape(3, 3)
    lib().or_reunit(_p(m))
    return m


def gauge_from_delta(dims, Delta, alpha: float):
    """g(x) (3, 3, V) from Delta (3, 3, V)."""
    Delta = _c128(Delta)
    g = np.empty_like(Delta)
    d = _dims(dims)
    lib().or_gauge_from_delta(_p(d), _p(Delta), float(alpha), _p(g))
    return g


def apply_gauge(dims, U, g):
    """U_mu(x) -> g(x) U_mu(x) g^dag(x+mu); returns a new array."""
    U = np.array(U, dtype=np.complex128, copy=True)
    g = _c128(g)
    d = _dims(dims)
    lib().or_apply_gauge(_p(d), _p(U), _p(g))
    return U


def reunit_links(dims, U):
    U = np.array(U, dtype=np.complex128, copy=True)
    d = _dims(dims)
    lib().or_reunit_links(_p(d), _p(U))
    return U


def set_fft_axis_order(order=(0, 1, 2, 3)):
    """Order in which the 4D transform takes the axes (a permutation of 0..3)."""
    o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    lib().or_set_fft_axis_order(_p(o))


def fix(dims, U, alpha=0.08, eps=1e-15, max_iter=100000, reunit_every=0, hist_cap=None, f32_storage=False,
        fft_axis_order=None, two_row=False):
    """Alg. 1 on a copy of U. Returns (iters, U_final, F_hist, theta_hist).

    f32_storage: links and g kept in single-precision 12-real storage
    (or_fix_f32_storage); U_final is then the stored links.
    two_row: the 12-real representation kept in FP64 (or_fix_two_row).
    fft_axis_order: the transform's axis order for this run (default x, y, z, t).
    """
    if fft_axis_order is not None:
        set_fft_axis_order(fft_axis_order)
        try:
            return fix(dims, U, alpha, eps, max_iter, reunit_every, hist_cap, f32_storage, two_row=two_row)
        finally:
            set_fft_axis_order()
    U = np.array(U, dtype=np.complex128, copy=True)
    d = _dims(dims)
    cap = int(max_iter) + 1 if hist_cap is None else int(hist_cap)
    cap = min(cap, 10_000_000)
    Fh = np.zeros(cap, dtype=np.float64)
    Th = np.zeros(cap, dtype=np.float64)
    f = lib().or_fix_f32_storage if f32_storage else (lib().or_fix_two_row if two_row else lib().or_fix)
    n = f(_p(d), _p(U), float(alpha), float(eps), int(max_iter), int(reunit_every), _p(Fh), _p(Th), cap)
    k = min(n + 1, cap)
    return int(n), U, Fh[:k].copy(), Th[:k].copy()


def rounding_spread(dims, U, alpha=0.08, eps=1e-15, max_iter=100000, reunit_every=0):
    """Per-iteration relative differences of F and theta between two FP64 runs of
    Alg. 1 that differ only in the transform's axis order (x, y, z, t against
    t, z, y, x): the spread of two correct implementations, over the iterations
    both made. Returns (dF, dtheta, iters_default, iters_reversed)."""
    n0, _, F0, T0 = fix(dims, U, alpha, eps, max_iter, reunit_every)
    n1, _, F1, T1 = fix(dims, U, alpha, eps, max_iter, reunit_every, fft_axis_order=(3, 2, 1, 0))
    k = min(len(F0), len(F1))
    dF = np.abs(F1[:k] - F0[:k]) / np.abs(F0[:k]).clip(1e-300)
    dT = np.abs(T1[:k] - T0[:k]) / np.abs(T0[:k]).clip(1e-300)
    return dF, dT, n0, n1


def store_f32(dims, M):
    """Single-precision 12-real storage (or_store_f32) of a copy of the matrix fields M [n][3][3][V]."""
    M = np.array(M, dtype=np.complex128, copy=True)
    d = _dims(dims)
    n = M.size // (9 * int(np.prod(dims)))
    lib().or_store_f32(_p(d), _p(M), n)
    return M


def philox4x32_10(ctr, key):
    """Philox4x32-10 block: four uint32 outputs for a 4-word counter and 2-word key."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def heatbath(dims, U, beta, n_sweeps, n_or=0, seed=0, sweep0=0):
    """Wilson-action heatbath + overrelaxation sweeps on a copy of U (every extent even)."""
    U = np.array(U, dtype=np.complex128, copy=True)
    d = _dims(dims)
    lib().or_heatbath(_p(d), _p(U), float(beta), int(n_sweeps), int(n_or), int(seed), int(sweep0))
    return U


def overrelax(dims, U, n):
    """n overrelaxation sweeps on a copy of U."""
    U = np.array(U, dtype=np.complex128, copy=True)
    d = _dims(dims)
    lib().or_overrelax(_p(d), _p(U), int(n))
    return U


def kp_samples(a, n, seed=0):
    """x0 of n Kennedy-Pendleton draws at parameter a (accepted ones)."""
    out = np.zeros(int(n), dtype=np.float64)
    m = lib().or_kp_samples(float(a), int(n), int(seed), _p(out))
    return out[:m]


def plaquette(dims, U):
    U = _c128(U)
    d = _dims(dims)
    return lib().or_plaquette(_p(d), _p(U))


def polyakov(dims, U):
    U = _c128(U)
    d = _dims(dims)
    re = ctypes.c_double()
    im = ctypes.c_double()
    lib().or_polyakov(_p(d), _p(U), ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def eigh3(Q):
    Q = np.array(Q, dtype=np.complex128, copy=True).reshape(3, 3)
    lam = np.empty(3)
    W = np.empty((3, 3), dtype=np.complex128)
    lib().or_eigh3(_p(Q), _p(lam), _p(W))
    return lam, W


def expi(Q):
    """exp(i Q) for one hermitian 3x3 Q."""
    Q = np.array(Q, dtype=np.complex128, copy=True).reshape(3, 3)
    out = np.empty((3, 3), dtype=np.complex128)
    lib().or_expi(_p(Q), _p(out))
    return out


def expi_frechet(Q, E):
    """Frechet derivative of exp at iQ in direction E."""
    Q = np.array(Q, dtype=np.complex128, copy=True).reshape(3, 3)
    E = np.array(E, dtype=np.complex128, copy=True).reshape(3, 3)
    out = np.empty((3, 3), dtype=np.complex128)
    lib().or_expi_frechet(_p(Q), _p(E), _p(out))
    return out


def gauge_from_omega(dims, omega):
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    g = np.empty((3, 3, _vol(dims)), dtype=np.complex128)
    d = _dims(dims)
    lib().or_gauge_from_omega(_p(d), _p(omega), _p(g))
    return g


def functional_g(dims, U, omega):
    U = _c128(U)
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    d = _dims(dims)
    return lib().or_functional_g(_p(d), _p(U), _p(omega))


def local_functional_g(dims, U, omega, site: int, w_site):
    U = _c128(U)
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    w = np.ascontiguousarray(w_site, dtype=np.float64)
    d = _dims(dims)
    return lib().or_local_functional_g(_p(d), _p(U), _p(omega), int(site), _p(w))


def grad_omega_sites(dims, U, omega, sites):
    U = _c128(U)
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(sites), 8), dtype=np.float64)
    d = _dims(dims)
    lib().or_grad_omega_sites(_p(d), _p(U), _p(omega), len(sites), _p(sites), _p(out))
    return out


def grad_links(dims, omega):
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    V = _vol(dims)
    out = np.empty((4, 3, 3, V), dtype=np.complex128)
    d = _dims(dims)
    lib().or_grad_links(_p(d), _p(omega), _p(out))
    return out
