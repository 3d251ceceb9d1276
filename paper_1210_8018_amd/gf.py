"""ctypes binding of ``libgfix.so`` (the C ABI declared in ``include/gf.h``).

Argument marshalling only: every step of the gauge-fixing iteration runs in
the library's HIP kernels. PyTorch provides device memory (links, workspace,
gradients) and the stream. There is no CPU fallback: if the library is
missing, loading it raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgfix.so")

GF_OK, GF_ERR_ARG, GF_ERR_SHAPE, GF_ERR_HIP, GF_ERR_NONFINITE, GF_ERR_MAXITER, GF_ERR_STATE = range(7)


class gf_params(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int32 * 4),
        ("alpha", ctypes.c_double),
        ("fft_prec", ctypes.c_int32),
        ("reunit_every", ctypes.c_int32),
        ("chunk", ctypes.c_int32),
        ("fft_schedule", ctypes.c_int32),
        ("link_prec", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("refine_theta", ctypes.c_double),
    ]


class GFError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = f"{where}: {strerror(status)}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)


_lib = None


def lib():
    """Load libgfix.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1210_8018_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I32, I64, D, S = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
        PP = ctypes.POINTER(gf_params)
        PD = ctypes.POINTER(ctypes.c_double)
        PI64 = ctypes.POINTER(ctypes.c_int64)
        st = ctypes.c_int
        sig = {
            "gf_workspace_bytes": (S, [PP]),
            "gf_workspace_bytes_batch": (S, [I32, PP]),
            "gf_init": (st, [ctypes.POINTER(P), PP, P, P, S, P]),
            "gf_workspace_bytes_functional": (S, [PP]),
            "gf_init_functional": (st, [ctypes.POINTER(P), PP, P, P, S, P]),
            "gf_init_batch": (st, [ctypes.POINTER(P), I32, PP, ctypes.POINTER(P), P, S, P]),
            "gf_functional": (st, [P, PD, PD]),
            "gf_functional_batch": (st, [P, PD, PD]),
            "gf_step": (st, [P, I32, PD, PD]),
            "gf_fix_until": (st, [P, D, I64, PI64, PD, PD]),
            "gf_fix_until_batch": (st, [P, D, I64, PI64, PD, PD]),
            "gf_fix_until_static": (st, [PP, P, D, I64, PI64, PD, PD, P]),
            "gf_history": (st, [P, I64, PD, PD, PI64]),
            "gf_history_batch": (st, [P, I32, I64, PD, PD, PI64]),
            "gf_delta": (st, [P, P]),
            "gf_gauge": (st, [P, P]),
            "gf_apply_gauge": (st, [P, P]),
            "gf_fft": (st, [P, P, I32, I32]),
            "gf_heatbath": (st, [P, D, I32, I32, ctypes.c_uint64, I64]),
            "gf_plaquette": (st, [P, PD]),
            "gf_functional_g": (st, [P, P, PD]),
            "gf_functional_g_backward": (st, [P, P, D, P, P]),
            "gf_destroy": (st, [P]),
            "gf_strerror": (ctypes.c_char_p, [st]),
            "gf_last_error": (ctypes.c_char_p, [P]),
            "gf_set_timing": (st, [P, I32]),
            "gf_kernel_count": (I32, [P]),
            "gf_kernel_name": (ctypes.c_char_p, [P, I32]),
            "gf_kernel_time": (st, [P, I32, PD, PI64]),
            "gf_reset_timing": (st, [P]),
            "gf_fft_schedule": (I32, [P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().gf_strerror(int(status)).decode()


def _check(status: int, where: str, ctx=None, ok=(GF_OK,)):
    if status not in ok:
        detail = lib().gf_last_error(ctx).decode() if ctx else ""
        raise GFError(status, where, detail)
    return status


def make_params(dims, alpha=0.08, fft_prec=0, reunit_every=0, chunk=0, fft_schedule=0, link_prec=0,
                refine_theta=0.0) -> gf_params:
    p = gf_params()
    for k in range(4):
        p.dims[k] = int(dims[k])
    p.alpha = float(alpha)
    p.fft_prec = int(fft_prec)
    p.reunit_every = int(reunit_every)
    p.chunk = int(chunk)
    p.fft_schedule = int(fft_schedule)
    p.link_prec = int(link_prec)
    p.reserved = 0
    p.refine_theta = float(refine_theta)
    return p


def _stream_ptr(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


# ---------------------------------------------------------------- C-ABI calls
def gf_workspace_bytes(params: gf_params) -> int:
    return int(lib().gf_workspace_bytes(ctypes.byref(params)))


def gf_workspace_bytes_batch(params_list) -> int:
    arr = (gf_params * len(params_list))(*params_list)
    return int(lib().gf_workspace_bytes_batch(len(params_list), arr))


def gf_init(params: gf_params, links: torch.Tensor, ws: torch.Tensor, stream=None):
    ctx = ctypes.c_void_p()
    st = lib().gf_init(ctypes.byref(ctx), ctypes.byref(params), _ptr(links), _ptr(ws), ws.numel() * ws.element_size(),
                       _stream_ptr(stream))
    _check(st, "gf_init")
    return ctx


def gf_workspace_bytes_functional(params: gf_params) -> int:
    return int(lib().gf_workspace_bytes_functional(ctypes.byref(params)))


def gf_init_functional(params: gf_params, links: torch.Tensor, ws: torch.Tensor, stream=None):
    ctx = ctypes.c_void_p()
    st = lib().gf_init_functional(ctypes.byref(ctx), ctypes.byref(params), _ptr(links), _ptr(ws),
                                  ws.numel() * ws.element_size(), _stream_ptr(stream))
    _check(st, "gf_init_functional")
    return ctx


def gf_init_batch(params_list, links_list, ws: torch.Tensor, stream=None):
    n = len(params_list)
    arr = (gf_params * n)(*params_list)
    ptrs = (ctypes.c_void_p * n)(*[_ptr(t) for t in links_list])
    ctx = ctypes.c_void_p()
    st = lib().gf_init_batch(ctypes.byref(ctx), n, arr, ptrs, _ptr(ws), ws.numel() * ws.element_size(),
                             _stream_ptr(stream))
    _check(st, "gf_init_batch")
    return ctx


def gf_functional(ctx):
    F, th = ctypes.c_double(), ctypes.c_double()
    _check(lib().gf_functional(ctx, ctypes.byref(F), ctypes.byref(th)), "gf_functional", ctx)
    return F.value, th.value


def gf_functional_batch(ctx, n: int):
    F = (ctypes.c_double * n)()
    th = (ctypes.c_double * n)()
    _check(lib().gf_functional_batch(ctx, F, th), "gf_functional_batch", ctx)
    return list(F), list(th)


def gf_step(ctx, n: int):
    F, th = ctypes.c_double(), ctypes.c_double()
    _check(lib().gf_step(ctx, int(n), ctypes.byref(F), ctypes.byref(th)), "gf_step", ctx)
    return F.value, th.value


def gf_fix_until(ctx, theta_eps: float, max_iter: int, allow_maxiter: bool = False):
    it = ctypes.c_int64()
    F, th = ctypes.c_double(), ctypes.c_double()
    ok = (GF_OK, GF_ERR_MAXITER) if allow_maxiter else (GF_OK,)
    st = lib().gf_fix_until(ctx, float(theta_eps), int(max_iter), ctypes.byref(it), ctypes.byref(F), ctypes.byref(th))
    _check(st, "gf_fix_until", ctx, ok)
    return int(it.value), F.value, th.value, st


GF_STATIC_SCRATCH_BYTES = 64 * 1024 * 1024  # include/gf.h


def gf_fix_until_static(params: gf_params, links: torch.Tensor, theta_eps: float, max_iter: int,
                        allow_maxiter: bool = False, stream=None):
    """The allocation-free gf_init + gf_fix_until + gf_destroy (workspace in the library's static array)."""
    it = ctypes.c_int64()
    F, th = ctypes.c_double(), ctypes.c_double()
    ok = (GF_OK, GF_ERR_MAXITER) if allow_maxiter else (GF_OK,)
    st = lib().gf_fix_until_static(ctypes.byref(params), _ptr(links), float(theta_eps), int(max_iter),
                                   ctypes.byref(it), ctypes.byref(F), ctypes.byref(th), _stream_ptr(stream))
    _check(st, "gf_fix_until_static", None, ok)
    return int(it.value), F.value, th.value, st


def gf_fix_until_batch(ctx, n: int, theta_eps: float, max_iter: int, allow_maxiter: bool = False):
    it = (ctypes.c_int64 * n)()
    F = (ctypes.c_double * n)()
    th = (ctypes.c_double * n)()
    ok = (GF_OK, GF_ERR_MAXITER) if allow_maxiter else (GF_OK,)
    st = lib().gf_fix_until_batch(ctx, float(theta_eps), int(max_iter), it, F, th)
    _check(st, "gf_fix_until_batch", ctx, ok)
    return list(it), list(F), list(th), st


def gf_history(ctx):
    n = ctypes.c_int64()
    _check(lib().gf_history(ctx, 0, None, None, ctypes.byref(n)), "gf_history", ctx)
    F = (ctypes.c_double * max(1, n.value))()
    T = (ctypes.c_double * max(1, n.value))()
    _check(lib().gf_history(ctx, n.value, F, T, ctypes.byref(n)), "gf_history", ctx)
    return list(F)[: n.value], list(T)[: n.value]


def gf_history_batch(ctx, k: int):
    n = ctypes.c_int64()
    _check(lib().gf_history_batch(ctx, int(k), 0, None, None, ctypes.byref(n)), "gf_history_batch", ctx)
    F = (ctypes.c_double * max(1, n.value))()
    T = (ctypes.c_double * max(1, n.value))()
    _check(lib().gf_history_batch(ctx, int(k), n.value, F, T, ctypes.byref(n)), "gf_history_batch", ctx)
    return list(F)[: n.value], list(T)[: n.value]


def gf_delta(ctx, out: torch.Tensor):
    _check(lib().gf_delta(ctx, _ptr(out)), "gf_delta", ctx)


def gf_gauge(ctx, out: torch.Tensor):
    _check(lib().gf_gauge(ctx, _ptr(out)), "gf_gauge", ctx)


def gf_apply_gauge(ctx, g: torch.Tensor):
    _check(lib().gf_apply_gauge(ctx, _ptr(g)), "gf_apply_gauge", ctx)


def gf_fft(ctx, fields: torch.Tensor, nfields: int, sign: int):
    _check(lib().gf_fft(ctx, _ptr(fields), int(nfields), int(sign)), "gf_fft", ctx)


def gf_heatbath(ctx, beta: float, n_sweeps: int, n_or: int = 0, seed: int = 0, sweep0: int = 0):
    _check(lib().gf_heatbath(ctx, float(beta), int(n_sweeps), int(n_or), int(seed), int(sweep0)), "gf_heatbath", ctx)


def gf_plaquette(ctx) -> float:
    P = ctypes.c_double()
    _check(lib().gf_plaquette(ctx, ctypes.byref(P)), "gf_plaquette", ctx)
    return P.value


def gf_functional_g(ctx, omega: torch.Tensor) -> float:
    F = ctypes.c_double()
    _check(lib().gf_functional_g(ctx, _ptr(omega), ctypes.byref(F)), "gf_functional_g", ctx)
    return F.value


def gf_functional_g_backward(ctx, omega: torch.Tensor, grad_out: float, d_omega=None, d_U=None):
    st = lib().gf_functional_g_backward(ctx, _ptr(omega), float(grad_out),
                                        None if d_omega is None else _ptr(d_omega),
                                        None if d_U is None else _ptr(d_U))
    _check(st, "gf_functional_g_backward", ctx)


def gf_destroy(ctx):
    if ctx:
        lib().gf_destroy(ctx)


def gf_set_timing(ctx, on: bool):
    _check(lib().gf_set_timing(ctx, 1 if on else 0), "gf_set_timing", ctx)


def gf_kernel_times(ctx):
    """{name: (total_ms, launches)} accumulated while timing was on."""
    out = {}
    for k in range(lib().gf_kernel_count(ctx)):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().gf_kernel_time(ctx, k, ctypes.byref(ms), ctypes.byref(n)), "gf_kernel_time", ctx)
        out[lib().gf_kernel_name(ctx, k).decode()] = (ms.value, n.value)
    return out


def gf_fft_schedule(ctx) -> int:
    return int(lib().gf_fft_schedule(ctx))


def gf_reset_timing(ctx):
    _check(lib().gf_reset_timing(ctx), "gf_reset_timing", ctx)
