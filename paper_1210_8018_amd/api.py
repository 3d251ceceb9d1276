"""High-level PyTorch front end of the gauge-fixing library.

Links are complex128 CUDA tensors of shape (4, 3, 3, Lt, Lz, Ly, Lx)
(structure of arrays, site s = x + Lx*(y + Ly*(z + Lz*t))), updated in place.
All arithmetic happens in the HIP library; this module allocates device
buffers with torch and passes pointers.
"""
from __future__ import annotations

from collections import OrderedDict

import torch

from . import gf

__all__ = ["GaugeFixer", "BatchGaugeFixer", "GaugeFunctional", "functional_g", "dims_of"]


def dims_of(links: torch.Tensor):
    if links.dim() != 7 or tuple(links.shape[:3]) != (4, 3, 3):
        raise ValueError("links must have shape (4, 3, 3, Lt, Lz, Ly, Lx)")
    Lt, Lz, Ly, Lx = links.shape[3:]
    return (int(Lx), int(Ly), int(Lz), int(Lt))


def _check_links(links: torch.Tensor):
    if links.dtype != torch.complex128 or not links.is_cuda or not links.is_contiguous():
        raise ValueError("links must be a contiguous complex128 CUDA tensor")


class GaugeFixer:
    """Fourier-accelerated steepest-descent Landau gauge fixing of one configuration."""

    def __init__(self, links: torch.Tensor, alpha: float = 0.08, fft_prec: int = 0, reunit_every: int = 0,
                 chunk: int = 0, fft_schedule: int = 0, link_prec: int = 0, refine_theta: float = 0.0):
        _check_links(links)
        self.links = links
        self.dims = dims_of(links)
        self.V = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]
        self.fft_prec = int(fft_prec)
        self.params = gf.make_params(self.dims, alpha, fft_prec, reunit_every, chunk, fft_schedule, link_prec,
                                     refine_theta)
        nbytes = gf.gf_workspace_bytes(self.params)
        if nbytes == 0:
            raise ValueError(f"unsupported parameters for dims {self.dims}")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=links.device)
        self.ctx = gf.gf_init(self.params, links, self.ws)

    def functional(self):
        """(F, theta) of the current links."""
        return gf.gf_functional(self.ctx)

    def step(self, n: int = 1):
        """n iterations regardless of theta; returns (F, theta) after them."""
        return gf.gf_step(self.ctx, n)

    def fix_until(self, theta_eps: float = 1e-15, max_iter: int = 1_000_000, allow_maxiter: bool = False):
        """Iterate until theta <= theta_eps; returns (iterations, F, theta)."""
        it, F, th, _ = gf.gf_fix_until(self.ctx, theta_eps, max_iter, allow_maxiter)
        return it, F, th

    def history(self):
        """Lists (F_k, theta_k), k = 0 (initial) .. number of updates."""
        return gf.gf_history(self.ctx)

    def delta(self) -> torch.Tensor:
        out = torch.empty((3, 3, self.V), dtype=torch.complex128, device=self.links.device)
        gf.gf_delta(self.ctx, out)
        return out

    def gauge(self) -> torch.Tensor:
        out = torch.empty((3, 3, self.V), dtype=torch.complex128, device=self.links.device)
        gf.gf_gauge(self.ctx, out)
        return out

    def apply_gauge(self, g: torch.Tensor):
        if g.dtype != torch.complex128 or not g.is_contiguous() or g.numel() != 9 * self.V:
            raise ValueError("g must be a contiguous complex128 tensor of 9 V entries")
        gf.gf_apply_gauge(self.ctx, g)

    def fft(self, fields: torch.Tensor, sign: int) -> torch.Tensor:
        """In-place 4D transform of (n, V) fields (complex128, or complex64 when fft_prec = 1)."""
        want = torch.complex64 if self.fft_prec else torch.complex128
        if fields.dtype != want or not fields.is_contiguous() or fields.numel() % self.V:
            raise ValueError("fields must be contiguous (n, V) of the context's transform precision")
        gf.gf_fft(self.ctx, fields, fields.numel() // self.V, sign)
        return fields

    @property
    def fft_schedule(self) -> int:
        return gf.gf_fft_schedule(self.ctx)

    def heatbath(self, beta: float, n_sweeps: int, n_or: int = 0, seed: int = 0, sweep0: int = 0):
        """Wilson-action heatbath + overrelaxation sweeps on the links (the input generator)."""
        gf.gf_heatbath(self.ctx, beta, n_sweeps, n_or, seed, sweep0)

    def plaquette(self) -> float:
        return gf.gf_plaquette(self.ctx)

    def set_timing(self, on: bool):
        gf.gf_set_timing(self.ctx, on)

    def kernel_times(self):
        return gf.gf_kernel_times(self.ctx)

    def reset_timing(self):
        gf.gf_reset_timing(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            gf.gf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchGaugeFixer:
    """Many independent configurations, possibly of different dims, in one context."""

    def __init__(self, links_list, alpha: float = 0.08, fft_prec: int = 1, reunit_every: int = 0, chunk: int = 0,
                 fft_schedule: int = 0, link_prec: int = 0, refine_theta: float = 0.0):
        for t in links_list:
            _check_links(t)
        self.links = list(links_list)
        self.n = len(self.links)
        self.params = [gf.make_params(dims_of(t), alpha, fft_prec, reunit_every, chunk, fft_schedule, link_prec,
                                      refine_theta) for t in self.links]
        nbytes = gf.gf_workspace_bytes_batch(self.params)
        if nbytes == 0:
            raise ValueError("unsupported batch parameters")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.links[0].device)
        self.ctx = gf.gf_init_batch(self.params, self.links, self.ws)

    def functional(self):
        return gf.gf_functional_batch(self.ctx, self.n)

    def fix_until(self, theta_eps: float = 1e-15, max_iter: int = 1_000_000, allow_maxiter: bool = False):
        it, F, th, _ = gf.gf_fix_until_batch(self.ctx, self.n, theta_eps, max_iter, allow_maxiter)
        return it, F, th

    def history(self, k: int):
        """Lists (F_j, theta_j) of configuration k, j = 0 (initial) .. its number of updates."""
        return gf.gf_history_batch(self.ctx, k)

    @property
    def fft_schedule(self) -> int:
        return gf.gf_fft_schedule(self.ctx)

    def set_timing(self, on: bool):
        gf.gf_set_timing(self.ctx, on)

    def kernel_times(self):
        return gf.gf_kernel_times(self.ctx)

    def reset_timing(self):
        gf.gf_reset_timing(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            gf.gf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_FN_CACHE_SIZE = 8
_fn_contexts = OrderedDict()


def _functional_context(U: torch.Tensor):
    """A functional-only library context for links U (cached per device,
    address, shape and stream; it holds no reference to U, only its address,
    and every call reads whatever U holds then)."""
    stream = torch.cuda.current_stream(U.device)
    key = (U.device.index, U.data_ptr(), dims_of(U), stream.cuda_stream)
    ent = _fn_contexts.get(key)
    if ent is not None:
        _fn_contexts.move_to_end(key)
        return ent[0]
    params = gf.make_params(dims_of(U))
    nbytes = gf.gf_workspace_bytes_functional(params)
    if nbytes == 0:
        raise ValueError(f"unsupported dims {dims_of(U)}")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=U.device)
    ctx = gf.gf_init_functional(params, U, ws, stream)
    _fn_contexts[key] = (ctx, ws)
    while len(_fn_contexts) > _FN_CACHE_SIZE:
        _, (old, _) = _fn_contexts.popitem(last=False)
        gf.gf_destroy(old)
    return ctx


def _check_omega(omega: torch.Tensor, U: torch.Tensor):
    V = U.numel() // 36
    if (omega.dtype != torch.float64 or not omega.is_cuda or omega.device != U.device
            or omega.dim() < 1 or omega.shape[0] != 8 or omega.numel() != 8 * V):
        raise ValueError(f"omega must be a float64 tensor of shape (8, V = {V}) on {U.device}")


class GaugeFunctional(torch.autograd.Function):
    """F_U[g] of Eq. 1 with g(x) = exp(i sum_a lambda_a omega_a(x)); differentiable in U and omega.

    U: complex128 (4, 3, 3, Lt, Lz, Ly, Lx) CUDA tensor; omega: float64 (8, V)
    on the same device. The gradient with respect to U follows torch's
    convention dF/dRe U + i dF/dIm U. Forward and backward run in a
    functional-only context (g and block partials, ~144 B per site), reused
    while U stays the same tensor.
    """

    @staticmethod
    def forward(ctx, U: torch.Tensor, omega: torch.Tensor):
        _check_links(U)
        _check_omega(omega, U)
        omega = omega.contiguous()
        F = gf.gf_functional_g(_functional_context(U), omega)
        ctx.save_for_backward(U, omega)
        return torch.tensor(F, dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, grad_out):
        U, omega = ctx.saved_tensors
        g = float(grad_out.detach().to("cpu"))
        d_omega = torch.empty_like(omega) if ctx.needs_input_grad[1] else None
        d_U = torch.empty_like(U) if ctx.needs_input_grad[0] else None
        if d_omega is not None or d_U is not None:
            gf.gf_functional_g_backward(_functional_context(U), omega, g, d_omega, d_U)
        return d_U, d_omega


def functional_g(U: torch.Tensor, omega: torch.Tensor) -> torch.Tensor:
    return GaugeFunctional.apply(U, omega)
