"""MI355X (gfx950) Fourier-accelerated steepest-descent Landau gauge fixing.

``inputs`` draws seeded synthetic link fields; ``gf`` is the ctypes binding of
the HIP library's C ABI (include/gf.h); ``api`` holds the torch front end
(GaugeFixer, BatchGaugeFixer, GaugeFunctional). The HIP library is loaded on
first use and its absence is an error.
"""

__all__ = ["inputs", "gf", "api", "build"]


def __getattr__(name):
    if name in ("gf", "api", "build", "inputs"):
        import importlib

        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
