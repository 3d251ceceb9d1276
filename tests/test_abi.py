"""The HIP library loads without a GPU and exports every entry point of include/gf.h."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "gf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gf_[a-z_]+)\s*\(", src)))


def test_header_declares_the_method_calls():
    names = declared_symbols()
    for n in ("gf_init", "gf_step", "gf_fix_until", "gf_functional", "gf_functional_g", "gf_functional_g_backward",
              "gf_init_batch", "gf_fix_until_batch"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1210_8018_amd import gf

    lib = gf.lib()
    for n in declared_symbols():
        assert hasattr(lib, n), n


def test_host_only_calls_without_gpu():
    from paper_1210_8018_amd import gf

    p = gf.make_params((32, 32, 32, 32))
    b64 = gf.gf_workspace_bytes(p)
    b32 = gf.gf_workspace_bytes(gf.make_params((32, 32, 32, 32), fft_prec=1))
    V = 32**4
    assert b64 > V * (64 + 144) and b32 < b64
    assert gf.gf_workspace_bytes(gf.make_params((6, 8, 8, 8))) > 0
    assert gf.gf_workspace_bytes(gf.make_params((10, 8, 8, 8))) == 0  # factor 5
    assert gf.gf_workspace_bytes(gf.make_params((8, 8, 8, 8), fft_prec=2)) == 0
    assert gf.strerror(gf.GF_ERR_MAXITER).startswith("iteration cap")
    pl = [gf.make_params((12, 12, 12, 12), fft_prec=1), gf.make_params((8, 8, 8, 16), fft_prec=1)]
    assert gf.gf_workspace_bytes_batch(pl) > 0
    pl[1] = gf.make_params((8, 8, 8, 16), fft_prec=0)  # one precision per batch
    assert gf.gf_workspace_bytes_batch(pl) == 0
    assert gf.lib().gf_init(None, None, None, None, 0, None) == gf.GF_ERR_ARG
    # the allocation-free call checks its arguments and the size of its static
    # array on the host before any HIP call
    assert gf.lib().gf_fix_until_static(None, None, 1e-15, 10, None, None, None, None) == gf.GF_ERR_ARG
    big = gf.make_params((32, 32, 16, 16))
    assert gf.gf_workspace_bytes(big) > gf.GF_STATIC_SCRATCH_BYTES
    assert gf.lib().gf_fix_until_static(ctypes.byref(big), ctypes.c_void_p(256), 1e-15, 10, None, None, None,
                                        None) == gf.GF_ERR_SHAPE
    # functional-only contexts need g and the block partials, not the iteration's buffers
    fp = gf.make_params((24, 24, 24, 24))
    assert 144 * 24**4 < gf.gf_workspace_bytes_functional(fp) < 160 * 24**4 < gf.gf_workspace_bytes(fp)
    small = gf.make_params((12, 12, 12, 12))
    assert 0 < gf.gf_workspace_bytes(small) <= gf.GF_STATIC_SCRATCH_BYTES


def test_params_layout_and_link_storage_options():
    """gf_params matches the C layout (56 bytes); single-precision link storage
    adds its buffers to the workspace; bad values are rejected."""
    import ctypes

    from paper_1210_8018_amd import gf

    assert ctypes.sizeof(gf.gf_params) == 56
    assert gf.gf_params.refine_theta.offset == 48 and gf.gf_params.link_prec.offset == 40
    V = 16**4
    b0 = gf.gf_workspace_bytes(gf.make_params((16, 16, 16, 16)))
    b1 = gf.gf_workspace_bytes(gf.make_params((16, 16, 16, 16), link_prec=1))
    assert b1 - b0 >= V * (2 * 192 + 48)
    assert gf.gf_workspace_bytes(gf.make_params((8, 8, 8, 8), link_prec=2)) == 0
    assert gf.gf_workspace_bytes(gf.make_params((8, 8, 8, 8), link_prec=1, refine_theta=-1.0)) == 0
    p = gf.make_params((8, 8, 8, 8))
    p.reserved = 1
    assert gf.gf_workspace_bytes(p) == 0
    pl = [gf.make_params((8, 8, 8, 8), link_prec=1), gf.make_params((8, 8, 8, 16), link_prec=0)]
    assert gf.gf_workspace_bytes_batch(pl) == 0  # one link storage per batch
