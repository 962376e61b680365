"""CPU checks of the C ABI library: it loads, exports every declared entry
point, and its host-side argument checks work without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msplat.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(msplat_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2606_03877_amd import _lib
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["msplat_create", "msplat_destroy", "msplat_render_forward",
                     "msplat_render_backward", "msplat_workspace_size", "msplat_debug_hits"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2606_03877_amd import _lib
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in _lib.EXPORTS, name


def test_status_strings_and_param_count(lib):
    from paper_2606_03877_amd import _lib, NetSpec
    assert lib.msplat_status_string(0) == b"ok"
    assert b"workspace" in lib.msplat_status_string(2)
    import synth
    for cfg in synth.CONFIGS:
        spec = NetSpec(cfg.num_prims, cfg.pe_freqs, cfg.hidden_width, cfg.hidden_layers, cfg.out_dim,
                       primitive=cfg.primitive)
        assert lib.msplat_num_params(ctypes.byref(spec.c())) == synth.num_params(cfg)
        out = ctypes.c_uint64()
        assert lib.msplat_workspace_size(ctypes.byref(spec.c()), 1000, 1000, ctypes.byref(out)) == _lib.MSPLAT_OK
    # the contact-point primitive: the paper's 72-32-32-4 network, 12 L inputs
    assert lib.msplat_num_params(ctypes.byref(NetSpec(4, 6, 32, 2, 4, primitive="contact").c())) == \
        72 * 32 + 32 + 32 * 32 + 32 + 32 * 4 + 4
    bad_kind = _lib.Model(8, 6, 32, 2, 4, 0, 7)
    assert lib.msplat_num_params(ctypes.byref(bad_kind)) == 0


def test_host_argument_checks(lib):
    from paper_2606_03877_amd import _lib, NetSpec, RenderOpts
    spec = NetSpec(8, 4, 32, 2, 4)
    opts = RenderOpts()
    null = ctypes.c_void_p()
    st = lib.msplat_render_forward(None, ctypes.byref(spec.c()), ctypes.byref(opts.c()),
                                   null, null, null, null, null, null, 0, null, null, null,
                                   null, 0, None, null)
    assert st == _lib.MSPLAT_E_INVALID
    bad = _lib.Model(0, 4, 32, 2, 4, 0)
    out = ctypes.c_uint64()
    assert lib.msplat_workspace_size(ctypes.byref(bad), 10, 10, ctypes.byref(out)) == _lib.MSPLAT_E_INVALID
    odd = _lib.Model(8, 5, 48, 2, 4, 0)
    assert lib.msplat_workspace_size(ctypes.byref(odd), 10, 10, ctypes.byref(out)) == _lib.MSPLAT_E_UNSUPPORTED
    ok = spec.c()
    assert lib.msplat_workspace_size(ctypes.byref(ok), 4096, 1000, ctypes.byref(out)) == _lib.MSPLAT_OK
    small = out.value
    assert lib.msplat_workspace_size(ctypes.byref(ok), 4096, 100000, ctypes.byref(out)) == _lib.MSPLAT_OK
    assert out.value > small
    # hit lists are addressed with 32-bit offsets: at most 2^31 - 1 hits and rays per call
    assert lib.msplat_workspace_size(ctypes.byref(ok), 4096, 2 ** 31 - 1, ctypes.byref(out)) == _lib.MSPLAT_OK
    assert lib.msplat_workspace_size(ctypes.byref(ok), 4096, 2 ** 31, ctypes.byref(out)) == _lib.MSPLAT_E_INVALID
    assert lib.msplat_workspace_size(ctypes.byref(ok), 2 ** 31, 10, ctypes.byref(out)) == _lib.MSPLAT_E_INVALID
    h = ctypes.c_void_p()
    assert lib.msplat_create(-1, ctypes.byref(h)) in (_lib.MSPLAT_E_INVALID, _lib.MSPLAT_E_HIP)
