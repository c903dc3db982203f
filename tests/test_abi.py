"""The C-ABI library loads on a host without a GPU and exports every entry
point that include/gx.h declares; the Python binding declares them too."""
import os
import re
import ctypes

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(gx_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = _declared()
    for core in ("gx_tree_build", "gx_gravity_forces", "gx_sph_density", "gx_sph_forces",
                 "gx_kick_drift"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2510_23330_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgx.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    from paper_2510_23330_amd import _lib
    assert set(_declared()) <= set(_lib.SIGNATURES)


def test_version_and_invalid_args_without_gpu():
    from paper_2510_23330_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgx.so not built")
    lib = _lib.load()
    assert b"gfx950" in lib.gx_version()
    # null out-pointer is rejected before any device call
    assert lib.gx_create(None, 0, None) == _lib.GX_EINVAL
    assert lib.gx_destroy(None) == _lib.GX_EINVAL


def test_unet_layer_table_matches_oracle():
    # the library's layer order and flat parameter offsets (host-only calls)
    # are the oracle network's
    from paper_2510_23330_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgx.so not built")
    import paper_2510_23330_amd as gx
    from oracle import unet as ounet
    for base, levels in ((32, 4), (16, 3), (16, 2)):
        tab, n, _ = ounet.layer_table(base, levels)
        assert gx.unet_sizes(levels, base, 8, 16) == (n, len(tab))
        got = gx.unet_layers(levels, base, 8, 16)
        assert [g[0] for g in got] == list(tab)
        for name, ci, co, k, wo, bo in got:
            d = tab[name]
            assert (ci, co, k, wo, bo) == (d["cin"], d["cout"], d["k"], d["w"][0], d["b"][0])
    lib = _lib.load()
    n = ctypes.c_int64(0)
    assert lib.gx_unet_sizes(1, 32, 8, 16, ctypes.byref(n), None) == _lib.GX_EINVAL
