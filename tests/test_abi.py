"""The C ABI library loads without a GPU and exports every entry point that
include/mpmrom.h declares; the Python binding declares each of them."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpmrom.h")
LIB = os.path.join(ROOT, "paper_2109_12390_amd", "libmpmrom.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    names = re.findall(r"\b((?:mpm|rom|mr)_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for required in ["mpm_p2g", "mpm_grid_update", "mpm_g2p", "rom_decode", "rom_decode_jac",
                     "rom_project", "rom_step"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libmpmrom.so not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    from paper_2109_12390_amd import binding
    assert sorted(binding.SIGNATURES) == declared_functions()
    lib = binding.load()
    assert binding.version().startswith("mpmrom")
    assert lib is binding.load()


def declared_arity():
    """Parameter count of every function the header declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    out = {}
    for m in re.finditer(r"\b((?:mpm|rom|mr)_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", text, flags=re.S):
        args = m.group(2).strip()
        out[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_binding_argument_counts_match_the_header():
    from paper_2109_12390_amd import binding
    arity = declared_arity()
    bad = {n: (len(args), arity[n]) for n, (_, args) in binding.SIGNATURES.items()
           if n in arity and len(args) != arity[n]}
    assert not bad, bad
    assert set(binding.SIGNATURES) <= set(arity)


def test_host_side_validation_without_gpu():
    """Entry points reject bad arguments on the host before touching HIP."""
    from paper_2109_12390_amd import binding as B
    lib = B.load()
    g = B.Grid(4, [8, 8, 8], 0.1).c()          # dim 4 is invalid
    assert lib.mpm_workspace_bytes(ctypes.byref(g), 10) == -1
    g = B.Grid(3, [16, 16, 16], 1 / 16).c()
    assert lib.mpm_workspace_bytes(ctypes.byref(g), 1000) > 0
    assert lib.mpm_grid_update(None, 0.1, None, None, 0, None) == B.MR_EINVAL
    h = ctypes.c_void_p()
    assert lib.rom_decoder_create(4, 3, 8, 2, None, None, None, None, None, 1, 0,
                                  ctypes.byref(h)) == B.MR_EINVAL
    opts = B.gn_opts(max_backtrack=-1)
    assert lib.rom_project(None, 1, 1, None, 1, None, None, None, None, None, None, 0.1,
                           ctypes.byref(opts), None, None, None, None, None, None, 0,
                           None) == B.MR_EINVAL
    assert lib.rom_project_workspace_bytes(None, 1, 1, ctypes.byref(opts)) == B.MR_EINVAL
