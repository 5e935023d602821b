"""The C-ABI library loads and exports every entry point include/nqs.h declares
(CPU only: no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nqs.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nqs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib_path():
    from paper_2206_14307_amd import LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_2206_14307_amd import build
        build.build()
    return LIB_PATH


def test_header_declares_the_hot_path_calls():
    names = declared()
    for n in ("nqs_sample", "nqs_logpsi", "nqs_eloc", "nqs_lanczos_moments", "nqs_grad",
              "nqs_sr_solve", "nqs_create", "nqs_set_params"):
        assert n in names


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    for n in declared():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True)
    exported = set(re.findall(r" T (nqs_[a-z0-9_]+)", out.stdout))
    assert set(declared()) <= exported


def test_binding_declares_the_same_symbols():
    from paper_2206_14307_amd import EXPORTS
    assert sorted(EXPORTS) == declared()


def test_header_compiles_as_c():
    src = f'#include "{HEADER}"\nint main(void) {{ return (int)sizeof(nqs_model_desc); }}\n'
    r = subprocess.run(["gcc", "-x", "c", "-std=c99", "-fsyntax-only", "-I/opt/rocm/include",
                        "-D__HIP_PLATFORM_AMD__", "-"], input=src, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_status_strings_without_a_device(lib_path):
    from paper_2206_14307_amd import load_library
    lib = load_library()
    assert lib.nqs_status_str(0) == b"ok"
    assert lib.nqs_status_str(6).startswith(b"matrix")
    assert lib.nqs_status_str(7).startswith(b"iterative solver")
    assert lib.nqs_num_params(None) == -1
    assert lib.nqs_workspace_bytes(None, 0, 10) == 0
