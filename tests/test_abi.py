"""The C ABI as a contract (CPU only, no compute call).

The shared library must load, export every function that include/infuse.h
declares (and no other im_* symbol), and the Python binding must declare
exactly that set.  Without the built library the binding must fail loudly:
there is no CPU fallback.
"""

import os
import re
import subprocess

import pytest

from paper_2008_03095_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "infuse.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    # a declaration: return type, name, '(' at the start of a statement
    names = re.findall(r"(?:^|;|\})\s*(?:const\s+)?[A-Za-z_][\w]*\s*\**\s*(im_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_parses():
    names = header_functions()
    for must in ("im_ctx_create", "im_graph_load_csr", "im_set_params", "im_select_seeds",
                 "im_estimate_sigma", "im_server_submit", "im_batch_select"):
        assert must in names
    assert len(names) >= 30


def test_binding_declares_exactly_the_header():
    assert sorted(_lib.SIGNATURES) == header_functions()


def test_library_exports_every_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines() if re.search(r"\sT\s+im_\w+$", ln)})
    assert exported == header_functions()


def test_library_loads_and_resolves():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = _lib.load()
    for name in header_functions():
        assert getattr(lib, name) is not None
    assert lib.im_version().decode()


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libinfuse.so"))
    with pytest.raises(ImportError):
        _lib.load()


def test_no_device_is_an_error_not_a_fallback():
    """Without a GPU, creating a context reports IM_ERR_DEVICE."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("a device is present")
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    import ctypes as C

    lib = _lib.load()
    out = C.c_void_p()
    st = lib.im_ctx_create(0, None, None, 0, C.byref(out))
    assert st == 4  # IM_ERR_DEVICE
    assert not out.value
