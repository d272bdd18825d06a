"""Host-side checks of the C-ABI library: it loads without a GPU, exports
every entry point include/gtod.h declares, and the binding's ctypes
structs have the C layout.  No compute calls."""
import ctypes
import os
import re

import pytest

from paper_2604_23305_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "gtod.h")).read()
    return sorted(set(re.findall(r"^\s*(?:gtod_status|const char\*|void)\s+"
                                 r"(gtod_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_five_calls():
    fns = header_functions()
    for name in ("gtod_sim_init", "gtod_load_screen", "gtod_load_filters",
                 "gtod_simulate_tod", "gtod_free"):
        assert name in fns


def test_library_exports_every_declared_symbol():
    lib = _abi.load()
    for name in header_functions():
        assert hasattr(lib, name), name
    assert sorted(_abi.SYMBOLS) == header_functions()


def test_struct_layouts_match_c():
    lib = _abi.load()
    out = (ctypes.c_int64 * 6)()
    lib.gtod_abi_sizes(out)
    assert list(out) == _abi.struct_sizes()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_abi, "_lib", None)
    monkeypatch.setattr(_abi, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        _abi.load()


def test_init_without_gpu_reports_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2604_23305_amd import GtodError, sim_init
    with pytest.raises(GtodError):
        sim_init()
