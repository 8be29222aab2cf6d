"""The C-ABI library loads on the CPU host and exports every declared symbol.

No compute call is made (there is no GPU here); loading the shared object
only needs the HIP runtime library.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpo.h")
LIB = os.path.join(ROOT, "paper_2407_14675_amd", "libdpo.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dpo_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2407_14675_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dpo_create", "dpo_bellman_sweep", "dpo_policy_eval_sweep", "dpo_solve_vi",
                     "dpo_solve_pi", "dpo_extract_feedback", "dpo_value_at"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_last_error_without_context(lib):
    lib.dpo_last_error.restype = ctypes.c_char_p
    lib.dpo_last_error.argtypes = [ctypes.c_void_p]
    assert isinstance(lib.dpo_last_error(None), bytes)


def test_binding_refuses_to_run_without_library(monkeypatch, tmp_path):
    """The product path has no CPU fallback: a missing library is an error."""
    from paper_2407_14675_amd import dpo
    monkeypatch.setattr(dpo, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(dpo, "_lib", None)
    with pytest.raises(ImportError):
        dpo.load()
