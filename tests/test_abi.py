"""Host-side checks of the C ABI (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2103_16841_amd import build as stb_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "stb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(stb_[a-zA-Z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(stb_build.LIB):
        pytest.fail("libstb.so not built")
    lib = ctypes.CDLL(stb_build.LIB)
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_symbol():
    from paper_2103_16841_amd import stb
    assert sorted(stb.EXPORTS) == _declared()


def test_status_strings_and_defaults():
    from paper_2103_16841_amd import stb
    L = stb.load()
    assert L.stb_status_str(0) == b"ok"
    assert L.stb_status_str(2) == b"invalid mesh"
    p = stb.default_params()
    assert (p.m_q, p.n_g, p.prec) == (3, 16, 0)


def test_null_arguments_are_rejected():
    from paper_2103_16841_amd import stb
    L = stb.load()
    assert L.stb_ctx_create(0, None) == 1
    assert L.stb_mat_info(None, None, None, None, None) == 1
    assert L.stb_mat_to_dense(None, None) == 1
