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
    assert (p.m_q, p.n_g, p.prec, p.lit_search, p.n_min) == (3, 16, 0, stb.STB_LIT_FLAT, 64)


def test_null_arguments_are_rejected():
    from paper_2103_16841_amd import stb
    L = stb.load()
    assert L.stb_ctx_create(0, None) == 1
    assert L.stb_mat_info(None, None, None, None, None) == 1
    assert L.stb_mat_to_dense(None, None) == 1


def _exported_stb_symbols():
    """Names of the stb_* functions the library exports (defined, global)."""
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", stb_build.LIB], stdout=subprocess.PIPE,
                         text=True, check=True).stdout
    names = set()
    for line in out.splitlines():
        parts = line.split()
        if len(parts) == 3 and parts[1] in ("T", "W") and re.fullmatch(r"stb_[A-Za-z0-9_]+", parts[2]):
            names.add(parts[2])
    return sorted(names)


def test_library_exports_nothing_undeclared():
    """Every exported stb_* function is declared in include/stb.h: no debug
    or internal entry point leaks into the product library's interface."""
    if not os.path.exists(stb_build.LIB):
        pytest.fail("libstb.so not built")
    extra = sorted(set(_exported_stb_symbols()) - set(_declared()))
    assert not extra, extra


def test_binding_rejects_misshaped_arrays():
    """The binding checks array shapes before a pointer reaches the library
    (which reads and writes as many values as the mesh or matrix says)."""
    import numpy as np
    from paper_2103_16841_amd import stb

    class FakeMesh:
        nt, nv, h = 10, 8, None

    class FakeCtx:
        h = None

    m, c = FakeMesh(), FakeCtx()
    with pytest.raises(ValueError):
        stb.potential_S(c, m, np.zeros(9), np.zeros((3, 4)))
    with pytest.raises(ValueError):
        stb.potential_S(c, m, np.zeros(10), np.zeros((3, 3)))
    with pytest.raises(ValueError):
        stb.potential_D(c, m, np.zeros(10), np.zeros((3, 4)))
    with pytest.raises(ValueError):
        stb.dl_energetic(c, m, np.zeros(7))
    with pytest.raises(ValueError):
        stb.inner_values(c, m, np.zeros((3, 4)), np.zeros(2, dtype=np.int32))
    with pytest.raises(ValueError):
        stb.outer_rhs(c, m, np.zeros((10, 35)))
    with pytest.raises(ValueError):
        stb.Mesh(c, np.zeros((4, 3)), np.zeros((1, 4), dtype=np.int32))

    class FakeMatrix(stb.Matrix):
        def __init__(self):
            self.n, self.ctx, self.h = 10, c, None

    with pytest.raises(ValueError):
        FakeMatrix().apply(np.zeros(11))
    with pytest.raises(ValueError):
        FakeMatrix().apply(np.zeros((9, 16)))
    with pytest.raises(ValueError):
        stb.solve_gmres(c, FakeMatrix(), np.zeros(9))

    class FakeServer(stb.Server):
        def __init__(self):
            self._sizes = {0: 10}
            self.h = None

    S = FakeServer()
    with pytest.raises(ValueError):
        S.submit_matvec(0, np.zeros((10, 8)))
    with pytest.raises(ValueError):
        S.submit_matvec(1, np.zeros((10, 16)))
    with pytest.raises(ValueError):
        S.submit_potential(0, np.zeros(9), np.zeros((5, 4)))
    with pytest.raises(ValueError):
        S.submit_potential(0, np.zeros(10), np.zeros(5))
