"""Plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``stb_oracle.c`` (plain C,
OpenMP over rows) through ctypes and shares no code with the HIP path.

What it computes, with citations, is described in ``stb_oracle.c``.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stb_oracle.c")
_LIB = os.path.join(_HERE, "libstb_oracle.so")
_lib = None


def build(force=True):
    """Compile the oracle with gcc -O2 (no fast-math), OpenMP."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall",
           "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


class Stats(ctypes.Structure):
    _fields_ = [("n_eval", ctypes.c_int64), ("n_sub", ctypes.c_int64),
                ("n_bp", ctypes.c_int64), ("n_lit", ctypes.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        i64, i32, c_int = ctypes.c_int64, ctypes.c_int32, ctypes.c_int
        P = ctypes.POINTER
        L.orc_gauss_legendre01.argtypes = [c_int, _D, _D]
        L.orc_inner.argtypes = [_D, _D, c_int, _D, P(Stats)]
        L.orc_L.argtypes = [_D, _D, ctypes.c_double, _D]
        L.orc_panel_frame.argtypes = [_D, _D, _D, _D, _D]
        L.orc_outer_points.argtypes = [_D, c_int, _D, _D]
        L.orc_entry.argtypes = [_D, _I32, i64, i64, c_int, c_int, _D, P(Stats)]
        L.orc_assemble_rows.argtypes = [i64, _D, i64, _I32, i64, _I64, c_int, c_int, _D,
                                        P(Stats)]
        L.orc_assemble_rows_mag.argtypes = [i64, _D, i64, _I32, i64, _I64, c_int, c_int, _D, _D,
                                            P(Stats)]
        L.orc_matvec_rows.argtypes = [i64, _D, i64, _I32, i64, _I64, c_int, c_int, _D, _D]
        L.orc_potential.argtypes = [i64, _D, i64, _I32, _D, i64, _D, c_int, _D]
        L.orc_lit.argtypes = [_D, _D, _D, _D]
        L.orc_pair_causal.argtypes = [_D, _I32, i64, i64, c_int]
        L.orc_count_causal_rows.argtypes = [i64, _D, i64, _I32, i64, _I64, c_int]
        L.orc_count_causal_rows.restype = i64
        L.orc_count_causal_per_row.argtypes = [i64, _D, i64, _I32, i64, _I64, c_int, _I64]
        L.orc_num_threads.argtypes = []
        L.orc_breakpoints.argtypes = [_D, _D, _D, c_int]
        L.orc_inner_dl.argtypes = [_D, _D, _D, _D, c_int, _D]
        L.orc_potential_dl.argtypes = [i64, _D, i64, _I32, _D, _D, i64, _D, c_int, _D]
        L.orc_l2_points.argtypes = [_D, _D, _D]
        L.orc_l2_projection.argtypes = [i64, _D, i64, _I32, _D, _D]
        L.orc_dl_energetic_rows.argtypes = [i64, _D, i64, _I32, _D, _D, i64, _I64, c_int, c_int,
                                            ctypes.c_double, _D]
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_D)


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_I32)


def _i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_I64)


def _check(rc, what):
    if rc < 0:
        raise ValueError("oracle %s failed with code %d" % (what, rc))
    return rc


DEFAULT_NG = 16
DEFAULT_MQ = 3


def gauss_legendre01(n):
    x = np.zeros(n)
    w = np.zeros(n)
    _check(lib().orc_gauss_legendre01(n, x.ctypes.data_as(_D), w.ctypes.data_as(_D)), "gl")
    return x, w


def inner(x4, tet, n_g=DEFAULT_NG, stats=None):
    """V phi_sigma(x) for one point x=(t,x,y,z) and one panel tet (4x4)."""
    x4, px = _d(x4)
    tet, pt = _d(tet)
    out = ctypes.c_double()
    st = stats if stats is not None else Stats()
    _check(lib().orc_inner(px, pt, n_g, ctypes.byref(out), ctypes.byref(st)), "inner")
    return out.value


def L(x4, tet, phi):
    x4, px = _d(x4)
    tet, pt = _d(tet)
    out = ctypes.c_double()
    _check(lib().orc_L(px, pt, float(phi), ctypes.byref(out)), "L")
    return out.value


def panel_frame(tet):
    tet, pt = _d(tet)
    o, e1, e2, n = (np.zeros(3) for _ in range(4))
    _check(lib().orc_panel_frame(pt, *(v.ctypes.data_as(_D) for v in (o, e1, e2, n))), "frame")
    return o, e1, e2, n


def outer_points(tet, m_q=DEFAULT_MQ):
    tet, pt = _d(tet)
    pts = np.zeros((4 * m_q * m_q, 4))
    w = np.zeros(4 * m_q * m_q)
    n = _check(lib().orc_outer_points(pt, m_q, pts.ctypes.data_as(_D), w.ctypes.data_as(_D)),
               "outer_points")
    return pts[:n].copy(), w[:n].copy()


def entry(vtx, tets, i, j, m_q=DEFAULT_MQ, n_g=DEFAULT_NG):
    vtx, pv = _d(vtx)
    tets, pt = _i32(tets)
    out = ctypes.c_double()
    _check(lib().orc_entry(pv, pt, i, j, m_q, n_g, ctypes.byref(out), None), "entry")
    return out.value


def assemble_rows(vtx, tets, rows=None, m_q=DEFAULT_MQ, n_g=DEFAULT_NG, stats=None, mag=False):
    """Rows of A (all columns).  mag=True: also the size of each entry's
    outer-sum terms, sum_q |w_q I_q| (returns (A, M))."""
    vtx, pv = _d(vtx)
    tets, pt = _i32(tets)
    nt = tets.shape[0]
    rows = np.arange(nt) if rows is None else rows
    rows, pr = _i64(rows)
    out = np.zeros((rows.shape[0], nt))
    M = np.zeros((rows.shape[0], nt)) if mag else None
    st = stats if stats is not None else Stats()
    _check(lib().orc_assemble_rows_mag(vtx.shape[0], pv, nt, pt, rows.shape[0], pr, m_q, n_g,
                                       out.ctypes.data_as(_D),
                                       M.ctypes.data_as(_D) if mag else None, ctypes.byref(st)),
           "assemble_rows")
    return (out, M) if mag else out


def matvec_rows(vtx, tets, w, rows=None, m_q=DEFAULT_MQ, n_g=DEFAULT_NG):
    vtx, pv = _d(vtx)
    tets, pt = _i32(tets)
    nt = tets.shape[0]
    rows = np.arange(nt) if rows is None else rows
    rows, pr = _i64(rows)
    w, pw = _d(w)
    y = np.zeros(rows.shape[0])
    _check(lib().orc_matvec_rows(vtx.shape[0], pv, nt, pt, rows.shape[0], pr, m_q, n_g, pw,
                                 y.ctypes.data_as(_D)), "matvec_rows")
    return y


def potential(vtx, tets, w, pts, n_g=DEFAULT_NG):
    vtx, pv = _d(vtx)
    tets, pt = _i32(tets)
    w, pw = _d(w)
    pts, pp = _d(np.asarray(pts).reshape(-1, 4))
    out = np.zeros(pts.shape[0])
    _check(lib().orc_potential(vtx.shape[0], pv, tets.shape[0], pt, pw, pts.shape[0], pp, n_g,
                               out.ctypes.data_as(_D)), "potential")
    return out


def lit(x4, tet):
    x4, px = _d(x4)
    tet, pt = _d(tet)
    mn = ctypes.c_double()
    mx = ctypes.c_double()
    r = _check(lib().orc_lit(px, pt, ctypes.byref(mn), ctypes.byref(mx)), "lit")
    return bool(r), mn.value, mx.value


def pair_causal(vtx, tets, i, j, m_q=DEFAULT_MQ):
    vtx, pv = _d(vtx)
    tets, pt = _i32(tets)
    return bool(_check(lib().orc_pair_causal(pv, pt, i, j, m_q), "pair_causal"))


def count_causal_per_row(vtx, tets, rows=None, m_q=DEFAULT_MQ):
    vtx, pv = _d(vtx)
    tets, pt = _i32(tets)
    nt = tets.shape[0]
    rows = np.arange(nt) if rows is None else rows
    rows, pr = _i64(rows)
    out = np.zeros(rows.shape[0], dtype=np.int64)
    _check(lib().orc_count_causal_per_row(vtx.shape[0], pv, nt, pt, rows.shape[0], pr, m_q,
                                          out.ctypes.data_as(_I64)), "count_causal")
    return out


def num_threads():
    return int(lib().orc_num_threads())


def breakpoints(x4, tet):
    x4, px = _d(x4)
    tet, pt = _d(tet)
    out = np.zeros(64)
    n = _check(lib().orc_breakpoints(px, pt, out.ctypes.data_as(_D), 64), "breakpoints")
    return out[:n].copy()


def inner_dl(x4, tet, nrm, vv, n_g=DEFAULT_NG):
    """Retarded double-layer potential (eq. dlp) at x = (t,x,y,z) of the
    density that is linear on the panel tet (4x4) with values vv at its 4
    vertices; nrm = the outward spatial normal of the panel (any length)."""
    x4, px = _d(x4)
    tet, pt = _d(tet)
    nrm, pn = _d(nrm)
    vv, pvv = _d(vv)
    out = ctypes.c_double()
    _check(lib().orc_inner_dl(px, pt, pn, pvv, n_g, ctypes.byref(out)), "inner_dl")
    return out.value


def potential_dl(vtx, tets, nrm, v, pts, n_g=DEFAULT_NG):
    """u(p) = D v (p) for v in V_h^1 given by its vertex values v (eq. dlp);
    nrm = per-panel outward spatial normals (nt x 3)."""
    vtx, pv = _d(vtx)
    tets, pt = _i32(tets)
    nrm, pn = _d(np.asarray(nrm).reshape(-1, 3))
    v, pvv = _d(v)
    pts, pp = _d(np.asarray(pts).reshape(-1, 4))
    out = np.zeros(pts.shape[0])
    _check(lib().orc_potential_dl(vtx.shape[0], pv, tets.shape[0], pt, pn, pvv, pts.shape[0], pp,
                                  n_g, out.ctypes.data_as(_D)), "potential_dl")
    return out


def dl_energetic_rows(vtx, tets, nrm, v, rows, c_id=0.0, m_q=DEFAULT_MQ, n_g=DEFAULT_NG):
    """c_id b_I(v, phi_i) + b_K(v, phi_i) for the test panels in rows (eq.
    int_bform with A = I, K); v in V_h^1 by vertex values."""
    vtx, pv = _d(vtx)
    tets, pt = _i32(tets)
    nrm, pn = _d(np.asarray(nrm).reshape(-1, 3))
    v, pvv = _d(v)
    rows, pr = _i64(rows)
    out = np.zeros(rows.shape[0])
    _check(lib().orc_dl_energetic_rows(vtx.shape[0], pv, tets.shape[0], pt, pn, pvv, rows.shape[0],
                                       pr, m_q, n_g, float(c_id), out.ctypes.data_as(_D)),
           "dl_energetic_rows")
    return out


def l2_points(tet):
    """The 27 points and weights of the projection rule on one panel."""
    tet, pt = _d(tet)
    pts = np.zeros((27, 4))
    w = np.zeros(27)
    _check(lib().orc_l2_points(pt, pts.ctypes.data_as(_D), w.ctypes.data_as(_D)), "l2_points")
    return pts, w


def l2_projection(vtx, tets, gq):
    """Vertex values of Q_h^1 g from g at every panel's 27 rule points."""
    vtx, pv = _d(vtx)
    tets, pt = _i32(tets)
    gq, pg = _d(np.asarray(gq).reshape(-1))
    out = np.zeros(vtx.shape[0])
    _check(lib().orc_l2_projection(vtx.shape[0], pv, tets.shape[0], pt, pg, out.ctypes.data_as(_D)),
           "l2_projection")
    return out
