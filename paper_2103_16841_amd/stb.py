"""ctypes binding of libstb (include/stb.h): argument marshalling only.

Every step of the method runs in the HIP library.  Loading fails loudly
when the library is not built; there is no fallback.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

STB_FP64, STB_MIXED = 0, 1
STATUS = {0: "STB_OK", 1: "STB_E_INVALID_ARG", 2: "STB_E_INVALID_MESH", 3: "STB_E_NO_MEMORY",
          4: "STB_E_DEVICE", 5: "STB_E_NOT_FOUND", 6: "STB_E_BUSY", 7: "STB_E_INTERNAL"}

# Every symbol declared in include/stb.h
EXPORTS = ["stb_default_params", "stb_ctx_create", "stb_ctx_destroy", "stb_status_str",
           "stb_last_error", "stb_mesh_create", "stb_mesh_destroy", "stb_mesh_size",
           "stb_assemble_V", "stb_mat_destroy", "stb_mat_info", "stb_mat_to_dense", "stb_mat_get",
           "stb_apply", "stb_apply_dev", "stb_apply16_noalloc", "stb_potential_S", "stb_potential_S_dev",
           "stb_inner_values", "stb_last_timings", "stb_last_work", "stb_last_lit_search", "stb_last_path_counts", "stb_mesh_create_dev",
           "stb_outer_points", "stb_outer_rhs", "stb_solve_gmres", "stb_solve_mot", "stb_mesh_set_normals", "stb_potential_D",
           "stb_potential_D_dev", "stb_inner_values_D", "stb_dl_energetic",
           "stb_l2_points", "stb_project_V1",
           "stb_last_kernel_times", "stb_mat_export", "stb_batch_assemble", "stb_autotune",
           "stb_set_tuning", "stb_set_pair_lists", "stb_server_create", "stb_server_add_mesh", "stb_server_submit",
           "stb_server_wait", "stb_server_destroy"]

STB_REQ_MATVEC16, STB_REQ_POTENTIAL = 0, 1

KERNEL_KINDS = ["lit", "breakpoints", "empty_test", "mixed_restore", "nodes_fp64", "nodes_fp32",
                "sums_store", "mixed_redo_nodes"]


STB_LIT_TREE, STB_LIT_FLAT = 0, 1


class QuadParams(ctypes.Structure):
    _fields_ = [("m_q", ctypes.c_int32), ("n_g", ctypes.c_int32), ("eta_far", ctypes.c_double),
                ("prec", ctypes.c_int), ("lit_search", ctypes.c_int32), ("n_min", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("mesh", ctypes.c_int32), ("np", ctypes.c_int64),
                ("w", ctypes.c_void_p), ("pts", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class StbError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)
_VP = ctypes.c_void_p


def lib_path():
    return _build.LIB


def load():
    """Load the in-tree libstb.so (built by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        raise ImportError("libstb.so is not built: run __graft_entry__.build() (hipcc, gfx950)")
    L = ctypes.CDLL(_build.LIB)
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    L.stb_default_params.restype = QuadParams
    L.stb_ctx_create.argtypes = [i32, ctypes.POINTER(_VP)]
    L.stb_ctx_destroy.argtypes = [_VP]
    L.stb_ctx_destroy.restype = None
    L.stb_status_str.argtypes = [ctypes.c_int]
    L.stb_status_str.restype = ctypes.c_char_p
    L.stb_last_error.argtypes = [_VP]
    L.stb_last_error.restype = ctypes.c_char_p
    L.stb_mesh_create.argtypes = [_VP, i64, _D, i64, _I32, ctypes.POINTER(_VP)]
    L.stb_mesh_destroy.argtypes = [_VP]
    L.stb_mesh_destroy.restype = None
    L.stb_mesh_size.argtypes = [_VP]
    L.stb_mesh_size.restype = i64
    L.stb_assemble_V.argtypes = [_VP, _VP, ctypes.POINTER(QuadParams), ctypes.POINTER(_VP)]
    L.stb_mat_destroy.argtypes = [_VP]
    L.stb_mat_destroy.restype = None
    L.stb_mat_info.argtypes = [_VP, _I64, _I64, _I64, _I64]
    L.stb_mat_to_dense.argtypes = [_VP, _D]
    L.stb_mat_get.argtypes = [_VP, i64, _I32, _I32, _D]
    L.stb_apply.argtypes = [_VP, _VP, i32, _D, _D]
    L.stb_apply_dev.argtypes = [_VP, _VP, i32, _VP, _VP, _VP]
    L.stb_apply16_noalloc.argtypes = [_VP, _VP, _VP, _VP, _VP]
    L.stb_potential_S.argtypes = [_VP, _VP, ctypes.POINTER(QuadParams), _D, i64, _D, _D]
    L.stb_last_timings.argtypes = [_VP, _D]
    L.stb_inner_values.argtypes = [_VP, _VP, ctypes.POINTER(QuadParams), i64, _D, _I32, _D]
    L.stb_mesh_set_normals.argtypes = [_VP, _VP, _D]
    L.stb_potential_D.argtypes = [_VP, _VP, ctypes.POINTER(QuadParams), _D, i64, _D, _D]
    L.stb_potential_D_dev.argtypes = [_VP, _VP, ctypes.POINTER(QuadParams), _VP, i64, _VP, _VP, _VP]
    L.stb_inner_values_D.argtypes = [_VP, _VP, ctypes.POINTER(QuadParams), i64, _D, _I32, _D]
    L.stb_dl_energetic.argtypes = [_VP, _VP, ctypes.POINTER(QuadParams), _D, ctypes.c_double, _D]
    L.stb_l2_points.argtypes = [_VP, _VP, _D, _D]
    L.stb_project_V1.argtypes = [_VP, _VP, _D, _D, ctypes.POINTER(ctypes.c_int32)]
    L.stb_last_work.argtypes = [_VP, _I64]
    L.stb_last_lit_search.argtypes = [_VP, _I64]
    L.stb_last_path_counts.argtypes = [_VP, _I64]
    L.stb_outer_points.argtypes = [_VP, _VP, i32, _D, _D, _I32]
    L.stb_outer_rhs.argtypes = [_VP, _VP, i32, _D, _D]
    L.stb_solve_gmres.argtypes = [_VP, _VP, _D, _D, i32, i32, ctypes.c_double, _I32,
                                  ctypes.POINTER(ctypes.c_double)]
    L.stb_solve_mot.argtypes = [_VP, _VP, _VP, _D, _D, _D]
    L.stb_last_kernel_times.argtypes = [_VP, _D, _I64, _I64]
    L.stb_mat_export.argtypes = [_VP, _I64, _I32, _D]
    L.stb_autotune.argtypes = [_VP, _VP, ctypes.POINTER(QuadParams), _I32]
    L.stb_server_create.argtypes = [_VP, i64, i32, ctypes.POINTER(_VP)]
    L.stb_server_add_mesh.argtypes = [_VP, _VP, _VP, ctypes.POINTER(ctypes.c_int32)]
    L.stb_server_submit.argtypes = [_VP, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.stb_server_wait.argtypes = [_VP, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
    L.stb_server_destroy.argtypes = [_VP]
    L.stb_server_destroy.restype = None
    L.stb_set_tuning.argtypes = [_VP, _I32]
    L.stb_set_pair_lists.argtypes = [_VP, i64, i64, i64]
    L.stb_batch_assemble.argtypes = [_VP, i32, ctypes.POINTER(_VP), ctypes.POINTER(QuadParams),
                                     i64, ctypes.POINTER(_VP), i32, ctypes.POINTER(_VP),
                                     ctypes.POINTER(_VP), _I64]
    L.stb_mesh_create_dev.argtypes = [_VP, i64, _VP, i64, _VP, _VP, ctypes.POINTER(_VP)]
    L.stb_potential_S_dev.argtypes = [_VP, _VP, ctypes.POINTER(QuadParams), _VP, i64, _VP, _VP,
                                      _VP]
    _lib = L
    return L


def _chk(st, ctx=None):
    if st != 0:
        msg = load().stb_last_error(ctx)
        raise StbError(st, msg.decode() if msg else "")


def default_params(n_g=None, m_q=None, prec=None, eta_far=None, lit_search=None, n_min=None):
    p = load().stb_default_params()
    if lit_search is not None:
        p.lit_search = lit_search
    if n_min is not None:
        p.n_min = n_min
    if n_g is not None:
        p.n_g = n_g
    if m_q is not None:
        p.m_q = m_q
    if prec is not None:
        p.prec = prec
    if eta_far is not None:
        p.eta_far = eta_far
    return p


def _d(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a, a.ctypes.data_as(_D)


def _vec(a, n, what):
    """A contiguous FP64 vector of exactly n entries (ValueError otherwise):
    the library reads and writes as many as the mesh or matrix says."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 1 or a.shape[0] != n:
        raise ValueError("%s must have shape (%d,), got %s" % (what, n, a.shape))
    return a, a.ctypes.data_as(_D)


def _points(pts):
    """Points as a contiguous (k, 4) FP64 array (t, x, y, z)."""
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    if pts.ndim == 1 and pts.size == 0:
        pts = pts.reshape(0, 4)
    if pts.ndim != 2 or pts.shape[1] != 4:
        raise ValueError("points must have shape (k, 4) (t, x, y, z), got %s" % (pts.shape,))
    return pts, pts.ctypes.data_as(_D)


class Context:
    def __init__(self, device=0):
        L = load()
        h = _VP()
        _chk(L.stb_ctx_create(device, ctypes.byref(h)), None)
        self.h = h

    def close(self):
        if self.h:
            load().stb_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def timings(self):
        out = np.zeros(4)
        _chk(load().stb_last_timings(self.h, out.ctypes.data_as(_D)), self.h)
        return dict(geometry_ms=out[0], cull_ms=out[1], quadrature_ms=out[2], total_ms=out[3])

    def kernel_times(self):
        """{kind: (total ms, launches, work units)} of the pair pipeline's last run."""
        ms = np.zeros(8)
        n = np.zeros(8, dtype=np.int64)
        u = np.zeros(8, dtype=np.int64)
        _chk(load().stb_last_kernel_times(self.h, ms.ctypes.data_as(_D), n.ctypes.data_as(_I64),
                                          u.ctypes.data_as(_I64)), self.h)
        return {k: (float(ms[i]), int(n[i]), int(u[i])) for i, k in enumerate(KERNEL_KINDS)}

    def work(self):
        out = np.zeros(4, dtype=np.int64)
        _chk(load().stb_last_work(self.h, out.ctypes.data_as(_I64)), self.h)
        return dict(L_evals=int(out[0]), lit_pairs=int(out[1]), apex_pairs=int(out[2]),
                    pieces=int(out[3]))

    def lit_search(self):
        """The last potential's lit search: (point, leaf) pairs kept by the
        tree, panels in those leaves (|X_N| summed over the points), candidates
        after the per-panel bound test."""
        out = np.zeros(3, dtype=np.int64)
        _chk(load().stb_last_lit_search(self.h, out.ctypes.data_as(_I64)), self.h)
        return dict(leaf_pairs=int(out[0]), leaf_panels=int(out[1]), candidates=int(out[2]))

    def path_counts(self):
        """Evaluations of L in the FP64 Gauss-node launches of the last run by
        path (recipe1, recipe2, full), and the pieces found empty by the ray
        test without evaluating L (ray_empty_pieces)."""
        out = np.zeros(4, dtype=np.int64)
        _chk(load().stb_last_path_counts(self.h, out.ctypes.data_as(_I64)), self.h)
        return dict(recipe1=int(out[0]), recipe2=int(out[1]), full=int(out[2]),
                    ray_empty_pieces=int(out[3]))


class Mesh:
    def __init__(self, ctx, vtx, tets, _handle=None, _nt=None, _nv=None):
        L = load()
        self.ctx = ctx
        if _handle is not None:
            self.h, self.nt, self.nv = _handle, _nt, _nv
            return
        vtx, pv = _d(vtx)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        if vtx.ndim != 2 or vtx.shape[1] != 4 or tets.ndim != 2 or tets.shape[1] != 4:
            raise ValueError("vertices must be (nv, 4) (t, x, y, z) and panels (nt, 4), got %s, %s"
                             % (vtx.shape, tets.shape))
        h = _VP()
        _chk(L.stb_mesh_create(ctx.h, vtx.shape[0], pv, tets.shape[0],
                               tets.ctypes.data_as(_I32), ctypes.byref(h)), ctx.h)
        self.h = h
        self.nt = int(tets.shape[0])
        self.nv = int(vtx.shape[0])

    @classmethod
    def from_device(cls, ctx, vtx_ptr, nv, tet_ptr, nt, stream=None):
        """Mesh from device arrays (e.g. torch tensors' data_ptr())."""
        h = _VP()
        _chk(load().stb_mesh_create_dev(ctx.h, nv, _VP(vtx_ptr), nt, _VP(tet_ptr),
                                        _VP(stream) if stream else None, ctypes.byref(h)), ctx.h)
        return cls(ctx, None, None, _handle=h, _nt=int(nt), _nv=int(nv))

    def set_normals(self, nrm):
        """Outward spatial normals of the panels (nt x 3), for the double layer."""
        nrm, pn = _d(nrm, (-1, 3))
        if nrm.shape[0] != self.nt:
            raise ValueError("need one normal per panel")
        _chk(load().stb_mesh_set_normals(self.ctx.h, self.h, pn), self.ctx.h)

    def close(self):
        if self.h:
            load().stb_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Matrix:
    def __init__(self, ctx, h):
        self.ctx = ctx
        self.h = h
        n, nc, ns, nb = (ctypes.c_int64() for _ in range(4))
        _chk(load().stb_mat_info(h, ctypes.byref(n), ctypes.byref(nc), ctypes.byref(ns),
                                 ctypes.byref(nb)), ctx.h)
        self.n, self.n_causal, self.n_stored, self.bytes = n.value, nc.value, ns.value, nb.value

    def close(self):
        if self.h:
            load().stb_mat_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def to_dense(self):
        out = np.zeros((self.n, self.n))
        _chk(load().stb_mat_to_dense(self.h, out.ctypes.data_as(_D)), self.ctx.h)
        return out

    def export(self):
        """(rowptr, cols, vals) of the CSR store (host copies)."""
        rp = np.zeros(self.n + 1, dtype=np.int64)
        cols = np.zeros(self.n_stored, dtype=np.int32)
        vals = np.zeros(self.n_stored)
        _chk(load().stb_mat_export(self.h, rp.ctypes.data_as(_I64), cols.ctypes.data_as(_I32),
                                   vals.ctypes.data_as(_D)), self.ctx.h)
        return rp, cols, vals

    def get(self, rows, cols):
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        out = np.zeros(rows.shape[0])
        _chk(load().stb_mat_get(self.h, rows.shape[0], rows.ctypes.data_as(_I32),
                                cols.ctypes.data_as(_I32), out.ctypes.data_as(_D)), self.ctx.h)
        return out

    def apply(self, w):
        w = np.ascontiguousarray(w, dtype=np.float64)
        if w.ndim not in (1, 2) or w.shape[0] != self.n or (w.ndim == 2 and w.shape[1] < 1):
            raise ValueError("w must have shape (%d,) or (%d, nrhs), got %s" % (self.n, self.n, w.shape))
        nrhs = 1 if w.ndim == 1 else w.shape[1]
        y = np.zeros_like(w)
        _chk(load().stb_apply(self.ctx.h, self.h, nrhs, w.ctypes.data_as(_D),
                              y.ctypes.data_as(_D)), self.ctx.h)
        return y

    def apply_dev(self, w_ptr, y_ptr, nrhs, stream=None):
        """Device-pointer product (e.g. torch tensors' data_ptr())."""
        _chk(load().stb_apply_dev(self.ctx.h, self.h, nrhs, _VP(w_ptr), _VP(y_ptr),
                                  _VP(stream) if stream else None), self.ctx.h)

    def apply16_noalloc(self, w_ptr, y_ptr, stream=None):
        """16-RHS product that allocates nothing (device pointers, n x 16);
        enqueued on the stream, not synchronised."""
        _chk(load().stb_apply16_noalloc(self.ctx.h, self.h, _VP(w_ptr), _VP(y_ptr),
                                        _VP(stream) if stream else None), self.ctx.h)


def autotune(ctx, mesh, params=None):
    """Tune the pipeline's launch shapes on mesh; returns (blocks[8], per_cu[8])."""
    p = params if params is not None else default_params()
    cfg = np.zeros(16, dtype=np.int32)
    _chk(load().stb_autotune(ctx.h, mesh.h, ctypes.byref(p), cfg.ctypes.data_as(_I32)), ctx.h)
    return cfg[:8].tolist(), cfg[8:].tolist()


def set_tuning(ctx, blocks=None, per_cu=None):
    """Set launch shapes (None: defaults)."""
    if blocks is None:
        _chk(load().stb_set_tuning(ctx.h, None), ctx.h)
        return
    cfg = np.asarray(list(blocks) + list(per_cu), dtype=np.int32)
    _chk(load().stb_set_tuning(ctx.h, cfg.ctypes.data_as(_I32)), ctx.h)


def set_pair_lists(ctx, max_cand=0, max_combo=0, max_piece=0):
    """Limit the pair pipeline's list lengths per chunk (0: no limit)."""
    _chk(load().stb_set_pair_lists(ctx.h, max_cand, max_combo, max_piece), ctx.h)


def batch_assemble(ctx, meshes, params=None, hbm_budget=0, keep=True, W_ptrs=None, Y_ptrs=None,
                   nrhs=16, causal=None):
    """Assemble several meshes in one pass of the pair pipeline.  keep: return
    the matrices; W_ptrs/Y_ptrs: device pointers per mesh for Y_m = A_m W_m;
    causal: optional int64 array receiving the causal pairs per mesh."""
    p = params if params is not None else default_params()
    n = len(meshes)
    hs = (_VP * n)(*[m.h for m in meshes])
    outs = (_VP * n)() if keep else None
    W = (_VP * n)(*[_VP(x) for x in W_ptrs]) if W_ptrs is not None else None
    Y = (_VP * n)(*[_VP(x) for x in Y_ptrs]) if Y_ptrs is not None else None
    nc = None
    if causal is not None:
        assert causal.dtype == np.int64 and causal.size == n
        nc = causal.ctypes.data_as(_I64)
    _chk(load().stb_batch_assemble(ctx.h, n, hs, ctypes.byref(p), hbm_budget, outs, nrhs, W, Y, nc),
         ctx.h)
    return [Matrix(ctx, _VP(outs[k])) for k in range(n)] if keep else None


def assemble_V(ctx, mesh, params=None):
    p = params if params is not None else default_params()
    h = _VP()
    _chk(load().stb_assemble_V(ctx.h, mesh.h, ctypes.byref(p), ctypes.byref(h)), ctx.h)
    return Matrix(ctx, h)


def potential_S(ctx, mesh, w, pts, params=None):
    p = params if params is not None else default_params()
    w, pw = _vec(w, mesh.nt, "w")
    pts, pp = _points(pts)
    out = np.zeros(pts.shape[0])
    _chk(load().stb_potential_S(ctx.h, mesh.h, ctypes.byref(p), pw, pts.shape[0], pp,
                                out.ctypes.data_as(_D)), ctx.h)
    return out


def outer_points(ctx, mesh, m_q=3):
    """The outer rule of every panel: points [nt][4 m_q^2][4], weights
    [nt][4 m_q^2], counts [nt] (entries past a panel's count are zero)."""
    maxq = 4 * m_q * m_q
    pts = np.zeros((mesh.nt, maxq, 4))
    w = np.zeros((mesh.nt, maxq))
    n = np.zeros(mesh.nt, dtype=np.int32)
    _chk(load().stb_outer_points(ctx.h, mesh.h, m_q, pts.ctypes.data_as(_D), w.ctypes.data_as(_D),
                                 n.ctypes.data_as(_I32)), ctx.h)
    return pts, w, n


def energetic_rhs(ctx, mesh, g, m_q=3):
    """b_i = sum_q w_iq g(x_q): the right-hand side of the indirect system
    for boundary data g (a function of an array [k][4] of points (t,x,y,z)).
    The caller's g is sampled at the outer points; the sum runs in the
    library (stb_outer_rhs)."""
    pts, w, n = outer_points(ctx, mesh, m_q)
    vals = np.asarray(g(pts.reshape(-1, 4)), dtype=np.float64)
    if vals.shape != (pts.shape[0] * pts.shape[1],):
        raise ValueError("g must return one value per point")
    return outer_rhs(ctx, mesh, vals.reshape(w.shape), m_q)


def outer_rhs(ctx, mesh, gq, m_q=3):
    """b_i = sum_q w_iq gq[i, q] for data gq at the outer points [nt][4 m_q^2]."""
    gq = np.ascontiguousarray(gq, dtype=np.float64)
    if gq.shape != (mesh.nt, 4 * m_q * m_q):
        raise ValueError("gq must be [%d, %d]" % (mesh.nt, 4 * m_q * m_q))
    b = np.zeros(mesh.nt)
    _chk(load().stb_outer_rhs(ctx.h, mesh.h, m_q, gq.ctypes.data_as(_D), b.ctypes.data_as(_D)),
         ctx.h)
    return b


def solve_gmres(ctx, A, b, x0=None, restart=100, maxit=2000, rtol=1e-10):
    """x with A x = b by restarted GMRES on the device; returns (x, products,
    relative residual)."""
    b, pb = _vec(b, A.n, "b")
    x = np.zeros(A.n) if x0 is None else _vec(np.array(x0, dtype=np.float64), A.n, "x0")[0]
    it = ctypes.c_int32(0)
    rr = ctypes.c_double(0.0)
    _chk(load().stb_solve_gmres(ctx.h, A.h, pb, x.ctypes.data_as(_D), restart, maxit, rtol,
                                ctypes.byref(it), ctypes.byref(rr)), ctx.h)
    return x, it.value, rr.value


def solve_mot(ctx, mesh, A, b):
    """x with A x = b by marching-on-in-time (slab-structured, unjittered
    meshes); returns (x, info) with info = dict(slabs, panels_per_slab,
    inversion_ms, march_ms)."""
    b, pb = _vec(b, A.n, "b")
    x = np.zeros(A.n)
    info = np.zeros(4)
    _chk(load().stb_solve_mot(ctx.h, mesh.h, A.h, pb, x.ctypes.data_as(_D), info.ctypes.data_as(_D)),
         ctx.h)
    return x, dict(slabs=int(info[0]), panels_per_slab=int(info[1]), inversion_ms=float(info[2]),
                   march_ms=float(info[3]))


def inner_values(ctx, mesh, pts, panels, params=None):
    """V phi_panel (pt) for each (point, panel) pair."""
    p = params if params is not None else default_params()
    pts, pp = _points(pts)
    panels = np.ascontiguousarray(panels, dtype=np.int32)
    if panels.ndim != 1 or panels.shape[0] != pts.shape[0]:
        raise ValueError("one panel index per point")
    out = np.zeros(pts.shape[0])
    _chk(load().stb_inner_values(ctx.h, mesh.h, ctypes.byref(p), pts.shape[0], pp,
                                 panels.ctypes.data_as(_I32), out.ctypes.data_as(_D)), ctx.h)
    return out


def potential_D(ctx, mesh, v, pts, params=None):
    """Retarded double-layer potential of the V_h^1 density with vertex
    values v at points (t,x,y,z); the mesh needs its outward normals."""
    p = params if params is not None else default_params()
    v, pv = _vec(v, mesh.nv, "v (vertex values)")
    pts, pp = _points(pts)
    out = np.zeros(pts.shape[0])
    _chk(load().stb_potential_D(ctx.h, mesh.h, ctypes.byref(p), pv, pts.shape[0], pp,
                                out.ctypes.data_as(_D)), ctx.h)
    return out


def potential_D_dev(ctx, mesh, v_ptr, np_, pts_ptr, out_ptr, params=None, stream=None):
    """Double-layer potential with device pointers (vertex values, points, output)."""
    p = params if params is not None else default_params()
    _chk(load().stb_potential_D_dev(ctx.h, mesh.h, ctypes.byref(p), _VP(v_ptr), np_, _VP(pts_ptr),
                                    _VP(out_ptr), _VP(stream) if stream else None), ctx.h)


def dl_energetic(ctx, mesh, v, c_id=0.0, params=None):
    """c_id b_I(v, phi_i) + b_K(v, phi_i) for every test panel (outer rule of
    eq. int_bform); c_id = 1/2: the interior direct method's right-hand side."""
    p = params if params is not None else default_params()
    v, pv = _vec(v, mesh.nv, "v (vertex values)")
    out = np.zeros(mesh.nt)
    _chk(load().stb_dl_energetic(ctx.h, mesh.h, ctypes.byref(p), pv, float(c_id),
                                 out.ctypes.data_as(_D)), ctx.h)
    return out


L2_POINTS = 27


def l2_points(ctx, mesh):
    """Points [nt][27][4] and weights [nt][27] of the projection's rule."""
    pts = np.zeros((mesh.nt, L2_POINTS, 4))
    w = np.zeros((mesh.nt, L2_POINTS))
    _chk(load().stb_l2_points(ctx.h, mesh.h, pts.ctypes.data_as(_D), w.ctypes.data_as(_D)), ctx.h)
    return pts, w


def project_V1(ctx, mesh, gq, nv=None):
    """Vertex values of the L2 projection Q_h^1 g from g at the l2_points;
    returns them and the CG steps taken."""
    nv = mesh.nv if nv is None else nv
    gq, pg = _d(gq, (-1,))
    if gq.shape[0] != mesh.nt * L2_POINTS:
        raise ValueError("need g at the %d points of every panel" % L2_POINTS)
    out = np.zeros(nv)
    it = ctypes.c_int32()
    _chk(load().stb_project_V1(ctx.h, mesh.h, pg, out.ctypes.data_as(_D), ctypes.byref(it)), ctx.h)
    return out, it.value


def inner_values_D(ctx, mesh, pts, panels, params=None):
    """Double-layer potentials of the 4 hat functions of each panel at each
    point: [k, 4], column q for the panel's q-th vertex."""
    p = params if params is not None else default_params()
    pts, pp = _points(pts)
    panels = np.ascontiguousarray(panels, dtype=np.int32)
    if panels.ndim != 1 or panels.shape[0] != pts.shape[0]:
        raise ValueError("one panel index per point")
    out = np.zeros((pts.shape[0], 4))
    _chk(load().stb_inner_values_D(ctx.h, mesh.h, ctypes.byref(p), pts.shape[0], pp,
                                   panels.ctypes.data_as(_I32), out.ctypes.data_as(_D)), ctx.h)
    return out


def potential_S_dev(ctx, mesh, w_ptr, np_, pts_ptr, out_ptr, params=None, stream=None):
    """Potential with device pointers (density, points (t,x,y,z), output)."""
    p = params if params is not None else default_params()
    _chk(load().stb_potential_S_dev(ctx.h, mesh.h, ctypes.byref(p), _VP(w_ptr), np_, _VP(pts_ptr),
                                    _VP(out_ptr), _VP(stream) if stream else None), ctx.h)


class Server:
    """Continuous-batching server on resident meshes (stb_server_*).  The
    arrays of a request are kept alive here until its ticket is waited on."""

    def __init__(self, ctx, hbm_budget=0, nslots=4):
        h = _VP()
        _chk(load().stb_server_create(ctx.h, hbm_budget, nslots, ctypes.byref(h)), ctx.h)
        self.ctx, self.h = ctx, h
        self._live = {}
        self._sizes = {}
        self._lock = __import__("threading").Lock()

    def add_mesh(self, mesh, mat=None):
        i = ctypes.c_int32()
        _chk(load().stb_server_add_mesh(self.h, mesh.h, mat.h if mat is not None else None,
                                        ctypes.byref(i)), self.ctx.h)
        self._sizes[i.value] = mesh.nt
        return i.value

    def _submit(self, req, keep):
        t = ctypes.c_uint64()
        _chk(load().stb_server_submit(self.h, ctypes.byref(req), ctypes.byref(t)), None)
        with self._lock:
            self._live[t.value] = keep
        return t.value

    def submit_matvec(self, mesh_id, W):
        W = np.ascontiguousarray(W, dtype=np.float64)
        n = self._sizes.get(mesh_id)
        if n is None:
            raise ValueError("unknown mesh id %r" % (mesh_id,))
        if W.shape != (n, 16):
            raise ValueError("W must have shape (%d, 16), got %s" % (n, W.shape))
        out = np.empty_like(W)
        req = Request(STB_REQ_MATVEC16, mesh_id, 0, W.ctypes.data, None, out.ctypes.data)
        return self._submit(req, (W, out))

    def submit_potential(self, mesh_id, w, pts):
        n = self._sizes.get(mesh_id)
        if n is None:
            raise ValueError("unknown mesh id %r" % (mesh_id,))
        w, _ = _vec(w, n, "w")
        pts, _ = _points(pts)
        out = np.empty(pts.shape[0])
        req = Request(STB_REQ_POTENTIAL, mesh_id, pts.shape[0], w.ctypes.data, pts.ctypes.data,
                      out.ctypes.data)
        return self._submit(req, (w, pts, out))

    def wait(self, ticket):
        """(result array, latency in seconds)."""
        lat = ctypes.c_double()
        st = load().stb_server_wait(self.h, ticket, ctypes.byref(lat))
        with self._lock:
            keep = self._live.pop(ticket, None)
        _chk(st, None)
        return keep[-1], lat.value

    def close(self):
        if self.h:
            load().stb_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
