"""The allocation-free 16-RHS product (stb_apply16_noalloc) against the
allocating one (stb_apply_dev, nrhs = 16) through the C ABI: the same kernels
on the same inputs, so the results must agree bit for bit.  Two calls in a
row share the static scratch array, the second with a smaller matrix and
input; a matrix without its matrix-core copy is refused."""
import ctypes

import numpy as np
import pytest

from paper_2103_16841_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stb():
    import torch
    torch.cuda.init()
    from paper_2103_16841_amd import stb as s
    s.load()
    return s


def _case(stb, ctx, mesh, seed):
    import torch
    dev = torch.device("cuda:0")
    m = stb.Mesh(ctx, mesh.vtx, mesh.tets)
    A = stb.assemble_V(ctx, m)
    W = torch.from_numpy(np.random.default_rng(seed).standard_normal((mesh.nt, 16))).to(dev)
    Y1 = torch.full_like(W, np.nan)
    Y2 = torch.full_like(W, np.nan)
    torch.cuda.synchronize()
    return m, A, W, Y1, Y2


def test_noalloc_equals_allocating_product(stb):
    import torch
    ctx = stb.Context(0)
    big = inputs.icosphere_mesh(level=1, S=12, T=4.0, jitter=0.2, seed=31)   # 2,880 panels
    small = inputs.cube_mesh()                                               # 144 panels
    L = stb.load()
    for mesh, seed in ((big, 1), (small, 2)):
        print("case: no-alloc product,", mesh.name, "N =", mesh.nt, flush=True)
        m, A, W, Y1, Y2 = _case(stb, ctx, mesh, seed)
        # refused before the matrix-core copy exists
        st = L.stb_apply16_noalloc(ctx.h, A.h, ctypes.c_void_p(W.data_ptr()),
                                   ctypes.c_void_p(Y2.data_ptr()), None)
        assert st == 1
        A.apply_dev(W.data_ptr(), Y1.data_ptr(), 16)          # allocating entry point
        torch.cuda.synchronize()
        st = L.stb_apply16_noalloc(ctx.h, A.h, ctypes.c_void_p(W.data_ptr()),
                                   ctypes.c_void_p(Y2.data_ptr()), None)
        assert st == 0
        torch.cuda.synchronize()          # the call only enqueues on the context stream
        y1, y2 = Y1.cpu().numpy(), Y2.cpu().numpy()
        assert np.all(np.isfinite(y2))
        assert np.array_equal(y1, y2)
        # and the product itself against the FP64 store (FP32 matrix cores)
        y64 = np.stack([A.apply(np.ascontiguousarray(W.cpu().numpy()[:, c])) for c in range(16)], axis=1)
        rp, cols, vals = A.export()
        from scipy.sparse import csr_matrix
        absAW = csr_matrix((np.abs(vals), cols, rp), shape=(mesh.nt, mesh.nt)) @ np.abs(W.cpu().numpy())
        assert np.all(np.abs(y2 - y64) <= 2e-6 * absAW)
        A.close()
        m.close()
    ctx.close()
