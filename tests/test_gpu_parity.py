"""GPU path vs the FP64 oracle (element by element), through the C ABI.

Tolerance (plain FP64), per entry: |A_gpu - A_orc| <= 1e-10 M_ij + 2 P_ij
with M_ij = sum_q |w_q I_q| the size of the entry's outer-sum terms (eq.
int_bform) and P_ij the change of the oracle's entry when the vertex
coordinates move by two ulps (tests/_tol.py); entries of non-causal pairs
must be exactly +0.0 on both sides, and the causal-pair count must agree
exactly.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2103_16841_amd import inputs

pytestmark = pytest.mark.gpu

from _tol import RTOL, assert_entries, oracle_rows, row_bound


@pytest.fixture(scope="module")
def stb():
    import torch
    torch.cuda.init()          # torch's HIP state first, then the library
    from paper_2103_16841_amd import stb as s
    print("loading", s.lib_path(), flush=True)
    s.load()
    return s


@pytest.fixture(scope="module")
def ctx(stb):
    c = stb.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def cube():
    return inputs.cube_mesh()


@pytest.fixture(scope="module")
def cube_AMP(cube):
    return oracle_rows(cube.vtx, cube.tets)


@pytest.fixture(scope="module")
def cube_ref(cube_AMP):
    return cube_AMP[0]


@pytest.fixture(scope="module")
def cube_M(cube_AMP):
    return cube_AMP[1]


@pytest.fixture(scope="module")
def cube_P(cube_AMP):
    return cube_AMP[2]


@pytest.fixture(scope="module")
def cube_gpu(stb, ctx, cube):
    m = stb.Mesh(ctx, cube.vtx, cube.tets)
    A = stb.assemble_V(ctx, m)
    return m, A


def test_cube_full_matrix(cube_gpu, cube_ref, cube_M, cube_P):
    print("case: cube N=144 full matrix", flush=True)
    _, A = cube_gpu
    D = A.to_dense()
    assert_entries(D, cube_ref, cube_M, cube_P, what="cube")
    zero = cube_ref == 0.0
    assert np.all(D[~zero] != 0.0)


def test_cube_causal_count(cube, cube_gpu, cube_ref):
    _, A = cube_gpu
    per_row = oracle.count_causal_per_row(cube.vtx, cube.tets)
    assert A.n_causal == per_row.sum() == np.count_nonzero(cube_ref)
    assert A.n_stored == A.n_causal           # the store keeps the causal pairs only


def test_cube_matvec(cube, cube_gpu, cube_M, cube_P):
    _, A = cube_gpu
    w = inputs.density_normal(cube.nt, seed=0)
    y = A.apply(w)
    yo = oracle.matvec_rows(cube.vtx, cube.tets, w)
    assert np.all(np.abs(y - yo) <= row_bound(cube_M, w, cube_P))


def test_cube_matvec_16rhs_matrix_cores(cube, cube_gpu, cube_ref):
    """16 right-hand sides on the FP32 matrix cores vs the FP64 product."""
    _, A = cube_gpu
    W = np.random.default_rng(1).standard_normal((cube.nt, 16))
    Y = A.apply(W)
    ref = cube_ref @ W
    scale = np.abs(cube_ref) @ np.abs(W)
    assert np.all(np.abs(Y - ref) <= 2e-6 * scale)
    # FP32 rounding really happened (not an FP64 path)
    assert np.abs(Y - ref).max() > 0.0


def test_matrix_core_product_many_columns(stb, ctx):
    """The 16-RHS FP32 matrix-core product on a 3,840-panel icosphere, whose
    16-row blocks span thousands of columns (several LDS tiles per block in
    the blocked copy), against the FP64 product of the same matrix (itself
    checked against the oracle elsewhere), column by column."""
    mesh = inputs.icosphere_mesh(level=1, S=16, T=4.0, jitter=0.2, seed=8)
    m = stb.Mesh(ctx, mesh.vtx, mesh.tets)
    A = stb.assemble_V(ctx, m)
    W = np.random.default_rng(5).standard_normal((mesh.nt, 16))
    Y = A.apply(W)
    Y64 = np.stack([A.apply(np.ascontiguousarray(W[:, c])) for c in range(16)], axis=1)
    from scipy.sparse import csr_matrix
    rowptr, cols, vals = A.export()
    absAW = csr_matrix((np.abs(vals), cols, rowptr), shape=(mesh.nt, mesh.nt)) @ np.abs(W)
    err = np.abs(Y - Y64) / np.maximum(absAW, 1e-300)
    print("16-RHS vs FP64: worst |dY| / (|A| |W|) = %.3e" % err.max(), flush=True)
    assert np.all(np.abs(Y - Y64) <= 2e-6 * absAW)
    A.close()
    m.close()


def test_entries_get(cube_gpu, cube_ref, cube_M, cube_P):
    _, A = cube_gpu
    rng = np.random.default_rng(0)
    r = rng.integers(0, 144, 500)
    c = rng.integers(0, 144, 500)
    v = A.get(r, c)
    assert_entries(v, cube_ref[r, c], cube_M[r, c], cube_P[r, c], what="get")


@pytest.mark.parametrize("S,T,jit,L", [(3, 1.5, 0.0, None), (5, 2.5, 0.2, 0), (2, 3.0, 0.2, 1)])
def test_small_meshes_full(stb, ctx, S, T, jit, L):
    """Ragged sizes: several tiles per row with a ragged last tile."""
    mesh = inputs.cube_mesh(S=S, T=T, jitter=jit, seed=3) if L is None else \
        inputs.icosphere_mesh(level=L, S=S, T=T, jitter=jit, seed=4)
    print("case:", mesh, flush=True)
    ref, mag, pert = oracle_rows(mesh.vtx, mesh.tets)
    m = stb.Mesh(ctx, mesh.vtx, mesh.tets)
    A = stb.assemble_V(ctx, m)
    D = A.to_dense()
    assert_entries(D, ref, mag, pert, what=str(mesh))
    assert A.n_causal == np.count_nonzero(ref)


@pytest.mark.parametrize("n_g,m_q", [(8, 3), (24, 2), (16, 1)])
def test_quadrature_parameters(stb, ctx, cube, n_g, m_q):
    rows = np.arange(0, cube.nt, 5)
    ref, mag, pert = oracle_rows(cube.vtx, cube.tets, rows=rows, n_g=n_g, m_q=m_q)
    m = stb.Mesh(ctx, cube.vtx, cube.tets)
    A = stb.assemble_V(ctx, m, stb.default_params(n_g=n_g, m_q=m_q))
    D = A.to_dense()[rows]
    assert_entries(D, ref, mag, pert, what="n_g %d m_q %d" % (n_g, m_q))


@pytest.fixture(scope="module")
def ico2():
    return inputs.icosphere_mesh(level=2, S=32, T=4.0, jitter=0.2, seed=2)


@pytest.fixture(scope="module")
def ico2_gpu(stb, ctx, ico2):
    print("case: icosphere L2 S32 N=30720 assembly", flush=True)
    m = stb.Mesh(ctx, ico2.vtx, ico2.tets)
    A = stb.assemble_V(ctx, m)
    print("assembled: causal", A.n_causal, "stored", A.n_stored, ctx.timings(), flush=True)
    return m, A


@pytest.fixture(scope="module")
def ico2_rows(ico2):
    """256 seeded rows of the full-size workload, every column (oracle)."""
    rows = np.sort(np.random.default_rng(7).choice(ico2.nt, 256, replace=False))
    return (rows,) + oracle_rows(ico2.vtx, ico2.tets, rows=rows)


def test_icosphere_sampled_rows(ico2, ico2_gpu, ico2_rows):
    """Full-size workload: 256 seeded rows, every column, vs the oracle."""
    _, A = ico2_gpu
    rows, ref, mag, pert = ico2_rows
    rr = np.repeat(rows, ico2.nt).astype(np.int32)
    cc = np.tile(np.arange(ico2.nt), rows.size).astype(np.int32)
    got = A.get(rr, cc).reshape(rows.size, ico2.nt)
    print("rows", rows[:8], "...", flush=True)
    assert_entries(got, ref, mag, pert, what="icosphere rows")
    assert np.array_equal(got != 0.0, ref != 0.0)


def test_icosphere_matvec_sampled_rows(ico2, ico2_gpu, ico2_rows):
    """The bench step's product (w ~ N(0,1), seed 0) on the same 256 rows."""
    _, A = ico2_gpu
    rows, ref_rows, mag, pert = ico2_rows
    w = inputs.density_normal(ico2.nt, seed=0)
    y = A.apply(w)
    yo = oracle.matvec_rows(ico2.vtx, ico2.tets, w, rows=rows)
    assert np.all(np.abs(y[rows] - yo) <= row_bound(mag, w, pert))


def test_icosphere_causal_count_property(ico2, ico2_gpu):
    """Exact causal count vs the oracle's per-row counts on sampled rows:
    the GPU count over all rows is checked through its stored nonzeros."""
    _, A = ico2_gpu
    rows = np.sort(np.random.default_rng(9).choice(ico2.nt, 64, replace=False))
    per = oracle.count_causal_per_row(ico2.vtx, ico2.tets, rows=rows)
    rr = np.repeat(rows, ico2.nt).astype(np.int32)
    cc = np.tile(np.arange(ico2.nt), rows.size).astype(np.int32)
    got = A.get(rr, cc).reshape(rows.size, ico2.nt)
    assert np.array_equal((got != 0).sum(axis=1), per)
    assert A.n_causal > 0.9 * per.mean() * ico2.nt / 2
    assert A.n_stored == A.n_causal
    rp, cols, vals = A.export()
    assert np.all(vals != 0.0) and np.all(np.diff(rp) >= 0)
    assert all(np.all(np.diff(cols[rp[i]:rp[i + 1]]) > 0) for i in range(0, ico2.nt, 97))


def test_bench_potential_sampled_points(stb, ctx, ico2, ico2_gpu):
    """The bench step's potential (1,000 shell points, |x| in [1.5, 3], t in
    [0, T], density N(0,1) seed 5) on the 30,720-panel mesh, in the launch
    the bench times (all 1,000 points in one call): 64 seeded points against
    the oracle, each to 1e-10 of sum_j |w_j| V phi_j (p)."""
    m, _ = ico2_gpu
    w = inputs.density_normal(ico2.nt, seed=5)
    pts = inputs.shell_points(1000, ico2.T, seed=4)
    u = stb.potential_S(ctx, m, w, pts)
    k = np.sort(np.random.default_rng(23).choice(1000, 64, replace=False))
    print("case: bench potential, points", k[:8], "...", flush=True)
    uo = oracle.potential(ico2.vtx, ico2.tets, w, pts[k])
    absref = oracle.potential(ico2.vtx, ico2.tets, np.abs(w), pts[k])
    err = np.abs(u[k] - uo) / np.maximum(absref, 1e-300)
    print("worst |du| / S|w| = %.3e" % err.max(), flush=True)
    assert np.all(np.abs(u[k] - uo) <= RTOL * absref)
    assert np.all((u[k] == 0.0) == (absref == 0.0))


def test_potential_vs_oracle(stb, ctx):
    mesh = inputs.icosphere_mesh(level=1, S=8, T=4.0, jitter=0.2, seed=5)
    m = stb.Mesh(ctx, mesh.vtx, mesh.tets)
    w = inputs.density_normal(mesh.nt, seed=3)
    pts = inputs.shell_points(300, mesh.T, seed=4)
    u = stb.potential_S(ctx, m, w, pts)
    uo = oracle.potential(mesh.vtx, mesh.tets, w, pts)
    # norm-wise: relative to sum_j |w_j| V phi_j (p)
    absref = oracle.potential(mesh.vtx, mesh.tets, np.abs(w), pts)
    assert np.all(np.abs(u - uo) <= RTOL * np.maximum(absref, 1e-300))


def test_potential_near_and_on_surface(stb, ctx):
    mesh = inputs.cube_mesh(S=4, T=2.0)
    m = stb.Mesh(ctx, mesh.vtx, mesh.tets)
    w = inputs.density_time(mesh, lambda t: np.sin(np.pi * t / 2) ** 2)
    rng = np.random.default_rng(6)
    pts = np.concatenate([rng.uniform(0.2, 2.0, (60, 1)), rng.uniform(-0.6, 0.6, (60, 3))], axis=1)
    pts[:10, 3] = 0.5                       # on a face plane
    u = stb.potential_S(ctx, m, w, pts)
    uo = oracle.potential(mesh.vtx, mesh.tets, w, pts)
    assert np.allclose(u, uo, rtol=RTOL, atol=1e-14)


def test_errors(stb, ctx):
    vtx = np.array([[0, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [1, 0, 0, 0.3]], float)
    with pytest.raises(stb.StbError) as e:
        stb.Mesh(ctx, vtx, np.array([[0, 1, 2, 3]]))          # not vertical
    assert e.value.status == 2
    vtx2 = vtx.copy()
    vtx2[3, 3] = 0.0
    vtx2[1, 2] = np.nan
    with pytest.raises(stb.StbError) as e:
        stb.Mesh(ctx, vtx2, np.array([[0, 1, 2, 3]]))
    assert e.value.status == 2
    with pytest.raises(stb.StbError) as e:
        stb.Mesh(ctx, vtx, np.array([[0, 1, 2, 7]]))          # bad index
    assert e.value.status == 2
    good = vtx.copy()
    good[3, 3] = 0.0
    m = stb.Mesh(ctx, good, np.array([[0, 1, 2, 3]]))
    with pytest.raises(stb.StbError) as e:
        stb.assemble_V(ctx, m, stb.default_params(n_g=0))
    assert e.value.status == 1


def test_unshared_faces_equal_shared(stb, ctx):
    """The FP64 assembly evaluates each face shared by two panels once.  The
    same mesh with every panel on vertices of its own shares no face, so
    each face is evaluated per panel: the matrices agree to rounding, with
    the same causal pairs, and both match the oracle."""
    mesh = inputs.icosphere_mesh(level=0, S=4, T=2.5, jitter=0.2, seed=7)
    vtx_split = mesh.vtx[mesh.tets].reshape(-1, 4).copy()
    tets_split = np.arange(4 * mesh.nt, dtype=np.int32).reshape(mesh.nt, 4)
    print("case: icosphere L0 S4 shared vs unshared faces", flush=True)
    A1 = stb.assemble_V(ctx, stb.Mesh(ctx, mesh.vtx, mesh.tets))
    A2 = stb.assemble_V(ctx, stb.Mesh(ctx, vtx_split, tets_split))
    D1, D2 = A1.to_dense(), A2.to_dense()
    assert A1.n_causal == A2.n_causal
    assert np.array_equal(D1 != 0.0, D2 != 0.0)
    ref, mag, pert = oracle_rows(mesh.vtx, mesh.tets)
    assert_entries(D1, ref, mag, pert, what="shared faces")
    assert_entries(D2, ref, mag, pert, what="unshared faces")
    assert np.all(np.abs(D1 - D2) <= 2 * (RTOL * mag + 2 * pert))


def test_single_panel_and_empty_points(stb, ctx):
    vtx = np.array([[0, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [1, 0, 0, 0]], float)
    tets = np.array([[0, 1, 2, 3]])
    m = stb.Mesh(ctx, vtx, tets)
    A = stb.assemble_V(ctx, m)
    ref, mag, pert = oracle_rows(vtx, tets)
    assert_entries(A.to_dense(), ref, mag, pert, what="one panel")
    assert stb.potential_S(ctx, m, np.ones(1), np.zeros((0, 4))).shape == (0,)


def test_device_pointer_paths(stb, ctx):
    """Mesh ingest, products and potential from device-resident inputs."""
    import torch
    mesh = inputs.icosphere_mesh(level=0, S=6, T=3.0, jitter=0.2, seed=12)
    dev = torch.device("cuda:0")
    vtx = torch.from_numpy(mesh.vtx).to(dev)
    tet = torch.from_numpy(mesh.tets).to(dev)
    torch.cuda.synchronize()
    m = stb.Mesh.from_device(ctx, vtx.data_ptr(), mesh.nv, tet.data_ptr(), mesh.nt)
    A = stb.assemble_V(ctx, m)
    ref, mag, pert = oracle_rows(mesh.vtx, mesh.tets)
    assert_entries(A.to_dense(), ref, mag, pert, what="device pointers")
    w = inputs.density_normal(mesh.nt, seed=1)
    wd = torch.from_numpy(w).to(dev)
    yd = torch.empty_like(wd)
    torch.cuda.synchronize()
    A.apply_dev(wd.data_ptr(), yd.data_ptr(), 1)
    torch.cuda.synchronize()
    assert np.all(np.abs(yd.cpu().numpy() - ref @ w) <= row_bound(mag, w, pert))
    W = np.random.default_rng(2).standard_normal((mesh.nt, 16))
    Wd = torch.from_numpy(W).to(dev)
    Yd = torch.empty_like(Wd)
    torch.cuda.synchronize()
    A.apply_dev(Wd.data_ptr(), Yd.data_ptr(), 16)
    torch.cuda.synchronize()
    assert np.all(np.abs(Yd.cpu().numpy() - ref @ W) <= 2e-6 * (np.abs(ref) @ np.abs(W)))
    pts = inputs.shell_points(64, mesh.T, seed=3)
    pd = torch.from_numpy(pts).to(dev)
    ud = torch.empty(64, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    stb.potential_S_dev(ctx, m, wd.data_ptr(), 64, pd.data_ptr(), ud.data_ptr())
    uo = oracle.potential(mesh.vtx, mesh.tets, w, pts)
    absref = oracle.potential(mesh.vtx, mesh.tets, np.abs(w), pts)
    assert np.all(np.abs(ud.cpu().numpy() - uo) <= RTOL * np.maximum(absref, 1e-300))
    bad = tet.clone()
    bad[3, 2] = mesh.nv + 5
    torch.cuda.synchronize()
    with pytest.raises(stb.StbError) as e:
        stb.Mesh.from_device(ctx, vtx.data_ptr(), mesh.nv, bad.data_ptr(), mesh.nt)
    assert e.value.status == 2


def _unique_outer_points(mesh):
    """The outer points of every panel (oracle), each shared point once: a
    face with nu_t != 0 belongs to two panels, which evaluate the same
    points (up to rounding)."""
    seen, pts = set(), []
    for i in range(mesh.nt):
        P, _ = oracle.outer_points(mesh.vtx[mesh.tets[i]])
        for x in P:
            key = tuple(np.round(x, 9))
            if key not in seen:
                seen.add(key)
                pts.append(x)
    return np.array(pts)


def test_work_counters(stb, ctx, cube):
    """FP64 work per distinct (outer point, panel) pair against the oracle
    run on the same pairs: each face's points are evaluated once for the
    two panels that share the face."""
    m = stb.Mesh(ctx, cube.vtx, cube.tets)
    stb.assemble_V(ctx, m)
    w = ctx.work()
    pts = _unique_outer_points(cube)
    st = oracle.Stats()
    for x in pts:
        for j in range(cube.nt):
            oracle.inner(x, cube.vtx[cube.tets[j]], stats=st)
    print("case: cube, %d distinct outer points" % len(pts), w, st.as_dict(), flush=True)
    # the same rule: lit (outer point, panel) pairs and L evaluations (piece
    # tests and Gauss nodes) agree up to decisions taken within rounding: a
    # sliver piece between two nearly coincident breakpoints where L is
    # rounding noise (~1e-17) on one side and exactly 0 on the other costs
    # n_g node evaluations that contribute nothing
    # pieces the ray test finds empty skip the three evaluations of the
    # empty-piece test
    pc = ctx.path_counts()
    assert pc["ray_empty_pieces"] > 0
    assert abs(w["lit_pairs"] - st.n_lit) <= 0.01 * st.n_lit
    evals = w["L_evals"] + 3 * pc["ray_empty_pieces"]
    assert abs(evals - st.n_eval) <= 0.03 * st.n_eval
