"""Lit-panel search of single points (Sec. 3.3, Exp. 1) on the GPU.

For a point x at time t = T the lit set Sigma_N(x) (panels its backward
light cone meets) is a two-dimensional slice of the three-dimensional
space-time boundary, so |Sigma_N(x)| grows like N^(2/3) under uniform
refinement in space and time; the cluster tree's candidate set X_N(x) (the
panels of the leaves that Alg. lit_leaves keeps, tested with Theorem
phi_xi_sphere) stays within a bounded factor of it, for every leaf size
n_min (the factor settles once the leaves are small against the cone); the
per-panel bound test then leaves a subset of the flat cull's candidates.  The domains of Exp. 1: the cube (-1/2, 1/2)^3 with T = 1 and the
unit ball with T = 5, about one slab per spatial mesh width, and the three
points x_A = 0, x_B = (1, 1, 1)/sqrt 3, x_C = (-1, -sqrt 2/2, -1/pi) at
t = T.  The tree and the flat cull must find the same lit sets (both feed
the exact lit test), so the potentials through either search agree to
rounding, and both agree with the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2103_16841_amd import inputs

pytestmark = pytest.mark.gpu

POINTS = {"x_A": (0.0, 0.0, 0.0), "x_B": tuple(np.ones(3) / np.sqrt(3.0)),
          "x_C": (-1.0, -np.sqrt(2.0) / 2.0, -1.0 / np.pi)}
NMIN = (1, 5, 50)


@pytest.fixture(scope="module")
def stb():
    import torch
    torch.cuda.init()
    from paper_2103_16841_amd import stb as s
    s.load()
    return s


@pytest.fixture(scope="module")
def ctx(stb):
    c = stb.Context(0)
    yield c
    c.close()


def _meshes(domain):
    if domain == "cube":
        return 1.0, [inputs.cube_mesh(S=2 ** (L + 1), T=1.0, level=L) for L in range(5)]
    return 5.0, [inputs.icosphere_mesh(level=L, S=5 * 2 ** L, T=5.0, jitter=0.0, seed=0)
                 for L in range(4)]


@pytest.mark.parametrize("domain", ["cube", "ball"])
def test_exp1_lit_and_candidate_sets(stb, ctx, domain):
    T, meshes = _meshes(domain)
    res = {}
    for mesh in meshes:
        m = stb.Mesh(ctx, mesh.vtx, mesh.tets)
        w = inputs.density_normal(mesh.nt, seed=3)
        aw = np.abs(w)
        flat = stb.default_params(lit_search=stb.STB_LIT_FLAT)
        ref = {}
        for name, x in POINTS.items():
            pt = np.array([[T, *x]])
            u_f = stb.potential_S(ctx, m, w, pt, flat)
            wk = ctx.work()
            ref[name] = (u_f[0], wk["lit_pairs"], wk["apex_pairs"],
                         stb.potential_S(ctx, m, aw, pt, flat)[0])
        for nmin in NMIN:
            p = stb.default_params(lit_search=stb.STB_LIT_TREE, n_min=nmin)
            for name, x in POINTS.items():
                u_t = stb.potential_S(ctx, m, w, np.array([[T, *x]]), p)
                wk, ls = ctx.work(), ctx.lit_search()
                u_f, lit_f, cand_f, scale = ref[name]
                # the same lit set: the same count, the same potential to rounding
                assert wk["lit_pairs"] == lit_f, (mesh.name, name, nmin)
                assert abs(u_t[0] - u_f) <= 1e-14 * max(scale, 1e-300)
                assert wk["apex_pairs"] == ls["candidates"] <= cand_f
                assert ls["leaf_panels"] >= ls["candidates"] >= wk["lit_pairs"]
                res[(mesh.nt, name, nmin)] = (wk["lit_pairs"], ls["leaf_panels"])
        print("case: %s N %d: (|Sigma_N|, |X_N|) for n_min %s: %s" %
              (mesh.name, mesh.nt, NMIN,
               {name: [res[(mesh.nt, name, k)] for k in NMIN] for name in POINTS}), flush=True)
        m.close()
    ns = np.array([mm.nt for mm in meshes], dtype=np.float64)
    for name in POINTS:
        lit = np.array([res[(int(n), name, 1)][0] for n in ns], dtype=np.float64)
        slope = np.polyfit(np.log(ns[1:]), np.log(lit[1:]), 1)[0]
        print("%s %s: |Sigma_N| slope in log N %.3f (2/3 expected)" % (domain, name, slope), flush=True)
        assert 0.6 <= slope <= 0.73
        for nmin in NMIN:
            ratio = np.array([res[(int(n), name, nmin)][1] / max(res[(int(n), name, nmin)][0], 1)
                              for n in ns])
            print("   n_min %d: |X_N|/|Sigma_N| %s" % (nmin, np.round(ratio, 2)), flush=True)
            assert ratio[-1] <= 1.3 * ratio[-2]          # bounded: it grows ever slower
            assert ratio[-1] <= {1: 4.0, 5: 9.0, 50: 16.0}[nmin]


def test_tree_potential_vs_oracle(stb, ctx):
    """Many points through the tree against the oracle and the flat search,
    on a jittered icosphere, on-surface and near-surface points included."""
    mesh = inputs.icosphere_mesh(level=1, S=8, T=4.0, jitter=0.2, seed=5)
    m = stb.Mesh(ctx, mesh.vtx, mesh.tets)
    w = inputs.density_normal(mesh.nt, seed=3)
    rng = np.random.default_rng(12)
    pts = np.concatenate([inputs.shell_points(200, mesh.T, seed=4),
                          np.concatenate([rng.uniform(0.3, 4.0, (100, 1)),
                                          rng.uniform(-1.1, 1.1, (100, 3))], axis=1)])
    P, _ = oracle.outer_points(mesh.vtx[mesh.tets[17]])
    pts = np.concatenate([pts, P[:6]])                  # points on a panel face
    u = stb.potential_S(ctx, m, w, pts, stb.default_params(lit_search=stb.STB_LIT_TREE))
    uf = stb.potential_S(ctx, m, w, pts, stb.default_params(lit_search=stb.STB_LIT_FLAT))
    uo = oracle.potential(mesh.vtx, mesh.tets, w, pts)
    absref = oracle.potential(mesh.vtx, mesh.tets, np.abs(w), pts)
    assert np.all(np.abs(u - uo) <= 1e-10 * np.maximum(absref, 1e-300))
    assert np.all(np.abs(u - uf) <= 1e-14 * np.maximum(absref, 1e-300))
    for nmin in (1, 3, 64, 4096):
        un = stb.potential_S(ctx, m, w, pts, stb.default_params(lit_search=stb.STB_LIT_TREE, n_min=nmin))
        assert np.all(np.abs(un - uf) <= 1e-14 * np.maximum(absref, 1e-300)), nmin
    with pytest.raises(stb.StbError):
        stb.potential_S(ctx, m, w, pts, stb.default_params(lit_search=stb.STB_LIT_TREE, n_min=0))
