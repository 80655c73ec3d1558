"""Stored oracle values (tests/golden/cube_S4_T2.txt, written by
tests/golden/make_golden.py from the oracle alone): the oracle must still
produce them, and the HIP path must match them to the parity tolerance
(per entry 1e-10 of the size of its outer-sum terms, stored beside it;
zeros exact; the causal count exact)."""
import numpy as np
import pytest

import oracle
from paper_2103_16841_amd import inputs
from _golden import load_cube
from _tol import RTOL, assert_entries


def test_oracle_reproduces_golden():
    causal, rows, cols, vals, mags, y, yb = load_cube()
    mesh = inputs.cube_mesh(S=4, T=2.0)
    got = np.array([oracle.entry(mesh.vtx, mesh.tets, int(i), int(j)) for i, j in zip(rows, cols)])
    assert np.all(np.abs(got - vals) <= 1e-14 * np.abs(vals).max())
    assert np.all((got == 0.0) == (vals == 0.0))
    assert int(oracle.count_causal_per_row(mesh.vtx, mesh.tets).sum()) == causal
    yo = oracle.matvec_rows(mesh.vtx, mesh.tets, inputs.density_normal(mesh.nt, seed=0))
    assert np.all(np.abs(yo - y) <= 1e-14 * np.abs(y).max())


@pytest.mark.gpu
def test_gpu_matches_golden():
    import torch
    torch.cuda.init()
    from paper_2103_16841_amd import stb
    stb.load()
    causal, rows, cols, vals, mags, y, yb = load_cube()
    mesh = inputs.cube_mesh(S=4, T=2.0)
    ctx = stb.Context(0)
    try:
        m = stb.Mesh(ctx, mesh.vtx, mesh.tets)
        A = stb.assemble_V(ctx, m)
        assert A.n_causal == causal
        got = A.get(rows, cols)
        assert_entries(got, vals, mags, what="golden")
        yg = A.apply(inputs.density_normal(mesh.nt, seed=0))
        assert np.all(np.abs(yg - y) <= RTOL * yb)
        A.close()
        m.close()
    finally:
        ctx.close()
