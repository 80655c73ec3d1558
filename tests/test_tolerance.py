"""The parity bound of tests/_tol.py is not vacuous: on the cube and on a
jittered icosphere, the conditioning term P_ij (the oracle's own change
under vertex coordinates moved by two ulps) is below 1e-13 of M_ij for
the median entry and exceeds 1e-10 M_ij only for a few barely lit pairs;
the bound therefore stays at the 1e-10 M_ij level for almost every entry."""
import numpy as np

from paper_2103_16841_amd import inputs
from _tol import oracle_rows


def _ratios(mesh):
    A, M, P = oracle_rows(mesh.vtx, mesh.tets)
    nz = M > 0.0
    return (P[nz] / M[nz]), A, M


def test_conditioning_term_is_small_for_almost_all_entries():
    for mesh in (inputs.cube_mesh(), inputs.icosphere_mesh(level=0, S=5, T=4.0, jitter=0.2, seed=4)):
        r, A, M = _ratios(mesh)
        print(mesh.name, "P/M quantiles 50/99/99.9/max:", np.quantile(r, [0.5, 0.99, 0.999, 1.0]))
        assert np.median(r) < 1e-13
        assert np.quantile(r, 0.999) < 1e-10
        assert (r > 1e-10).sum() <= 1e-3 * r.size
