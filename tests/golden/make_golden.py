"""Writes tests/golden/cube_S4_T2.txt from the oracle alone (no HIP code):
the 144-panel cube workload (surface of (-1/2, 1/2)^3 x (0, 2), 4 slabs,
no jitter; Sec. 4's domain): its exact causal-pair count, 200 seeded
entries A_ij = b_V(phi_j, phi_i) (eq. int_bform, m_q = 3, n_g = 16), each
with the size of its outer-sum terms M_ij = sum_q |w_q I_q|, and the
product y = A w for w ~ N(0, 1) (seed 0) with its bound sum_j M_ij |w_j|.  The paper prints no numbers for
this case; the file lets the tests check the oracle against its own past
output and the HIP path against stored values.

Run from the repository root: python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2103_16841_amd import inputs  # noqa: E402


def main():
    mesh = inputs.cube_mesh(S=4, T=2.0)
    A, M = oracle.assemble_rows(mesh.vtx, mesh.tets, mag=True)
    causal = int(oracle.count_causal_per_row(mesh.vtx, mesh.tets).sum())
    rng = np.random.default_rng(0)
    nz = np.argwhere(A != 0.0)
    pick = nz[rng.choice(len(nz), 150, replace=False)]
    zero = np.argwhere(A == 0.0)
    pick = np.concatenate([pick, zero[rng.choice(len(zero), 50, replace=False)]])
    w = inputs.density_normal(mesh.nt, seed=0)
    y = oracle.matvec_rows(mesh.vtx, mesh.tets, w)
    yb = M @ np.abs(w)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cube_S4_T2.txt")
    with open(out, "w") as f:
        f.write("# cube (-1/2,1/2)^3 x (0,2), 4 slabs, no jitter: 144 panels; m_q 3, n_g 16\n")
        f.write("# written by tests/golden/make_golden.py from the oracle\n")
        f.write("causal %d\n" % causal)
        for i, j in pick:
            f.write("entry %d %d %.17g %.17g\n" % (i, j, A[i, j], M[i, j]))
        for i, v in enumerate(y):
            f.write("matvec %d %.17g %.17g\n" % (i, v, yb[i]))


if __name__ == "__main__":
    main()
