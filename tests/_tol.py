"""Parity tolerances shared by the GPU tests.

A matrix entry of eq. int_bform is an outer sum A_ij = sum_q w_q I_q whose
top- and bottom-face terms cancel (the weights are +-|T_i| / m_q^2), so the
accuracy that two implementations of the same rule can share is set by the
size of the terms, M_ij = sum_q |w_q I_q| (oracle.assemble_rows(mag=True)),
not by |A_ij|: an inner integral I_q reproduced to relative 1e-10 moves the
entry by up to 1e-10 |w_q I_q|.  The bound is therefore per entry,
|A_gpu - A_orc| <= rtol * M_ij  (M_ij >= |A_ij|, and M_ij = 0 exactly where
the pair is not causal, so those entries must agree exactly: +0.0 on both
sides).  A product y = A w inherits sum_j M_ij |w_j| per row.

Barely lit pairs (a cone grazing a panel: a sliver of the panel is lit) are
ill-conditioned in the geometry: moving the vertices by a couple of ulps
moves such an entry by more than 1e-10 M_ij in the oracle itself, and two
correct implementations round the same geometry differently (frames, face
planes, apex data).  The bound therefore adds the conditioning the oracle
shows, P_ij = max over four meshes whose vertex coordinates are scaled by
1 + 2u r (r ~ U(-1, 1), u = 2^-53) of |A'_ij - A_ij|:
|A_gpu - A_orc| <= 1e-10 M_ij + 2 P_ij  (oracle_rows()).
"""
import numpy as np

import oracle

RTOL = 1e-10
U = 2.0 ** -53
NPERTURB = 4


def perturbed_vertices(vtx, seed, ulps=2):
    """Vertex coordinates scaled by 1 + ulps u r, r ~ U(-1, 1) (seeded)."""
    r = np.random.default_rng(1000 + seed).uniform(-1.0, 1.0, vtx.shape)
    return vtx * (1.0 + ulps * U * r)


def oracle_rows(vtx, tets, rows=None, nperturb=NPERTURB, **kw):
    """Rows of A from the oracle with the two scales of the parity bound:
    (A, M, P), M the size of each entry's outer-sum terms, P its change under
    vertex coordinates perturbed by two ulps (max over nperturb meshes)."""
    A, M = oracle.assemble_rows(vtx, tets, rows=rows, mag=True, **kw)
    P = np.zeros_like(A)
    for s in range(nperturb):
        Ap = oracle.assemble_rows(perturbed_vertices(vtx, s), tets, rows=rows, **kw)
        np.maximum(P, np.abs(Ap - A), out=P)
    return A, M, P


def limit(mag, pert=None, rtol=RTOL):
    """The per-entry parity bound rtol M_ij + 2 P_ij."""
    lim = rtol * np.asarray(mag)
    return lim if pert is None else lim + 2.0 * np.asarray(pert)


def assert_entries(got, ref, mag, pert=None, rtol=RTOL, what="entries"):
    """|got - ref| <= rtol M + 2 P elementwise; non-causal entries +0.0
    exactly (M = 0 there)."""
    got = np.asarray(got, dtype=np.float64)
    d = np.abs(got - ref)
    lim = limit(mag, pert, rtol)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(mag > 0.0, d / np.where(mag > 0.0, mag, 1.0), np.where(d == 0.0, 0.0, np.inf))
    if e.size:
        k = np.unravel_index(np.argmax(e), e.shape)
        print("%s: %d entries, largest |d|/M %.3e at %s (got %.17g oracle %.17g M %.3e P %.3e)" %
              (what, e.size, e[k], k, got[k], ref[k], mag[k],
               0.0 if pert is None else pert[k]), flush=True)
    bad = d > lim
    if np.any(bad):
        k = np.unravel_index(np.argmax(np.where(bad, d - lim, -np.inf)), d.shape)
        print("%s: %d entries over the bound, e.g. %s: got %.17g oracle %.17g M %.3e P %.3e" %
              (what, int(bad.sum()), k, got[k], ref[k], mag[k], 0.0 if pert is None else pert[k]),
              flush=True)
    assert not np.any(bad)
    zero = mag == 0.0
    assert np.all(got[zero] == 0.0)
    assert not np.any(np.signbit(got[zero]))


def row_bound(mag, w, pert=None):
    """Per-row bound of |sum_j dA_ij w_j| under the entrywise tolerance."""
    return limit(mag, pert) @ np.abs(np.asarray(w))


MTOL = 1e-6


def assert_entries_mixed(got, ref, mag, pert=None, mtol=MTOL, rtol=RTOL, what="entries"):
    """Mixed precision: |got - ref| <= mtol |A_ij| + rtol M_ij + 2 P_ij
    (relative 1e-6 of the entry itself, plus the FP64 parity allowance for
    entries that the mixed path recomputes in FP64); non-causal entries
    +0.0 exactly."""
    got = np.asarray(got, dtype=np.float64)
    d = np.abs(got - ref)
    lim = mtol * np.abs(ref) + limit(mag, pert, rtol)
    bad = d > lim
    if np.any(bad):
        with np.errstate(divide="ignore", invalid="ignore"):
            k = np.unravel_index(np.argmax(np.where(lim > 0, d / lim, np.inf)), d.shape)
        print("%s: worst %s got %.17g oracle %.17g M %.3e |d| %.3e limit %.3e" %
              (what, k, got[k], ref[k], mag[k], d[k], lim[k]), flush=True)
    assert not np.any(bad)
    zero = mag == 0.0
    assert np.all(got[zero] == 0.0)
    assert not np.any(np.signbit(got[zero]))


def rel_err_entries(got, ref):
    """max |got - ref| / |ref| over the non-zero entries (the figure reported)."""
    nz = ref != 0.0
    return float((np.abs(got[nz] - ref[nz]) / np.abs(ref[nz])).max()) if np.any(nz) else 0.0
