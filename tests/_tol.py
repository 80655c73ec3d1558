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
"""
import numpy as np

RTOL = 1e-10


def entry_err(got, ref, mag):
    """Per-entry error in units of M_ij (inf where M_ij = 0 and got != ref)."""
    got = np.asarray(got, dtype=np.float64)
    d = np.abs(got - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(mag > 0.0, d / np.where(mag > 0.0, mag, 1.0), np.where(d == 0.0, 0.0, np.inf))
    return e


def assert_entries(got, ref, mag, rtol=RTOL, what="entries"):
    """|got - ref| <= rtol M elementwise; non-causal entries +0.0 exactly."""
    got = np.asarray(got, dtype=np.float64)
    e = entry_err(got, ref, mag)
    if e.size and e.max() > rtol:
        k = np.unravel_index(np.argmax(e), e.shape)
        print("%s: worst %s got %.17g oracle %.17g M %.3e err/M %.3e" %
              (what, k, got[k], ref[k], mag[k], e[k]), flush=True)
    assert e.size == 0 or e.max() <= rtol, e.max()
    zero = mag == 0.0
    assert np.all(got[zero] == 0.0)
    assert not np.any(np.signbit(got[zero]))


def row_bound(mag, w):
    """Per-row bound of |sum_j dA_ij w_j| under the entrywise tolerance."""
    return np.asarray(mag) @ np.abs(np.asarray(w))


MTOL = 1e-6


def assert_entries_mixed(got, ref, mag, mtol=MTOL, rtol=RTOL, what="entries"):
    """Mixed precision: |got - ref| <= mtol |A_ij| + rtol M_ij (relative 1e-6
    of the entry itself, plus the FP64 parity allowance for entries that the
    mixed path recomputes in FP64); non-causal entries +0.0 exactly."""
    got = np.asarray(got, dtype=np.float64)
    d = np.abs(got - ref)
    lim = mtol * np.abs(ref) + rtol * mag
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
