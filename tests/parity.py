"""Parity measures shared by the GPU tests (test infrastructure).

Error measure (the relative error near Upsilon = 0 is floored):
    err = |U - U_ref| / max(|U_ref|, 2 N_eff)
with N_eff the number of non-empty segments of the row (its expected value
in pure noise is 2 N_eff: each non-empty segment term is chi^2 with two
degrees of freedom under the noise normalisation of eqn:inner_prod).  N_eff
is counted on the oracle's edges.

Edges are integers and are held to bit-exactness.  The one allowance: an
equal-[h|h] edge b_n = min{k : C(k) >= (n/N) C(k_hi)} may differ where the
oracle's cumulative sits within rounding of the target, so that the two sides'
FP64 sums decide the comparison differently.  Such a row passes only if
  - every bin between the two edges has the oracle's C(k) within
    1e-12 C(k_hi) of the target (checked from the oracle's own cumulative),
  - and its Upsilon matches the oracle evaluated on the GPU's edges
    (explicit-edge mode), to the same tolerance as every other row.
"""
from __future__ import annotations

import numpy as np

import oracle as O

TOL64 = 1e-9
TOLMIX = 1e-5
EDGE_TIE = 1e-12


def n_eff(bounds):
    """Non-empty segments per row of bounds [P, N+1]."""
    b = np.asarray(bounds)
    return np.sum(b[:, 1:] > b[:, :-1], axis=1)


def floored(got, ref, neff):
    """|got - ref| / max(|ref|, 2 N_eff), N_eff >= 1 so that an empty
    support (both zero) reads 0."""
    neff = np.maximum(np.asarray(neff), 1)
    return np.abs(np.asarray(got) - np.asarray(ref)) / np.maximum(np.abs(np.asarray(ref)), 2.0 * neff)


def tied_rows(grid, model, psd, theta, gpu_bnd, ref_bnd, G, mode=O.SEG_EQUAL_SNR):
    """Rows whose edges differ from the oracle's.  Asserts that supports are
    equal, that only equal-[h|h] inner edges differ, and that every
    differing edge is a rounding tie of the oracle's cumulative (module
    docstring).  Returns the indices of the differing rows."""
    gpu_bnd = np.asarray(gpu_bnd, dtype=np.int64)
    ref_bnd = np.asarray(ref_bnd, dtype=np.int64)
    assert gpu_bnd.shape == ref_bnd.shape
    N = gpu_bnd.shape[1] - 1
    rows = np.flatnonzero(~np.all(gpu_bnd == ref_bnd, axis=1))
    if rows.size:
        print(f"edge rows differing from the oracle: {rows.size} of {len(gpu_bnd)} ({rows[:8]})")
    for p in rows:
        assert mode == O.SEG_EQUAL_SNR, f"row {p}: uniform / explicit edges are exact integer work"
        ns = np.flatnonzero(gpu_bnd[p] != ref_bnd[p])
        assert ns.min() > 0 and ns.max() < N, f"row {p}: support differs"
        for n in ns:
            a, b = sorted((int(gpu_bnd[p, n]), int(ref_bnd[p, n])))
            ks = np.arange(a, b)
            Ck, tot, _ = O.edge_cumulative(grid, model, psd, theta[p], G, ks)
            tgt = (n / N) * tot
            gap = np.abs(Ck - tgt).max()
            assert gap <= EDGE_TIE * tot, f"row {p} edge {n}: gpu {gpu_bnd[p, n]} oracle {ref_bnd[p, n]}, " \
                                          f"|C - target| = {gap / tot:.3g} C_tot"
    return rows


def check_rows(ds, theta, got, ref, gpu_bnd, G, tol, mode=O.SEG_EQUAL_SNR, what="", model=None):
    """Floored error of got against the oracle's ref['ups'] on every row with
    the oracle's edges, and against the oracle on the GPU's own edges for the
    tied rows; asserts < tol and returns the max error.  theta, got, ref and
    gpu_bnd hold the same rows; ref must carry 'bounds'."""
    model = ds.model if model is None else model
    got = np.asarray(got)
    ref_ups = ref["ups"]
    ok = ~np.isnan(ref_ups)
    assert np.array_equal(np.isnan(got), ~ok), f"{what}: NaN rows differ"
    tied = tied_rows(ds.grid, model, ds.psd, theta, gpu_bnd, ref["bounds"], G, mode)
    same = ok.copy()
    same[tied] = False
    err = floored(got[same], ref_ups[same], n_eff(ref["bounds"])[same])
    emax = float(err.max()) if err.size else 0.0
    N = ref["bounds"].shape[1] - 1
    for p in tied:
        r = O.evaluate(ds.grid, model, ds.d_ri, ds.psd, theta[p:p + 1], N, O.SEG_EXPLICIT, 1,
                       np.asarray(gpu_bnd[p], dtype=np.int64), want_bounds=True)
        e = float(floored(got[p:p + 1], r["ups"], n_eff(r["bounds"]))[0])
        emax = max(emax, e)
    print(f"{what}: max floored rel err {emax:.3g} over {int(ok.sum())} rows ({len(tied)} tied)")
    assert emax < tol, (what, emax)
    return emax
