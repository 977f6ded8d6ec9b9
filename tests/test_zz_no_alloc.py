"""scs_evaluate_noalloc: the evaluation without any allocation, its buffers
in the library's static device scratch.

Two calls in a row on one context, the second with a smaller swarm (and
below the support-sort threshold, so that it takes the unsorted path), each
compared with scs_evaluate on the same particles: the launch shape and the
arithmetic are the same, so the results are equal bit for bit, and a few
rows of each are held to the oracle at the FP64 and mixed bars.  A request
too large for the scratch is refused before anything is queued.  Collected
last, so a failure here hides no other test.
"""
import numpy as np
import pytest

import oracle as O
from tests import datasets as D
from tests import parity as PT

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2408_13170_amd import B  # noqa: E402


def _ctx(ds, N, G=16):
    g = ds.grid
    h = B.scs_ctx_create(0)
    B.scs_load_data(h, np.ascontiguousarray(ds.d_ri), np.ascontiguousarray(ds.psd), g.k0 * g.df, g.df)
    m = ds.model
    B.scs_set_model(h, m.pn_order, m.response, m.support, m.t_obs)
    B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, G)
    return h


@pytest.mark.parametrize("prec", [B.SCS_PREC_FP64, B.SCS_PREC_MIXED])
def test_noalloc_equals_evaluate_on_two_calls(prec):
    ds = D.lisa_small(seed=41)
    N, G = 16, 16
    tol = PT.TOL64 if prec == B.SCS_PREC_FP64 else PT.TOLMIX
    h = _ctx(ds, N, G)
    try:
        for P, seed, with_seg in ((600, 141, False), (90, 142, True)):
            print(f"noalloc prec {prec} P {P} seg {with_seg}", flush=True)
            theta = D.lisa_particles(P, seed=seed)
            th = torch.tensor(np.ascontiguousarray(theta), device="cuda")
            u_ref = torch.empty(P, dtype=torch.float64, device="cuda")
            u_na = torch.full((P,), -7.0, dtype=torch.float64, device="cuda")
            s_ref = torch.empty((P, N, 3), dtype=torch.float64, device="cuda") if with_seg else None
            s_na = torch.full((P, N, 3), -7.0, dtype=torch.float64, device="cuda") if with_seg else None
            B.scs_evaluate(h, th, u_ref, prec, seg=s_ref)
            torch.cuda.synchronize()
            _, bnd = B.scs_last_bounds(h, P, N)
            B.scs_evaluate_noalloc(h, th, u_na, prec, seg=s_na)
            torch.cuda.synchronize()
            got, ref = u_na.cpu().numpy(), u_ref.cpu().numpy()
            assert np.array_equal(got, ref, equal_nan=True), np.nanmax(np.abs(got - ref))
            if with_seg:
                assert np.array_equal(s_na.cpu().numpy(), s_ref.cpu().numpy(), equal_nan=True)
            _, bnd_na = B.scs_last_bounds(h, P, N)
            assert np.array_equal(bnd_na, bnd)
            rows = np.arange(0, P, max(1, P // 6))
            r = O.evaluate(ds.grid, ds.model, ds.d_ri, ds.psd, theta[rows], N, O.SEG_EQUAL_SNR, G, want_bounds=True)
            PT.check_rows(ds, theta[rows], got[rows], r, bnd[rows], G, tol, what=f"noalloc P={P}")
    finally:
        B.scs_ctx_destroy(h)


def test_noalloc_refuses_what_the_scratch_cannot_hold():
    ds = D.lisa_small(seed=42)
    N = 64
    h = _ctx(ds, N)
    try:
        # 200000 particles: 90 MB of particle records alone
        P = 200000
        th = torch.tensor(np.tile(D.lisa_particles(100, seed=143), (P // 100, 1)), device="cuda")
        u = torch.full((P,), -7.0, dtype=torch.float64, device="cuda")
        with pytest.raises(B.ScsError) as ei:
            B.scs_evaluate_noalloc(h, th, u)
        assert ei.value.code == B.SCS_EINVAL and "scratch" in str(ei.value)
        torch.cuda.synchronize()
        assert bool(torch.all(u == -7.0))
        # host arrays are refused by the binding
        with pytest.raises(ValueError):
            B.scs_evaluate_noalloc(h, np.ascontiguousarray(D.lisa_particles(4, seed=1)), np.zeros(4))
    finally:
        B.scs_ctx_destroy(h)
