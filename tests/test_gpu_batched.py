"""Batched evaluation of uneven swarms and its HIP-graph replay equal the
solo evaluations."""
import numpy as np
import pytest

import synth
from tests import datasets as D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2408_13170_amd import B  # noqa: E402


def test_batched_and_graph_equal_solo():
    ds = D.lisa_small(seed=9)
    g = ds.grid
    h = B.scs_ctx_create(0)
    try:
        B.scs_load_data(h, np.ascontiguousarray(ds.d_ri), np.ascontiguousarray(ds.psd), g.k0 * g.df, g.df)
        B.scs_set_model(h, 7, 1, 1, ds.model.t_obs)
        B.scs_define_segmentation(h, 1, B.SCS_SEG_EQUAL_SNR, 16)
        shapes = [(256, 700), (64, 300), (16, 129), (1, 64)]
        items, solo = [], []
        for i, (N, P) in enumerate(shapes):
            th = torch.tensor(D.lisa_particles(P, seed=100 + i), device="cuda")
            ups = torch.full((P,), -1.0, dtype=torch.float64, device="cuda")
            items.append((h, N, th, ups))
        for prec in (B.SCS_PREC_FP64, B.SCS_PREC_MIXED):
            B.scs_evaluate_batched(items, prec)
            torch.cuda.synchronize()
            batched = [it[3].cpu().numpy().copy() for it in items]
            for (hh, N, th, _), bv in zip(items, batched):
                B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, 16)
                u = torch.empty(th.shape[0], dtype=torch.float64, device="cuda")
                B.scs_evaluate(h, th, u, prec)
                torch.cuda.synchronize()
                assert np.array_equal(u.cpu().numpy(), bv), (N, prec)
            graph = B.scs_graph_create(items, prec)
            for rep in range(3):
                for it in items:
                    it[3].fill_(-1.0)
                torch.cuda.synchronize()
                B.scs_graph_launch(graph)
                torch.cuda.synchronize()
                for it, bv in zip(items, batched):
                    assert np.array_equal(it[3].cpu().numpy(), bv), rep
            B.scs_graph_destroy(graph)
    finally:
        B.scs_ctx_destroy(h)
