"""Batched evaluation of uneven swarms (one fused persistent launch per
channel count) and its HIP-graph replay equal the solo evaluations bit for
bit, and agree with the oracle."""
import numpy as np
import pytest

import oracle as O
import synth
from tests import datasets as D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2408_13170_amd import B  # noqa: E402


def _ctx(ds, N=1, G=16):
    g = ds.grid
    h = B.scs_ctx_create(0)
    B.scs_load_data(h, np.ascontiguousarray(ds.d_ri), np.ascontiguousarray(ds.psd), g.k0 * g.df, g.df)
    m = ds.model
    B.scs_set_model(h, m.pn_order, m.response, m.support, m.t_obs)
    B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, G)
    return h


def test_batched_and_graph_equal_solo():
    lisa = D.lisa_small(seed=9)
    white = D.white16k()
    hl, hw = _ctx(lisa), _ctx(white, G=1)
    try:
        wth = synth.workload_particles(synth.workload("white16k"))
        # (context, dataset, N, P, theta)
        shapes = [(hl, lisa, 256, 700, D.lisa_particles(700, seed=100)),
                  (hw, white, 16, 64, wth),
                  (hl, lisa, 64, 300, D.lisa_particles(300, seed=101)),
                  (hl, lisa, 16, 129, D.lisa_particles(129, seed=102)),
                  (hw, white, 4, 33, wth[:33]),
                  (hl, lisa, 1, 64, D.lisa_particles(64, seed=103))]
        items = []
        for h, ds, N, P, th in shapes:
            items.append((h, N, torch.tensor(np.ascontiguousarray(th), device="cuda"),
                          torch.full((P,), -1.0, dtype=torch.float64, device="cuda")))
        for prec in (B.SCS_PREC_FP64, B.SCS_PREC_MIXED):
            B.scs_evaluate_batched(items, prec)
            torch.cuda.synchronize()
            batched = [it[3].cpu().numpy().copy() for it in items]
            for (h, ds, N, P, th), bv in zip(shapes, batched):
                B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, 1 if ds is white else 16)
                u = torch.empty(P, dtype=torch.float64, device="cuda")
                B.scs_evaluate(h, torch.tensor(np.ascontiguousarray(th), device="cuda"), u, prec)
                torch.cuda.synchronize()
                assert np.array_equal(u.cpu().numpy(), bv), (N, P, prec)
            if prec == B.SCS_PREC_FP64:
                # oracle spot check on two items of different channel counts
                for k in (0, 1):
                    h, ds, N, P, th = shapes[k]
                    ref = O.evaluate(ds.grid, ds.model, ds.d_ri, ds.psd, th[:6], N, O.SEG_EQUAL_SNR,
                                     1 if ds is white else 16)
                    e = np.abs(batched[k][:6] - ref["ups"]) / np.maximum(np.abs(ref["ups"]), 2.0 * N)
                    print("batched vs oracle, item", k, e.max())
                    assert e.max() < 1e-9
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
        B.scs_ctx_destroy(hl)
        B.scs_ctx_destroy(hw)
