"""The block-length search of the prologue takes its remainder bounds as
falling with frequency over a support: both grow with the time left to
coalescence at the block start, t_c - t(f), so they fall wherever the
stationary-phase time t(f) rises with f (the source chirps up).  The search
then finds, by bisection, the first bin from which a longer block meets the
bounds.  This checks that premise on the oracle's own SPA time (Sec 4,
waveform paragraph) for the prior boxes of tab:GW150914-like_injection and
tab:GW190521-like_injection, circular and eccentric over the e0 prior
[0.005, 0.1], across the whole band the grids cover: t(f) rises strictly and
stays before coalescence."""
import numpy as np

import oracle as O
import synth


def _times(model, theta, f):
    _, _, t, tc = O.phase(model, theta, f)
    return t, tc


def test_spa_time_rises_across_the_band():
    f = np.geomspace(0.014, 0.032, 4001)  # every support of the boxes lies inside
    boxes = [(synth.GW150914_PRIOR_LO, synth.GW150914_PRIOR_HI), (synth.GW190521_PRIOR_LO, synth.GW190521_PRIOR_HI)]
    checked = 0
    for bi, (lo, hi) in enumerate(boxes):
        th = synth.particles(lo, hi, 64, seed=2408 + bi)
        for ecc in (0, 1):
            m = O.Model(pn_order=7, response=O.RESP_LISA_LF_AE, support=O.SUPPORT_TOBS, t_obs=6.5536e7,
                        eccentric=ecc)
            rng = np.random.default_rng(13170 + bi)
            for row in th:
                theta = np.concatenate([row, [rng.uniform(0.005, 0.1)]]) if ecc else row
                fs = f[f >= row[2]]
                t, tc = _times(m, theta, fs)
                assert np.all(np.isfinite(t))
                assert np.all(np.diff(t) > 0.0), "SPA time not rising with f"
                assert np.all(t < tc), "band reaches coalescence"
                checked += 1
    assert checked == 256
