"""What the paper's sparse-grid evaluation (Sec 4: waveform and response on a
grid coarser than the FFT grid by 1000, cubic-spline interpolated onto it)
would cost in accuracy, measured with the oracle on the 2^20-bin workload:
the interpolated phase against the exact one at every in-support bin, and
the overlap lost at the injection.  The library evaluates the phase per
block with a remainder bound of 1e-12 cycles instead (no interpolation)."""
import math

import numpy as np
import pytest

import oracle as O
import synth

interpolate = pytest.importorskip("scipy.interpolate")


def test_cubic_spline_on_a_grid_coarser_by_1000():
    w = synth.workload("lisa1m")
    g = w.grid
    m = O.Model(pn_order=7, response=O.RESP_LISA_LF_AE, support=O.SUPPORT_TOBS, t_obs=g.t_obs)
    f = (g.k0 + np.arange(g.K)) * g.df
    frac, whole, t, _ = O.phase(m, w.injection, f)
    k = np.flatnonzero((f >= w.injection[2]) & (t < g.t_obs))
    # the phase relative to its value at the first support bin, so that the
    # differences keep their precision in double
    ph = (whole[k] - whole[k[0]]) + (frac[k] - frac[k[0]])
    nodes = np.append(np.arange(0, k.size, 1000), k.size - 1)
    sp = interpolate.CubicSpline(f[k][nodes], ph[nodes])
    err = sp(f[k]) - ph
    emax = np.abs(err).max()
    print(f"{k.size} bins, {nodes.size} nodes: spline phase error max {emax:.3g} cycles, "
          f"median {np.median(np.abs(err)):.3g}")
    # about 1e-6 cycles: far above the 1e-12-cycle bound of the block polynomials ...
    assert 1e-8 < emax < 1e-4
    # ... yet second order in Upsilon: the overlap of e^{2 pi i err} with 1
    loss = 1.0 - abs(np.mean(np.exp(2j * math.pi * err)))
    print(f"overlap lost at the injection: {loss:.3g}")
    assert loss < 1e-9
