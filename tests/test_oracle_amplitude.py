"""Pin of the absolute amplitude from the luminosity distance (Sec 4: D_L
enters as a 1/D_L prefactor; the coherent likelihood of Sec 2.1 needs the
absolute amplitude): the two injections of the paper at their printed
distances, evaluated with the full frequency-domain response (A, E, T) and
the TDI noise PSDs over the whole inspiral in the LISA band, reach the SNRs
the paper prints for them (38 at 50 Mpc, 21.45 at 200 Mpc) to within the
differences of the two models (response conventions, noise model,
eccentricity): 0.8 .. 1.25 of the printed values for both.  A factor of
sqrt 2, 2 or pi^2/3 anywhere in the amplitude moves one of them out."""
import json
import math
import os

import numpy as np

import oracle as O
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


def _snr(inj, dl_mpc, f_lo=0.0125, f_hi=0.5, df=2e-6):
    k0 = int(round(f_lo / df))
    K = int(round((f_hi - f_lo) / df))
    g = O.Grid(K, k0, df, 3)
    # support from f_low up to the band's end (t_obs beyond the merger)
    m = O.Model(pn_order=7, response=O.RESP_LISA_FD, support=O.SUPPORT_TOBS, t_obs=10 * 3.15576e7)
    h = O.template(g, m, inj)
    f = (k0 + np.arange(K)) * df
    S = synth.lisa_tdi_psd(f)[:3]
    return float(O.distance_amplitude(inj[0], dl_mpc)) * math.sqrt(4 * df * np.sum(np.abs(h) ** 2 / S))


def test_snr_of_the_paper_injections_from_their_distances():
    gold = json.load(open(GOLD))
    for key, inj in (("gw150914_like", synth.GW150914_LIKE), ("gw190521_like", synth.GW190521_LIKE)):
        src = gold[key]
        assert abs(inj[0] - src["Mc"]) < 1e-9 and abs(inj[2] - src["f_low"]) < 1e-12
        rho = _snr(inj, src["dl_mpc"])
        print(f"{key}: SNR {rho:.2f} at {src['dl_mpc']} Mpc, paper {src['snr']}")
        assert 0.8 < rho / src["snr"] < 1.25, (key, rho)


def test_amplitude_scales():
    """1/D_L and Mc^5/6 (the amplitude's dependence on the two parameters)."""
    a = O.distance_amplitude(30.0, 100.0)
    assert math.isclose(O.distance_amplitude(30.0, 200.0), a / 2, rel_tol=1e-15)
    assert math.isclose(O.distance_amplitude(60.0, 100.0), a * 2 ** (5 / 6), rel_tol=1e-15)


def test_amplitude_of_invalid_parameters_is_nan():
    a = O.distance_amplitude(np.array([30.0, -1.0, 30.0, np.nan]), np.array([-5.0, 100.0, 0.0, 100.0]))
    assert np.all(np.isnan(a))
