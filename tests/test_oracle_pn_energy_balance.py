"""Pin of the oracle's post-Newtonian phase coefficients (TaylorF2, the e0 -> 0
limit of the paper's waveform, Sec 4) by a route that never writes them down.

The stationary-phase time follows from energy balance: dt/dv = -E'(v)/F(v)
with the PN binding energy E(v) to 3PN and the gravitational-wave flux F(v)
to 3.5PN (including its 3PN logarithm), as given in Blanchet's review of PN
theory (Living Rev. Relativ. 17, 2, 2014).  The test divides the two series
(to relative order v^7), integrates term by term in 40-digit arithmetic and
compares the result with the oracle's t(f) - t_c.  TaylorF2 is exactly that
re-expanded ratio integrated, so the two agree to rounding; a wrong
coefficient, sign, eta power or log term anywhere in psi_2..psi_7 (the
2.5PN and 3PN logarithms and the Euler-gamma term included) moves t by far
more than the tolerance.  The v-independent part of psi_5 is a constant
phase and does not enter t; the test of the SPA time against the phase
derivative (test_oracle_pins) ties t back to the phase.
"""
import math

import numpy as np
import pytest

import oracle as O

mp = pytest.importorskip("mpmath")

TSUN = 1.32712440018e20 / 299792458.0 ** 3  # G M_sun / c^3 [s], IAU nominal solar mass parameter


def _t_minus_tc(eta, v, order=7):
    """t(v) - t_c in units of the total mass from -E'/F, with no integration
    constant (the oracle's t_c is defined the same way: the series in v has
    no v^0 term)."""
    with mp.workdps(40):
        e, pi, gam = mp.mpf(eta), mp.pi, mp.euler
        # E(v) = -(eta M v^2 / 2) (1 + e2 v^2 + e4 v^4 + e6 v^6)
        e2 = -mp.mpf(3) / 4 - e / 12
        e4 = -mp.mpf(27) / 8 + mp.mpf(19) / 8 * e - e ** 2 / 24
        e6 = (-mp.mpf(675) / 64 + (mp.mpf(34445) / 576 - mp.mpf(205) / 96 * pi ** 2) * e
              - mp.mpf(155) / 96 * e ** 2 - mp.mpf(35) / 5184 * e ** 3)
        # F(v) = (32/5) eta^2 v^10 (1 + sum_k fk v^k), f6 + f6_log ln v at 3PN
        fk = [mp.mpf(1), 0, -mp.mpf(1247) / 336 - mp.mpf(35) / 12 * e, 4 * pi,
              -mp.mpf(44711) / 9072 + mp.mpf(9271) / 504 * e + mp.mpf(65) / 18 * e ** 2,
              -(mp.mpf(8191) / 672 + mp.mpf(583) / 24 * e) * pi,
              (mp.mpf(6643739519) / 69854400 + mp.mpf(16) / 3 * pi ** 2 - mp.mpf(1712) / 105 * gam
               - mp.mpf(856) / 105 * mp.log(16)
               + (-mp.mpf(134543) / 7776 + mp.mpf(41) / 48 * pi ** 2) * e
               - mp.mpf(94403) / 3024 * e ** 2 - mp.mpf(775) / 324 * e ** 3),
              (-mp.mpf(16285) / 504 + mp.mpf(214745) / 1728 * e + mp.mpf(193385) / 3024 * e ** 2) * pi]
        f6_log = -mp.mpf(1712) / 105  # -(856/105) ln(16 v^2) = -(856/105) ln 16 - (1712/105) ln v
        # -E'(v) = eta M v (1 + 2 e2 v^2 + 3 e4 v^4 + 4 e6 v^6)
        num = [mp.mpf(1), 0, 2 * e2, 0, 3 * e4, 0, 4 * e6, 0]
        # q = num / (1 + sum fk v^k) to order v^7; the log enters at v^6 only
        q = []
        for k in range(8):
            q.append(num[k] - sum(fk[i] * q[k - i] for i in range(1, k + 1)))
        q6_log = -f6_log
        v = mp.mpf(v)
        # dt/dv = (5 M / (32 eta)) v^-9 (sum q_k v^k + q6_log v^6 ln v)
        s = sum(q[k] * v ** (k - 8) / (k - 8) for k in range(order + 1))
        if order >= 6:
            s += q6_log * (-mp.log(v) / (2 * v ** 2) - 1 / (4 * v ** 2))
        return float(5 / (32 * e) * s)


@pytest.mark.parametrize("eta", [0.25, 0.2, 0.1, 0.03])
def test_spa_time_from_energy_balance(eta):
    model = O.Model(pn_order=7, response=O.RESP_LISA_LF_AE, support=1, t_obs=6e7)
    Mc = 28.0
    M = Mc * eta ** -0.6 * TSUN
    # f_low near the top of the range keeps t_c small, so t - t_c keeps its digits
    th = np.array([Mc, eta, 30.0, 1.0, 0.3, 0.5, 0.2])
    v = np.linspace(0.05, 0.3, 11)
    f = v ** 3 / (math.pi * M)
    _, _, t, tc = O.phase(model, th, f)
    want = np.array([_t_minus_tc(eta, (math.pi * M * fi) ** (1.0 / 3.0)) * M for fi in f])
    rel = np.abs((t - tc) / want - 1)
    assert rel.max() < 1e-12, rel
    # the test resolves the highest order: dropping the 3.5PN term of the
    # series moves t at the top of the range by far more than the tolerance
    top = (math.pi * M * f[-1]) ** (1.0 / 3.0)
    assert abs(_t_minus_tc(eta, top, order=6) / _t_minus_tc(eta, top) - 1) > 1e-5
