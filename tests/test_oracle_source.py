"""The full source of Eq. (4) in the FP64 oracle: Townsend ionisation
gamma v_d with a separate attachment rate, and electron-ion recombination
-r_ei n^2.  Pins that do not restate the oracle's formulas:

* Stoletov's point: with gamma = A p exp(-B p/E) and v_d = mu_e E, the
  ionisation per unit field squared, nu_i/(mu_e E^2) = gamma/E, peaks at
  E/p = B with the value A/(B e) (e = Euler's number), for any A, B, p;
* the zero-field limit is the attachment rate alone;
* the recombination coefficient of Sec. II.A evaluated by hand at
  T_e = 2 eV;
* pure recombination dn/dt = -r n^2 has the exact solution
  n0/(1 + r n0 t): forward Euler reaches it with first-order error;
* with a constant net rate nu > 0 the update's fixed point is nu / r."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_13276_amd import workloads as W

QE, ME = 1.602176634e-19, 9.1093837015e-31


def _cfg(**over):
    return W.make(16, 8, 32, "uniform", 1, **over)


@pytest.mark.parametrize("A,B,p", [(15.0, 365.0, 700.0), (8.0, 210.0, 100.0)])
def test_townsend_stoletov_point(A, B, p):
    cfg = _cfg(source_model="townsend", A_town=A, B_town=B, nu_att=0.0, p_torr=p)
    omega = 2 * math.pi * cfg["freq_hz"]
    nu_m = 5.3e9 * p                      # Sec. II.A
    mu_e = QE / (ME * nu_m)
    fac = 1.0 + omega ** 2 / nu_m ** 2    # E_rms^2 = E_eff^2 (1 + w^2/nu_m^2)

    def per_field2(e_eff):
        return O.nu_net(cfg, e_eff ** 2 * fac) / (mu_e * e_eff ** 2)

    e_star = 100.0 * B * p                # E/p = B in V/(cm Torr), as V/m
    peak = A / (B * math.e)               # per volt (cm Torr cancels)
    assert per_field2(e_star) == pytest.approx(peak, rel=1e-12)
    for f in (0.9, 0.99, 1.01, 1.1, 2.0, 0.5):
        assert per_field2(f * e_star) < per_field2(e_star)


def test_zero_field_is_attachment():
    cfg = _cfg(source_model="townsend", nu_att=4.2e7)
    assert O.nu_net(cfg, 0.0) == -4.2e7


def test_recombination_coefficient():
    # T_e = 2 eV = 2 * 11604.518 K = 23209.04 K; sqrt(300 / 23209.04) = 0.113693
    cfg = _cfg(beta_rec=1.0, te_ev=2.0)
    assert O.r_ei(cfg) == pytest.approx(1.13693e-14, rel=2e-5)
    assert O.r_ei(_cfg(beta_rec=0.0)) == 0.0


def _uniform_run(cfg, n0, e2, t_end, k):
    n = np.full((5, 5), n0)
    erms2 = np.full((5, 5), e2)
    dtn = t_end / k
    for _ in range(k):
        n = O.continuity_apply(cfg, n, erms2, 1e-3, dtn)
    return n[2, 2]


def test_recombination_decay_first_order():
    cfg = _cfg(beta_rec=2.0, A_ion=0.0, d_mode="const", d_const=0.0)
    r = O.r_ei(cfg)
    n0, T = 1e21, 2e-7                    # r n0 T ~ 4.5: far into the decay
    exact = n0 / (1.0 + r * n0 * T)
    err = [abs(_uniform_run(cfg, n0, 0.0, T, k) - exact) / exact for k in (200, 400, 800)]
    assert err[2] < 5e-3
    assert 1.8 < err[0] / err[1] < 2.2 and 1.8 < err[1] / err[2] < 2.2


def test_logistic_fixed_point():
    cfg = _cfg(beta_rec=2.0, d_mode="const", d_const=0.0)
    e2 = (4.0e6) ** 2
    nu = O.nu_net(cfg, e2)
    assert nu > 0
    r = O.r_ei(cfg)
    n = _uniform_run(cfg, 1e15, e2, 400.0 / nu, 4000)
    assert n == pytest.approx(nu / r, rel=1e-9)
