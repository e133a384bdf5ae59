"""Pins of the oracle's derived constants against scalars the paper prints
(tests/golden/paper_scalars.json, each with its section)."""
import json
import math
import os

import pytest

from paper_2105_13276_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_scalars.json")))


def _cfg(**over):
    return W.make(64, 32, 32, "uniform", 1, **over)


def test_effective_field(oracle_mod):
    g = GOLD["E_eff_for_Erms_3p5"]
    inp = g["inputs"]
    cfg = _cfg(freq_hz=inp["omega"] / (2 * math.pi), p_torr=inp["nu_m"] / 5.3e9)
    d = oracle_mod.derived(cfg)
    e_eff = inp["E_rms"] * math.sqrt(d["eeff_fac"])
    assert e_eff == pytest.approx(g["value"], rel=g["rtol"])


def test_cutoff_density(oracle_mod):
    g = GOLD["n_cutoff_110GHz_atm"]
    cfg = _cfg(freq_hz=g["inputs"]["freq_hz"], p_torr=g["inputs"]["p_torr"])
    d = oracle_mod.derived(cfg)
    n_cut = d["n_c"] * d["nu_m"] / d["omega"]
    assert n_cut == pytest.approx(g["value"], rel=g["rtol"])
    # the critical density is the one at which omega_pe = omega
    e, m, eps0 = 1.602176634e-19, 9.1093837015e-31, 8.8541878128e-12
    assert math.sqrt(d["n_c"] * e * e / (m * eps0)) == pytest.approx(d["omega"], rel=1e-12)


def test_free_diffusion(oracle_mod):
    g = GOLD["D_e_atm"]
    cfg = _cfg(p_torr=g["inputs"]["p_torr"], te_ev=g["inputs"]["te_ev"])
    assert oracle_mod.derived(cfg)["D_e"] == pytest.approx(g["value"], rel=g["rtol"])


def test_ionisation_calibration(oracle_mod):
    g = GOLD["nu_i_unperturbed"]
    inp = g["inputs"]
    cfg = _cfg(p_torr=inp["p_torr"], freq_hz=inp["freq_hz"])
    nu = oracle_mod.nu_net(cfg, inp["E_rms"] ** 2)
    assert nu == pytest.approx(g["value"], rel=g["rtol"])


def test_breakdown_threshold_is_zero_net_rate(oracle_mod):
    # E_rms = E_bd makes E_eff equal to E_cr: net ionisation vanishes there,
    # is positive above and negative (attachment) below
    for f, p in ((35e9, 100.0), (110e9, 700.0), (170e9, 760.0)):
        cfg = _cfg(freq_hz=f, p_torr=p)
        ebd = oracle_mod.derived(cfg)["E_bd"]
        scale = oracle_mod.derived(cfg)["nu_att"]
        assert abs(oracle_mod.nu_net(cfg, ebd ** 2)) < 1e-9 * scale
        assert oracle_mod.nu_net(cfg, (1.1 * ebd) ** 2) > 0
        assert oracle_mod.nu_net(cfg, (0.9 * ebd) ** 2) < 0


def test_peak_amplitude_convention(oracle_mod):
    g = GOLD["E0_peak_for_Erms_3p5"]
    cfg = _cfg(p_torr=760.0)
    ebd = oracle_mod.derived(cfg)["E_bd"]
    cfg = _cfg(p_torr=760.0, erms_over_ebd=g["inputs"]["E_rms"] / ebd)
    assert oracle_mod.derived(cfg)["E0"] == pytest.approx(g["value"], rel=g["rtol"])


def test_collision_frequency(oracle_mod):
    g = GOLD["nu_m_per_torr"]
    for p in (100.0, 700.0, 760.0):
        assert oracle_mod.derived(_cfg(p_torr=p))["nu_m"] / p == pytest.approx(g["value"], rel=g["rtol"])


def test_effective_diffusion_limits(oracle_mod):
    # free diffusion at the low-density front, ambipolar in the dense bulk
    # (Sec. II.A); the blend between them is a reading (parity unpinned)
    cfg = _cfg()
    d = oracle_mod.derived(cfg)
    assert oracle_mod.d_eff(cfg, 1e6) == pytest.approx(d["D_e"], rel=1e-8)
    assert oracle_mod.d_eff(cfg, 1e30) == pytest.approx(d["D_a"], rel=1e-6)
    mid = oracle_mod.d_eff(cfg, d["n_amb"])
    assert mid == pytest.approx(0.5 * (d["D_e"] + d["D_a"]), rel=1e-12)


def test_steps_per_period(oracle_mod):
    # S = 0.5: 2 N_lambda steps per period on every level
    for npl in (32, 64):
        d = oracle_mod.derived(W.make(64, 32, npl, "uniform", 1))
        assert d["steps_per_period"] == 2 * npl
        assert 2 * math.pi / d["omega"] / d["dt"] == pytest.approx(2 * npl, rel=1e-12)
