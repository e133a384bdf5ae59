"""Front speed of the continuity step (Eq. (4)): with a fixed field the
density spreads as a pulled front whose speed is 2 sqrt(D nu) in the
continuum (the Fisher-KPP speed the paper uses to read its front
velocities, Sec. IV.D).  For the discrete scheme (forward Euler, 3-point
flux) the asymptotic speed of a level set is exactly
    v* = min_mu ln(1 + nu dt + 4 (D dt/dx^2) sinh^2(mu/2)) / mu   [cells/step],
the slowest exponential profile exp(-mu x/dx) that the scheme carries.  The
oracle's level set must move at v* (up to the known ln t transient) and v*
must sit within the discretisation error of 2 sqrt(D nu)."""
import numpy as np
from scipy.optimize import minimize_scalar

from paper_2105_13276_amd import workloads as W


def _level_set(n, level):
    """x (in cells) where log n crosses log level, right of the maximum."""
    ln = np.log(np.maximum(n, 1e-300))
    i = int(np.argmax(ln))
    t = np.log(level)
    k = i + int(np.argmax(ln[i:] < t))
    a, b = ln[k - 1], ln[k]
    return k - 1 + (a - t) / (a - b)


def test_pulled_front_speed(oracle_mod):
    cfg = W.make(64, 32, 64, "uniform", 1, d_mode="const")
    nx, ny = 1400, 2
    dx = 299792458.0 / cfg["freq_hz"] / 64
    erms2 = 1.6 * (oracle_mod.derived(cfg)["E_bd"]) ** 2
    nu = oracle_mod.nu_net(cfg, erms2)
    assert nu > 0
    a, b = 0.02, 0.1                      # nu dt and D dt / dx^2
    dtn = a / nu
    cfg["d_const"] = b * dx * dx / dtn
    D = cfg["d_const"]
    assert abs(oracle_mod.d_eff(cfg, 1.0) - D) < 1e-12 * D
    n = np.zeros((ny + 1, nx + 1))
    n[:, 60] = 1.0                        # a line source, uniform in y
    e = np.full_like(n, erms2)
    pos = {}
    for step in range(1, 6001):
        n = oracle_mod.continuity_apply(cfg, n, e, dx, dtn)
        if step in (3000, 4500, 6000):
            pos[step] = _level_set(n[1], 1.0)
    assert np.allclose(n[0], n[2]) and np.allclose(n[0], n[1])   # stays 1-D
    v_meas = (pos[6000] - pos[3000]) / 3000.0
    v_late = (pos[6000] - pos[4500]) / 1500.0
    res = minimize_scalar(lambda mu: np.log1p(a + 4 * b * np.sinh(mu / 2) ** 2) / mu,
                          bounds=(1e-3, 5.0), method="bounded")
    v_star, mu_star = res.fun, res.x
    # ln t transient of a level set: dx/dt ~ v* - 1/(2 mu* t)
    corr = np.log(6000 / 3000) / (2 * mu_star) / 3000.0
    print("front: measured %.6f (late %.6f), discrete v* %.6f, ln-t corrected %.6f, "
          "continuum %.6f cells/step" % (v_meas, v_late, v_star, v_star - corr,
                                         2 * np.sqrt(a * b)))
    assert abs(v_meas - (v_star - corr)) < 2e-3 * v_star
    assert abs(v_late - v_star) < abs(v_meas - v_star) + 1e-4   # approaches v*
    # the scheme's speed against the continuum Fisher-KPP speed 2 sqrt(D nu)
    v_cont = 2 * np.sqrt(D * nu) * dtn / dx
    assert abs(v_star / v_cont - 1) < 0.03
