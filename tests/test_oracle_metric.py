"""Pins of the oracle's Kerr-Schild metric (App. A) against what the paper and
the mathematics fix, independent of the oracle's own formulas:

* gamma^ij is the matrix inverse of gamma_ij and sqrt(gamma)^2 = det gamma_ij;
* the 3+1 pieces rebuild the printed 4-metric through eq. metric
  (g_tt = beta_i beta^i - alpha^2, g_ti = beta_i);
* M = a = 0 is flat space in spherical coordinates; a = 0 is Schwarzschild
  in ingoing Kerr-Schild form;
* the analytic derivatives agree with finite differences of the values;
* the four periodic geodesics of Table tab:paths start at radial turning
  points, and the Schwarzschild one has the textbook energy.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc


def _mats(m):
    g = np.array([[m["g_rr"], 0.0, m["g_rph"]], [0.0, m["g_thth"], 0.0], [m["g_rph"], 0.0, m["g_phph"]]])
    h = np.array([[m["h_rr"], 0.0, m["h_rph"]], [0.0, m["h_thth"], 0.0], [m["h_rph"], 0.0, m["h_phph"]]])
    return g, h


def _points(n=200, seed=1):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        M = rng.choice([1.0, 0.5, 2.0])
        a = M * rng.uniform(-0.999, 0.999)
        r = rng.uniform(0.5, 60.0) * M
        th = rng.uniform(0.05, math.pi - 0.05)
        yield a, M, r, th


def test_inverse_and_determinant():
    for a, M, r, th in _points():
        m = orc.metric(a, M, r, th)
        g, h = _mats(m)
        np.testing.assert_allclose(g @ h, np.eye(3), atol=1e-13 * np.abs(g).max() * np.abs(h).max())
        assert m["sqrtg"] ** 2 == pytest.approx(np.linalg.det(g), rel=1e-12)


def test_rebuilds_printed_four_metric():
    """eq. metric with eq. ks-coefficients: g_tt = z - 1, g_tr = z,
    g_tph = -a z sin^2 (M = 1 in the paper; z = 2Mr/rho^2 in general)."""
    for a, M, r, th in _points(seed=2):
        m = orc.metric(a, M, r, th)
        g, _ = _mats(m)
        beta_up = np.array([m["beta"], 0.0, 0.0])
        beta_dn = g @ beta_up
        rho2 = r * r + a * a * math.cos(th) ** 2
        z = 2.0 * M * r / rho2
        assert beta_dn @ beta_up - m["alpha"] ** 2 == pytest.approx(z - 1.0, rel=1e-12, abs=1e-14)
        assert beta_dn[0] == pytest.approx(z, rel=1e-12)
        assert beta_dn[2] == pytest.approx(-a * z * math.sin(th) ** 2, rel=1e-12, abs=1e-15)


def test_flat_and_schwarzschild_limits():
    r, th = 3.7, 0.9
    m = orc.metric(0.0, 0.0, r, th)
    assert (m["alpha"], m["beta"]) == (1.0, 0.0)
    np.testing.assert_allclose([m["g_rr"], m["g_thth"], m["g_phph"], m["g_rph"]],
                               [1.0, r * r, (r * math.sin(th)) ** 2, 0.0], rtol=1e-15)
    np.testing.assert_allclose([m["sqrtg"]], [r * r * math.sin(th)], rtol=1e-15)
    # Schwarzschild, ingoing Kerr-Schild: ds^2 = -(1-2M/r)dt^2 + 4M/r dt dr + (1+2M/r) dr^2 + r^2 dOmega^2
    M = 1.3
    m = orc.metric(0.0, M, r, th)
    assert m["g_rr"] == pytest.approx(1 + 2 * M / r, rel=1e-15)
    assert m["alpha"] == pytest.approx(1 / math.sqrt(1 + 2 * M / r), rel=1e-15)
    assert m["beta"] == pytest.approx((2 * M / r) / (1 + 2 * M / r), rel=1e-15)
    assert m["h_rr"] == pytest.approx(1 / (1 + 2 * M / r), rel=1e-14)


@pytest.mark.parametrize("key", orc.METRIC_DKEYS)
def test_derivatives_match_finite_differences(key):
    for a, M, r, th in _points(n=60, seed=3):
        hr, ht = 1e-3 * r, 1e-3 * min(th, math.pi - th)
        # 4th-order central differences
        def fd(f, x, h):
            return (-f(x + 2 * h) + 8 * f(x + h) - 8 * f(x - h) + f(x - 2 * h)) / (12 * h)
        d_r = fd(lambda x: orc.metric(a, M, x, th)[key], r, hr)
        d_t = fd(lambda x: orc.metric(a, M, r, x)[key], th, ht)
        m = orc.metric(a, M, r, th)
        scale_r = abs(m[key]) / r + 1e-12
        scale_t = abs(m[key]) + 1e-12
        assert m["dr_" + key] == pytest.approx(d_r, abs=1e-7 * scale_r, rel=1e-7)
        assert m["dth_" + key] == pytest.approx(d_t, abs=1e-7 * scale_t, rel=1e-7)


class _G:
    """Grid used only to map (r, theta) to the oracle's grid units."""
    a = 0.0
    M = 1.0
    nr = nth = 512
    guard = 2
    pitch = 517
    lnr0 = 0.0
    dlnr = 0.01
    dth = math.pi / 512


def _grid_for(a):
    g = _G()
    g.a = a
    return g


@pytest.mark.parametrize("name", ["(2,0,1)", "(3,3,1)", "(3,3,2)", "(4,3,1)"])
def test_table_geodesics_start_at_turning_points(tab_paths, name):
    row = tab_paths[name]
    g = _grid_for(row["a"])
    xi = (math.log(row["r"]) - g.lnr0) / g.dlnr
    eta = row["theta"] / g.dth
    f = orc.rhs(g, [xi, eta, 0.0, *row["u"]])
    dr_dt = f[0] * row["r"] * g.dlnr
    # the table prints 6-7 significant digits; a turning point gives |dr/dt| ~ 1e-7
    assert abs(dr_dt) < 1e-6, dr_dt
    assert abs(f[1]) < 1e-9          # equatorial, u_th = 0


def test_schwarzschild_orbit_energy(tab_paths):
    """(2,0,1) at a = 0: E = -u_0 = alpha sqrt(1 + u^2) - beta^r u_r equals the
    apastron value sqrt((1 - 2/r)(1 + L^2/r^2)) of a Schwarzschild orbit."""
    row = tab_paths["(2,0,1)"]
    r, (ur, uth, uph) = row["r"], row["u"]
    m = orc.metric(0.0, 1.0, r, row["theta"])
    uu = m["h_rr"] * ur * ur + 2 * m["h_rph"] * ur * uph + m["h_thth"] * uth ** 2 + m["h_phph"] * uph ** 2
    E = m["alpha"] * math.sqrt(1 + uu) - m["beta"] * ur
    E_closed = math.sqrt((1 - 2 / r) * (1 + uph ** 2 / r ** 2))
    assert E == pytest.approx(E_closed, abs=2e-6)
