"""Pins of oracle parts against published closed forms and stated values.

The synthetic family's phase is pinned through the stationary-phase relation
dPsi/df = 2 pi t(f) against the published time-to-coalescence series of a
quasi-circular inspiral (non-spinning terms through 3.5PN: Blanchet, Living
Rev. Relativ. 17, 2 (2014), the series t(x); spin-orbit at 1.5PN and
spin-spin at 2PN: Cutler & Flanagan, PRD 49, 2658 (1994), Eq. 3.2, with the
spin-spin sigma of Kidder, PRD 52, 821 (1995) and the black-hole
quadrupole-monopole term of Poisson, PRD 57, 5287 (1998)).  The mode
amplitudes and the analytic PSD are pinned against hand evaluations of the
workload definitions (tests/golden/).
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import physics as ph

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EULER_GAMMA = 0.57721566490153286061


def _ratio_to_newtonian_time(m1, m2, c1, c2, v):
    """(dPsi/df / 2 pi) / t_N with t_N = -5 M / (256 eta v^8), by the complex
    step through the oracle's phase: the factor multiplying the Newtonian time
    to coalescence."""
    m_s, eta, _ = ph.mass_params(m1, m2)
    f = v ** 3 / (math.pi * m_s)
    h = 1e-20 * f
    dpsi = np.imag(ph.pn_phase_22(f + 1j * h, m1, m2, c1, c2)) / h
    return (dpsi / (2.0 * math.pi)) / (-5.0 * m_s / (256.0 * eta * v ** 8))


def _published_time_series_nonspinning(eta, v):
    """1 + sum_k tau_k v^k of the time to coalescence, t = t_c - 5M/(256 eta v^8) (...),
    written as published in terms of x = v^2 (Blanchet 2014, the series t(x))."""
    pi = math.pi
    x = v ** 2
    t2 = 743.0 / 252.0 + 11.0 / 3.0 * eta
    t3 = -32.0 / 5.0 * pi
    t4 = 3058673.0 / 508032.0 + 5429.0 / 504.0 * eta + 617.0 / 72.0 * eta ** 2
    t5 = (-7729.0 / 252.0 + 13.0 / 3.0 * eta) * pi
    t6 = (-10052469856691.0 / 23471078400.0 + 128.0 / 3.0 * pi ** 2 + 6848.0 / 105.0 * EULER_GAMMA
          + (3147553127.0 / 3048192.0 - 451.0 / 12.0 * pi ** 2) * eta
          - 15211.0 / 1728.0 * eta ** 2 + 25565.0 / 1296.0 * eta ** 3
          + 3424.0 / 105.0 * np.log(16.0 * x))
    t7 = (-15419335.0 / 127008.0 - 75703.0 / 756.0 * eta + 14809.0 / 378.0 * eta ** 2) * pi
    return 1.0 + t2 * x + t3 * x ** 1.5 + t4 * x ** 2 + t5 * x ** 2.5 + t6 * x ** 3 + t7 * x ** 3.5


@pytest.mark.parametrize("m1,m2", [(5.0, 5.0), (8.0, 1.4), (30.0, 3.0)])
def test_phase_nonspinning_equals_published_time_series_through_3p5pn(m1, m2):
    """Without spins the phase's derivative must reproduce the published time
    series term for term, 2.5PN, 3PN (with its log) and 3.5PN included.  A 1%
    slip in any coefficient of the phase moves the ratio by >= 1e-6 somewhere
    on v in [0.05, 0.3]; rounding leaves ~1e-13."""
    _, eta, _ = ph.mass_params(m1, m2)
    v = np.linspace(0.05, 0.3, 200)
    got = _ratio_to_newtonian_time(m1, m2, 0.0, 0.0, v)
    want = _published_time_series_nonspinning(eta, v)
    assert np.max(np.abs(got - want)) < 1e-10


def _fit_time_series(m1, m2, c1, c2):
    """Least-squares coefficients of the ratio on 1, v^2 .. v^7 and v^6 log v
    (the complete set of powers the phase produces)."""
    v = np.linspace(0.02, 0.3, 160)
    r = _ratio_to_newtonian_time(m1, m2, c1, c2, v)
    basis = np.stack([np.ones_like(v), v ** 2, v ** 3, v ** 4, v ** 5, v ** 6, v ** 6 * np.log(v), v ** 7], axis=1)
    coef, *_ = np.linalg.lstsq(basis, r, rcond=None)
    return coef


@pytest.mark.parametrize("m1,m2,c1,c2", [(8.0, 1.4, 0.9, -0.8), (5.0, 5.0, 0.6, 0.6), (15.0, 3.0, -0.7, 0.4),
                                          (20.0, 1.0, 0.3, 0.0)])
def test_phase_spin_orbit_and_spin_spin_equal_published_coefficients(m1, m2, c1, c2):
    """With aligned spins the time series' 1.5PN coefficient is
    -(8/5)(4 pi - beta) with the spin-orbit beta = (1/12) sum_i chi_i
    (113 m_i^2/M^2 + 75 eta), and the 2PN coefficient is the non-spinning one
    minus 2 sigma with, for aligned black-hole spins (quadrupole-monopole
    constant 1), sigma = eta (721/48 - 247/48) chi1 chi2 + sum_i (m_i/M)^2
    [(720 - 1)/96 - (240 - 7)/96] chi_i^2.  Written per component here; the
    oracle writes the same terms in chi_s, chi_a, delta."""
    M = m1 + m2
    _, eta, _ = ph.mass_params(m1, m2)
    chi = (c1, c2)
    mm = (m1 / M, m2 / M)
    beta = sum(chi[i] * (113.0 * mm[i] ** 2 + 75.0 * eta) for i in range(2)) / 12.0
    sigma = eta * (721.0 / 48.0 - 247.0 / 48.0) * c1 * c2
    sigma += sum(mm[i] ** 2 * ((720.0 - 1.0) / 96.0 - (240.0 - 7.0) / 96.0) * chi[i] ** 2 for i in range(2))
    tau3 = -8.0 / 5.0 * (4.0 * math.pi - beta)
    tau4 = 3058673.0 / 508032.0 + 5429.0 / 504.0 * eta + 617.0 / 72.0 * eta ** 2 - 2.0 * sigma
    coef = _fit_time_series(m1, m2, c1, c2)
    assert coef[0] == pytest.approx(1.0, abs=1e-9)
    assert coef[1] == pytest.approx(743.0 / 252.0 + 11.0 / 3.0 * eta, rel=1e-8)
    # the fit recovers these to ~1e-9; a 1% slip in a spin term moves them by >= 1e-3
    assert coef[2] == pytest.approx(tau3, rel=1e-7, abs=1e-7)
    assert coef[3] == pytest.approx(tau4, rel=1e-7, abs=1e-7)


def test_spin_spin_changes_the_2pn_term_as_published():
    """The fitted 2PN coefficient moves with the spins by exactly -2 sigma
    (difference of a spinning and a non-spinning fit at equal masses, spins
    equal and opposite so that the 1.5PN spin-orbit term cancels)."""
    m1 = m2 = 6.0
    eta = 0.25
    c = 0.7
    a = _fit_time_series(m1, m2, c, -c)
    b = _fit_time_series(m1, m2, 0.0, 0.0)
    sigma = eta * (474.0 / 48.0) * (c * -c) + 2 * 0.25 * (486.0 / 96.0) * c ** 2
    assert a[2] == pytest.approx(b[2], abs=1e-8)            # beta = 0 for these spins
    assert a[3] - b[3] == pytest.approx(-2.0 * sigma, rel=1e-7)


# ---------------------------------------------------------------- chirp-time coordinates

@pytest.mark.parametrize("phys", [(8.0, 1.4, 0.3, 0.0), (5.31, 1.22, -0.69, -0.02), (15.0, 3.0, 0.5, 0.05),
                                  (10.0, 10.0, 0.4, -0.2)])
def test_theta3s_bar_uses_the_mass_weighted_effective_spin(phys):
    """Eq. metric_coords: theta3s_bar is theta3s with chi_r replaced by
    chi_eff = (m1 chi1 + m2 chi2) / M, both with the factor 113 / (192 eta).
    So theta3s_bar / theta3 = 113 chi_eff / (48 pi), and, because chi_r =
    chi_eff - 76 eta chi_s / 113, theta3s - theta3s_bar = -(19/48) chi_s
    (pi M f0)^(-2/3), independent of the mass ratio.  Checked with chi_eff
    and chi_s formed here from the components, not through the inverse map."""
    m1, m2, c1, c2 = phys
    f0 = 20.0
    th = ph.phys_to_theta(phys, f0)
    M = m1 + m2
    chi_eff = (m1 * c1 + m2 * c2) / M
    chi_s = 0.5 * (c1 + c2)
    u = math.pi * M * ph.MSUN_S * f0
    assert th[3] / th[1] == pytest.approx(113.0 * chi_eff / (48.0 * math.pi), rel=1e-13, abs=1e-15)
    assert th[2] - th[3] == pytest.approx(-19.0 / 48.0 * chi_s * u ** (-2.0 / 3.0), rel=1e-12, abs=1e-12)


def test_theta3s_bar_equal_spins_and_single_spin():
    """Equal component spins chi give chi_eff = chi at any masses; a spin on
    the heavier body alone gives chi_eff = m1 chi1 / M."""
    f0 = 15.0
    for m1, m2 in ((8.0, 1.4), (20.0, 2.0)):
        th = ph.phys_to_theta((m1, m2, 0.55, 0.55), f0)
        assert th[3] / th[1] == pytest.approx(113.0 * 0.55 / (48.0 * math.pi), rel=1e-13)
        th = ph.phys_to_theta((m1, m2, 0.8, 0.0), f0)
        assert th[3] / th[1] == pytest.approx(113.0 * (m1 * 0.8 / (m1 + m2)) / (48.0 * math.pi), rel=1e-13)


# ---------------------------------------------------------------- mode amplitudes

def test_mode_amplitudes_equal_hand_evaluated_values():
    """Each mode's amplitude, read off the waveform as |h_{l,-m}(f)| /
    (Amp f^-7/6) on its band, equals the hand-evaluated fraction of the
    workload's stated formula at the same masses (equal masses switch the
    odd-m modes off)."""
    with open(os.path.join(GOLDEN, "mode_amplitudes.json")) as fh:
        gold = json.load(fh)
    grid = ph.Grid(4096.0, 4.0, 20.0)
    for case in gold["cases"]:
        m1, m2 = case["m1"], case["m2"]
        _, eta, delta = ph.mass_params(m1, m2)
        assert delta == pytest.approx(float(Fraction(case["delta"])), rel=1e-14, abs=1e-15)
        assert eta == pytest.approx(float(Fraction(case["eta"])), rel=1e-14)
        amp0 = ph.newtonian_amplitude(m1, m2, 100.0)
        for key, frac in case["A"].items():
            l, m = (int(t) for t in key.split(","))
            want = float(Fraction(frac))
            assert ph.mode_amplitude(l, m, eta, delta) == pytest.approx(want, rel=1e-13, abs=1e-16)
            h = ph.waveform_mode(grid, l, m, (m1, m2, 0.2, -0.1), 100.0)
            j = np.nonzero(h)[0]
            if want == 0.0:
                assert j.size == 0 or np.max(np.abs(h)) == 0.0
                continue
            f = grid.freqs[j]
            got = np.abs(h[j]) * f ** (7.0 / 6.0) / amp0
            assert np.allclose(got, want, rtol=1e-12, atol=0)


# ---------------------------------------------------------------- PSD

def test_psd_at_hand_evaluated_points():
    """The analytic PSD at x = f / 215 Hz = 1, 2, sqrt 2 and 1/2 equals the
    hand evaluation of the stated formula (x = 1 gives exactly 33e-49), and
    the third-generation scale multiplies it by 0.1."""
    with open(os.path.join(GOLDEN, "psd_points.json")) as fh:
        gold = json.load(fh)
    xs = {"1": 1.0, "2": 2.0, "sqrt2": math.sqrt(2.0), "1/2": 0.5}
    for p in gold["points"]:
        x = xs[p["x"]]
        want = float(Fraction(p["rational"])) + (2.0 ** p["pow2"] if p["pow2"] is not None else 0.0)
        want *= 1e-49
        # abs=0: the values are ~1e-47, far below pytest.approx's default absolute tolerance
        assert ph.psd_analytic(np.array([215.0 * x]))[0] == pytest.approx(want, rel=1e-13, abs=0)
        assert ph.psd_analytic(np.array([215.0 * x]), 0.1)[0] == pytest.approx(0.1 * want, rel=1e-13, abs=0)
    # DC never contributes
    grid = ph.Grid(2048.0, 4.0, 20.0)
    assert np.isinf(ph.psd_on_grid(grid)[0])
