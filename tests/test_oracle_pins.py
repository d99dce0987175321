"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks one oracle part against something other than the oracle's
own formula: closed forms, invariants, brute force on small inputs, or
special cases that reduce to a textbook or library routine.
"""
import math

import numpy as np
import pytest
import scipy.fft

from oracle import likelihood as lk
from oracle import physics as ph
from oracle import startup as su
from paper_2508_04172_amd import workloads as wl

TINY = wl.CFG1.with_(name="tiny", seg_len=4.0, fs=1024.0, n_nodes=40, q=12, n_queries=200)
TINY_MULTI = wl.SMALL_MULTI.with_(name="tiny_multi", seg_len=4.0, fs=1024.0, n_nodes=60, q=10,
                                  n_queries=200)


@pytest.fixture(scope="module")
def tiny_art():
    return su.startup(TINY, wl.white_noise(TINY), workers=1)


@pytest.fixture(scope="module")
def multi_art():
    return su.startup(TINY_MULTI, wl.white_noise(TINY_MULTI), workers=1)


# ---------------------------------------------------------------- Halton

def test_halton_radical_inverse_known_values():
    # textbook van der Corput sequences
    assert [su.radical_inverse(i, 2) for i in range(1, 8)] == [0.5, 0.25, 0.75, 0.125, 0.625, 0.375, 0.875]
    got3 = [su.radical_inverse(i, 3) for i in range(1, 9)]
    want3 = [1 / 3, 2 / 3, 1 / 9, 4 / 9, 7 / 9, 2 / 9, 5 / 9, 8 / 9]
    assert np.allclose(got3, want3, rtol=0, atol=1e-16)
    assert su.radical_inverse(1, 7) == 1 / 7
    assert np.allclose(su.halton(1), [0.5, 1 / 3, 0.2, 1 / 7], atol=1e-16)


# ---------------------------------------------------------------- coordinates

@pytest.mark.parametrize("phys", [(8.0, 1.4, 0.3, 0.0), (5.31, 1.22, -0.69, -0.02), (15.0, 3.0, 0.5, 0.05),
                                  (20.0, 1.0, 0.95, -0.9)])
def test_theta_round_trip(phys):
    th = ph.phys_to_theta(phys, 20.0)
    m1, m2, c1, c2, eta = ph.theta_to_phys(th, 20.0)
    assert np.allclose([m1, m2, c1, c2], phys, rtol=1e-11, atol=1e-11)
    assert eta <= 0.25


def test_theta_ratio_gives_total_mass():
    # theta0 / theta3 = 5 / (32 pi (pi M f0)) independent of eta (Eq. metric_coords)
    th = ph.phys_to_theta((10.0, 2.0, 0.1, 0.0), 15.0)
    m_s = (12.0) * ph.MSUN_S
    assert th[0] / th[1] == pytest.approx(5.0 / (32.0 * math.pi * math.pi * m_s * 15.0), rel=1e-13)


# ---------------------------------------------------------------- waveform phase

def test_phase_newtonian_chirp_time():
    """Stationary phase: dPsi/df = 2 pi t(f), and at low frequency the time to
    coalescence tends to the quadrupole chirp time (5/256) Mc^(-5/3) (pi f)^(-8/3)."""
    m1, m2 = 8.0, 1.4
    mc = (m1 * m2) ** 0.6 / (m1 + m2) ** 0.2 * ph.MSUN_S
    for f in (1e-4, 1e-3):
        h = f * 1e-6
        dpsi = (ph.pn_phase_22(f + h, m1, m2, 0.0, 0.0) - ph.pn_phase_22(f - h, m1, m2, 0.0, 0.0)) / (2 * h)
        t = dpsi / (2 * math.pi)
        tau0 = 5.0 / 256.0 * mc ** (-5.0 / 3.0) * (math.pi * f) ** (-8.0 / 3.0)
        v2 = (math.pi * (m1 + m2) * ph.MSUN_S * f) ** (2.0 / 3.0)
        assert t < 0                                   # the signal precedes coalescence
        assert abs(-t / tau0 - 1.0) < 10 * v2


@pytest.mark.parametrize("m1,m2", [(5.0, 5.0), (30.0, 3.0)])
def test_phase_time_series_through_2pn(m1, m2):
    """Stationary phase fixes dPsi/df = 2 pi t(f), and the time to coalescence
    of a non-spinning binary has the classic post-Newtonian series
    t = -5M/(256 eta v^8) [1 + (743/252 + 11 eta/3) v^2 - (32 pi/5) v^3
    + (3058673/508032 + 5429 eta/504 + 617 eta^2/72) v^4 + O(v^5)].  The
    phase's derivative (complex step) divided by the Newtonian time is an
    exact finite series in 1, v^2 .. v^7 and v^6 log v; a least-squares fit
    over v in [0.02, 0.3] recovers its coefficients, and the 1PN, 1.5PN and
    2PN ones must be those of the time series (a slip in the phase's
    transcription of them fails here)."""
    m_s, eta, _ = ph.mass_params(m1, m2)
    v = np.linspace(0.02, 0.3, 120)
    f = v ** 3 / (math.pi * m_s)
    h = 1e-20 * f
    dpsi = np.imag(ph.pn_phase_22(f + 1j * h, m1, m2, 0.0, 0.0)) / h
    ratio = (dpsi / (2.0 * math.pi)) / (-5.0 * m_s / (256.0 * eta * v ** 8))
    basis = np.stack([np.ones_like(v), v ** 2, v ** 3, v ** 4, v ** 5, v ** 6, v ** 6 * np.log(v), v ** 7], axis=1)
    coef, *_ = np.linalg.lstsq(basis, ratio, rcond=None)
    tau2 = 743.0 / 252.0 + 11.0 * eta / 3.0
    tau3 = -32.0 * math.pi / 5.0
    tau4 = 3058673.0 / 508032.0 + 5429.0 * eta / 504.0 + 617.0 * eta ** 2 / 72.0
    # the fit recovers them to ~1e-10; a 1% slip in any of them moves its
    # coefficient by ~1e-2
    assert coef[0] == pytest.approx(1.0, abs=1e-9)
    assert coef[1] == pytest.approx(tau2, rel=1e-8)
    assert coef[2] == pytest.approx(tau3, rel=1e-8)
    assert coef[3] == pytest.approx(tau4, rel=1e-7)


def test_phase_spin_orbit_matches_reduced_spin_coordinate():
    """At low frequency the spin dependence of the phase is the 1.5PN
    spin-orbit term, which Eq. metric_coords writes as theta3s: the spin part
    equals 3/2 theta3s (f/f0)^(-2/3)."""
    phys = (8.0, 1.4, 0.6, -0.3)
    f0 = 20.0
    th = ph.phys_to_theta(phys, f0)
    for f in (1e-5, 1e-6):
        dpsi = ph.pn_phase_22(f, *phys) - ph.pn_phase_22(f, 8.0, 1.4, 0.0, 0.0)
        want = 1.5 * th[2] * (f / f0) ** (-2.0 / 3.0)
        v = (math.pi * 9.4 * ph.MSUN_S * f) ** (1.0 / 3.0)
        assert dpsi == pytest.approx(want, rel=30 * v)


def test_mode_band_and_amplitudes():
    grid = ph.Grid(2048.0, 4.0, 20.0)
    phys = (8.0, 1.4, 0.3, 0.0)
    f_isco = ph.f_isco_orbital(8.0, 1.4)
    assert 2 * f_isco == pytest.approx(1.0 / (6 ** 1.5 * math.pi * 9.4 * ph.MSUN_S))
    for (l, m) in wl.ALL_MODES:
        h = ph.waveform_mode(grid, l, m, phys, 100.0)
        nz = np.nonzero(h)[0]
        f = grid.freqs[nz]
        assert f.min() >= 20.0 and f.max() < m * f_isco
        assert f.max() + grid.df >= min(m * f_isco, grid.fs / 2 - grid.df)
    # (2,2) amplitude follows f^-7/6 exactly
    h = ph.waveform_mode(grid, 2, 2, phys, 100.0)
    j = np.nonzero(h)[0]
    ratio = np.abs(h[j]) * grid.freqs[j] ** (7.0 / 6.0)
    assert np.allclose(ratio, ratio[0], rtol=1e-13)


# ---------------------------------------------------------------- noise and inner product

def test_noise_colouring_statistics():
    """Over seeds, <h|n> has zero mean and variance <h|h> (Eq. innerProduct
    with one-sided PSD and the stated colouring)."""
    cfg = wl.CFG1.with_(fs=256.0, seg_len=4.0, f_low=20.0)
    grid = ph.Grid(cfg.fs, cfg.seg_len, cfg.f_low)
    psd = ph.psd_on_grid(grid)
    h = ph.waveform_mode(grid, 2, 2, (8.0, 1.4, 0.0, 0.0), 100.0)
    hh = ph.inner(h, h, psd, grid)
    vals = []
    for seed in range(600):
        w = wl.white_noise(cfg.with_(noise_seed=seed))
        ev = su.make_event(cfg.with_(inj_snr=1e-30), w, np.zeros(5))
        n = ev.data[0] - 0.0
        vals.append(ph.inner(h, n, psd, grid))
    vals = np.array(vals)
    n_s = len(vals)
    assert abs(vals.mean()) < 4 * math.sqrt(hh / n_s)
    assert abs(vals.var() / hh - 1.0) < 4 * math.sqrt(2.0 / n_s)


def test_snr_scaling_of_injection():
    cfg = TINY
    ev = su.make_event(cfg, None, wl.injection_extrinsics(cfg))
    rho2 = sum(ph.inner(ev.data[k], ev.data[k], ev.psd[k], ev.grid) for k in range(ev.n_det))
    assert math.sqrt(rho2) == pytest.approx(cfg.inj_snr, rel=1e-12)


# ---------------------------------------------------------------- harmonics and antenna patterns

def test_swsh_closed_form_and_orthonormality():
    for iota in (0.0, 0.4, 1.3, 2.9):
        for phi in (0.0, 1.1):
            want = math.sqrt(5.0 / (64.0 * math.pi)) * (1 + math.cos(iota)) ** 2 * complex(math.cos(2 * phi), math.sin(2 * phi))
            assert ph.ylm(2, 2, iota, phi) == pytest.approx(want, abs=1e-14)
            want21 = math.sqrt(5.0 / (16.0 * math.pi)) * math.sin(iota) * (1 + math.cos(iota)) * complex(math.cos(phi), math.sin(phi))
            assert ph.ylm(2, 1, iota, phi) == pytest.approx(want21, abs=1e-14)
    # orthonormality by Gauss-Legendre x trapezoid quadrature on the sphere
    xg, wg = np.polynomial.legendre.leggauss(24)
    phis = np.linspace(0, 2 * math.pi, 32, endpoint=False)
    lms = [(l, m) for l in (2, 3, 4) for m in range(-l, l + 1)]
    vals = np.array([[[ph.ylm(l, m, math.acos(c), p) for p in phis] for c in xg] for (l, m) in lms])
    gram = np.einsum("aij,bij,i->ab", np.conj(vals), vals, wg) * (2 * math.pi / len(phis))
    assert np.allclose(gram, np.eye(len(lms)), atol=1e-12)


def test_swsh_conjugation_relation():
    # conj(sY_lm) = (-1)^(s+m) (-s)Y_{l,-m}
    for (l, m) in [(2, 2), (2, -1), (3, 3), (3, -2), (4, 4)]:
        for iota, phi in [(0.3, 0.7), (2.0, 5.0)]:
            lhs = np.conj(ph.swsh(-2, l, m, iota, phi))
            rhs = (-1) ** (-2 + m) * ph.swsh(2, l, -m, iota, phi)
            assert lhs == pytest.approx(rhs, abs=1e-14)


def test_antenna_patterns_textbook_properties():
    site = (0.6, 1.2, 0.4, math.pi / 2, wl.EARTH_RADIUS_LS)
    D, pos = ph.detector_geometry(site)
    assert np.allclose(D, D.T) and abs(np.trace(D)) < 1e-15
    # source at the zenith of a 90-degree detector: F+^2 + Fx^2 = 1 for any psi
    for psi in (0.0, 0.3, 2.0):
        fp, fc = ph.antenna_pattern(D, 1.2, 0.6, psi)
        assert fp * fp + fc * fc == pytest.approx(1.0, abs=1e-14)
    # psi covariance: F+ + iFx rotates by a phase of twice the angle, modulus invariant
    a, d = 2.1, -0.4
    fp0, fc0 = ph.antenna_pattern(D, a, d, 0.0)
    for psi in (0.2, 1.0, 2.5):
        fp, fc = ph.antenna_pattern(D, a, d, psi)
        z = (fp + 1j * fc) / (fp0 + 1j * fc0)
        assert abs(z) == pytest.approx(1.0, abs=1e-13)
        assert abs(abs(np.angle(z)) - (2 * psi) % (2 * math.pi)) < 1e-12 or \
            abs(abs(np.angle(z)) - (2 * math.pi - (2 * psi) % (2 * math.pi))) < 1e-12
    fpq, fcq = ph.antenna_pattern(D, a, d, math.pi / 2)
    assert (fpq, fcq) == pytest.approx((-fp0, -fc0), abs=1e-14)
    # delay of a source at the zenith: -R (arrives earlier than at the geocentre)
    assert ph.time_delay(pos, 1.2, 0.6) == pytest.approx(-wl.EARTH_RADIUS_LS, rel=1e-13)


# ---------------------------------------------------------------- likelihood identity

def test_factorised_equals_brute_force(multi_art):
    """Eq. logl_complete (corrected reading) = Eq. logl_basic at arbitrary parameters."""
    ev = multi_art.ev
    rng = np.random.default_rng(11)
    for _ in range(4):
        phys = (8.0 + rng.uniform(-0.3, 0.3), 1.4 + rng.uniform(-0.05, 0.05), rng.uniform(-0.5, 0.5), 0.01)
        ext = np.array([rng.uniform(0, 6.28), rng.uniform(-1.2, 1.2), rng.uniform(0, 3), rng.uniform(0.1, 3), rng.uniform(0, 6)])
        t_c = ev.t_trig + rng.uniform(-0.01, 0.01)
        d = ev.d_inj * rng.uniform(0.6, 1.8)
        b = lk.brute_lnl(ev, phys, ext, t_c, d)
        f = lk.factorised_lnl(ev, phys, ext, t_c, d)
        assert f == pytest.approx(b, rel=1e-11, abs=1e-9)


def test_printed_first_term_would_differ(multi_art):
    """The printed first term of Eq. logl_complete (Y_lm instead of Y_{l,-m})
    does not reproduce Eq. logl_basic, which is why the corrected reading is used."""
    ev = multi_art.ev
    phys = ev.inj_phys
    alpha, dec, psi, iota, phi = ev.inj_ext
    k = 0
    fp, fc = ph.antenna_pattern(ev.det_tensor[k], alpha, dec, psi)
    tau = ev.t_trig + ph.time_delay(ev.det_pos[k], alpha, dec)
    z = np.array([lk.exact_z(ev, phys, k, a, tau) for a in range(len(ev.modes))])
    good = sum((np.conj(ph.mode_factor(l, m, fp, fc, iota, phi)) * z[a]).real for a, (l, m) in enumerate(ev.modes))
    printed = sum((0.5 * ((-1) ** l * ph.ylm(l, m, iota, phi) * (fp + 1j * fc)
                          + np.conj(ph.ylm(l, m, iota, phi)) * (fp - 1j * fc)) * z[a]).real
                  for a, (l, m) in enumerate(ev.modes))
    h = ph.detector_signal(ev.grid, ev.modes, phys, ev.d_inj, ev.inj_ext, ev.t_trig, ev.det_tensor[k], ev.det_pos[k])
    direct = ph.inner(h, ev.data[k], ev.psd[k], ev.grid)
    assert good == pytest.approx(direct, rel=1e-11)
    assert abs(printed - direct) > 1e-3 * abs(direct)


# ---------------------------------------------------------------- start-up pieces

def test_time_series_fft_equals_direct_sum(tiny_art):
    """z at the window via the inverse FFT = the direct sum over the band."""
    art = tiny_art
    ev = art.ev
    for node in (0, 7, 31):
        phys = tuple(art.phys_nodes[node])
        for t in (0, 5, art.half_w, 2 * art.half_w):
            tau = ev.t_trig + (t - art.half_w) / ev.grid.fs
            want = lk.exact_z(ev, phys, 0, 0, tau)
            assert art.z_nodes[0, 0, node, t] == pytest.approx(want, rel=1e-11, abs=1e-10)


def test_sigma_hermitian_positive(multi_art):
    s = multi_art.sigma_nodes
    assert np.allclose(s, np.conj(np.swapaxes(s, -1, -2)), rtol=0, atol=1e-12 * np.abs(s).max())
    ev = s.reshape(-1, s.shape[-1], s.shape[-1])
    assert np.all(np.linalg.eigvalsh(ev) > -1e-10 * np.abs(s).max())
    assert np.all(np.real(np.einsum("...aa->...a", s)) > 0)


def test_svd_full_rank_and_eckart_young(tiny_art):
    Z = tiny_art.z_nodes[0, 0]
    r = min(Z.shape)
    B, C, s = su.svd_basis(Z, r)
    assert np.allclose(C @ B.T, Z, rtol=0, atol=1e-12 * np.abs(Z).max())
    assert np.allclose(B.conj().T @ B, np.eye(r), atol=1e-12)
    for q in (3, 8):
        Bq, Cq, _ = su.svd_basis(Z, q)
        resid = np.sum(np.abs(Z - Cq @ Bq.T) ** 2)
        assert resid == pytest.approx(np.sum(s[q:] ** 2), rel=1e-9)


def test_rbf_interpolates_nodes_and_reproduces_polynomials(tiny_art):
    art = tiny_art
    x = art.x_nodes
    Y = lk.rbf_eval(art, x)
    scale = np.abs(art.node_values).max(axis=0)
    assert np.all(np.abs(Y - art.node_values) <= 1e-9 * scale[None, :])
    # data from a degree-r polynomial is reproduced everywhere (RBF part zero)
    for degree in (1, 3):
        F = np.stack([1.0 + 2 * x[:, 0] - x[:, 3], 0.5 * x[:, 2]], axis=1)
        if degree == 3:
            F[:, 1] += x[:, 0] ** 3 - x[:, 1] * x[:, 2] * x[:, 3]
        W, _ = su.rbf_solve(x, F, 1.0, degree)
        assert np.abs(W[:x.shape[0]]).max() < 1e-6
        xq = wl.uniform_ball(np.random.default_rng(0), 50)
        P = su.poly_matrix(xq, degree)
        got = np.concatenate([su.gaussian_kernel(xq, x, 1.0), P], axis=1) @ W
        want = np.stack([1.0 + 2 * xq[:, 0] - xq[:, 3], 0.5 * xq[:, 2]], axis=1)
        if degree == 3:
            want[:, 1] += xq[:, 0] ** 3 - xq[:, 1] * xq[:, 2] * xq[:, 3]
        assert np.allclose(got, want, atol=1e-7)


def test_monomial_count():
    # M = C(r + d, r) with d = 4 (Eq. rbfcoeff)
    for r in range(4):
        assert len(su.monomial_exponents(r)) == math.comb(r + 4, r)


def test_spline_weights_closed_form():
    tab = lk.spline_table()
    w0 = lk.spline_weights(np.array([0.0, 1.0]), tab)
    assert np.allclose(w0[0], np.eye(10)[4], atol=1e-14)
    assert np.allclose(w0[1], np.eye(10)[5], atol=1e-14)
    f = np.linspace(0, 1, 17)
    w = lk.spline_weights(f, tab)
    assert np.allclose(w.sum(axis=1), 1.0, atol=1e-14)
    # cubic data is reproduced exactly (not-a-knot spline of a cubic is the cubic)
    s = np.arange(10.0)
    for coeffs in ([1, 0, 0, 0], [0.3, -1, 2, 0.5], [0, 0, 0, 1]):
        y = np.polyval(coeffs[::-1], s)
        got = w @ y
        want = np.polyval(coeffs[::-1], 4.0 + f)
        assert np.allclose(got, want, atol=1e-11)


def test_metric_against_brute_force_match():
    """1 - M(Theta_c + dTheta) -> g dTheta dTheta for small steps along each
    eigen-axis (Eq. MisMatch), the band frozen at the centre."""
    cfg = wl.CFG1.with_(seg_len=8.0)
    grid = ph.Grid(cfg.fs, cfg.seg_len, cfg.f_low)
    psd = ph.psd_on_grid(grid)
    g = su.metric(grid, psd, cfg.inj_phys)
    fr = su.frame(g, ph.phys_to_theta(cfg.inj_phys, cfg.f_low), cfg.match)
    def ratio(i, t):
        x = np.zeros(4)
        x[i] = t
        th = su.x_to_theta(fr, x[None])[0]
        m1, m2, c1, c2, _ = ph.theta_to_phys(th, cfg.f_low)
        mm = 1 - su.match_22(grid, psd, cfg.inj_phys, (m1, m2, c1, c2), band_phys=cfg.inj_phys)
        return mm / ((1 - cfg.match) * t * t)

    # r(t) = 1 + a t + b t^2 + ...: fit three steps and extrapolate to t = 0.
    # The degenerate (longest) axis is ~1e3 times longer, so its steps are smaller.
    for i, t in ((0, 0.01), (1, 0.01), (2, 0.01), (3, 0.001)):
        ts = np.array([0.5, 1.0, 2.0]) * t
        r0 = np.polyfit(ts, [ratio(i, v) for v in ts], 2)[-1]
        assert r0 == pytest.approx(1.0, abs=1e-3)


def test_nodes_inside_ellipsoid_and_physical(tiny_art):
    art = tiny_art
    fr = art.frame
    dth = su.x_to_theta(fr, art.x_nodes) - fr.theta_c[None, :]
    q = np.einsum("ni,ij,nj->n", dth, fr.metric, dth)
    assert np.all(q <= (1 - TINY.match) * (1 + 1e-10))
    m1, m2, c1, c2, eta = ph.theta_to_phys(su.x_to_theta(fr, art.x_nodes).T, TINY.f_low)
    assert np.all(eta <= 0.25) and np.all(np.abs(c1) <= 1) and np.all(np.abs(c2) <= 1)


# ---------------------------------------------------------------- online stage

def test_meshfree_equals_brute_force_at_nodes_full_rank():
    """Query at a node, full-rank basis, on-grid arrival times: the interpolant
    and the SVD are exact there and the spline passes through the samples, so
    meshfree ln L = brute-force ln L.  Three co-located detectors at the
    geocentre keep every arrival time on the sample grid."""
    sites = tuple((0.8, -2.0, az, math.pi / 2, 0.0) for az in (0.3, 1.1, 2.0))
    cfg = TINY_MULTI.with_(n_nodes=40, q=40, center_node=True, sites=sites)
    art = su.startup(cfg, wl.white_noise(cfg), workers=1)
    ev = art.ev
    rng = np.random.default_rng(5)
    for node in (0, 9, 33):
        ext = np.array([rng.uniform(0, 6.28), rng.uniform(-1.2, 1.2), rng.uniform(0, 3),
                        rng.uniform(0.1, 3), rng.uniform(0, 6)])
        d = art.d_ref * 1.3
        tc = ev.t_trig + 3.0 / ev.grid.fs
        got = lk.meshfree_lnl(art, art.x_nodes[node:node + 1] * art.frame.semi, ext[None],
                              np.array([tc]), np.array([d]))[0]
        want = lk.brute_lnl(ev, tuple(art.phys_nodes[node]), ext, tc, d)
        assert got == pytest.approx(want, rel=1e-9, abs=1e-8)


def test_zero_noise_injection_at_node_gives_half_snr_squared():
    cfg = TINY.with_(n_nodes=40, q=40, center_node=True)
    art = su.startup(cfg, None, workers=1)
    got = lk.meshfree_lnl(art, np.zeros((1, 4)), art.ev.inj_ext[None], np.array([art.ev.t_trig]),
                          np.array([art.d_ref]))[0]
    assert got == pytest.approx(cfg.inj_snr ** 2 / 2, rel=1e-9)
    assert lk.brute_lnl(art.ev, cfg.inj_phys, art.ev.inj_ext, art.ev.t_trig, art.d_ref) == \
        pytest.approx(cfg.inj_snr ** 2 / 2, rel=1e-12)


def test_distance_dependence_closed_form(multi_art):
    """ln L = r X - r^2 Y / 2 in r = d_ref / d_L; its maximum over d_L is X^2 / (2 Y)."""
    art = multi_art
    qd = wl.queries(TINY_MULTI, n=64)
    dE, ext, tc, _ = lk.query_params(art, qd)
    rs = [0.7, 1.0, 1.6]
    vals = [lk.meshfree_lnl(art, dE, ext, tc, art.d_ref / r * np.ones(len(qd))) for r in rs]
    ok = np.isfinite(vals[0])
    assert ok.sum() > 3
    X = (vals[1] * rs[2] ** 2 - vals[2] * rs[1] ** 2) / (rs[1] * rs[2] ** 2 - rs[2] * rs[1] ** 2)
    Y = 2 * (X * rs[1] - vals[1]) / rs[1] ** 2
    pred = rs[0] * X - rs[0] ** 2 * Y / 2
    assert np.allclose(vals[0][ok], pred[ok], rtol=1e-10, atol=1e-8)


def test_quadrupole_only_phase_distance_maximum(tiny_art):
    """(2,2)-only: max over phi and d_L of ln L is |z|^2 / (2 sigma22),
    independent of inclination and antenna pattern."""
    art = tiny_art
    ev = art.ev
    x = art.x_nodes[3:4]
    tc = np.array([ev.t_trig + 0.37 / ev.grid.fs])
    _, z, sig, _ = lk.meshfree_parts(art, x * art.frame.semi, ev.inj_ext[None], tc, np.array([art.d_ref]))
    want = abs(z[0, 0, 0]) ** 2 / (2 * sig[0, 0, 0, 0].real)
    best = -np.inf
    for iota in (0.5, 1.9):
        phis = np.linspace(0, 2 * math.pi, 721)
        ext = np.tile(ev.inj_ext, (phis.size, 1))
        ext[:, 3] = iota
        ext[:, 4] = phis
        n = phis.size
        l1 = lk.meshfree_lnl(art, np.repeat(x * art.frame.semi, n, 0), ext, np.repeat(tc, n), np.full(n, art.d_ref))
        l2 = lk.meshfree_lnl(art, np.repeat(x * art.frame.semi, n, 0), ext, np.repeat(tc, n), np.full(n, art.d_ref / 2))
        Y = 2 * l1 - l2                       # l(r) = r X - r^2 Y / 2 at r = 1, 2
        X = l1 + Y / 2
        best = np.max(np.where(X > 0, X * X / (2 * Y), 0.0))
        assert best == pytest.approx(want, rel=1e-4)


def test_domain_boundaries(tiny_art):
    art = tiny_art
    ev = art.ev
    # outside the ellipsoid
    dE = np.array([[1.01, 0, 0, 0]]) * art.frame.semi
    assert lk.meshfree_lnl(art, dE, ev.inj_ext[None], np.array([ev.t_trig]), np.array([art.d_ref]))[0] == -np.inf
    # outside the time window
    far = ev.t_trig + (art.half_w - 3) / ev.grid.fs
    assert lk.meshfree_lnl(art, np.zeros((1, 4)), ev.inj_ext[None], np.array([far]), np.array([art.d_ref]))[0] == -np.inf
    near = ev.t_trig + (art.half_w - 6) / ev.grid.fs
    assert np.isfinite(lk.meshfree_lnl(art, np.zeros((1, 4)), ev.inj_ext[None], np.array([near]), np.array([art.d_ref]))[0])


# ---------------------------------------------------------------- method-error parts

def test_exact_parts_projected_equals_meshfree_at_nodes(multi_art):
    """At a node the RBF interpolant reproduces the node values, so ln L from
    the exact outputs projected on the time basis equals the meshfree ln L
    there, for any q and any arrival time inside the window."""
    art = multi_art
    rng = np.random.default_rng(17)
    nodes = np.array([0, 7, 21, 40])
    n = nodes.size
    ext = np.stack([rng.uniform(0, 6.28, n), rng.uniform(-1.2, 1.2, n), rng.uniform(0, 3, n),
                    rng.uniform(0.1, 3, n), rng.uniform(0, 6, n)], axis=1)
    tc = art.ev.t_trig + rng.uniform(-0.02, 0.02, n)
    dl = art.d_ref * rng.uniform(0.6, 1.8, n)
    de = art.x_nodes[nodes] * art.frame.semi
    projected, _ = lk.exact_parts(art, de, ext, tc, dl)
    meshfree = lk.meshfree_lnl(art, de, ext, tc, dl)
    assert np.all(np.isfinite(meshfree))
    np.testing.assert_allclose(projected, meshfree, rtol=1e-8, atol=1e-7)


def test_exact_parts_samples_equal_brute_force_on_grid():
    """With every arrival time on the sample grid the spline returns the sample
    itself, so ln L from the exact window samples equals the brute-force ln L
    at any physical proposal, not only at the nodes.  Co-located detectors at
    the geocentre keep the arrival times on the grid."""
    sites = tuple((0.8, -2.0, az, math.pi / 2, 0.0) for az in (0.3, 1.1, 2.0))
    cfg = TINY_MULTI.with_(sites=sites)
    art = su.startup(cfg, wl.white_noise(cfg), workers=1)
    idx, jit = wl.node_jitter(12, cfg.n_nodes, seed=19)
    qd = wl.queries(cfg, n=12, seed=23).near_nodes(art.x_nodes, idx, jit)
    de, ext, tc, dl = lk.query_params(art, qd)
    tc = art.ev.t_trig + np.round((tc - art.ev.t_trig) * art.ev.grid.fs) / art.ev.grid.fs
    _, samples = lk.exact_parts(art, de, ext, tc, dl)
    ok = np.isfinite(samples)
    assert ok.sum() >= 6
    _, phys = su.physical_mask(art.frame, de[ok] / art.frame.semi, art.ev.grid.f_low, cfg.chi_max)
    want = [lk.brute_lnl(art.ev, tuple(p), e, t, d) for p, e, t, d in zip(phys, ext[ok], tc[ok], dl[ok])]
    np.testing.assert_allclose(samples[ok], want, rtol=1e-9, atol=1e-8)


def test_exact_parts_full_basis_projection_is_lossless():
    """With q = T the time basis spans every window series (it needs N >= T),
    so the projection loses nothing: both parts agree at any proposal and any
    arrival time; NaN inputs give NaN in both."""
    cfg = TINY.with_(half_window=0.01, n_nodes=40, q=21)
    art = su.startup(cfg, wl.white_noise(cfg), workers=1)
    assert art.basis.shape[2] == 21
    idx, jit = wl.node_jitter(10, cfg.n_nodes, seed=29)
    qd = wl.queries(cfg, n=10, seed=31).near_nodes(art.x_nodes, idx, jit)
    de, ext, tc, dl = lk.query_params(art, qd)
    tc = art.ev.t_trig + np.random.default_rng(3).uniform(-0.004, 0.004, 10)
    dl = dl.copy()
    dl[0] = np.nan
    projected, samples = lk.exact_parts(art, de, ext, tc, dl)
    assert np.isnan(projected[0]) and np.isnan(samples[0])
    ok = np.isfinite(samples)
    assert ok.sum() >= 5
    np.testing.assert_array_equal(ok, np.isfinite(projected))
    np.testing.assert_allclose(projected[ok], samples[ok], rtol=1e-9, atol=1e-8)


# ---------------------------------------------------------------- time/phase reference

def test_referenced_phase_vanishes_with_its_slope_at_f_ref():
    """Psi(f) - Psi(f_ref) - Psi'(f_ref)(f - f_ref): zero with zero slope at
    f_ref (central differences, independent of the complex step) and an
    affine function of f away from the PN phase (second differences vanish)."""
    phys = (8.0, 1.4, 0.3, -0.2)
    f_ref = 137.0
    h = 1e-3
    fr = np.array([f_ref - h, f_ref, f_ref + h])
    p = ph.referenced_phase_22(fr, *phys, f_ref)
    assert abs(p[1]) < 1e-9
    assert abs((p[2] - p[0]) / (2 * h)) < 1e-5
    f = np.linspace(30.0, 400.0, 7)
    diff = ph.referenced_phase_22(f, *phys, f_ref) - ph.pn_phase_22(f, *phys)
    assert np.allclose(np.diff(diff, 2), 0.0, atol=1e-6 * np.max(np.abs(diff)))


def test_reference_frequency_with_flat_weights_is_the_band_midpoint():
    """With S(f) = f^(-7/3) the weights are flat, so the weighted mean
    frequency is the mean of the band's bins."""
    grid = ph.Grid(2048.0, 8.0, 20.0)
    f = grid.freqs
    psd = np.full(grid.n_f, np.inf)
    psd[1:] = f[1:] ** (-7.0 / 3.0)
    phys = (8.0, 1.4, 0.3, 0.0)
    j0, j1 = ph.mode_band(grid, 2, phys[0], phys[1])
    assert ph.reference_frequency(grid, psd, phys) == pytest.approx(0.5 * (j0 + j1 - 1) * grid.df, rel=1e-12)


def test_match_does_not_depend_on_the_time_phase_reference():
    """Eq. Match maximises over time and phase, so moving the templates'
    reference (a shift affine in f) leaves every match unchanged."""
    a, b = (8.0, 1.4, 0.3, 0.0), (7.6, 1.45, 0.1, 0.4)
    vals = []
    for f_ref in (0.0, 60.0, 137.0):
        grid = ph.Grid(2048.0, 8.0, 20.0, f_ref)
        vals.append(su.match_22(grid, ph.psd_on_grid(grid), a, b))
    assert vals[0] < 0.999
    assert vals[1] == pytest.approx(vals[0], abs=1e-9) and vals[2] == pytest.approx(vals[0], abs=1e-9)


# ---------------------------------------------------------------- squeeze (Fig. 2)

def test_squeeze_stops_at_the_first_true_match_crossing():
    """The squeezed tip of the longest axis has true match M0 with the centre
    (Eq. Match, brute force), every point of the axis inside it at least M0
    (the first crossing, not a later one), and only that axis changes."""
    cfg = TINY.with_(squeeze=True)
    ev = su.make_event(cfg, None, wl.injection_extrinsics(cfg))
    g = su.metric(ev.grid, ev.psd[0], cfg.inj_phys)
    fr0 = su.frame(g, ph.phys_to_theta(cfg.inj_phys, ev.grid.f_low), cfg.match)
    fr, factor = su.squeeze(fr0, ev.grid, ev.psd[0], cfg.inj_phys, cfg.match, ev.grid.f_low)
    assert 0.0 < factor < 1.0
    np.testing.assert_array_equal(fr.semi[:3], fr0.semi[:3])
    assert fr.semi[3] == factor * fr0.semi[3]

    def match_at(s):
        x = np.zeros((1, 4))
        x[0, 3] = s
        ok, phys = su.physical_mask(fr0, x, ev.grid.f_low, np.inf)
        return su.match_22(ev.grid, ev.psd[0], cfg.inj_phys, tuple(phys[0])) if ok[0] else None

    tips = [match_at(sgn * factor) for sgn in (1.0, -1.0)]
    assert any(t is not None and abs(t - cfg.match) < 1e-9 for t in tips)
    for sgn in (1.0, -1.0):
        for s in np.linspace(0.02, 0.999, 25) * factor:
            m = match_at(sgn * s)
            assert m is None or m >= cfg.match - 1e-12
    art = su.startup(cfg, None, workers=1)
    assert art.squeeze_factor == factor
    assert np.all(np.sum(art.x_nodes ** 2, axis=1) <= 1.0)


# ---------------------------------------------------------------- SNR-optimised centre

def test_centre_optimum_reaches_the_cauchy_schwarz_bound():
    """One detector, the (2,2) mode, zero noise: the data are a template of
    the family, so the best network SNR is the injection's optimal SNR
    (Cauchy-Schwarz, equality only at the injected template); started from a
    seed inside the match ellipsoid (as a template bank's best match would
    be) with iota = phi = 0, the optimiser must reach it and return a centre
    whose template matches the injection."""
    cfg = TINY.with_(centre_offset=(0.002, 0.0, 0.01, 0.0))
    ev = su.make_event(cfg, None, wl.injection_extrinsics(cfg))
    phys, iota, phi, snr_seed, snr_opt = su.optimise_centre(ev, cfg.seed_phys, cfg.match, cfg.half_window)
    assert snr_seed < 0.99 * cfg.inj_snr
    assert cfg.inj_snr * (1 - 1e-4) <= snr_opt <= cfg.inj_snr * (1 + 1e-6)
    assert su.match_22(ev.grid, ev.psd[0], cfg.inj_phys, phys) > 0.9999
    # the objective at the injection itself is the bound (any iota, phi for the (2,2) mode)
    s2 = su.network_snr2(ev, cfg.inj_phys, 0.4, 1.0, cfg.half_window)
    assert s2 == pytest.approx(cfg.inj_snr ** 2, rel=1e-6)


# ---------------------------------------------------------------- rotating Earth

def test_rotating_signal_reduces_to_the_frozen_one():
    """With a vanishing rotation rate the rotating-Earth signal (per-bin
    antenna factors and delays at each mode's stationary-phase time) equals
    the frozen projected signal of Eq. projected_h_fd."""
    cfg = TINY_MULTI
    ev = su.make_event(cfg, None, wl.injection_extrinsics(cfg))
    ext = np.array([1.1, -0.4, 0.7, 1.2, 2.3])
    for k in range(ev.n_det):
        a = ph.detector_signal(ev.grid, ev.modes, cfg.inj_phys, 100.0, ext, ev.t_trig + 0.01, ev.det_tensor[k],
                               ev.det_pos[k])
        b = ph.detector_signal(ev.grid, ev.modes, cfg.inj_phys, 100.0, ext, ev.t_trig + 0.01, ev.det_tensor[k],
                               ev.det_pos[k], 1e-30, ev.t_trig)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_rotating_signal_closed_form_on_the_equator():
    """A face-on (2,2) source on the equator seen by an equatorial detector with
    arms along x and y at the geocentre: |F+ - i Fx| = |cos 2(lon)| / 2 with
    lon the source's Earth-fixed longitude, so |h_k(f)| / |h_22(f)| =
    |Y_22(0)| |cos 2(alpha - rate (t(f) - t_ref))| / 4 at every bin; alpha is
    off zero so that the sign of the rotation matters."""
    grid = ph.Grid(1024.0, 8.0, 20.0, 137.0)
    D = 0.5 * (np.outer([1.0, 0, 0], [1.0, 0, 0]) - np.outer([0, 1.0, 0], [0, 1.0, 0]))
    pos = np.zeros(3)
    phys = (8.0, 1.4, 0.3, 0.0)
    alpha, rate, t_c, t_ref = 0.3, 0.02, 5.0, 4.0
    ext = np.array([alpha, 0.0, 0.0, 0.0, 0.0])
    h = ph.detector_signal(grid, ((2, 2),), phys, 100.0, ext, t_c, D, pos, rate, t_ref)
    h22 = ph.waveform_mode(grid, 2, 2, phys, 100.0)
    j0, j1 = ph.mode_band(grid, 2, phys[0], phys[1])
    f = np.arange(j0, j1) * grid.df
    t = ph.spa_time(f, 2, phys, grid.f_ref, t_c)
    want = abs(ph.ylm(2, 2, 0.0, 0.0)) * np.abs(np.cos(2.0 * (alpha - rate * (t - t_ref)))) / 4.0
    got = np.abs(h[j0:j1]) / np.abs(h22[j0:j1])
    assert np.allclose(got, want, rtol=1e-10, atol=1e-12)
    # the band spans a sizeable rotation, and the (2,2) mode passes f_ref at t_c
    assert np.ptp(rate * t) > 0.05
    assert ph.spa_time(np.array([grid.f_ref]), 2, phys, grid.f_ref, t_c)[0] == pytest.approx(t_c, abs=1e-9)


def test_artefacts_from_exports_evaluate_like_the_originals(multi_art):
    """The evaluation-parity glue: artefacts rebuilt from another start-up's
    arrays (here the oracle's own) give the same online-stage ln L bit for bit."""
    art = multi_art
    fr = art.frame
    rebuilt = su.artefacts_from_exports(TINY_MULTI, art.ev.inj_ext, fr.theta_c, fr.metric, fr.vecs, fr.lam, fr.semi,
                                        art.x_nodes, art.phys_nodes, art.W, art.basis, art.half_w, art.d_ref,
                                        art.ev.grid.f_ref)
    qd = wl.queries(TINY_MULTI, n=300, seed=3)
    a = lk.meshfree_lnl(art, *lk.query_params(art, qd))
    b = lk.meshfree_lnl(rebuilt, *lk.query_params(rebuilt, qd))
    assert np.isfinite(a).sum() > 0
    assert np.array_equal(a, b)


def test_choose_eps_is_the_smallest_integer_under_the_condition_bar(tiny_art):
    """The automatic shape parameter (a workload with eps = 0): the chosen
    integer's system has a 1-norm condition number <= the bar and the next
    smaller integer's does not (or it is 1); a looser bar never picks more."""
    x = tiny_art.x_nodes
    for bar in (1e6, 1e9, 1e12):
        eps = su.choose_eps(x, 1, cond_max=bar)
        assert np.linalg.cond(su.rbf_system(x, eps, 1), 1) <= bar or eps == 8
        if eps > 1:
            assert np.linalg.cond(su.rbf_system(x, eps - 1, 1), 1) > bar
    assert su.choose_eps(x, 1, cond_max=1e12) <= su.choose_eps(x, 1, cond_max=1e6)
