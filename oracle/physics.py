"""Oracle physics: inner product, PSD, waveform family, coordinates, detector response.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain float64 numpy.

Parity unpinned against the literature: the spin-orbit terms of pn_phase_22
at 2.5PN, 3PN and 3.5PN and its 3PN spin-spin term (every non-spinning order
through 3.5PN, the 1.5PN spin-orbit and the 2PN spin-spin terms are pinned;
see its docstring).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

MSUN_S = 4.925490947641267e-06          # G Msun / c^3 [s]
MPC_S = 3.0856775814913673e22 / 299792458.0   # 1 Mpc / c [s]
EULER_GAMMA = 0.5772156649015329


# ----------------------------------------------------------------------------
# Frequency grid and the noise-weighted inner product (Eq. innerProduct)
# ----------------------------------------------------------------------------

@dataclass
class Grid:
    """DFT grid of a segment: f_j = j / seg_len, j = 0 .. n_s/2.  f_ref is the
    templates' time/phase reference frequency (0: the formal coalescence)."""
    fs: float
    seg_len: float
    f_low: float
    f_ref: float = 0.0

    @property
    def n_s(self) -> int:
        return int(round(self.fs * self.seg_len))

    @property
    def n_f(self) -> int:
        return self.n_s // 2 + 1

    @property
    def df(self) -> float:
        return 1.0 / self.seg_len

    @property
    def freqs(self) -> np.ndarray:
        return np.arange(self.n_f) * self.df

    @property
    def j_lo(self) -> int:
        """First bin with f_j >= f_low (and never DC)."""
        return max(1, int(math.ceil(self.f_low * self.seg_len - 1e-9)))

    @property
    def j_hi(self) -> int:
        """One past the last band bin: the Nyquist bin is excluded."""
        return self.n_s // 2

    def band(self) -> slice:
        return slice(self.j_lo, self.j_hi)


def psd_analytic(f: np.ndarray, scale: float = 1.0) -> np.ndarray:
    """aLIGO-like analytic one-sided PSD, x = f / 215 Hz (workload definition).
    Pinned at hand-evaluated points (x = 1 gives 33e-49)."""
    x = np.asarray(f, dtype=np.float64) / 215.0
    return scale * 1e-49 * (x ** -4.14 - 5.0 * x ** -2 + 111.0 * (1.0 - x ** 2 + 0.5 * x ** 4) / (1.0 + 0.5 * x ** 2))


def psd_on_grid(grid: Grid, scale: float = 1.0) -> np.ndarray:
    """PSD on every bin; DC gets +inf so that it never contributes."""
    s = np.full(grid.n_f, np.inf)
    s[1:] = psd_analytic(grid.freqs[1:], scale)
    return s


def overlap(a: np.ndarray, b: np.ndarray, psd: np.ndarray, grid: Grid) -> complex:
    """Complex overlap (a|b) = 4 df sum_band conj(a) b / S; <a|b> is its real part."""
    sl = grid.band()
    return complex(4.0 * grid.df * np.sum(np.conj(a[sl]) * b[sl] / psd[sl]))


def inner(a, b, psd, grid) -> float:
    """Noise-weighted inner product <a|b> (Eq. innerProduct)."""
    return overlap(a, b, psd, grid).real


# ----------------------------------------------------------------------------
# Mass/spin parameters and the chirp-time coordinates (Eq. metric_coords)
# ----------------------------------------------------------------------------

def mass_params(m1, m2):
    """Total mass [s], symmetric mass ratio, asymmetric mass ratio delta."""
    mt = m1 + m2
    return mt * MSUN_S, m1 * m2 / mt ** 2, (m1 - m2) / mt


def phys_to_theta(phys, f0: float) -> np.ndarray:
    """(m1, m2, chi1, chi2) -> (theta0, theta3, theta3s, theta3s_bar), Eq. metric_coords.
    Pinned: theta3s through the 1.5PN spin-orbit phase, theta3s_bar through the
    mass-weighted effective spin and the mass-ratio-free difference
    theta3s - theta3s_bar = -(19/48) chi_s (pi M f0)^(-2/3)."""
    m1, m2, c1, c2 = (np.asarray(p, dtype=np.float64) for p in phys)
    m_s, eta, delta = mass_params(m1, m2)
    chi_s = 0.5 * (c1 + c2)
    chi_a = 0.5 * (c1 - c2)
    chi_r = chi_s + delta * chi_a - 76.0 * eta * chi_s / 113.0
    chi_eff = (m1 * c1 + m2 * c2) / (m1 + m2)
    u = math.pi * m_s * f0
    th0 = 5.0 / (128.0 * eta) * u ** (-5.0 / 3.0)
    th3 = math.pi / (4.0 * eta) * u ** (-2.0 / 3.0)
    th3s = 113.0 * chi_r / (192.0 * eta) * u ** (-2.0 / 3.0)
    th3b = 113.0 * chi_eff / (192.0 * eta) * u ** (-2.0 / 3.0)
    return np.array([th0, th3, th3s, th3b])


def theta_to_phys(theta, f0: float):
    """Closed-form inverse of phys_to_theta.  Returns (m1, m2, chi1, chi2, eta).

    From the ratios of the coordinates: pi M f0 = 5 theta3 / (32 pi theta0),
    eta = pi/(4 theta3) (pi M f0)^(-2/3), chi_r = 48 pi theta3s / (113 theta3),
    chi_eff = 48 pi theta3s_bar / (113 theta3), and chi_eff - chi_r =
    76 eta chi_s / 113.  eta is returned unclipped so callers can test the
    physical boundary eta <= 1/4; m1, m2, chi are NaN where eta > 1/4.
    """
    th0, th3, th3s, th3b = (np.asarray(t) for t in theta)
    with np.errstate(invalid="ignore", divide="ignore"):
        u = 5.0 * th3 / (32.0 * math.pi * th0)            # pi M f0
        m_s = u / (math.pi * f0)
        eta = math.pi / (4.0 * th3) * u ** (-2.0 / 3.0)
        chi_r = 48.0 * math.pi * th3s / (113.0 * th3)
        chi_eff = 48.0 * math.pi * th3b / (113.0 * th3)
        delta = np.sqrt(1.0 - 4.0 * eta)
        chi_s = 113.0 * (chi_eff - chi_r) / (76.0 * eta)
        chi_a = (chi_eff - chi_s) / delta
    m_tot = m_s / MSUN_S
    m1 = 0.5 * m_tot * (1.0 + delta)
    m2 = 0.5 * m_tot * (1.0 - delta)
    return m1, m2, chi_s + chi_a, chi_s - chi_a, eta


# ----------------------------------------------------------------------------
# Synthetic multimode inspiral family (TaylorF2-like phase, f^-7/6 amplitude)
# ----------------------------------------------------------------------------

def pn_phase_22(f, m1, m2, chi1, chi2):
    """(2,2) SPA phase Psi(f) at template t_c = phi_c = 0:

    Psi = -pi/4 + 3/(128 eta v^5) sum_k (phi_k + phi_kl log-terms) v^k, v = (pi M f)^(1/3),
    with 3.5PN non-spinning coefficients and aligned-spin spin-orbit /
    spin-spin terms (literature values).  Pinned in the tests through
    dPsi/df = 2 pi t(f) against the published time-to-coalescence series:
    every non-spinning term through 3.5PN (with the 3PN logarithm), the 1.5PN
    spin-orbit term and the 2PN spin-spin term; the spin-orbit terms at 2.5PN,
    3PN and 3.5PN and the 3PN spin-spin term are parity unpinned against the
    literature.
    """
    m_s, eta, delta = mass_params(m1, m2)
    chi_s = 0.5 * (chi1 + chi2)
    chi_a = 0.5 * (chi1 - chi2)
    pi = math.pi
    u = pi * m_s * np.asarray(f)
    v = u ** (1.0 / 3.0) if np.iscomplexobj(u) else np.cbrt(u.astype(np.float64))
    logv = np.log(v)
    p2 = 3715.0 / 756.0 + 55.0 * eta / 9.0
    p3 = (-16.0 * pi + 113.0 / 3.0 * delta * chi_a
          + (113.0 / 3.0 - 76.0 * eta / 3.0) * chi_s)
    p4 = (15293365.0 / 508032.0 + 27145.0 * eta / 504.0 + 3085.0 * eta ** 2 / 72.0
          + (-405.0 / 8.0 + 200.0 * eta) * chi_a ** 2
          - 405.0 / 4.0 * delta * chi_a * chi_s
          + (-405.0 / 8.0 + 5.0 * eta / 2.0) * chi_s ** 2)
    p5 = (pi * (38645.0 / 756.0 - 65.0 * eta / 9.0)
          + delta * chi_a * (-732985.0 / 2268.0 - 140.0 * eta / 9.0)
          + chi_s * (-732985.0 / 2268.0 + 24260.0 * eta / 81.0 + 340.0 * eta ** 2 / 9.0))
    p6 = (11583231236531.0 / 4694215680.0 - 640.0 * pi ** 2 / 3.0 - 6848.0 * EULER_GAMMA / 21.0
          + eta * (-15737765635.0 / 3048192.0 + 2255.0 * pi ** 2 / 12.0)
          + 76055.0 * eta ** 2 / 1728.0 - 127825.0 * eta ** 3 / 1296.0
          + pi * (2270.0 / 3.0 * delta * chi_a + (2270.0 / 3.0 - 520.0 * eta) * chi_s)
          + (75515.0 / 144.0 - 8225.0 * eta / 18.0) * delta * chi_a * chi_s
          + (75515.0 / 288.0 - 263245.0 * eta / 252.0 - 480.0 * eta ** 2) * chi_a ** 2
          + (75515.0 / 288.0 - 232415.0 * eta / 504.0 + 1255.0 * eta ** 2 / 9.0) * chi_s ** 2)
    p6l = -6848.0 / 21.0
    p7 = (pi * (77096675.0 / 254016.0 + 378515.0 * eta / 1512.0 - 74045.0 * eta ** 2 / 756.0)
          + delta * chi_a * (-25150083775.0 / 3048192.0 + 26804935.0 * eta / 6048.0
                             - 1985.0 * eta ** 2 / 48.0)
          + chi_s * (-25150083775.0 / 3048192.0 + 10566655595.0 * eta / 762048.0
                     - 1042165.0 * eta ** 2 / 3024.0 + 5345.0 * eta ** 3 / 36.0))
    series = (1.0 + p2 * v ** 2 + p3 * v ** 3 + p4 * v ** 4
              + p5 * (1.0 + 3.0 * logv) * v ** 5
              + (p6 + p6l * (math.log(4.0) + logv)) * v ** 6
              + p7 * v ** 7)
    return -pi / 4.0 + 3.0 / (128.0 * eta * v ** 5) * series


def referenced_phase_22(f, m1, m2, chi1, chi2, f_ref: float):
    """The (2,2) phase with the template's time and phase referenced at f_ref
    (the values a LAL-style approximant fixes at a reference frequency):
    Psi(f) - Psi(f_ref) - Psi'(f_ref) (f - f_ref), so that the shifted phase
    and its slope vanish at f_ref and t_c, phi_c become the time and phase at
    which the (2,2) mode passes f_ref.  Psi' by the complex step
    Im Psi(f_ref + i h) / h (exact to rounding).  f_ref <= 0: Psi itself."""
    psi = pn_phase_22(f, m1, m2, chi1, chi2)
    if f_ref <= 0.0:
        return psi
    h = 1e-20 * f_ref
    p0 = float(np.real(pn_phase_22(np.array([f_ref]), m1, m2, chi1, chi2))[0])
    dp = float(np.imag(pn_phase_22(np.array([f_ref + 1j * h]), m1, m2, chi1, chi2))[0]) / h
    return psi - p0 - dp * (np.asarray(f) - f_ref)


def reference_frequency(grid: Grid, psd: np.ndarray, phys) -> float:
    """Mean frequency of the (2,2) band of `phys` under the weights
    |h22|^2 / S = f^(-7/3) / S (the metric's weights)."""
    j0, j1 = mode_band(grid, 2, phys[0], phys[1])
    f = np.arange(j0, j1) * grid.df
    w = f ** (-7.0 / 3.0) / psd[j0:j1]
    return float(np.sum(f * w) / np.sum(w))


def mode_amplitude(l: int, m: int, eta: float, delta: float) -> float:
    """Relative mode amplitudes of the synthetic family: A22 = 1, A21 = 0.1 delta,
    A33 = 0.3 delta, A32 = 0.05 (1 - 3 eta), A44 = 0.1 (1 - 3 eta).  Pinned,
    through the waveform, at hand-evaluated fractions for three mass pairs."""
    table = {(2, 2): 1.0, (2, 1): 0.1 * delta, (3, 3): 0.3 * delta,
             (3, 2): 0.05 * (1.0 - 3.0 * eta), (4, 4): 0.1 * (1.0 - 3.0 * eta)}
    return table[(l, m)]


def newtonian_amplitude(m1, m2, d_mpc):
    """SPA amplitude constant sqrt(5/24) pi^(-2/3) Mc^(5/6) / d (geometric units, seconds)."""
    mc = (m1 * m2) ** 0.6 / (m1 + m2) ** 0.2 * MSUN_S
    return math.sqrt(5.0 / 24.0) * math.pi ** (-2.0 / 3.0) * mc ** (5.0 / 6.0) / (d_mpc * MPC_S)


def f_isco_orbital(m1, m2) -> float:
    """Orbital frequency at the Schwarzschild ISCO (r = 6M): 1 / (2 pi 6^(3/2) M)."""
    return 1.0 / (2.0 * math.pi * 6.0 ** 1.5 * (m1 + m2) * MSUN_S)


def mode_band(grid: Grid, m: int, m1, m2):
    """Bins where mode |m| is non-zero: f_low <= f_j < m * F_isco and j < n_s/2."""
    j_cut = int(math.ceil(m * f_isco_orbital(m1, m2) * grid.seg_len))   # first bin with f >= cut
    return grid.j_lo, max(grid.j_lo, min(j_cut, grid.j_hi))


def waveform_mode(grid: Grid, l: int, m: int, phys, d_mpc: float) -> np.ndarray:
    """h_{l,-m}(f_j) on the whole grid (zeros outside the mode's band):

    h_{l,-m}(f) = A_lm * Amp * f^(-7/6) * exp(-i (m/2) Psi(2 f / m)),
    Psi referenced at grid.f_ref.
    """
    m1, m2, c1, c2 = phys
    _, eta, delta = mass_params(m1, m2)
    out = np.zeros(grid.n_f, dtype=np.complex128)
    j0, j1 = mode_band(grid, m, m1, m2)
    if j1 <= j0:
        return out
    f = np.arange(j0, j1) * grid.df
    psi = referenced_phase_22(2.0 * f / m, m1, m2, c1, c2, grid.f_ref)
    amp = mode_amplitude(l, m, eta, delta) * newtonian_amplitude(m1, m2, d_mpc) * f ** (-7.0 / 6.0)
    out[j0:j1] = amp * np.exp(-1j * (0.5 * m) * psi)
    return out


# ----------------------------------------------------------------------------
# Spin-weighted spherical harmonics (Eq. h_spherical_harmonic_basis)
# ----------------------------------------------------------------------------

def wigner_d(l: int, mp: int, m: int, beta: float) -> float:
    """Wigner small-d matrix element d^l_{mp,m}(beta) by the explicit finite sum."""
    f = math.factorial
    c = math.cos(0.5 * beta)
    s = math.sin(0.5 * beta)
    pre = math.sqrt(f(l + mp) * f(l - mp) * f(l + m) * f(l - m))
    total = 0.0
    for k in range(0, 2 * l + 1):
        a1, a2, a3, a4 = l + m - k, k, mp - m + k, l - mp - k
        if min(a1, a2, a3, a4) < 0:
            continue
        total += ((-1.0) ** (mp - m + k) * pre / (f(a1) * f(a2) * f(a3) * f(a4))
                  * c ** (2 * l + m - mp - 2 * k) * s ** (mp - m + 2 * k))
    return total


def swsh(s: int, l: int, m: int, theta: float, phi: float) -> complex:
    """Spin-weighted harmonic sY_lm(theta, phi) = (-1)^s sqrt((2l+1)/4pi) d^l_{m,-s}(theta) e^{i m phi}."""
    return ((-1.0) ** s * math.sqrt((2 * l + 1) / (4.0 * math.pi))
            * wigner_d(l, m, -s, theta) * complex(math.cos(m * phi), math.sin(m * phi)))


def ylm(l: int, m: int, iota: float, phi: float) -> complex:
    """Spin -2 harmonic (the symbol -2 is dropped in the paper's equations)."""
    return swsh(-2, l, m, iota, phi)


# ----------------------------------------------------------------------------
# Detector geometry and response (Eqs. projected_h_td / projected_h_fd)
# ----------------------------------------------------------------------------

def detector_geometry(site):
    """Detector tensor D = (u u^T - v v^T)/2 and position [light-seconds] in
    Earth-fixed coordinates from (lat, lon, x-arm azimuth from north toward
    east, opening angle, distance from the geocentre)."""
    lat, lon, az, opening, radius = site
    east = np.array([-math.sin(lon), math.cos(lon), 0.0])
    north = np.array([-math.sin(lat) * math.cos(lon), -math.sin(lat) * math.sin(lon), math.cos(lat)])
    up = np.array([math.cos(lat) * math.cos(lon), math.cos(lat) * math.sin(lon), math.sin(lat)])
    u = math.cos(az) * north + math.sin(az) * east
    v = math.cos(az + opening) * north + math.sin(az + opening) * east
    return 0.5 * (np.outer(u, u) - np.outer(v, v)), radius * up


def antenna_pattern(D: np.ndarray, alpha: float, dec: float, psi: float):
    """F+ = D:e+, Fx = D:ex with the wave-frame axes X = -cos(psi) e_alpha +
    sin(psi) e_dec, Y = sin(psi) e_alpha + cos(psi) e_dec (Earth-fixed sky,
    Greenwich sidereal time taken as zero, patterns frozen in time)."""
    e_a = np.array([-math.sin(alpha), math.cos(alpha), 0.0])
    e_d = np.array([-math.sin(dec) * math.cos(alpha), -math.sin(dec) * math.sin(alpha), math.cos(dec)])
    X = -math.cos(psi) * e_a + math.sin(psi) * e_d
    Y = math.sin(psi) * e_a + math.cos(psi) * e_d
    ep = np.outer(X, X) - np.outer(Y, Y)
    ec = np.outer(X, Y) + np.outer(Y, X)
    return float(np.sum(D * ep)), float(np.sum(D * ec))


def time_delay(pos: np.ndarray, alpha: float, dec: float) -> float:
    """Arrival time at the detector minus geocentric time: -r . s_hat."""
    s_hat = np.array([math.cos(dec) * math.cos(alpha), math.cos(dec) * math.sin(alpha), math.sin(dec)])
    return float(-np.dot(pos, s_hat))


def mode_factor(l: int, m: int, fp: float, fc: float, iota: float, phi: float) -> complex:
    """A_{lm} = 1/2 [(F+ + i Fx) Y_{l,-m} + (-1)^l (F+ - i Fx) conj(Y_{l,m})]:
    the detector response is sum_lm A_lm h_{l,-m}(f) by Eqs. hplus_hcross_decomposed1/2."""
    return 0.5 * ((fp + 1j * fc) * ylm(l, -m, iota, phi)
                  + (-1.0) ** l * (fp - 1j * fc) * np.conj(ylm(l, m, iota, phi)))


def polarizations(grid: Grid, modes, phys, d_mpc, iota, phi):
    """h+(f), hx(f) from the negative-m modes, Eqs. hplus_hcross_decomposed1/2."""
    hp = np.zeros(grid.n_f, dtype=np.complex128)
    hc = np.zeros(grid.n_f, dtype=np.complex128)
    for (l, m) in modes:
        h = waveform_mode(grid, l, m, phys, d_mpc)
        y_neg = ylm(l, -m, iota, phi)
        y_pos_c = np.conj(ylm(l, m, iota, phi))
        sgn = (-1.0) ** l
        hp += 0.5 * (y_neg + sgn * y_pos_c) * h
        hc += 0.5j * (y_neg - sgn * y_pos_c) * h
    return hp, hc


def spa_time(f: np.ndarray, m: int, phys, f_ref: float, t_c: float) -> np.ndarray:
    """Stationary-phase time at which mode m has frequency f: the slope of its
    phase (m/2) Psi(2f/m), i.e. t_c + Psi'(2f/m) / (2 pi) with the referenced
    phase Psi; the derivative by the complex step."""
    x = 2.0 * np.asarray(f, dtype=np.float64) / m
    h = 1e-20 * x
    d = np.imag(referenced_phase_22(x + 1j * h, *phys, f_ref)) / h
    return t_c + d / (2.0 * math.pi)


def rotating_detector_signal(grid: Grid, modes, phys, d_mpc, ext, t_c, D, pos, rate: float, t_ref: float):
    """Projected signal on a rotating Earth: mode (l, m) at frequency f is
    emitted at its stationary-phase time t_a(f), when the source (fixed right
    ascension alpha) sits at Earth-fixed longitude alpha - rate (t_a - t_ref);
    its antenna factor and delay are taken there:
    sum_lm A_lm(t_a) h_{l,-m}(f) e^{-2 pi i f (t_c + dt(t_a))}."""
    alpha, dec, psi, iota, phi = ext
    out = np.zeros(grid.n_f, dtype=np.complex128)
    m1, m2 = phys[0], phys[1]
    for (l, m) in modes:
        j0, j1 = mode_band(grid, m, m1, m2)
        if j1 <= j0:
            continue
        j = np.arange(j0, j1)
        f = j * grid.df
        h = waveform_mode(grid, l, m, phys, d_mpc)[j0:j1]
        ta = spa_time(f, m, phys, grid.f_ref, t_c)
        for i in range(0, f.size, 65536):
            sl = slice(i, min(f.size, i + 65536))
            al = alpha - rate * (ta[sl] - t_ref)
            # the frozen pattern's formulas, for an array of longitudes
            e_a = np.stack([-np.sin(al), np.cos(al), np.zeros_like(al)], axis=1)
            e_d = np.stack([-math.sin(dec) * np.cos(al), -math.sin(dec) * np.sin(al),
                            np.full_like(al, math.cos(dec))], axis=1)
            X = -math.cos(psi) * e_a + math.sin(psi) * e_d
            Y = math.sin(psi) * e_a + math.cos(psi) * e_d
            fp = np.einsum("ij,ni,nj->n", D, X, X) - np.einsum("ij,ni,nj->n", D, Y, Y)
            fc = np.einsum("ij,ni,nj->n", D, X, Y) + np.einsum("ij,ni,nj->n", D, Y, X)
            s_hat = np.stack([math.cos(dec) * np.cos(al), math.cos(dec) * np.sin(al),
                              np.full_like(al, math.sin(dec))], axis=1)
            dt = -(s_hat @ pos)
            A = 0.5 * ((fp + 1j * fc) * ylm(l, -m, iota, phi)
                       + (-1.0) ** l * (fp - 1j * fc) * np.conj(ylm(l, m, iota, phi)))
            tau = t_c + dt
            n = np.rint(tau * grid.fs).astype(np.int64)
            rem = tau - n / grid.fs
            frac = ((j[sl] * (n % grid.n_s)) % grid.n_s).astype(np.float64) / grid.n_s
            out[j0 + i:j0 + i + f[sl].size] += A * h[sl] * np.exp(-2j * math.pi * (frac + f[sl] * rem))
    return out


def detector_signal(grid: Grid, modes, phys, d_mpc, ext, t_c, D, pos, rate: float = 0.0, t_ref: float = 0.0):
    """Projected signal (Eq. projected_h_fd): [F+ h+ + Fx hx] e^{-2 pi i f (t_c + dt_k)};
    on a rotating Earth (rate != 0) rotating_detector_signal."""
    if rate != 0.0:
        return rotating_detector_signal(grid, modes, phys, d_mpc, ext, t_c, D, pos, rate, t_ref)
    alpha, dec, psi, iota, phi = ext
    fp, fc = antenna_pattern(D, alpha, dec, psi)
    hp, hc = polarizations(grid, modes, phys, d_mpc, iota, phi)
    tau = t_c + time_delay(pos, alpha, dec)
    return (fp * hp + fc * hc) * shift_factor(grid, tau)


def shift_factor(grid: Grid, tau: float) -> np.ndarray:
    """exp(-2 pi i f_j tau) on the grid.  tau is split into a whole number of
    samples n (whose phase j n / n_s is reduced exactly in integers) plus a
    remainder, so that long segments keep full double precision."""
    n = int(round(tau * grid.fs))
    rem = tau - n / grid.fs
    j = np.arange(grid.n_f, dtype=np.int64)
    frac = ((j * n) % grid.n_s).astype(np.float64) / grid.n_s
    return np.exp(-2j * math.pi * (frac + grid.freqs * rem))
