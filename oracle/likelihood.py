"""Oracle likelihoods: brute force (Eq. logl_basic), mode-factorised
(Eq. logl_complete, corrected) and the meshfree online stage (Sec. II D).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain float64 numpy.

Reading of Eq. logl_complete used here (the printed form has a Y_lm where
Y_{l,-m} belongs in its first term, drops the real part and the -1/2 of
the second term):

  ln L = sum_k [ r Re sum_a conj(A_ka) z_ka(tau_k)
                 - r^2/2 Re sum_ab conj(A_ka) A_kb sigma_k,ab ],
  A_k,lm = [(F+ + i Fx) Y_{l,-m} + (-1)^l (F+ - i Fx) conj(Y_{lm})] / 2,
  z_ka(tau) = 4 df sum_f conj(h_a) d_k e^{+2 pi i f tau} / S_k,
  sigma_k,ab = 4 df sum_f conj(h_a) h_b / S_k,  r = d_ref / d_L,
  tau_k = t_c + dt_k.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.interpolate import CubicSpline

from . import physics as ph
from .startup import Artefacts, Event, gaussian_kernel, output_layout, poly_matrix


# ----------------------------------------------------------------------------
# Brute force and the exact mode-factorised form
# ----------------------------------------------------------------------------

def brute_lnl(ev: Event, phys, ext, t_c: float, d_l: float) -> float:
    """ln L = sum_k <h_k|d_k> - 1/2 <h_k|h_k> with the projected signal of
    Eq. projected_h_fd (Eq. logl_basic); on a rotating Earth (ev.earth_rate)
    with each mode's antenna factor and delay at its stationary-phase time."""
    total = 0.0
    for k in range(ev.n_det):
        h = ph.detector_signal(ev.grid, ev.modes, phys, d_l, ext, t_c, ev.det_tensor[k], ev.det_pos[k],
                               ev.earth_rate, ev.t_trig)
        total += ph.inner(h, ev.data[k], ev.psd[k], ev.grid) - 0.5 * ph.inner(h, h, ev.psd[k], ev.grid)
    return total


def exact_z(ev: Event, phys, k: int, a: int, tau: float) -> complex:
    """z_ka(tau) by the direct sum over the band (no FFT, no interpolation)."""
    l, m = ev.modes[a]
    h = ph.waveform_mode(ev.grid, l, m, phys, ev.d_inj)
    return ph.overlap(h * ph.shift_factor(ev.grid, tau), ev.data[k], ev.psd[k], ev.grid)


def exact_sigma(ev: Event, phys, k: int) -> np.ndarray:
    hs = [ph.waveform_mode(ev.grid, l, m, phys, ev.d_inj) for (l, m) in ev.modes]
    n = len(hs)
    out = np.zeros((n, n), dtype=np.complex128)
    for a in range(n):
        for b in range(n):
            out[a, b] = ph.overlap(hs[a], hs[b], ev.psd[k], ev.grid)
    return out


def combine(A: np.ndarray, z: np.ndarray, sigma: np.ndarray, r) -> np.ndarray:
    """One detector's term: r Re sum_a conj(A_a) z_a - r^2/2 Re sum_ab conj(A_a) A_b sigma_ab.
    A, z: [..., n]; sigma: [..., n, n]."""
    zt = np.real(np.sum(np.conj(A) * z, axis=-1))
    st = np.real(np.einsum("...a,...b,...ab->...", np.conj(A), A, sigma))
    return r * zt - 0.5 * r * r * st


def band_overlap(a: np.ndarray, b: np.ndarray, psd: np.ndarray, grid, j0: int, j1: int) -> complex:
    """(a|b) over the bins j0 .. j1 - 1 only."""
    sl = slice(j0, j1)
    return complex(4.0 * grid.df * np.sum(np.conj(a[sl]) * b[sl] / psd[sl]))


def band_alpha(ev: Event, alpha, t_c, t_band):
    """Right ascension as the rotating Earth sees it at time t_c + t_band:
    alpha - rate (t_c + t_band - t_trig) (the Earth-fixed frame is taken at
    the trigger time, as in the exact rotating-Earth likelihood)."""
    return alpha - ev.earth_rate * (t_c + t_band - ev.t_trig)


def banded_signal(ev: Event, phys, ext, t_c: float, d_l: float, bands, k: int) -> np.ndarray:
    """The signal the time-banded form models in detector k: in band b every
    mode a takes its antenna factor and delay at its band time t_ba
    (startup.time_bands), sum_a A_a(t_ba) h_a(f) e^{-2 pi i f (t_c + dt(t_ba))}."""
    edges, times = bands
    alpha, dec, psi, iota, phi = ext
    out = np.zeros(ev.grid.n_f, dtype=np.complex128)
    for a, (l, m) in enumerate(ev.modes):
        h = ph.waveform_mode(ev.grid, l, m, phys, d_l)
        for b in range(len(edges) - 1):
            sl = slice(edges[b], edges[b + 1])
            al = band_alpha(ev, alpha, t_c, times[b, a])
            fp, fc = ph.antenna_pattern(ev.det_tensor[k], al, dec, psi)
            tau = t_c + ph.time_delay(ev.det_pos[k], al, dec)
            out[sl] += ph.mode_factor(l, m, fp, fc, iota, phi) * h[sl] * ph.shift_factor(ev.grid, tau)[sl]
    return out


def factorised_lnl_banded(ev: Event, phys, ext, t_c: float, d_l: float, bands) -> float:
    """Eq. logl_complete (corrected reading) with time-banded antenna
    patterns, z and sigma computed exactly over each band's bins: block
    (detector k, band b) is the frozen-pattern form over the band with mode
    a's factor A_ba and delay at its band time.  The overlaps carry no delay,
    so the cross terms between modes drop the phase 2 pi f (dt_ba - dt_bc)
    their delays would give them (the one approximation beyond
    banded_signal: with a single mode the two agree exactly)."""
    edges, times = bands
    alpha, dec, psi, iota, phi = ext
    r = ev.d_inj / d_l
    hs = [ph.waveform_mode(ev.grid, l, m, phys, ev.d_inj) for (l, m) in ev.modes]
    n = len(hs)
    total = 0.0
    for k in range(ev.n_det):
        for b in range(len(edges) - 1):
            A = np.zeros(n, dtype=np.complex128)
            z = np.zeros(n, dtype=np.complex128)
            for a, (l, m) in enumerate(ev.modes):
                al = band_alpha(ev, alpha, t_c, times[b, a])
                fp, fc = ph.antenna_pattern(ev.det_tensor[k], al, dec, psi)
                tau = t_c + ph.time_delay(ev.det_pos[k], al, dec)
                A[a] = ph.mode_factor(l, m, fp, fc, iota, phi)
                z[a] = band_overlap(hs[a] * ph.shift_factor(ev.grid, tau), ev.data[k], ev.psd[k], ev.grid,
                                    edges[b], edges[b + 1])
            sig = np.array([[band_overlap(hs[i], hs[j], ev.psd[k], ev.grid, edges[b], edges[b + 1])
                             for j in range(n)] for i in range(n)])
            total += float(combine(A, z, sig, r))
    return total


def factorised_lnl(ev: Event, phys, ext, t_c: float, d_l: float) -> float:
    """Eq. logl_complete (corrected reading) with z and sigma computed exactly."""
    alpha, dec, psi, iota, phi = ext
    r = ev.d_inj / d_l
    total = 0.0
    for k in range(ev.n_det):
        fp, fc = ph.antenna_pattern(ev.det_tensor[k], alpha, dec, psi)
        tau = t_c + ph.time_delay(ev.det_pos[k], alpha, dec)
        A = np.array([ph.mode_factor(l, m, fp, fc, iota, phi) for (l, m) in ev.modes])
        z = np.array([exact_z(ev, phys, k, a, tau) for a in range(len(ev.modes))])
        total += float(combine(A, z, exact_sigma(ev, phys, k), r))
    return total


# ----------------------------------------------------------------------------
# Sub-sample time interpolation (Sec. II D: cubic spline through ~10 samples)
# ----------------------------------------------------------------------------

def spline_table() -> np.ndarray:
    """w[s][p]: the not-a-knot cubic spline through 10 samples at abscissae
    0..9, evaluated at 4 + f (f in [0, 1)), equals sum_s w_s(f) y_s with
    w_s(f) = sum_p w[s][p] f^p.  Obtained by splining each unit vector."""
    xs = np.arange(10.0)
    tab = np.zeros((10, 4))
    for s in range(10):
        e = np.zeros(10)
        e[s] = 1.0
        c = CubicSpline(xs, e, bc_type="not-a-knot").c[:, 4]   # (x-4)^3, ^2, ^1, ^0
        tab[s] = c[::-1]
    return tab


def spline_weights(f: np.ndarray, tab: np.ndarray) -> np.ndarray:
    """[n][10] weights at fractional offsets f."""
    f = np.asarray(f, dtype=np.float64)
    return tab[None, :, 0] + f[:, None] * (tab[None, :, 1] + f[:, None] * (tab[None, :, 2] + f[:, None] * tab[None, :, 3]))


# ----------------------------------------------------------------------------
# Vectorised extrinsic factors
# ----------------------------------------------------------------------------

def antenna_patterns(D: np.ndarray, alpha, dec, psi):
    alpha, dec, psi = (np.asarray(v, dtype=np.float64) for v in (alpha, dec, psi))
    zero = np.zeros_like(alpha)
    e_a = np.stack([-np.sin(alpha), np.cos(alpha), zero], axis=-1)
    e_d = np.stack([-np.sin(dec) * np.cos(alpha), -np.sin(dec) * np.sin(alpha), np.cos(dec)], axis=-1)
    X = -np.cos(psi)[..., None] * e_a + np.sin(psi)[..., None] * e_d
    Y = np.sin(psi)[..., None] * e_a + np.cos(psi)[..., None] * e_d
    fp = np.einsum("ij,ni,nj->n", D, X, X) - np.einsum("ij,ni,nj->n", D, Y, Y)
    fc = np.einsum("ij,ni,nj->n", D, X, Y) + np.einsum("ij,ni,nj->n", D, Y, X)
    return fp, fc


def time_delays(pos: np.ndarray, alpha, dec):
    s = np.stack([np.cos(dec) * np.cos(alpha), np.cos(dec) * np.sin(alpha), np.sin(dec)], axis=-1)
    return -(s @ pos)


def ylm_vec(l, m, iota, phi):
    iota = np.asarray(iota, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    d = np.array([ph.wigner_d(l, m, 2, float(b)) for b in iota.ravel()]).reshape(iota.shape)
    return math.sqrt((2 * l + 1) / (4.0 * math.pi)) * d * np.exp(1j * m * phi)


def mode_factors(modes, fp, fc, iota, phi) -> np.ndarray:
    """[n_q][n_modes] A_{k,lm} for one detector."""
    out = []
    for (l, m) in modes:
        out.append(0.5 * ((fp + 1j * fc) * ylm_vec(l, -m, iota, phi)
                          + (-1.0) ** l * (fp - 1j * fc) * np.conj(ylm_vec(l, m, iota, phi))))
    return np.stack(out, axis=-1)


# ----------------------------------------------------------------------------
# Meshfree online stage
# ----------------------------------------------------------------------------

def rbf_eval(art: Artefacts, x: np.ndarray) -> np.ndarray:
    """Y(x) = sum_i W_i phi(|x - x_i|) + sum_j W_{N+j} p_j(x) (Eq. rbfcoeff), [n][K]."""
    basis = np.concatenate([gaussian_kernel(x, art.x_nodes, art.eps), poly_matrix(x, art.degree)], axis=1)
    return basis @ art.W


def domain(art: Artefacts, x: np.ndarray) -> np.ndarray:
    """Inside the unit ball (the ellipsoid) and physical (eta <= 1/4, |chi| <= chi_max)."""
    from .startup import physical_mask
    inside = np.sum(x * x, axis=1) <= 1.0
    ok, _ = physical_mask(art.frame, x, art.ev.grid.f_low, art.cfg.chi_max)
    return inside & ok


def virtual_detectors(art: Artefacts, alpha, t_c):
    """The blocks of interpolated outputs, each with its detector and the
    right ascensions its modes see, grouped: without time bands block k is
    detector k with the source's alpha for all modes (patterns frozen,
    Sec. II B); with B time bands block v = k B + b is detector k over band
    b, mode a at band_alpha(alpha, t_c, t_ba).  Returns [(detector,
    [(alpha, mode indices)])]."""
    ev = art.ev
    n_modes = len(ev.modes)
    if art.bands is None:
        return [(k, [(alpha, list(range(n_modes)))]) for k in range(ev.n_det)]
    times = art.bands[1]
    return [(k, [(band_alpha(ev, alpha, t_c, times[b, a]), [a]) for a in range(n_modes)])
            for k in range(ev.n_det) for b in range(times.shape[0])]


def meshfree_parts(art: Artefacts, delta_e: np.ndarray, ext: np.ndarray, t_c: np.ndarray, d_l: np.ndarray,
                   Y: np.ndarray | None = None):
    """Online stage for a batch.  delta_e: [n][4] displacement along the
    eigen-axes; ext: [n][5] (alpha, dec, psi, iota, phi); t_c, d_l: [n].
    Returns (ln L [n] with -inf outside the domain or the time window,
    z [n][n_v][n_modes], sigma [n][n_v][n][n], valid mask), n_v the
    detectors or, with time bands, the (detector, band) blocks."""
    ev = art.ev
    x = delta_e / art.frame.semi[None, :]
    n_q = x.shape[0]
    valid = domain(art, x)
    if Y is None:
        Y = rbf_eval(art, x)
    n_modes = len(ev.modes)
    alpha, dec, psi, iota, phi = (ext[:, i] for i in range(5))
    blocks = virtual_detectors(art, alpha, t_c)
    K, coef_off, sig_off = output_layout(len(blocks), n_modes, art.q)
    tab = spline_table()
    T = art.basis.shape[2]
    r = art.d_ref / d_l
    lnl = np.zeros(n_q)
    zs = np.zeros((n_q, len(blocks), n_modes), dtype=np.complex128)
    sigs = np.zeros((n_q, len(blocks), n_modes, n_modes), dtype=np.complex128)
    for k, (det, groups) in enumerate(blocks):
        A = np.zeros((n_q, n_modes), dtype=np.complex128)
        for al, members in groups:
            # antenna factors and arrival-time stencil of the modes that see
            # right ascension al in block k
            fp, fc = antenna_patterns(ev.det_tensor[det], al, dec, psi)
            A_all = mode_factors(ev.modes, fp, fc, iota, phi)
            s = (t_c + time_delays(ev.det_pos[det], al, dec) - ev.t_trig) * ev.grid.fs + art.half_w
            n0 = np.floor(s)
            f = s - n0
            n0 = n0.astype(np.int64)
            ok = (n0 >= 4) & (n0 <= T - 6)
            valid &= ok
            n0c = np.where(ok, n0, 4)
            w = spline_weights(f, tab)                                   # [n][10]
            rows = n0c[:, None] + np.arange(-4, 6)[None, :]              # [n][10]
            for a in members:
                A[:, a] = A_all[:, a]
                o = coef_off[k][a]
                C = Y[:, o:o + 2 * art.q:2] + 1j * Y[:, o + 1:o + 2 * art.q:2]
                btilde = np.einsum("ns,nsi->ni", w, art.basis[k, a][rows])
                zs[:, k, a] = np.sum(C * btilde, axis=1)
        o = sig_off[k]
        for a in range(n_modes):
            sigs[:, k, a, a] = Y[:, o + a]
        p = o + n_modes
        for a in range(n_modes):
            for b in range(a + 1, n_modes):
                sigs[:, k, a, b] = Y[:, p] + 1j * Y[:, p + 1]
                sigs[:, k, b, a] = Y[:, p] - 1j * Y[:, p + 1]
                p += 2
        lnl += combine(A, zs[:, k], sigs[:, k], r)
    lnl = np.where(valid, lnl, -np.inf)
    return lnl, zs, sigs, valid


def meshfree_lnl(art: Artefacts, delta_e, ext, t_c, d_l) -> np.ndarray:
    return meshfree_parts(art, delta_e, ext, t_c, d_l)[0]


def exact_parts(art: Artefacts, delta_e, ext, t_c, d_l):
    """The online stage's approximations taken one at a time (Sec. II D).
    At each proposal the quantities the interpolants stand for are computed
    exactly, with the start-up's own definitions applied to the proposal's
    template: z at the window samples and the mode overlaps.  Returns two
    ln L arrays (-inf / NaN as meshfree_lnl):
      projected: the window series projected on the time basis (exact SVD
                 coefficients) and the exact overlaps, through the online
                 stage -- everything but the RBF interpolation;
      samples:   the spline through the exact window samples, no basis --
                 everything but the basis truncation and the RBF."""
    from .startup import node_series_and_overlaps, physical_mask
    if art.bands is not None:
        raise NotImplementedError("exact_parts covers frozen antenna patterns only")
    ev = art.ev
    n_q = delta_e.shape[0]
    x = delta_e / art.frame.semi[None, :]
    valid = domain(art, x)
    nan_in = np.any(np.isnan(np.concatenate([delta_e, ext, t_c[:, None], d_l[:, None]], axis=1)), axis=1)
    idx = np.flatnonzero(valid & ~nan_in)
    n_modes = len(ev.modes)
    K, coef_off, sig_off = output_layout(ev.n_det, n_modes, art.q)
    T = art.basis.shape[2]
    Z = np.zeros((ev.n_det, n_modes, n_q, T), dtype=np.complex128)
    S = np.zeros((ev.n_det, n_q, n_modes, n_modes), dtype=np.complex128)
    if idx.size:
        _, phys = physical_mask(art.frame, x[idx], ev.grid.f_low, art.cfg.chi_max)
        z, sig = node_series_and_overlaps(ev, phys, art.cfg.half_window)
        Z[:, :, idx] = z
        S[:, idx] = sig
    # outputs in the interpolants' layout, from the exact series and overlaps
    Y = np.zeros((n_q, K))
    for k in range(ev.n_det):
        for a in range(n_modes):
            Cc = Z[k, a] @ np.conj(art.basis[k, a])            # C_i = sum_t z(t) conj(B[t, i])
            o = coef_off[k][a]
            Y[:, o:o + 2 * art.q:2] = Cc.real
            Y[:, o + 1:o + 2 * art.q:2] = Cc.imag
        o = sig_off[k]
        for a in range(n_modes):
            Y[:, o + a] = S[k, :, a, a].real
        p = o + n_modes
        for a in range(n_modes):
            for b in range(a + 1, n_modes):
                Y[:, p] = S[k, :, a, b].real
                Y[:, p + 1] = S[k, :, a, b].imag
                p += 2
    projected = meshfree_parts(art, delta_e, ext, t_c, d_l, Y=Y)[0]
    # spline through the exact samples
    tab = spline_table()
    r = art.d_ref / d_l
    alpha, dec, psi, iota, phi = (ext[:, i] for i in range(5))
    samples = np.zeros(n_q)
    ok_all = valid.copy()
    for k in range(ev.n_det):
        fp, fc = antenna_patterns(ev.det_tensor[k], alpha, dec, psi)
        s = (t_c + time_delays(ev.det_pos[k], alpha, dec) - ev.t_trig) * ev.grid.fs + art.half_w
        with np.errstate(invalid="ignore"):
            n0 = np.floor(s)
        f = s - n0
        ok = np.isfinite(n0) & (n0 >= 4) & (n0 <= T - 6)
        ok_all &= ok
        n0c = np.where(ok, n0, 4).astype(np.int64)
        w = spline_weights(np.where(ok, f, 0.0), tab)
        rows = n0c[:, None] + np.arange(-4, 6)[None, :]
        z = np.stack([np.sum(w * np.take_along_axis(Z[k, a], rows, axis=1), axis=1) for a in range(n_modes)], axis=-1)
        A = mode_factors(ev.modes, fp, fc, iota, phi)
        samples += combine(A, z, S[k], r)
    samples = np.where(ok_all, samples, -np.inf)
    samples = np.where(nan_in, np.nan, samples)
    projected = np.where(nan_in, np.nan, projected)
    return projected, samples


def query_params(art: Artefacts, qd) -> tuple:
    """Turn a normalised query draw into the paper's coordinates with this
    side's own frame and reference distance."""
    delta_e = qd.x * art.frame.semi[None, :]
    return delta_e, qd.ext, art.ev.t_trig + qd.dt, art.d_ref * qd.dist_ratio
