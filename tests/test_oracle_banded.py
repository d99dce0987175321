"""Pins of the oracle's time-banded antenna patterns (the meshfree
likelihood for long signals on a rotating Earth; Sec. II B freezes the
patterns, Sec. IV names their time dependence as the next step).

Reading: the frequency axis is cut into B bands holding equal shares of the
centre template's (2,2) gravitational-wave phase; in band b mode a takes its
antenna factor and delay at one time t_ba, the f^2-weighted mean of its own
stationary-phase times over its bins in the band.  Each (detector, band) is
then one more block of Eq. logl_complete's terms, with band-restricted z and
sigma and per-mode factors.
"""
import math

import numpy as np
import pytest

from oracle import likelihood as lk
from oracle import physics as ph
from oracle import startup as su
from paper_2508_04172_amd import workloads as wl

TINY_MULTI = wl.SMALL_MULTI.with_(name="tiny_multi_banded", seg_len=4.0, fs=1024.0, n_nodes=60, q=10,
                                  n_queries=200)


def _ext(rng):
    return np.array([rng.uniform(0, 6.28), rng.uniform(-1.2, 1.2), rng.uniform(0, 3), rng.uniform(0.1, 3),
                     rng.uniform(0, 6)])


def test_bands_hold_equal_shares_of_the_gw_phase():
    cfg = TINY_MULTI.with_(modes=wl.ALL_MODES)
    ev = su.make_event(cfg, None, wl.injection_extrinsics(cfg))
    B = 4
    edges, times = su.time_bands(ev.grid, ev.psd[0], cfg.seed_phys, ev.modes, B)
    assert edges[0] == ev.grid.j_lo and edges[-1] == ev.grid.j_hi
    assert np.all(np.diff(edges) > 0) and times.shape == (B, 5)
    m1, m2 = cfg.seed_phys[0], cfg.seed_phys[1]
    j0, j1 = ph.mode_band(ev.grid, 2, m1, m2)
    f = np.arange(j0, j1) * ev.grid.df
    # the GW phase 2 pi f t(f) - Psi(f) by a plain trapezoid sum of
    # 2 pi f dt along the track (not its closed form): each inner edge is where
    # the running share crosses b / B, to within the bins' own step
    t = ph.spa_time(f, 2, cfg.seed_phys, ev.grid.f_ref, 0.0)
    run = np.concatenate([[0.0], np.cumsum(math.pi * (f[1:] + f[:-1]) * np.diff(t))])
    share = run / run[-1]
    for b in range(1, B):
        i = edges[b] - j0
        assert share[i - 1] <= b / B + 1e-6 and share[i] >= b / B - 1e-6
    # mode a's band time: its stationary-phase times over its bins in the band,
    # weighted by f^(-1/3) / S, so it lies inside their range; a mode absent
    # from a band has time 0
    for a, (l, m) in enumerate(ev.modes):
        a0, a1 = ph.mode_band(ev.grid, m, m1, m2)
        for b in range(B):
            lo, hi = max(edges[b], a0), min(edges[b + 1], a1)
            if hi <= lo:
                assert times[b, a] == 0.0
                continue
            fb = np.arange(lo, hi) * ev.grid.df
            tb = ph.spa_time(fb, m, cfg.seed_phys, ev.grid.f_ref, 0.0)
            assert tb.min() <= times[b, a] <= tb.max()
            # mode m at f is the (2,2) track at 2 f / m
            assert tb[0] == pytest.approx(ph.spa_time(np.array([2 * fb[0] / m]), 2, cfg.seed_phys,
                                                      ev.grid.f_ref, 0.0)[0], rel=1e-12)


def test_banded_equals_frozen_without_rotation():
    """Bands partition the bins, so with a zero rotation rate the banded form
    is the frozen Eq. logl_complete exactly (sums regrouped)."""
    cfg = TINY_MULTI.with_(modes=wl.ALL_MODES)
    ev = su.make_event(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg))
    bands = su.time_bands(ev.grid, ev.psd[0], cfg.seed_phys, ev.modes, 3)
    rng = np.random.default_rng(3)
    for _ in range(3):
        ext = _ext(rng)
        tc = ev.t_trig + rng.uniform(-0.01, 0.01)
        a = lk.factorised_lnl(ev, cfg.inj_phys, ext, tc, ev.d_inj * 1.2)
        b = lk.factorised_lnl_banded(ev, cfg.inj_phys, ext, tc, ev.d_inj * 1.2, bands)
        assert b == pytest.approx(a, rel=1e-11, abs=1e-10)


def test_banded_factorisation_of_one_mode_is_its_banded_signal():
    """With one mode the overlaps have no cross terms, so the factorised
    banded form is exactly <h|d> - <h|h>/2 of the signal it models (each
    band's bins with the mode's antenna factor and delay at its band time)."""
    cfg = TINY_MULTI.with_(modes=((3, 3),), earth_rate=3e-2)
    ev = su.make_event(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg))
    bands = su.time_bands(ev.grid, ev.psd[0], cfg.seed_phys, ev.modes, 5)
    rng = np.random.default_rng(8)
    for _ in range(3):
        ext = _ext(rng)
        tc = ev.t_trig + rng.uniform(-0.01, 0.01)
        d = ev.d_inj * 0.9
        want = 0.0
        for k in range(ev.n_det):
            h = lk.banded_signal(ev, cfg.inj_phys, ext, tc, d, bands, k)
            want += ph.inner(h, ev.data[k], ev.psd[k], ev.grid) - 0.5 * ph.inner(h, h, ev.psd[k], ev.grid)
        got = lk.factorised_lnl_banded(ev, cfg.inj_phys, ext, tc, d, bands)
        assert got == pytest.approx(want, rel=1e-10, abs=1e-9)
        # and the rotation matters: the frozen form differs
        assert abs(lk.factorised_lnl(ev, cfg.inj_phys, ext, tc, d) - want) > 1e-4


def test_banded_signal_converges_to_the_rotating_signal():
    """All five modes, a 64 s segment holding the whole 41 s signal, rotation
    27 times the sidereal rate: the banded signal's squared distance to the
    exact rotating-Earth signal (every bin's factor and delay at its own
    stationary-phase time), summed over the detectors, falls roughly as 1/B^2
    -- at least 4x per 4x more bands, below 1e-3 of the frozen one at 64."""
    cfg = wl.SMALL_MULTI.with_(name="banded_64s", seg_len=64.0, fs=1024.0, modes=wl.ALL_MODES, earth_rate=2e-3,
                               inj_snr=30.0)
    ev = su.make_event(cfg, None, wl.injection_extrinsics(cfg))
    phys = tuple(cfg.seed_phys)
    ext = np.array([1.3, 0.4, 0.6, 0.9, 2.0])
    tc = ev.t_trig + 0.004
    exact = [ph.detector_signal(ev.grid, ev.modes, phys, ev.d_inj, ext, tc, ev.det_tensor[k], ev.det_pos[k],
                                ev.earth_rate, ev.t_trig) for k in range(ev.n_det)]
    frozen = [ph.detector_signal(ev.grid, ev.modes, phys, ev.d_inj, ext, tc, ev.det_tensor[k], ev.det_pos[k],
                                 0.0, ev.t_trig) for k in range(ev.n_det)]

    def dist2(hs):
        return sum(ph.inner(e - h, e - h, ev.psd[k], ev.grid) for k, (e, h) in enumerate(zip(exact, hs)))

    d_frozen = dist2(frozen)
    d = [dist2([lk.banded_signal(ev, phys, ext, tc, ev.d_inj, su.time_bands(ev.grid, ev.psd[0], phys, ev.modes, B),
                                 k) for k in range(ev.n_det)]) for B in (4, 16, 64)]
    assert d_frozen > 1e-2                      # the rotation matters at this rate
    assert d[0] < d_frozen and d[1] < d[0] / 4 and d[2] < d[1] / 4
    assert d[2] < 1e-3 * d_frozen * 4


def test_banded_meshfree_equals_banded_factorised_at_nodes_full_rank():
    """At a node, with a full-rank basis, the banded online stage reproduces
    the banded factorised ln L (every approximation of the meshfree method is
    exact there: the spline of the window series at a node is the series at
    on-grid arrival times, here all detectors at the Earth's centre)."""
    sites = tuple((0.8, -2.0, az, math.pi / 2, 0.0) for az in (0.3, 1.1, 2.0))
    cfg = TINY_MULTI.with_(n_nodes=40, q=40, center_node=True, sites=sites, earth_rate=1e-3, n_bands=3,
                           modes=((2, 2), (3, 3), (2, 1)))
    art = su.startup(cfg, wl.white_noise(cfg), workers=1)
    ev = art.ev
    assert art.bands is not None and art.W.shape[1] == 3 * 3 * (2 * 40 * 3 + 9)
    rng = np.random.default_rng(5)
    for node in (0, 9, 33):
        ext = _ext(rng)
        d = art.d_ref * 1.3
        tc = ev.t_trig + 3.0 / ev.grid.fs
        got = lk.meshfree_lnl(art, art.x_nodes[node:node + 1] * art.frame.semi, ext[None],
                              np.array([tc]), np.array([d]))[0]
        want = lk.factorised_lnl_banded(ev, tuple(art.phys_nodes[node]), ext, tc, d, art.bands)
        assert got == pytest.approx(want, rel=1e-9, abs=1e-8)
