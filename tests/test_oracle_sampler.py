"""Pins of the sampler oracle: the Philox4x32-10 known-answer vectors of its
authors' distribution, the stationary distribution of the move on targets
with known moments, and the reweighting Jacobian against the forward map."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import physics as ph
from oracle import sampler as sm
from oracle import startup as su
from paper_2508_04172_amd import workloads as wl


def test_philox_known_answers():
    # Random123 known-answer vectors for philox4x32, 10 rounds
    cases = [((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
             ((0xffffffff,) * 4, (0xffffffff, 0xffffffff), (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
             ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
              (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1))]
    for ctr, key, want in cases:
        got = tuple(int(v) for v in sm.philox4x32_10(ctr, key))
        assert got == want


def test_uniforms_in_open_interval_and_uniform():
    u0, u1 = sm.uniform_pair(12345, np.arange(20000), 7, 1, 2)
    u = np.concatenate([u0, u1])
    assert u.min() > 0.0 and u.max() < 1.0
    assert stats.kstest(u, "uniform").pvalue > 1e-3


@pytest.fixture(scope="module")
def frame_tiny():
    cfg = wl.CFG1.with_(name="tiny_frame", seg_len=4.0, fs=1024.0)
    ev = su.make_event(cfg, None, wl.injection_extrinsics(cfg))
    g = su.metric(ev.grid, ev.psd[0], cfg.inj_phys)
    return cfg, su.frame(g, ph.phys_to_theta(cfg.inj_phys, ev.grid.f_low), cfg.match)


def test_de_moves_sample_a_gaussian_and_the_prior(frame_tiny):
    """Stationary distribution of the move: a Gaussian likelihood in Delta e
    (narrow against the ellipsoid, so the prior's edges do not matter) gives
    the Gaussian's moments; the extrinsic parameters, with a flat likelihood,
    follow the prior (cos iota, sin dec, t_c, d uniform)."""
    cfg, fr = frame_tiny
    prior = sm.Prior(t_lo=10.0, t_hi=10.1, d_lo=50.0, d_hi=150.0, d_exp=0.0)
    sig = 0.02 * fr.semi
    W = 1024
    X = sm.init_walkers(fr, cfg.f_low, cfg.chi_max, prior, seed=3, W=W)
    X[0:4] = 0.05 * sig[:, None] * np.random.default_rng(0).standard_normal((4, W))

    def lnl(P):
        return -0.5 * np.sum((P[0:4] / sig[:, None]) ** 2, axis=0)

    def lp(P):
        return sm.log_prior(fr, cfg.f_low, cfg.chi_max, prior, P)

    lnl_x, lp_x = lnl(X), lp(X)
    samples = []
    for step in range(400):
        for half in (0, 1):
            sm.de_half_step(X, lnl_x, lp_x, 3, step, half, 2.38 / math.sqrt(22.0), 0.1, lnl, lp)
        if step >= 150 and step % 10 == 0:
            samples.append(X.copy())
    S = np.concatenate(samples, axis=1)
    for d in range(4):
        assert abs(np.mean(S[d])) < 0.1 * sig[d]
        assert np.std(S[d]) == pytest.approx(sig[d], rel=0.1)
    last = samples[-1]
    assert stats.kstest(np.cos(last[7]), "uniform", args=(-1, 2)).pvalue > 1e-3
    assert stats.kstest(np.sin(last[5]), "uniform", args=(-1, 2)).pvalue > 1e-3
    assert stats.kstest(last[9], "uniform", args=(prior.t_lo, prior.t_hi - prior.t_lo)).pvalue > 1e-3
    assert stats.kstest(last[10], "uniform", args=(prior.d_lo, prior.d_hi - prior.d_lo)).pvalue > 1e-3


def test_reweighting_jacobian_inverts_the_forward_map(frame_tiny):
    """|det d phys / d Theta| (complex step through the inverse map) times
    |det d Theta / d phys| (central differences of Eq. metric_coords) = 1."""
    cfg, fr = frame_tiny
    rng = np.random.default_rng(5)
    x = rng.uniform(-0.3, 0.3, (20, 4))
    ok, phys = su.physical_mask(fr, x, cfg.f_low, cfg.chi_max)
    P = np.zeros((11, ok.sum()))
    P[0:4] = (x[ok] * fr.semi).T
    P[10] = 100.0
    box = (0, 100, 0, 100, -1, 1, -1, 1)
    logw = sm.log_prior_weights(fr, cfg.f_low, P, box, 0.0)
    assert np.all(np.isfinite(logw))
    for i, p in enumerate(phys[ok]):
        J = np.empty((4, 4))
        for m in range(4):
            h = 1e-6 * max(abs(p[m]), 1e-3)
            a, b = p.copy(), p.copy()
            a[m] += h
            b[m] -= h
            J[:, m] = (ph.phys_to_theta(a, cfg.f_low) - ph.phys_to_theta(b, cfg.f_low)) / (2 * h)
        assert logw[i] + math.log(abs(np.linalg.det(J))) == pytest.approx(0.0, abs=1e-6)
    # outside the box, and the distance factor
    assert sm.log_prior_weights(fr, cfg.f_low, P, (0, 1, 0, 1, -1, 1, -1, 1), 0.0)[0] == -np.inf
    assert sm.log_prior_weights(fr, cfg.f_low, P, box, 2.0)[0] == pytest.approx(logw[0] + 2 * math.log(100.0))


def test_log_prior_closed_form(frame_tiny):
    cfg, fr = frame_tiny
    prior = sm.Prior(t_lo=0.0, t_hi=1.0, d_lo=10.0, d_hi=20.0, d_exp=2.0)
    P = np.zeros((11, 3))
    P[5] = [0.3, 0.3, 2.0]          # dec (third out of range)
    P[7] = [1.1, 1.1, 1.1]
    P[9] = [0.5, 1.5, 0.5]          # t_c (second out of range)
    P[10] = [15.0, 15.0, 15.0]
    lp = sm.log_prior(fr, cfg.f_low, cfg.chi_max, prior, P)
    assert lp[0] == pytest.approx(math.log(math.cos(0.3)) + math.log(math.sin(1.1)) + 2 * math.log(15.0))
    assert lp[1] == -np.inf and lp[2] == -np.inf


def test_smc_stage_effective_size_and_systematic_resampling():
    """The chosen increment gives the target effective sample size; every
    walker is copied floor or ceil of W w_i / sum w times (systematic
    resampling); a constant ln L takes the whole remaining step at once and
    adds exactly that constant times the step to log Z."""
    rng = np.random.default_rng(8)
    W = 4000
    lnl = rng.normal(0.0, 30.0, W)
    lnl[:5] = -np.inf
    db, idx, dz = sm.smc_stage(lnl, 0.2, 0.5, 17, 3)
    assert 0.0 < db < 0.8
    w = np.where(np.isfinite(lnl), np.exp(db * (lnl - lnl[np.isfinite(lnl)].max())), 0.0)
    assert w.sum() ** 2 / (w * w).sum() == pytest.approx(0.5 * W, rel=1e-9)
    counts = np.bincount(idx, minlength=W)
    expect = W * w / w.sum()
    assert np.all(counts >= np.floor(expect) - 1e-9) and np.all(counts <= np.ceil(expect) + 1e-9)
    assert np.all(counts[:5] == 0)
    assert dz == pytest.approx(math.log(np.mean(np.exp(db * lnl[5:])) * (W - 5) / W), rel=1e-9)
    db2, idx2, dz2 = sm.smc_stage(np.full(W, 7.0), 0.25, 0.5, 17, 4)
    assert db2 == 0.75 and dz2 == pytest.approx(7.0 * 0.75, rel=1e-14)
    assert np.array_equal(np.sort(idx2), np.arange(W))
