"""The GPU ensemble sampler (rbfl_sampler_*) and the prior reweighting
(rbfl_prior_weights) against the oracle: the initial draw and prior-only
steps bit for bit up to rounding (same Philox stream, same moves), a step
on the posterior with the oracle's own ln L, the prior as the stationary
distribution of prior-only runs, a posterior run on a small configuration,
and the reweighting's log weights."""
import dataclasses
import math

import numpy as np
import pytest
from scipy import stats

from oracle import likelihood as lk
from oracle import sampler as sm
from oracle import startup as su
from paper_2508_04172_amd import rbfl
from paper_2508_04172_amd import workloads as wl

from test_gpu_parity import both

pytestmark = pytest.mark.gpu

GAMMA = 2.38 / math.sqrt(22.0)
TABLE1_BOX = (5.0, 20.0, 1.0, 3.0, -0.998, 0.998, -0.05, 0.05)


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def frame_of(h):
    fr = h.frame()
    return su.Frame(theta_c=fr["theta_c"], metric=fr["metric"], vecs=fr["vecs"], lam=fr["lam"], semi=fr["semi"])


def prior_for(cfg, h, d_exp=0.0):
    return sm.Prior(t_lo=cfg.t_trig - cfg.tc_span, t_hi=cfg.t_trig + cfg.tc_span, d_lo=0.5 * h.d_ref(),
                    d_hi=2.0 * h.d_ref(), d_exp=d_exp)


def make_sampler(h, pr, W, seed, prior_only=False, stream=0, anneal_steps=0, beta0=1.0):
    return rbfl.Sampler(h, W, (pr.t_lo, pr.t_hi), (pr.d_lo, pr.d_hi), seed=seed, d_exp=pr.d_exp,
                        p_jump=0.1, prior_only=prior_only, stream=stream, anneal_steps=anneal_steps, beta0=beta0)


def test_initial_walkers_match_oracle():
    cfg, art, h = both("small_multi")
    pr = prior_for(cfg, h)
    W = 256
    s = make_sampler(h, pr, W, seed=11, prior_only=True)
    got = s.walkers_state()
    want = sm.init_walkers(frame_of(h), cfg.f_low, cfg.chi_max, pr, 11, W)
    print(f"[sampler] init: max |d| {np.abs(got[:11] - want).max():.3e}", flush=True)
    s.close()
    np.testing.assert_allclose(got[:11], want, rtol=1e-12, atol=1e-12)
    assert np.all(got[11] == 0.0)


def test_prior_only_steps_match_oracle():
    """Without ln L every decision depends on the prior alone, computed the
    same way on both sides: the walkers after several steps agree to rounding."""
    cfg, art, h = both("small_multi")
    pr = prior_for(cfg, h)
    W = 512
    s = make_sampler(h, pr, W, seed=13, prior_only=True)
    X = s.walkers_state()[:11].copy()
    s.run(4)
    got = s.walkers_state()
    steps, acc = s.stats()
    s.close()
    fr = frame_of(h)

    def lp(P):
        return sm.log_prior(fr, cfg.f_low, cfg.chi_max, pr, P)

    lnl = np.zeros(W)
    lpx = lp(X)
    for step in range(4):
        for half in (0, 1):
            sm.de_half_step(X, lnl, lpx, 13, step, half, GAMMA, 0.1, lambda P: np.zeros(P.shape[1]), lp)
    d = np.abs(got[:11] - X).max()
    print(f"[sampler] prior-only 4 steps: max |d| {d:.3e}, acceptance {acc:.3f}", flush=True)
    assert steps == 4
    np.testing.assert_allclose(got[:11], X, rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("anneal_steps,beta0", [(0, 1.0), (100, 0.01)])
def test_posterior_step_matches_oracle(anneal_steps, beta0):
    """One step on the posterior (plain, and the first step of an annealed
    start, ln L weighted by beta0): the oracle moves the same walkers with its
    own meshfree ln L (at the library's frame); decisions can differ only
    where the two ln L values straddle the acceptance threshold."""
    cfg, art, h = both("small_multi")
    pr = prior_for(cfg, h)
    W = 1024
    s = make_sampler(h, pr, W, seed=5, anneal_steps=anneal_steps, beta0=beta0)
    st0 = s.walkers_state()
    s.run(1)
    got = s.walkers_state()
    s.close()
    fr = frame_of(h)
    art_g = dataclasses.replace(art, frame=fr)

    def lnl_fn(P):
        return lk.meshfree_lnl(art_g, P[0:4].T, P[4:9].T, P[9], P[10])

    def lp(P):
        return sm.log_prior(fr, cfg.f_low, cfg.chi_max, pr, P)

    X = st0[:11].copy()
    lnl = st0[11].copy()
    lpx = lp(X)
    beta = sm.anneal_beta(0, anneal_steps, beta0) if anneal_steps else 1.0
    for half in (0, 1):
        sm.de_half_step(X, lnl, lpx, 5, 0, half, GAMMA, 0.1, lnl_fn, lp, beta=beta)
    same = np.all(np.isclose(got[:11], X, rtol=1e-9, atol=1e-9), axis=0)
    fin = np.isfinite(lnl) & same
    dl = np.abs(got[11][fin] - lnl[fin])
    print(f"[sampler] posterior step: {same.mean():.4f} of walkers identical, max |d lnL| {dl.max():.3e}",
          flush=True)
    assert same.mean() >= 0.98
    assert dl.max() <= 1e-3


def test_prior_only_chain_keeps_the_prior():
    """Prior-only walkers start from the prior; after many moves they must still
    follow it: KS tests of every extrinsic parameter, and of the intrinsic
    radius against rejection samples of the ball and the physical region."""
    cfg, art, h = both("small_multi")
    pr = prior_for(cfg, h)
    W = 4096
    s = make_sampler(h, pr, W, seed=21, prior_only=True)
    s.run(150)
    X = s.walkers_state()[:11]
    steps, acc = s.stats()
    s.close()
    p = {"cos iota": stats.kstest(np.cos(X[7]), "uniform", args=(-1, 2)).pvalue,
         "sin dec": stats.kstest(np.sin(X[5]), "uniform", args=(-1, 2)).pvalue,
         "alpha": stats.kstest(X[4], "uniform", args=(0, 2 * math.pi)).pvalue,
         "psi": stats.kstest(X[6], "uniform", args=(0, math.pi)).pvalue,
         "phi": stats.kstest(X[8], "uniform", args=(0, 2 * math.pi)).pvalue,
         "t_c": stats.kstest(X[9], "uniform", args=(pr.t_lo, pr.t_hi - pr.t_lo)).pvalue,
         "d_L": stats.kstest(X[10], "uniform", args=(pr.d_lo, pr.d_hi - pr.d_lo)).pvalue}
    fr = frame_of(h)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (200000, 4))
    x = x[np.sum(x * x, axis=1) <= 1.0]
    ok, _ = su.physical_mask(fr, x, cfg.f_low, cfg.chi_max)
    ref = np.linalg.norm(x[ok], axis=1)
    r = np.linalg.norm(X[0:4].T / fr.semi[None, :], axis=1)
    p["radius"] = stats.ks_2samp(r, ref).pvalue
    p["x3"] = stats.ks_2samp(X[3] / fr.semi[3], x[ok][:, 3]).pvalue
    print(f"[sampler] prior-only {steps} steps, acceptance {acc:.3f}, KS p-values "
          + ", ".join(f"{k} {v:.3f}" for k, v in p.items()), flush=True)
    assert 0.05 < acc < 0.95
    assert min(p.values()) > 1e-4


def test_smc_first_stage_matches_oracle():
    """The first tempered stage: the library's beta increment and evidence
    increment from its walkers' ln L equal the oracle's smc_stage on the same
    values; after the resampling and one move the walkers agree with the
    oracle's (its own ln L) up to decisions at the acceptance threshold."""
    cfg, art, h = both("squeezed")
    pr = prior_for(cfg, h)
    W = 2048
    s = make_sampler(h, pr, W, seed=9)
    st0 = s.walkers_state()
    lz, stages, beta = s.smc(ess_frac=0.5, moves=1, max_stages=1)
    got = s.walkers_state()
    s.close()
    db, idx, dz = sm.smc_stage(st0[11], 0.0, 0.5, 9, 0)
    print(f"[sampler] SMC stage 1: beta {beta:.6g} (oracle {db:.6g}), log Z {lz:.6f} (oracle {dz:.6f})", flush=True)
    assert stages == 1
    assert beta == pytest.approx(db, rel=1e-12) and lz == pytest.approx(dz, rel=1e-12, abs=1e-12)
    fr = frame_of(h)
    art_g = dataclasses.replace(art, frame=fr)
    X = st0[:11][:, idx].copy()
    lnl = st0[11][idx].copy()

    def lp(P):
        return sm.log_prior(fr, cfg.f_low, cfg.chi_max, pr, P)

    lpx = lp(X)
    for half in (0, 1):
        sm.de_half_step(X, lnl, lpx, 9, 0, half, GAMMA, 0.1,
                        lambda P: lk.meshfree_lnl(art_g, P[0:4].T, P[4:9].T, P[9], P[10]), lp, beta=db)
    same = np.all(np.isclose(got[:11], X, rtol=1e-9, atol=1e-9), axis=0)
    print(f"[sampler] after resampling and one move: {same.mean():.4f} of walkers identical", flush=True)
    assert same.mean() >= 0.98


def test_smc_posterior_and_reweighting():
    """Parameter estimation on the small 3-detector case with the squeezed
    ellipsoid: a tempered SMC start from the prior reaches beta = 1, the
    walkers sit at the likelihood peak (t_c within a millisecond or two of
    the injection), and the samples reweighted to Table I's mass and spin box
    keep a usable effective size; the log weights match the oracle's."""
    torch = _torch()
    cfg, art, h = both("squeezed")
    pr = prior_for(cfg, h)
    W = 8192
    stream = torch.cuda.current_stream().cuda_stream
    s = make_sampler(h, pr, W, seed=2, stream=stream)
    lz, stages, beta = s.smc(ess_frac=0.5, moves=10, max_stages=100, stream=stream)
    slots = 4
    chain = torch.empty((12, slots, W), dtype=torch.float64, device="cuda")
    s.run(100, thin=25, chain_ptr=chain.data_ptr(), slots=slots, stream=stream)
    torch.cuda.synchronize()
    steps, acc = s.stats()
    s.close()
    C = chain.cpu().numpy()
    lnl = C[11].ravel()
    tc = C[9].ravel()
    inj_lnl = h_lnl_at_injection(h, cfg)
    print(f"[sampler] SMC: {stages} stages to beta {beta}, log Z {lz:.2f}, {steps} steps, acceptance {acc:.3f}, "
          f"ln L median {np.median(lnl):.2f} (injection {inj_lnl:.2f}), "
          f"|t_c - t_inj| median {np.median(np.abs(tc - cfg.t_trig)) * 1e3:.2f} ms", flush=True)
    assert beta == 1.0 and stages < 100
    assert np.median(lnl) > inj_lnl - 15.0
    assert np.median(np.abs(tc - cfg.t_trig)) < 2e-3
    logw = torch.empty(slots * W, dtype=torch.float64, device="cuda")
    n_eff = rbfl.prior_weights(h, chain.data_ptr(), slots * W, slots * W, TABLE1_BOX, 0.0, logw.data_ptr(),
                               stream=stream)
    lw = logw.cpu().numpy()
    print(f"[sampler] reweighting to Table I's box: N_eff {n_eff:.1f} of {lw.size}, "
          f"{np.isfinite(lw).mean():.3f} inside", flush=True)
    assert n_eff > 50
    P = C[:11].reshape(11, -1)[:, :400]
    want = sm.log_prior_weights(frame_of(h), cfg.f_low, P, TABLE1_BOX, 0.0)
    fin = np.isfinite(want)
    np.testing.assert_array_equal(fin, np.isfinite(lw[:400]))
    assert np.abs(lw[:400][fin] - want[fin]).max() <= 1e-5


def h_lnl_at_injection(h, cfg):
    torch = _torch()
    inj = wl.injection_extrinsics(cfg)
    p = np.zeros((11, 1))
    p[4:9, 0] = inj
    p[9, 0] = cfg.t_trig
    p[10, 0] = h.d_ref()
    t = torch.from_numpy(p).cuda()
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    h.eval(t.data_ptr(), 1, out.data_ptr(), rbfl.FORM_FP64, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return float(out.cpu()[0])
