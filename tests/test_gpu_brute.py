"""Exact ln L on the GPU (rbfl_brute) against the oracle's brute force.

Both sides form each proposal's templates on the frequency grid and sum the
band directly (Eq. logl_basic for the projected signal of Eq.
projected_h_fd); they differ only in summation order, so they agree to
rounding (1e-9 of max(1, |ln L|)).  Also: the zero-noise injection gives
rho^2 / 2 exactly, NaN and unphysical inputs, and the meshfree method's error
against the exact value near the nodes (reported; bounded loosely).
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import likelihood as lk
from oracle import physics as ph
from oracle import startup as su
from paper_2508_04172_amd import rbfl
from paper_2508_04172_amd import workloads as wl

from test_gpu_parity import both, gpu_eval

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def gpu_brute(h, params):
    torch = _torch()
    p = torch.from_numpy(np.ascontiguousarray(params)).cuda()
    n = params.shape[1]
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    h.brute(p.data_ptr(), n, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def oracle_brute(art, h, params, cfg):
    """The oracle's brute force at the physical points the library's own frame
    gives these parameters (so both sides evaluate the same binary; the two
    frames agree only to ~1e-9), -inf if unphysical."""
    fr = h.frame()
    theta = fr["theta_c"][None, :] + params[0:4].T @ fr["vecs"].T
    m1, m2, c1, c2, eta = ph.theta_to_phys(theta.T, cfg.f_low)
    with np.errstate(invalid="ignore"):
        ok = (eta <= 0.25) & (np.abs(c1) <= cfg.chi_max) & (np.abs(c2) <= cfg.chi_max) & np.isfinite(c1 + c2)
    out = np.full(params.shape[1], -np.inf)
    for i in np.flatnonzero(ok):
        out[i] = lk.brute_lnl(art.ev, (m1[i], m2[i], c1[i], c2[i]), params[4:9, i], params[9, i], params[10, i])
    return out


@pytest.mark.parametrize("name", ["cfg1", "small_multi"])
def test_brute_matches_oracle(name):
    cfg, art, h = both(name)
    n = 24
    idx, jit = wl.node_jitter(n, cfg.n_nodes, seed=29)
    qd = wl.queries(cfg, n=n, seed=31)
    params = rbfl.params_soa(h, qd.near_nodes(h.nodes(), idx, jit), cfg.t_trig)
    lg = gpu_brute(h, params)
    lo = oracle_brute(art, h, params, cfg)
    fin = np.isfinite(lo)
    assert np.array_equal(fin, np.isfinite(lg))
    assert fin.sum() >= n // 2
    d = np.abs(lg[fin] - lo[fin])
    print(f"[brute] {name}: {fin.sum()} physical, max |d lnL| vs oracle brute force {d.max():.3e}", flush=True)
    assert np.all(d <= 1e-9 * np.maximum(1.0, np.abs(lo[fin])))


def test_brute_zero_noise_injection():
    """Zero noise, the injection's own parameters: ln L = rho^2 / 2."""
    cfg = wl.CFG1.with_(seg_len=8.0, n_nodes=60, q=60, center_node=True)
    inj = wl.injection_extrinsics(cfg)
    h = rbfl.Handle.from_config(cfg, None, inj)
    qd = wl.queries(cfg, n=1)
    qd.x[:] = 0.0
    qd.dt[:] = 0.0
    qd.ext[0, 4] = inj[4]
    qd.dist_ratio[:] = 1.0
    lg = gpu_brute(h, rbfl.params_soa(h, qd, cfg.t_trig))
    assert lg[0] == pytest.approx(cfg.inj_snr ** 2 / 2, rel=1e-10)


def test_brute_nan_and_unphysical():
    cfg, art, h = both("small_multi")
    qd = wl.queries(cfg, n=3)
    p = rbfl.params_soa(h, qd, cfg.t_trig)
    p[6, 0] = np.nan                   # psi
    p[0:4, 1] = 1e6 * h.frame()["semi"]  # far outside any physical region
    lg = gpu_brute(h, p)
    assert math.isnan(lg[0]) and lg[1] == -np.inf


def test_meshfree_equals_exact_at_nodes():
    """Where the method makes no approximation -- proposals exactly at the
    nodes, t_c on the sample grid, q = N (the basis holds every node's time
    series) -- the meshfree ln L equals the exact one up to the solve's
    rounding."""
    cfg = wl.CFG1.with_(seg_len=8.0, n_nodes=60, q=60)
    inj = wl.injection_extrinsics(cfg)
    h = rbfl.Handle.from_config(cfg, wl.white_noise(cfg), inj)
    n = 60
    qd = wl.queries(cfg, n=n, seed=43)
    qd.x[:] = h.nodes()
    qd.dt[:] = np.round(qd.dt * cfg.fs) / cfg.fs
    params = rbfl.params_soa(h, qd, cfg.t_trig)
    lm = gpu_eval(h, qd, cfg.t_trig)
    lb = gpu_brute(h, params)
    fin = np.isfinite(lm)
    assert fin.sum() >= n // 2
    d = np.abs(lm[fin] - lb[fin])
    print(f"[brute] at the nodes: {fin.sum()} points, max |meshfree - exact| {d.max():.3e}", flush=True)
    assert np.all(d <= 1e-6 * np.maximum(1.0, np.abs(lb[fin])))


def test_meshfree_method_error_near_nodes():
    """The method's own error (interpolation, basis truncation, spline) against
    the exact ln L near the nodes of a small configuration: reported."""
    cfg, art, h = both("small_multi")
    n = 2000
    idx, jit = wl.node_jitter(n, cfg.n_nodes, seed=37)
    qd = wl.queries(cfg, n=n, seed=41).near_nodes(h.nodes(), idx, jit)
    p = rbfl.params_soa(h, qd, cfg.t_trig)
    lm = gpu_eval(h, qd, cfg.t_trig)
    lb = gpu_brute(h, p)
    fin = np.isfinite(lm)
    assert fin.sum() > n // 4 and np.all(np.isfinite(lb[fin]))
    d = np.abs(lm[fin] - lb[fin])
    q = np.quantile(d, [0.5, 0.9, 0.99, 1.0])
    print(f"[brute] small_multi (N=150, q=12) method error: median {q[0]:.3e}, 90% {q[1]:.3e}, "
          f"99% {q[2]:.3e}, max {q[3]:.3e} (|lnL| median {np.median(np.abs(lb[fin])):.1f})", flush=True)


def gpu_parts(h, params):
    torch = _torch()
    p = torch.from_numpy(np.ascontiguousarray(params)).cuda()
    n = params.shape[1]
    out = torch.empty((2, n), dtype=torch.float64, device="cuda")
    h.exact_parts(p.data_ptr(), n, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("name", ["cfg1", "small_multi"])
def test_exact_parts_match_oracle(name):
    """rbfl_exact_parts against the oracle's exact_parts on the same
    proposals: the oracle takes the library's frame (the two frames agree
    only to ~1e-9, and ln L is steep in the physical point), its own basis."""
    cfg, art, h = both(name)
    n = 40
    idx, jit = wl.node_jitter(n, cfg.n_nodes, seed=47)
    qd = wl.queries(cfg, n=n, seed=53).near_nodes(h.nodes(), idx, jit)
    qd.dt[:6] = np.array([-0.2, 0.2, 0.049, -0.049, 0.0, 0.01])   # outside / at the edges of the window
    params = rbfl.params_soa(h, qd, cfg.t_trig)
    params[10, 6] = np.nan
    got = gpu_parts(h, params)
    fr = h.frame()
    art_g = dataclasses.replace(art, frame=su.Frame(theta_c=fr["theta_c"], metric=fr["metric"], vecs=fr["vecs"],
                                                    lam=fr["lam"], semi=fr["semi"]))
    pj, sm = lk.exact_parts(art_g, params[0:4].T, params[4:9].T, params[9], params[10])
    for label, g, o in (("projected", got[0], pj), ("samples", got[1], sm)):
        np.testing.assert_array_equal(np.isnan(g), np.isnan(o))
        np.testing.assert_array_equal(np.isneginf(g), np.isneginf(o))
        fin = np.isfinite(o)
        assert fin.sum() >= n // 3
        d = np.abs(g[fin] - o[fin])
        print(f"[parts] {name} {label}: {fin.sum()} valid, max |d lnL| vs oracle {d.max():.3e}", flush=True)
        assert np.all(d <= 1e-8 * np.maximum(1.0, np.abs(o[fin])))


def test_exact_parts_bracket_the_method_error():
    """The two parts sit between the meshfree and the exact ln L: at the
    nodes with q = N and on-grid times all four agree; near the nodes the
    differences are reported per approximation."""
    cfg = wl.CFG1.with_(seg_len=8.0, n_nodes=60, q=60)
    h = rbfl.Handle.from_config(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg))
    n = 60
    qd = wl.queries(cfg, n=n, seed=43)
    qd.x[:] = h.nodes()
    qd.dt[:] = np.round(qd.dt * cfg.fs) / cfg.fs
    params = rbfl.params_soa(h, qd, cfg.t_trig)
    parts = gpu_parts(h, params)
    lb = gpu_brute(h, params)
    lm = gpu_eval(h, qd, cfg.t_trig)
    fin = np.isfinite(lm)
    assert fin.sum() >= n // 2
    for v in (parts[0], parts[1], lm):
        assert np.all(np.abs(v[fin] - lb[fin]) <= 1e-6 * np.maximum(1.0, np.abs(lb[fin])))
    # near the nodes of the small multi-detector case: report the split
    cfg2, art, h2 = both("small_multi")
    m = 500
    idx, jit = wl.node_jitter(m, cfg2.n_nodes, seed=59)
    q2 = wl.queries(cfg2, n=m, seed=61).near_nodes(h2.nodes(), idx, jit)
    p2 = rbfl.params_soa(h2, q2, cfg2.t_trig)
    pr = gpu_parts(h2, p2)
    ex = gpu_brute(h2, p2)
    mf = gpu_eval(h2, q2, cfg2.t_trig)
    ok = np.isfinite(mf)
    med = lambda a, b: float(np.median(np.abs(a[ok] - b[ok])))
    print(f"[parts] small_multi medians: rbf {med(mf, pr[0]):.3e}, truncation {med(pr[0], pr[1]):.3e}, "
          f"spline {med(pr[1], ex):.3e}, total {med(mf, ex):.3e}", flush=True)


def test_optimised_centre_matches_oracle():
    """The library's gradient ascent and the oracle's Nelder-Mead on the same
    network-SNR objective (one detector, (2,2) mode, zero noise, an offset
    seed): both reach the injection's optimal SNR; the frame is built at the
    optimum."""
    cfg = wl.CFG1.with_(name="cfg1_offset_seed", seg_len=8.0, n_nodes=60, q=20, optimise_centre=True,
                        centre_offset=(0.002, 0.0, 0.01, 0.0))
    inj = wl.injection_extrinsics(cfg)
    h = rbfl.Handle.from_config(cfg, None, inj)
    got = h.centre()
    ev = su.make_event(cfg, None, inj)
    phys, iota, phi, snr_seed, snr_opt = su.optimise_centre(ev, cfg.seed_phys, cfg.match, cfg.half_window)
    m = su.match_22(ev.grid, ev.psd[0], cfg.inj_phys, tuple(got["phys"]))
    print(f"[centre] seed SNR {got['snr_seed']:.6f} (oracle {snr_seed:.6f}), optimum {got['snr_opt']:.6f} "
          f"(oracle {snr_opt:.6f}, bound {cfg.inj_snr}), centre {np.round(got['phys'], 4)}, match to injection {m:.7f}",
          flush=True)
    assert got["snr_seed"] == pytest.approx(snr_seed, rel=1e-9)
    assert got["snr_opt"] == pytest.approx(snr_opt, rel=1e-4)
    assert got["snr_opt"] <= cfg.inj_snr * (1 + 1e-6)
    assert m > 0.9999
    fr = h.frame()
    assert np.allclose(fr["theta_c"], ph.phys_to_theta(got["phys"], cfg.f_low), rtol=1e-12)


def test_rotating_earth_brute_matches_oracle():
    """The exact ln L on a rotating Earth (each mode's frequency at its own
    stationary-phase time, antenna factors and delays there), with an
    injection synthesised the same way, against the oracle's brute force; the
    rate is exaggerated so that an 8 s segment sees the patterns move."""
    cfg = wl.SMALL_MULTI.with_(name="small_rotating", earth_rate=200 * 7.2921150e-5, n_nodes=40, q=8)
    white = wl.white_noise(cfg)
    inj = wl.injection_extrinsics(cfg)
    h = rbfl.Handle.from_config(cfg, white, inj)
    ev = su.make_event(cfg, white, inj)
    assert h.d_ref() == pytest.approx(ev.d_inj, rel=1e-10)
    n = 8
    idx, jit = wl.node_jitter(n, cfg.n_nodes, seed=97)
    qd = wl.queries(cfg, n=n, seed=101).near_nodes(h.nodes(), idx, jit)
    params = rbfl.params_soa(h, qd, cfg.t_trig)
    lg = gpu_brute(h, params)
    fr = h.frame()
    theta = fr["theta_c"][None, :] + params[0:4].T @ fr["vecs"].T
    m1, m2, c1, c2, _ = ph.theta_to_phys(theta.T, cfg.f_low)
    d = []
    for i in range(n):
        if not np.isfinite(lg[i]):
            continue
        lo = lk.brute_lnl(ev, (m1[i], m2[i], c1[i], c2[i]), params[4:9, i], params[9, i], params[10, i])
        d.append(abs(lg[i] - lo) / max(1.0, abs(lo)))
    frozen = dataclasses.replace(ev, earth_rate=0.0)
    i0 = int(np.flatnonzero(np.isfinite(lg))[0])
    l_frozen = lk.brute_lnl(frozen, (m1[i0], m2[i0], c1[i0], c2[i0]), params[4:9, i0], params[9, i0], params[10, i0])
    print(f"[brute] rotating Earth: {len(d)} proposals, max relative |d lnL| vs oracle {max(d):.3e}; "
          f"proposal {i0}: {lg[i0]:.4f} rotating, {l_frozen:.4f} frozen", flush=True)
    assert len(d) >= n // 2 and max(d) <= 1e-9
