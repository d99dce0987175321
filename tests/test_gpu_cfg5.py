"""The third-generation-like workload at full size: 2048 s at 4096 Hz from
5 Hz, a co-located 60-degree triangle, five modes, SNR 200, N = 3000 nodes,
q = 80, K = 2475.  The oracle cannot run its start-up at this size (45,000
transforms of 8.4 M points), so it checks samples one by one: the frame and
the nodes, the overlap time series and mode overlaps at three nodes, and the
exact ln L at two proposals; the interpolant's exactness at the nodes is
checked as a property.  The method's error against the exact ln L and the
surrogate's held-out check are reported."""
import time

import numpy as np
import pytest

from full_size import handle
from oracle import likelihood as lk
from oracle import physics as ph
from oracle import startup as su
from paper_2508_04172_amd import rbfl
from paper_2508_04172_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def cfg5():
    cfg, h = handle("cfg5")          # shared with the eval-parity tier: one start-up per process
    print("[cfg5] oracle event", flush=True)
    ev = su.make_event(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg))
    return cfg, h, ev


def gpu_call(h, fn, params):
    torch = _torch()
    p = torch.from_numpy(np.ascontiguousarray(params)).cuda()
    n = params.shape[1]
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    fn(p.data_ptr(), n, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.timeout(1200)
def test_cfg5_frame_nodes_and_series(cfg5):
    cfg, h, ev = cfg5
    assert h.d_ref() == pytest.approx(ev.d_inj, rel=1e-10)
    assert h.f_ref() == pytest.approx(ev.grid.f_ref, rel=1e-12)
    g = su.metric(ev.grid, ev.psd[0], cfg.seed_phys)
    fr = su.frame(g, ph.phys_to_theta(cfg.seed_phys, ev.grid.f_low), cfg.match)
    frg = h.frame()
    assert np.allclose(frg["theta_c"], fr.theta_c, rtol=1e-13)
    assert np.allclose(frg["semi"], fr.semi, rtol=1e-8)
    x, phys = su.place_nodes(fr, cfg.n_nodes, ev.grid.f_low, cfg.chi_max, cfg.center_node)
    assert np.allclose(h.nodes(), x, rtol=0, atol=1e-15)
    idx = np.array([0, 1234, cfg.n_nodes - 1])
    print("[cfg5] oracle series at 3 nodes", flush=True)
    z, sig = su.node_series_and_overlaps(ev, phys[idx], cfg.half_window, workers=8)
    zg = h.z_nodes()[:, :, idx, :]
    scale = np.abs(z).max()
    dz = np.abs(zg - z).max() / scale
    nv = h.node_values()[idx]
    K, coef_off, sig_off = su.output_layout(ev.n_det, len(ev.modes), cfg.q)
    ds = 0.0
    for k in range(ev.n_det):
        for a in range(len(ev.modes)):
            ds = max(ds, np.abs(nv[:, sig_off[k] + a] - sig[k, :, a, a].real).max() / np.abs(sig[k, :, a, a]).max())
    print(f"[cfg5] z at 3 nodes: max |dz| / max |z| {dz:.3e}; sigma diagonals: {ds:.3e}", flush=True)
    assert dz <= 1e-8 and ds <= 1e-10


@pytest.mark.timeout(1200)
def test_cfg5_interpolant_reproduces_the_nodes(cfg5):
    """Eq. rbfcoeff interpolates: at the nodes the FP64 interpolant returns the
    node values (to the solve's conditioning)."""
    cfg, h, ev = cfg5
    nodes = h.nodes()
    sel = np.arange(0, cfg.n_nodes, 47)
    fr = h.frame()
    params = np.zeros((11, sel.size))
    params[0:4] = (nodes[sel] * fr["semi"][None, :]).T
    params[4:9] = np.asarray(wl.injection_extrinsics(cfg))[:, None]
    params[9] = cfg.t_trig
    params[10] = h.d_ref()
    K = h.sizes()["K"]
    torch = _torch()
    p = torch.from_numpy(np.ascontiguousarray(params)).cuda()
    out = torch.empty((sel.size, K), dtype=torch.float64, device="cuda")
    h.interp(p.data_ptr(), sel.size, out.data_ptr(), rbfl.FORM_FP64, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    Y = out.cpu().numpy()
    nv = h.node_values()[sel]
    col = np.abs(h.node_values()).max(axis=0)
    col = np.maximum(col, 1e-9 * col.max())     # columns that vanish in exact arithmetic hold rounding noise
    err = (np.abs(Y - nv) / col[None, :]).max()
    print(f"[cfg5] interpolant at {sel.size} nodes: max column-relative error {err:.3e}", flush=True)
    assert err <= 1e-6


@pytest.mark.timeout(1200)
def test_cfg5_exact_lnl_matches_oracle_and_method_error(cfg5):
    cfg, h, ev = cfg5
    n = 2
    idx, jit = wl.node_jitter(n, cfg.n_nodes, seed=71)
    qd = wl.queries(cfg, n=n, seed=73).near_nodes(h.nodes(), idx, jit)
    params = rbfl.params_soa(h, qd, cfg.t_trig)
    lb = gpu_call(h, h.brute, params)
    lm = gpu_call(h, lambda p, n_, o, s: h.eval(p, n_, o, rbfl.FORM_FP64, s), params)
    fr = h.frame()
    theta = fr["theta_c"][None, :] + params[0:4].T @ fr["vecs"].T
    m1, m2, c1, c2, _ = ph.theta_to_phys(theta.T, cfg.f_low)
    print("[cfg5] oracle brute force at 2 proposals", flush=True)
    for i in range(n):
        lo = lk.brute_lnl(ev, (m1[i], m2[i], c1[i], c2[i]), params[4:9, i], params[9, i], params[10, i])
        print(f"[cfg5] proposal {i}: exact GPU {lb[i]:.6f}, oracle {lo:.6f}, meshfree {lm[i]:.6f}", flush=True)
        assert abs(lb[i] - lo) <= 1e-9 * max(1.0, abs(lo))
    # the method's error near the nodes (reported)
    m = 256
    idx, jit = wl.node_jitter(m, cfg.n_nodes, seed=79)
    qd = wl.queries(cfg, n=m, seed=83).near_nodes(h.nodes(), idx, jit)
    params = rbfl.params_soa(h, qd, cfg.t_trig)
    lb = gpu_call(h, h.brute, params)
    lm = gpu_call(h, lambda p, n_, o, s: h.eval(p, n_, o, rbfl.FORM_FP64, s), params)
    fin = np.isfinite(lm)
    d = np.abs(lm[fin] - lb[fin])
    print(f"[cfg5] method error near the nodes: {fin.sum()} valid, median {np.median(d):.3e}, max {d.max():.3e} "
          f"(|ln L| median {np.median(np.abs(lb[fin])):.1f})", flush=True)
    assert fin.sum() > 0 and np.all(np.isfinite(lb[fin]))
    # ln L finished inside the contraction (the order the autotuner picks at
    # this size) agrees with the default order to rounding
    h.fuse_epilogue(True)
    try:
        lf = gpu_call(h, lambda p, n_, o, s: h.eval(p, n_, o, rbfl.FORM_FP64, s), params)
    finally:
        h.fuse_epilogue(False)
    assert np.array_equal(fin, np.isfinite(lf))
    df = np.abs(lf[fin] - lm[fin]).max()
    print(f"[cfg5] ln L inside the contraction vs the default order: max |d| {df:.3e}", flush=True)
    assert df <= 1e-9 * max(1.0, np.abs(lm[fin]).max())


@pytest.mark.timeout(1200)
def test_cfg5_surrogate_reported(cfg5):
    """The learned form on this workload (MLP 4 -> 256 -> 256 -> K trained by
    the library's kernels on proposals the FP64 interpolant labels): its
    held-out check against 1e-3 in ln L (at SNR 200, 5e-8 relative) is
    reported; when it fails, the surrogate form returns the interpolant's
    ln L exactly."""
    torch = _torch()
    cfg, h, ev = cfg5
    K = h.sizes()["K"]
    hidden = 256
    z = wl.mlp_normals(rbfl.mlp_param_count(4, hidden, K))

    def dev(m, seed):
        idx, jit = wl.node_jitter(m, cfg.n_nodes, seed=seed)
        qd = wl.queries(cfg, n=m, seed=seed).near_nodes(h.nodes(), idx, jit)
        return torch.from_numpy(np.ascontiguousarray(rbfl.params_soa(h, qd, cfg.t_trig))).cuda()

    tr = dev(100000, 5)
    ho = dev(4096, 6)
    st = h.surrogate_train(z, tr.data_ptr(), 100000, ho.data_ptr(), 4096, hidden=hidden, batch=1024, epochs=10,
                           lr=1e-3, threshold=1e-3)
    print(f"[cfg5] surrogate: {st}", flush=True)
    assert st["last_loss"] < st["first_loss"]
    q = dev(2048, 7)
    sp = torch.cuda.current_stream().cuda_stream
    a = torch.empty(2048, dtype=torch.float64, device="cuda")
    b = torch.empty(2048, dtype=torch.float64, device="cuda")
    h.eval(q.data_ptr(), 2048, a.data_ptr(), rbfl.FORM_FP64, sp)
    h.eval(q.data_ptr(), 2048, b.data_ptr(), rbfl.FORM_SURROGATE, sp)
    torch.cuda.synchronize()
    if not st["accepted"]:
        assert torch.equal(torch.nan_to_num(a, neginf=0.0), torch.nan_to_num(b, neginf=0.0))


@pytest.mark.timeout(1200)
def test_cfg5_rotating_earth_reported():
    """The meshfree method freezes the antenna patterns at t_c (Sec. II B); the
    third-generation signal lasts ~28 minutes from 5 Hz, over which the Earth
    turns by ~7 degrees.  With the injection and the exact ln L on a rotating
    Earth (sidereal rate), the meshfree ln L's error near the nodes is
    reported beside the frozen case's, and the exact ln L with and without
    rotation at the same proposals."""
    torch = _torch()
    cfg = wl.CFG5.with_(name="cfg5_rotating", earth_rate=7.2921150e-5)
    h = rbfl.Handle.from_config(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg))
    m = 256
    idx, jit = wl.node_jitter(m, cfg.n_nodes, seed=79)
    qd = wl.queries(cfg, n=m, seed=83).near_nodes(h.nodes(), idx, jit)
    params = rbfl.params_soa(h, qd, cfg.t_trig)
    lb = gpu_call(h, h.brute, params)
    lm = gpu_call(h, lambda p, n_, o, s: h.eval(p, n_, o, rbfl.FORM_FP64, s), params)
    fin = np.isfinite(lm)
    d = np.abs(lm[fin] - lb[fin])
    print(f"[cfg5] rotating Earth: meshfree (frozen patterns) vs exact, {fin.sum()} valid: median {np.median(d):.3e}, "
          f"90% {np.quantile(d, 0.9):.3e}, max {d.max():.3e} (|ln L| median {np.median(np.abs(lb[fin])):.1f})",
          flush=True)
    assert fin.sum() > 0 and np.all(np.isfinite(lb[fin]))
