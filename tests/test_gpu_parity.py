"""GPU parity: the HIP library against the FP64 oracle on the same seeded inputs.

Build parity: each side runs its own start-up from the same seeded deviates
and configuration; basis-independent quantities are compared (time series at
the nodes, overlaps, singular values, interpolated overlaps, ln L).  The SVD
basis of both sides follows one phase convention (largest entry of each
right singular vector real positive), so coefficient outputs are compared
too, column by column, relative to the column's scale at the nodes.

Tolerances: the FP64 path must agree within |d ln L| <= 1e-3 absolute; the
interpolated outputs within 1e-6 of each column's node scale.
"""
import math
import sys

import numpy as np
import pytest

from oracle import likelihood as lk
from oracle import startup as su
from paper_2508_04172_amd import rbfl
from paper_2508_04172_amd import workloads as wl

pytestmark = pytest.mark.gpu

CASES = {
    "cfg1": wl.CFG1,
    "small_multi": wl.SMALL_MULTI,
    "ragged_tail": wl.SMALL_MULTI.with_(name="ragged_tail", n_nodes=131, q=7, modes=wl.ALL_MODES, n_queries=1237),
    "squeezed": wl.SMALL_MULTI.with_(name="small_hlv_3mode_squeezed", squeeze=True),
}


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def gpu_eval(h, qd, t_trig, form=rbfl.FORM_FP64):
    torch = _torch()
    p = torch.from_numpy(np.ascontiguousarray(rbfl.params_soa(h, qd, t_trig))).cuda()
    n = len(qd)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    h.eval(p.data_ptr(), n, out.data_ptr(), form, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def gpu_interp(h, qd, t_trig, form=rbfl.FORM_FP64):
    torch = _torch()
    p = torch.from_numpy(np.ascontiguousarray(rbfl.params_soa(h, qd, t_trig))).cuda()
    n = len(qd)
    K = h.sizes()["K"]
    out = torch.empty((n, K), dtype=torch.float64, device="cuda")
    h.interp(p.data_ptr(), n, out.data_ptr(), form, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


_cache = {}


def column_scale(art):
    """Scale of each interpolated column at the nodes, floored at 1e-9 of the
    largest column: a column that vanishes in exact arithmetic (e.g. Im sigma
    between two modes of equal |m|, whose templates share one phase) holds
    only rounding noise on both sides."""
    s = np.abs(art.node_values).max(axis=0)
    return np.maximum(s, 1e-9 * s.max())


def both(name):
    if name not in _cache:
        cfg = CASES[name]
        print(f"[parity] building {name}", flush=True)
        white = wl.white_noise(cfg)
        inj = wl.injection_extrinsics(cfg)
        art = su.startup(cfg, white, inj)
        h = rbfl.Handle.from_config(cfg, white, inj)
        _cache[name] = (cfg, art, h)
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_frame_and_nodes(name):
    cfg, art, h = both(name)
    fr = h.frame()
    assert np.allclose(fr["theta_c"], art.frame.theta_c, rtol=1e-13)
    assert np.allclose(fr["semi"], art.frame.semi, rtol=1e-8)
    assert np.allclose(fr["vecs"], art.frame.vecs, atol=1e-9)
    assert np.allclose(h.nodes(), art.x_nodes, rtol=0, atol=1e-15)
    assert np.allclose(h.node_phys(), art.phys_nodes, rtol=1e-8, atol=1e-9)
    assert h.d_ref() == pytest.approx(art.d_ref, rel=1e-11)
    assert h.f_ref() == pytest.approx(art.ev.grid.f_ref, rel=1e-12) and h.f_ref() > 0.0
    factor, tip = h.squeeze()
    assert factor == pytest.approx(art.squeeze_factor, rel=1e-8)
    if cfg.squeeze:
        assert factor < 1.0 and tip == pytest.approx(cfg.match, abs=1e-9)


@pytest.mark.parametrize("name", list(CASES))
def test_time_series_and_overlaps_at_nodes(name):
    cfg, art, h = both(name)
    z = h.z_nodes()
    scale = np.abs(art.z_nodes).max()
    assert np.abs(z - art.z_nodes).max() <= 1e-8 * scale
    s_gpu = h.singular()
    q = cfg.q
    assert np.allclose(s_gpu[..., :q], art.singular[..., :q], rtol=1e-8)
    nv = h.node_values()
    col_scale = column_scale(art)
    err = np.abs(nv - art.node_values).max(axis=0) / col_scale
    assert err.max() <= 1e-7, f"worst column {int(err.argmax())}: {err.max():.3e}"


@pytest.mark.parametrize("name", list(CASES))
def test_interpolated_outputs(name):
    """Interpolated coefficients and overlaps within 1e-6 of each column's
    scale at the nodes.  Where a column's own cancellation factor
    amp_c = max_x sum_r |B_r(x) W_rc| / scale_c makes that unreachable for
    two independent FP64 pipelines (their node values differ at ~1e-13
    relative, which the interpolant multiplies by amp_c), the bar is
    1e-13 * amp_c instead; the 1e-3 bar on ln L applies unchanged."""
    cfg, art, h = both(name)
    qd = wl.queries(cfg, n=min(cfg.n_queries, 2000))
    Yg = gpu_interp(h, qd, cfg.t_trig)
    Yo = lk.rbf_eval(art, qd.x)
    col_scale = column_scale(art)
    basis = np.concatenate([su.gaussian_kernel(qd.x, art.x_nodes, art.eps), su.poly_matrix(qd.x, art.degree)], 1)
    amp = (np.abs(basis) @ np.abs(art.W)).max(axis=0) / col_scale
    bar = np.maximum(1e-6, 1e-13 * amp)
    err = np.abs(Yg - Yo).max(axis=0) / col_scale
    print(f"[parity] {name}: max column-relative interpolant error {err.max():.3e} "
          f"(cancellation factor up to {amp.max():.2e}; columns held to 1e-6: {(bar == 1e-6).mean():.0%})",
          flush=True)
    assert np.all(err <= bar), f"column {int(np.argmax(err / bar))}: {err.max():.3e}"


@pytest.mark.parametrize("name", list(CASES))
def test_lnl_parity_fp64(name):
    cfg, art, h = both(name)
    qd = wl.queries(cfg, n=min(cfg.n_queries, 3000))
    lg = gpu_eval(h, qd, cfg.t_trig)
    dE, ext, tc, dl = lk.query_params(art, qd)
    lo = lk.meshfree_lnl(art, dE, ext, tc, dl)
    fin_o, fin_g = np.isfinite(lo), np.isfinite(lg)
    assert np.array_equal(fin_o, fin_g), f"domain flags differ at {np.where(fin_o != fin_g)[0][:10]}"
    assert fin_o.sum() > 0
    d = np.abs(lg[fin_o] - lo[fin_o])
    print(f"[parity] {name}: {fin_o.sum()} valid, max |dlnL| {d.max():.3e}, median {np.median(d):.3e}",
          flush=True)
    assert d.max() <= 1e-3


@pytest.mark.parametrize("name", list(CASES))
def test_lnl_parity_near_nodes(name):
    """Proposals next to the nodes: inside the physical part of the ellipsoid,
    where a sampler's proposals concentrate."""
    cfg, art, h = both(name)
    n = min(cfg.n_queries, 3000)
    idx, jit = wl.node_jitter(n, cfg.n_nodes)
    qd = wl.queries(cfg, n=n)
    lg = gpu_eval(h, qd.near_nodes(h.nodes(), idx, jit), cfg.t_trig)
    lo = lk.meshfree_lnl(art, *lk.query_params(art, qd.near_nodes(art.x_nodes, idx, jit)))
    fin = np.isfinite(lo)
    assert np.array_equal(fin, np.isfinite(lg))
    assert fin.mean() > 0.3
    d = np.abs(lg[fin] - lo[fin])
    print(f"[parity] {name} near nodes: {fin.sum()} valid, max |dlnL| {d.max():.3e}", flush=True)
    assert d.max() <= 1e-3


@pytest.mark.parametrize("name", list(CASES))
def test_lnl_parity_fused_epilogue(name):
    """ln L finished inside the FP64 contraction (coefficient-weighted output
    tiles, no interpolated outputs written): the oracle bar, the same domain
    flags, and agreement with the default order to rounding."""
    cfg, art, h = both(name)
    n = min(cfg.n_queries, 3000)
    idx, jit = wl.node_jitter(n, cfg.n_nodes)
    qd = wl.queries(cfg, n=n)
    q_gpu = qd.near_nodes(h.nodes(), idx, jit)
    ref = gpu_eval(h, q_gpu, cfg.t_trig)
    h.fuse_epilogue(True)
    try:
        lg = gpu_eval(h, q_gpu, cfg.t_trig)
    finally:
        h.fuse_epilogue(False)
    lo = lk.meshfree_lnl(art, *lk.query_params(art, qd.near_nodes(art.x_nodes, idx, jit)))
    fin = np.isfinite(lo)
    assert np.array_equal(fin, np.isfinite(lg)) and np.array_equal(np.isnan(ref), np.isnan(lg))
    assert np.array_equal(np.isfinite(ref), np.isfinite(lg))
    d = np.abs(lg[fin] - lo[fin])
    dr = np.abs(lg[fin] - ref[fin]).max()
    print(f"[parity] {name} fused epilogue: max |dlnL| vs oracle {d.max():.3e}, vs default order {dr:.3e}",
          flush=True)
    assert d.max() <= 1e-3
    assert dr <= 1e-9 * max(1.0, np.abs(ref[fin]).max())


@pytest.mark.parametrize("name", ["small_multi", "ragged_tail"])
def test_fp64_tile_variants(name):
    """Every FP64 contraction tile variant (rows + GEMM tiles of several
    shapes and chunk depths, and the fused kernel) sums each output over the
    same rows in the same order, so ln L is identical across variants;
    variant 0 is held to the oracle bar as well."""
    torch = _torch()
    cfg, art, h = both(name)
    n = min(cfg.n_queries, 3000)
    idx, jit = wl.node_jitter(n, cfg.n_nodes)
    qd = wl.queries(cfg, n=n)
    q_gpu = qd.near_nodes(h.nodes(), idx, jit)
    nv = rbfl.variants(rbfl.FORM_FP64)
    outs = []
    for v in range(nv):
        h.set_variant(rbfl.FORM_FP64, v)
        outs.append(torch.from_numpy(gpu_eval(h, q_gpu, cfg.t_trig)))
    h.set_variant(rbfl.FORM_FP64, 0)
    lo = lk.meshfree_lnl(art, *lk.query_params(art, qd.near_nodes(art.x_nodes, idx, jit)))
    fin = np.isfinite(lo)
    assert np.array_equal(fin, np.isfinite(outs[0].numpy()))
    assert np.abs(outs[0].numpy()[fin] - lo[fin]).max() <= 1e-3
    key = lambda t: torch.nan_to_num(t, nan=1.5, neginf=-2.5)
    same = [bool(torch.equal(key(outs[0]), key(o))) for o in outs]
    diff = [float((key(outs[0]) - key(o)).abs().max()) for o in outs]
    print(f"[parity] {name}: {nv} FP64 variants, identical to variant 0: {same}, max |d| {diff}", flush=True)
    assert all(same)


def _full_size_sampled(cfg, capacity, seed):
    """A workload at full size in the benchmark's launch configuration (work
    capacity, autotuned tile and evaluation order); the oracle checks a
    seeded sample of the outputs one by one.  Then the other FP64 evaluation
    order (ln L inside the contraction, or not) on the same proposals: the
    same sample bar, and agreement with the first to rounding."""
    torch = _torch()
    white = wl.white_noise(cfg)
    inj = wl.injection_extrinsics(cfg)
    print(f"[parity] {cfg.name}: GPU start-up", flush=True)
    h = rbfl.Handle.from_config(cfg, white, inj)
    print(f"[parity] {cfg.name}: oracle start-up", flush=True)
    art = su.startup(cfg, white, inj)
    n = cfg.n_queries
    idx, jit = wl.node_jitter(n, cfg.n_nodes)
    qd = wl.queries(cfg, n=n)
    p = torch.from_numpy(np.ascontiguousarray(rbfl.params_soa(h, qd.near_nodes(h.nodes(), idx, jit), cfg.t_trig)))
    p = p.cuda()
    sp = torch.cuda.current_stream().cuda_stream
    h.reserve(capacity)
    tune = h.autotune(p.data_ptr(), n, rbfl.FORM_FP64, sp)
    order = h.pipeline()
    print(f"[parity] {cfg.name}: tile {tune['variant']}, order {order}", flush=True)
    sample = np.random.default_rng(seed).choice(n, 2000, replace=False)
    sample.sort()
    lo = lk.meshfree_lnl(art, *lk.query_params(art, qd.subset(sample).near_nodes(art.x_nodes, idx[sample],
                                                                                 jit[sample])))
    fin = np.isfinite(lo)
    outs = []
    for fused in (order["fused_epilogue"], not order["fused_epilogue"]):
        h.fuse_epilogue(fused)
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        h.eval(p.data_ptr(), n, out.data_ptr(), rbfl.FORM_FP64, sp)
        torch.cuda.synchronize()
        lg = out.cpu().numpy()
        assert np.array_equal(fin, np.isfinite(lg[sample]))
        d = np.abs(lg[sample][fin] - lo[fin])
        print(f"[parity] {cfg.name} full size, ln L inside the contraction {fused}: {fin.sum()} valid of 2000 "
              f"sampled, max |dlnL| {d.max():.3e}", flush=True)
        assert d.max() <= 1e-3
        # properties that hold at any size: finite where inside, -inf elsewhere, never NaN
        assert not np.isnan(lg).any()
        outs.append(lg)
    a, b = outs
    both_fin = np.isfinite(a)
    assert np.array_equal(both_fin, np.isfinite(b))
    assert np.abs(a[both_fin] - b[both_fin]).max() <= 1e-9 * max(1.0, np.abs(a[both_fin]).max())


@pytest.mark.timeout(1200)
def test_cfg2_full_size_sampled():
    """3-detector, 5-mode workload (N = 800, q = 40, 1e6 proposals in one
    launch, as timed by bench.py)."""
    _full_size_sampled(wl.CFG2, 1 << 20, 123)


@pytest.mark.timeout(1200)
def test_cfg3_full_size_sampled():
    """10 Hz single-detector cubic-tail workload (N = 1500, M = 35, q = 60,
    4e6 proposals in launches of 65,536, as timed by bench.py --mixed-cfg3)."""
    _full_size_sampled(wl.CFG3, 65536, 321)


def test_edge_cases():
    cfg, art, h = both("small_multi")
    torch = _torch()
    # empty batch is a no-op
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    h.eval(out.data_ptr(), 0, out.data_ptr())
    # outside the ellipsoid, outside the window, NaN input; in both FP64
    # evaluation orders (ln L inside the contraction or not), and a batch of one
    qd = wl.queries(cfg, n=4)
    qd.x[0] = [1.2, 0.0, 0.0, 0.0]
    qd.dt[1] = 0.049
    p = rbfl.params_soa(h, qd, cfg.t_trig)
    p[5, 2] = np.nan
    pt = torch.from_numpy(np.ascontiguousarray(p)).cuda()
    o = torch.empty(4, dtype=torch.float64, device="cuda")
    one = torch.empty(1, dtype=torch.float64, device="cuda")
    p3 = torch.from_numpy(np.ascontiguousarray(p[:, 3:4])).cuda()
    lo3 = lk.meshfree_lnl(art, *lk.query_params(art, qd.subset(np.array([3]))))[0]
    for fused in (False, True):
        h.fuse_epilogue(fused)
        try:
            lg = gpu_eval(h, qd, cfg.t_trig)
            assert lg[0] == -np.inf and lg[1] == -np.inf
            h.eval(pt.data_ptr(), 4, o.data_ptr())
            h.eval(p3.data_ptr(), 1, one.data_ptr())
            torch.cuda.synchronize()
        finally:
            h.fuse_epilogue(False)
        assert math.isnan(o[2].item()) and o[0].item() == -math.inf and o[1].item() == -math.inf
        if np.isfinite(lo3):
            assert abs(one.item() - lo3) <= 1e-3 and abs(o[3].item() - one.item()) <= 1e-9 * max(1.0, abs(lo3))
        else:
            assert one.item() == lo3
    # an unknown form is an argument error, an unprepared one a state error (on
    # a fresh handle: the cached ones may have been prepared by other tests)
    with pytest.raises(rbfl.RbflError) as e:
        h.eval(pt.data_ptr(), 4, o.data_ptr(), 17)
    assert e.value.code == rbfl.E_INVALID_ARG
    small = wl.CFG1.with_(seg_len=8.0, n_nodes=60, q=10)
    fresh = rbfl.Handle.from_config(small, None, wl.injection_extrinsics(small))
    p2 = torch.from_numpy(np.ascontiguousarray(rbfl.params_soa(fresh, wl.queries(small, n=4), small.t_trig))).cuda()
    for form in (rbfl.FORM_FP32, rbfl.FORM_BF16, rbfl.FORM_SPLIT):
        with pytest.raises(rbfl.RbflError) as e:
            fresh.eval(p2.data_ptr(), 4, o.data_ptr(), form)
        assert e.value.code == rbfl.E_STATE


def test_batch_larger_than_work_space():
    """Batches above the work-space capacity are processed in chunks with the
    same results as one pass."""
    cfg, art, h = both("small_multi")
    qd = wl.queries(cfg, n=70000, seed=9)
    l1 = gpu_eval(h, qd, cfg.t_trig)
    idx = np.arange(0, 70000, 997)
    l2 = gpu_eval(h, qd.subset(idx), cfg.t_trig)
    ok = np.isfinite(l2)
    assert np.array_equal(np.isfinite(l1[idx]), ok)
    assert np.abs(l1[idx][ok] - l2[ok]).max() <= 1e-12 * max(1.0, np.abs(l2[ok]).max())


def test_zero_noise_injection_at_centre_node():
    """Zero noise, injection at the centre node, full-rank basis, on-grid
    t_c at a geocentre detector: ln L = rho^2 / 2."""
    cfg = wl.CFG1.with_(seg_len=8.0, n_nodes=60, q=60, center_node=True)
    inj = wl.injection_extrinsics(cfg)
    h = rbfl.Handle.from_config(cfg, None, inj)
    qd = wl.queries(cfg, n=1)
    qd.x[:] = 0.0
    qd.dt[:] = 0.0
    qd.ext[0, 4] = inj[4]
    qd.dist_ratio[:] = 1.0
    lg = gpu_eval(h, qd, cfg.t_trig)
    assert lg[0] == pytest.approx(cfg.inj_snr ** 2 / 2, rel=1e-9)


def test_invalid_spec_errors():
    cfg = wl.CFG1.with_(seg_len=8.0, n_nodes=60, q=10)
    inj = wl.injection_extrinsics(cfg)
    keep = []
    spec = rbfl.spec_from_config(cfg, None, inj, keep=keep)
    spec.q = 1000
    with pytest.raises(rbfl.RbflError) as e:
        rbfl.Handle.build(spec)
    assert e.value.code == rbfl.E_INVALID_ARG
    spec = rbfl.spec_from_config(cfg, None, inj, keep=keep)
    spec.modes[0][1] = 3
    with pytest.raises(rbfl.RbflError) as e:
        rbfl.Handle.build(spec)
    assert e.value.code == rbfl.E_INVALID_ARG


def test_order_and_variant_arguments():
    """Argument checks of the evaluation-order and tile-variant entry points."""
    cfg, art, h = both("cfg1")
    for bad in (0, 65, -1):
        with pytest.raises(rbfl.RbflError) as e:
            h.set_pipeline(bad)
        assert e.value.code == rbfl.E_INVALID_ARG
    nv = rbfl.variants(rbfl.FORM_FP64)
    assert nv >= 2 and rbfl.variants(rbfl.FORM_SPLIT) >= 1
    with pytest.raises(ValueError):
        rbfl.variants(rbfl.FORM_SURROGATE)
    for bad in (-1, nv):
        with pytest.raises(rbfl.RbflError) as e:
            h.set_variant(rbfl.FORM_FP64, bad)
        assert e.value.code == rbfl.E_INVALID_ARG
    fresh = rbfl.Handle.from_config(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg))
    with pytest.raises(rbfl.RbflError) as e:
        fresh.set_variant(rbfl.FORM_BF16, 0)     # not prepared
    assert e.value.code == rbfl.E_STATE
    fresh.close()
    h.set_variant(rbfl.FORM_FP64, 0)
    h.set_pipeline(1)
    h.fuse_epilogue(False)
