"""Multi-event (ragged) batches: the persistent kernel and the captured plan
against the oracle and against per-event evaluation."""
import numpy as np
import pytest

from oracle import likelihood as lk
from oracle import startup as su
from paper_2508_04172_amd import rbfl
from paper_2508_04172_amd import workloads as wl

pytestmark = pytest.mark.gpu

EVENTS = wl.ragged_events(6, seed=11, seg_range=(4.0, 16.0), node_range=(60, 200), q_range=(5, 20),
                          base=wl.SMALL_MULTI)
COUNTS = [131, 700, 1, 257, 64, 383]          # tile remainders, a single proposal, exact tiles
_state = {}


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def events():
    if "h" not in _state:
        hs, arts = [], []
        for cfg in EVENTS:
            print(f"[ragged] building {cfg.name}: T={cfg.seg_len}s modes={len(cfg.modes)} N={cfg.n_nodes} q={cfg.q}",
                  flush=True)
            white = wl.white_noise(cfg)
            inj = wl.injection_extrinsics(cfg)
            hs.append(rbfl.Handle.from_config(cfg, white, inj))
            arts.append(su.startup(cfg, white, inj, workers=1))
            # the events leave eps open: both sides pick the smallest integer keeping cond <= 1e12
            assert hs[-1].eps() == arts[-1].eps, f"{cfg.name}: eps {hs[-1].eps()} vs oracle {arts[-1].eps}"
        _state["h"], _state["art"] = hs, arts
    return _state["h"], _state["art"]


def proposals(step):
    """Per event: near-node proposals (different draws per sampler step)."""
    hs, arts = events()
    gpu, cpu = [], []
    for e, (cfg, h, art) in enumerate(zip(EVENTS, hs, arts)):
        n = COUNTS[e]
        idx, jit = wl.node_jitter(n, cfg.n_nodes, seed=100 * step + e)
        qd = wl.queries(cfg, n=n, seed=1000 * step + e)
        gpu.append(rbfl.params_soa(h, qd.near_nodes(h.nodes(), idx, jit), cfg.t_trig))
        cpu.append(lk.query_params(art, qd.near_nodes(art.x_nodes, idx, jit)))
    return np.ascontiguousarray(np.concatenate(gpu, axis=1)), cpu


def per_event_gpu(hs, params):
    torch = _torch()
    out, off = [], 0
    for h, n in zip(hs, COUNTS):
        p = torch.from_numpy(np.ascontiguousarray(params[:, off:off + n])).cuda()
        o = torch.empty(n, dtype=torch.float64, device="cuda")
        h.eval(p.data_ptr(), n, o.data_ptr())
        torch.cuda.synchronize()
        out.append(o.cpu().numpy())
        off += n
    return np.concatenate(out)


def test_ragged_matches_oracle_and_per_event():
    torch = _torch()
    hs, arts = events()
    params, cpu = proposals(0)
    total = sum(COUNTS)
    p = torch.from_numpy(params).cuda()
    out = torch.empty(total, dtype=torch.float64, device="cuda")
    rbfl.eval_ragged(hs, COUNTS, p.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    lr = out.cpu().numpy()
    le = per_event_gpu(hs, params)
    fin = np.isfinite(le)
    assert np.array_equal(fin, np.isfinite(lr))
    assert np.abs(lr[fin] - le[fin]).max() <= 1e-12 * max(1.0, np.abs(le[fin]).max())
    off = 0
    for e, (art, n) in enumerate(zip(arts, COUNTS)):
        lo = lk.meshfree_lnl(art, *cpu[e])
        lg = lr[off:off + n]
        f = np.isfinite(lo)
        assert np.array_equal(f, np.isfinite(lg)), f"event {e}: domain flags differ"
        if f.any():
            d = np.abs(lg[f] - lo[f]).max()
            print(f"[ragged] event {e}: {f.sum()}/{n} valid, max |dlnL| vs oracle {d:.3e}", flush=True)
            assert d <= 1e-3
        off += n


def test_build_many_matches_single_builds():
    """rbfl_build_many (stages before and after the SVD on 3 host threads, the
    six events' SVDs in one batched call with their node counts padded to the
    largest) against one rbfl_build per event: nodes and frame identical, the
    leading q singular values within 1e-10 of the largest, each basis vector
    the same up to a phase, the ln L of every event within 1e-3 of the single
    build's and of the oracle's, with the same domain flags."""
    torch = _torch()
    hs, arts = events()
    items = [(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg)) for cfg in EVENTS]
    print(f"[ragged] build_many: {len(items)} events, node counts {[c.n_nodes for c in EVENTS]}", flush=True)
    hm = rbfl.Handle.from_configs(items, n_threads=3)
    params, cpu = proposals(0)
    lm = per_event_gpu(hm, params)
    le = per_event_gpu(hs, params)
    off = 0
    for e, (h1, h2, art, n) in enumerate(zip(hs, hm, arts, COUNTS)):
        assert np.array_equal(h1.nodes(), h2.nodes()) and h1.eps() == h2.eps()
        assert np.array_equal(h1.frame()["semi"], h2.frame()["semi"])
        q = h1.sizes()["q"]
        s1, s2 = h1.singular(), h2.singular()
        assert s1.shape == s2.shape
        ds = np.abs(s1[..., :q] - s2[..., :q]).max() / s1[..., 0].max()
        b1, b2 = h1.basis(), h2.basis()
        overlap = np.abs(np.einsum("vatq,vatq->vaq", b1.conj(), b2))
        # vectors compared where their singular value is apart from its
        # neighbours' (a near-repeated value leaves only the pair's plane fixed)
        sv = s1[..., :q + 1] / s1[..., :1]
        gap = np.minimum(np.diff(sv, prepend=np.inf)[..., :q] * -1.0, -np.diff(sv)[..., :q])
        sep = np.abs(gap) > 1e-6
        du = np.abs(1.0 - overlap[sep]).max() if sep.any() else 0.0
        a, b = le[off:off + n], lm[off:off + n]
        f = np.isfinite(a)
        assert np.array_equal(f, np.isfinite(b)), f"event {e}: domain flags differ"
        d = np.abs(a[f] - b[f]).max() if f.any() else 0.0
        lo = lk.meshfree_lnl(art, *cpu[e])
        do = np.abs(b[f] - lo[f]).max() if f.any() else 0.0
        print(f"[ragged] build_many event {e}: N {h1.sizes()['N']}, singular values {ds:.1e}, basis "
              f"{du:.1e}, max |dlnL| vs single build {d:.1e}, vs oracle {do:.1e}", flush=True)
        assert ds <= 1e-10 and du <= 1e-8 and d <= 1e-3 and do <= 1e-3
        off += n
    t = np.array([h.timing()[3] for h in hm])
    assert np.all(t == t[0]) and t[0] > 0     # one batched SVD stage for all
    for h in hm:
        h.close()


def test_build_many_single_event_is_rbfl_build():
    """rbfl_build_many over one event runs the same stages and the same
    unpadded SVD as rbfl_build: identical artefacts and ln L bit for bit."""
    torch = _torch()
    hs, _ = events()
    cfg = EVENTS[2]
    (h2,) = rbfl.Handle.from_configs([(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg))], n_threads=4)
    h1 = hs[2]
    assert np.array_equal(h1.weights(), h2.weights()) and np.array_equal(h1.singular(), h2.singular())
    assert np.array_equal(h1.basis(), h2.basis())
    n = 700
    idx, jit = wl.node_jitter(n, cfg.n_nodes, seed=5)
    qd = wl.queries(cfg, n=n, seed=6)
    p = torch.from_numpy(np.ascontiguousarray(rbfl.params_soa(h1, qd.near_nodes(h1.nodes(), idx, jit),
                                                              cfg.t_trig))).cuda()
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    h1.eval(p.data_ptr(), n, a.data_ptr())
    h2.eval(p.data_ptr(), n, b.data_ptr())
    torch.cuda.synchronize()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.array_equal(np.isfinite(a), np.isfinite(b))
    assert np.array_equal(a[np.isfinite(a)], b[np.isfinite(b)])
    h2.close()


def test_build_many_two_window_lengths():
    """rbfl_build_many over events with two window lengths (one SVD call per
    length: the second event's window is 30 ms instead of 50 ms) against one
    rbfl_build per event: same singular values, basis up to a phase, ln L
    within 1e-3 with the same domain flags."""
    torch = _torch()
    cfgs = [EVENTS[1], EVENTS[4].with_(name=EVENTS[4].name + "_w30", half_window=0.03), EVENTS[0]]
    items = [(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg)) for cfg in cfgs]
    hm = rbfl.Handle.from_configs(items, n_threads=2)
    Ts = [h.sizes()["T"] for h in hm]
    assert len(set(Ts)) == 2, Ts
    for e, (cfg, h2, (c, white, inj)) in enumerate(zip(cfgs, hm, items)):
        h1 = rbfl.Handle.from_config(cfg, white, inj)
        q = h1.sizes()["q"]
        ds = np.abs(h1.singular()[..., :q] - h2.singular()[..., :q]).max() / h1.singular()[..., 0].max()
        n = 512
        idx, jit = wl.node_jitter(n, cfg.n_nodes, seed=70 + e)
        qd = wl.queries(cfg, n=n, seed=80 + e)
        p = torch.from_numpy(np.ascontiguousarray(rbfl.params_soa(h1, qd.near_nodes(h1.nodes(), idx, jit),
                                                                  cfg.t_trig))).cuda()
        a = torch.empty(n, dtype=torch.float64, device="cuda")
        b = torch.empty(n, dtype=torch.float64, device="cuda")
        h1.eval(p.data_ptr(), n, a.data_ptr())
        h2.eval(p.data_ptr(), n, b.data_ptr())
        torch.cuda.synchronize()
        a, b = a.cpu().numpy(), b.cpu().numpy()
        f = np.isfinite(a)
        assert np.array_equal(f, np.isfinite(b)), f"event {e}: domain flags differ"
        d = np.abs(a[f] - b[f]).max() if f.any() else 0.0
        print(f"[ragged] build_many, two windows, event {e}: T {Ts[e]}, N {cfg.n_nodes}, {f.sum()}/{n} valid, "
              f"singular values {ds:.1e}, max |dlnL| vs single build {d:.1e}", flush=True)
        assert ds <= 1e-10 and d <= 1e-3
        h1.close()
    for h in hm:
        h.close()


def test_plan_graph_replays_follow_new_proposals():
    """Capture once, then per sampler step write new proposals into the same
    device buffer, with eager work in between, and check every replay."""
    torch = _torch()
    hs, _ = events()
    total = sum(COUNTS)
    params0, _ = proposals(0)
    p = torch.from_numpy(params0).cuda()
    out = torch.empty(total, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    plan = rbfl.Plan(hs, COUNTS, p.data_ptr(), out.data_ptr(), rbfl.PLAN_GRAPH | rbfl.PLAN_AUTOTUNE, stream)
    info = plan.info()
    print(f"[ragged] plan: {info}", flush=True)
    assert info["items"] > 0 and info["proposals"] == total
    for step in range(4):
        params, _ = proposals(step + 1)
        p.copy_(torch.from_numpy(params))
        torch.cuda.synchronize()
        plan.launch(stream)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        want = per_event_gpu(hs, params)
        fin = np.isfinite(want)
        assert np.array_equal(fin, np.isfinite(got)), f"replay {step}"
        assert np.abs(got[fin] - want[fin]).max() <= 1e-12 * max(1.0, np.abs(want[fin]).max()), f"replay {step}"
        _ = (torch.ones(1000, device="cuda") * 2).sum().item()   # unrelated eager work between replays
    plan.close()


def test_plan_rejects_bad_arguments():
    torch = _torch()
    hs, _ = events()
    buf = torch.zeros(11, dtype=torch.float64, device="cuda")
    with pytest.raises(rbfl.RbflError) as e:
        rbfl.Plan(hs[:2], [5, 0], buf.data_ptr(), buf.data_ptr(), 0)
    assert e.value.code == rbfl.E_INVALID_ARG


def _oracle_per_event(arts, cpu, lr, bar=1e-3, label="split plan"):
    off = 0
    worst = 0.0
    for e, (art, n) in enumerate(zip(arts, COUNTS)):
        lo = lk.meshfree_lnl(art, *cpu[e])
        lg = lr[off:off + n]
        f = np.isfinite(lo)
        assert np.array_equal(f, np.isfinite(lg)), f"{label} event {e}: domain flags differ"
        if f.any():
            d = np.abs(lg[f] - lo[f]).max()
            worst = max(worst, d)
            assert d <= bar, f"{label} event {e}: max |dlnL| {d:.3e}"
        off += n
    return worst


def test_split_plan_tuned_per_event_matches_oracle_and_replays():
    """The split form in one plan: each event's digit count tuned against the
    FP64 plan (within RBFL_SPLIT_TOL on the tuning proposals), the captured
    graph replayed on new proposals, every replay within 1e-3 of the oracle
    per event and within the split form's accuracy of the FP64 per-event
    evaluation."""
    torch = _torch()
    hs, arts = events()
    total = sum(COUNTS)
    params0, cpu0 = proposals(0)
    p = torch.from_numpy(params0).cuda()
    out = torch.empty(total, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    plan = rbfl.Plan(hs, COUNTS, p.data_ptr(), out.data_ptr(),
                     rbfl.PLAN_GRAPH | rbfl.PLAN_AUTOTUNE | rbfl.PLAN_SPLIT, stream)
    info = plan.info()
    print(f"[ragged] split plan: {info}", flush=True)
    assert info["form"] == "split" and info["variant"] == -1 and info["within_split_tol"] is True
    assert 5 <= info["slices_min"] <= info["slices_max"] <= 8 and len(info["tune_ms"]) == 4
    plan.launch(stream)
    torch.cuda.synchronize()
    lr = out.cpu().numpy()
    assert np.abs(lr[np.isfinite(lr)] - per_event_gpu(hs, params0)[np.isfinite(lr)]).max() <= rbfl.SPLIT_TOL
    worst = _oracle_per_event(arts, cpu0, lr)
    print(f"[ragged] split plan vs oracle: max |dlnL| {worst:.3e}", flush=True)
    for step in range(2):
        params, cpu = proposals(step + 1)
        p.copy_(torch.from_numpy(params))
        torch.cuda.synchronize()
        plan.launch(stream)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        want = per_event_gpu(hs, params)
        fin = np.isfinite(want)
        assert np.array_equal(fin, np.isfinite(got)), f"replay {step}"
        assert np.abs(got[fin] - want[fin]).max() <= 1e-3, f"replay {step}"
        _oracle_per_event(arts, cpu, got, label=f"split replay {step}")
        _ = (torch.ones(1000, device="cuda") * 2).sum().item()
    plan.close()


def test_split_plan_untuned_uses_each_handles_digits():
    """Without tuning every event keeps its handle's split variant (7 digits
    unless tuned on the handle) and matches the oracle within 1e-3."""
    torch = _torch()
    hs, arts = events()
    total = sum(COUNTS)
    params, cpu = proposals(5)
    p = torch.from_numpy(params).cuda()
    out = torch.empty(total, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    plan = rbfl.Plan(hs, COUNTS, p.data_ptr(), out.data_ptr(), rbfl.PLAN_SPLIT, stream)
    info = plan.info()
    assert info["form"] == "split" and info["within_split_tol"] is None
    plan.launch(stream)
    torch.cuda.synchronize()
    _oracle_per_event(arts, cpu, out.cpu().numpy(), label="untuned split plan")
    plan.close()
    with pytest.raises(rbfl.RbflError) as e:
        rbfl.Plan(hs, COUNTS, p.data_ptr(), out.data_ptr(), 0x80, stream)
    assert e.value.code == rbfl.E_INVALID_ARG


def test_fp64_plan_8_wave_tile_matches_per_event():
    """Every FP64 tile variant of the persistent contraction, the 8-wave
    128 x 128 one included, gives the per-event results to rounding."""
    torch = _torch()
    hs, _ = events()
    total = sum(COUNTS)
    params, _ = proposals(7)
    p = torch.from_numpy(params).cuda()
    out = torch.empty(total, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    plan = rbfl.Plan(hs, COUNTS, p.data_ptr(), out.data_ptr(), rbfl.PLAN_AUTOTUNE | rbfl.PLAN_GRAPH, stream)
    info = plan.info()
    print(f"[ragged] FP64 tile timings {info['tune_ms']}, chosen {info['variant']}", flush=True)
    assert len(info["tune_ms"]) == 6
    want = per_event_gpu(hs, params)
    fin = np.isfinite(want)
    for v in range(6):
        plan.set_variant(v, stream)
        plan.launch(stream)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(fin, np.isfinite(got)), f"variant {v}"
        assert np.abs(got[fin] - want[fin]).max() <= 1e-12 * max(1.0, np.abs(want[fin]).max()), f"variant {v}"
    plan.close()


def test_debug_bounds_checks_pass_on_every_layout(monkeypatch, tmp_path):
    """With RBFL_DEBUG set, the library checks on the host every offset its
    kernels index with -- each handle's output layout and device constants
    after build and load, and every work item of the FP64 plan (all six tile
    variants) and of the split plan replayed through the kernels' event
    lookup -- and raises RBFL_E_STATE on a violation.  Every layout here
    passes, and the results are those of the unchecked run."""
    torch = _torch()
    hs, _ = events()
    total = sum(COUNTS)
    params, _ = proposals(9)
    p = torch.from_numpy(params).cuda()
    out = torch.empty(total, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    want = per_event_gpu(hs, params)
    fin = np.isfinite(want)
    monkeypatch.setenv("RBFL_DEBUG", "1")
    # build and load under the checks (one small event, and a banded handle)
    cfg = EVENTS[2]
    h = rbfl.Handle.from_config(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg))
    h.save(str(tmp_path / "e.rbfl"))
    rbfl.Handle.load(str(tmp_path / "e.rbfl")).close()
    h.close()
    bcfg = wl.SMALL_BANDED.with_(name="debug_banded", seg_len=4.0, n_nodes=80, q=10, n_bands=3)
    rbfl.Handle.from_config(bcfg, wl.white_noise(bcfg), wl.injection_extrinsics(bcfg)).close()
    plan = rbfl.Plan(hs, COUNTS, p.data_ptr(), out.data_ptr(), rbfl.PLAN_AUTOTUNE, stream)
    for v in range(6):
        plan.set_variant(v, stream)
        plan.launch(stream)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(fin, np.isfinite(got))
        assert np.abs(got[fin] - want[fin]).max() <= 1e-12 * max(1.0, np.abs(want[fin]).max())
    plan.close()
    plan = rbfl.Plan(hs, COUNTS, p.data_ptr(), out.data_ptr(), rbfl.PLAN_SPLIT, stream)
    plan.launch(stream)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.array_equal(fin, np.isfinite(got))
    assert np.abs(got[fin] - want[fin]).max() <= 1e-3
    plan.close()
