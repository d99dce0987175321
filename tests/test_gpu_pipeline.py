"""Pipelined FP64 evaluation: chunks whose epilogues run on the handle's side
stream under the next chunk's basis rows and MFMA product.  Each proposal's
arithmetic is unchanged, so ln L must be bit-identical to the serial order:
for several chunk counts, over many chunks (both work-space halves reused),
on a non-default stream with back-to-back calls, with per-launch timing on,
and under graph capture (which keeps the serial order)."""
import numpy as np
import pytest

from paper_2508_04172_amd import rbfl
from paper_2508_04172_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def setup():
    torch = _torch()
    cfg = wl.CFG1
    print("[pipeline] building cfg1", flush=True)
    h = rbfl.Handle.from_config(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg))
    h.reserve(16384)                # two halves of 8192 proposals
    n = 50003                       # 7 chunks of at most 8192 at 4 chunks per call, ragged last
    idx, jit = wl.node_jitter(n, cfg.n_nodes, seed=11)
    qd = wl.queries(cfg, n=n, seed=12).near_nodes(h.nodes(), idx, jit)
    p = torch.from_numpy(np.ascontiguousarray(rbfl.params_soa(h, qd, cfg.t_trig))).cuda()
    return cfg, h, p, n


def run(h, p, n, chunks, stream=None):
    torch = _torch()
    h.set_pipeline(chunks)
    out = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
    st = stream or torch.cuda.current_stream()
    h.eval(p.data_ptr(), n, out.data_ptr(), rbfl.FORM_FP64, st.cuda_stream)
    st.synchronize()
    return out


def same(a, b):
    torch = _torch()
    return bool(torch.equal(torch.nan_to_num(a, nan=1.5, neginf=-2.5), torch.nan_to_num(b, nan=1.5, neginf=-2.5)))


def test_pipelined_equals_serial(setup):
    cfg, h, p, n = setup
    ref = run(h, p, n, 1)
    fin = int(ref.isfinite().sum())
    print(f"[pipeline] serial: {fin} of {n} finite", flush=True)
    assert fin > n // 4
    for chunks in (2, 3, 4, 8, 64):
        got = run(h, p, n, chunks)
        print(f"[pipeline] {chunks} chunks: identical {same(ref, got)}", flush=True)
        assert same(ref, got)
    h.set_pipeline(1)


def test_pipelined_back_to_back_on_a_side_stream(setup):
    """Two calls on a non-default stream without a host synchronisation
    between them (the second call's first products reuse the work-space
    halves that the first call's last epilogues read), then a serial check."""
    torch = _torch()
    cfg, h, p, n = setup
    ref = run(h, p, n, 1)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    h.set_pipeline(4)
    with torch.cuda.stream(st):
        h.eval(p.data_ptr(), n, a.data_ptr(), rbfl.FORM_FP64, st.cuda_stream)
        h.eval(p.data_ptr(), n, b.data_ptr(), rbfl.FORM_FP64, st.cuda_stream)
    st.synchronize()
    h.set_pipeline(1)
    assert same(ref, a) and same(ref, b)


def test_pipelined_profile_counts(setup):
    cfg, h, p, n = setup
    ref = run(h, p, n, 1)
    h.profile(True)
    got = run(h, p, n, 4)
    h.profile(False)
    ks = h.kernel_stats()
    print(f"[pipeline] profile: {ks}", flush=True)
    h.set_pipeline(1)
    assert same(ref, got)
    assert ks["contract_launches"] == ks["epilogue_launches"] == 7
    assert ks["contract_n"] == ks["epilogue_n"] == n
    assert ks["contract_ms"] > 0 and ks["epilogue_ms"] > 0


def test_graph_capture_keeps_serial_order(setup):
    """Under capture the call keeps the serial order; every replay, with
    eager work and synchronisations between replays, matches the eager
    result."""
    torch = _torch()
    cfg, h, p, n = setup
    m = 12000                       # within the work capacity: no allocation under capture
    ref = run(h, p[:, :m].contiguous(), m, 1)
    q = p[:, :m].contiguous()
    out = torch.zeros(m, dtype=torch.float64, device="cuda")
    h.set_pipeline(4)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        h.eval(q.data_ptr(), m, out.data_ptr(), rbfl.FORM_FP64, torch.cuda.current_stream().cuda_stream)
    for r in range(3):
        out.fill_(3.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        print(f"[pipeline] replay {r}: identical {same(ref, out)}", flush=True)
        assert same(ref, out)
        eager = run(h, p, n, 4)       # eager pipelined work between replays
        assert eager.isfinite().sum() > 0
    h.set_pipeline(1)
    del g


def test_autotune_sets_pipeline(setup):
    cfg, h, p, n = setup
    torch = _torch()
    h.autotune(p.data_ptr(), n, rbfl.FORM_FP64, torch.cuda.current_stream().cuda_stream)
    pl = h.pipeline()
    print(f"[pipeline] autotune: {pl}", flush=True)
    assert pl["chunks"] in (1, 2, 4, 8) and len(pl["ms"]) == 4
    ref = run(h, p, n, 1)
    got = run(h, p, n, pl["chunks"])
    assert same(ref, got)
    h.set_pipeline(1)


def test_fused_epilogue_chunks_profile_and_capture(setup):
    """ln L finished inside the contraction over several chunks of the work
    space (50003 proposals, capacity 16384), with per-launch timing on, and
    replayed from a captured graph: agreement with the default order to
    rounding, identical domain flags, every replay identical."""
    torch = _torch()
    cfg, h, p, n = setup
    ref = run(h, p, n, 1)
    h.fuse_epilogue(True)
    try:
        h.profile(True)
        got = run(h, p, n, 1)
        h.profile(False)
        ks = h.kernel_stats()
        m = 12000
        q = p[:, :m].contiguous()
        eager = run(h, q, m, 1)
        out = torch.zeros(m, dtype=torch.float64, device="cuda")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            h.eval(q.data_ptr(), m, out.data_ptr(), rbfl.FORM_FP64, torch.cuda.current_stream().cuda_stream)
        for r in range(3):
            out.fill_(3.0)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert same(eager, out), f"replay {r}"
            run(h, p, n, 1)
        del g
    finally:
        h.fuse_epilogue(False)
    fin = ref.isfinite()
    assert torch.equal(fin, got.isfinite()) and torch.equal(ref.isnan(), got.isnan())
    d = float((ref[fin] - got[fin]).abs().max())
    print(f"[pipeline] fused epilogue: max |d| vs default order {d:.3e}; profile {ks}", flush=True)
    assert d <= 1e-9 * max(1.0, float(ref[fin].abs().max()))
    assert ks["contract_launches"] == ks["epilogue_launches"] == ks["rows_launches"] == 4
    assert ks["contract_n"] == n
