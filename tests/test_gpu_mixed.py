"""Mixed-precision contraction forms against the FP64 oracle.

Split form: every product of int8 digits is summed exactly in int32, so its
only errors are the dropped digit pairs and the digit remainders, at most
(S + 3) 254^-S of s_q s_c per kernel row (s_q, s_c the power-of-two scales
of the proposal's row and of the weight column).  With its default S = 7 it
is held to the FP64 bars: |d ln L| <= 1e-3 and, per interpolated column, the
FP64 bar widened by that worst-case bound.  After rbfl_autotune (which keeps
only digit counts within 1e-4 of the FP64 form on the tuning proposals) it is
held to 1e-3 against the oracle on other proposals.

FP32 and BF16 forms: reported, not held to 1e-3 (their kernel rows, weights
and sums lose what the interpolant's cancellation amplifies); the tests check
only that they run, keep the FP64 domain flags and stay finite where those
are set.
"""
import numpy as np
import pytest

from oracle import likelihood as lk
from oracle import startup as su
from paper_2508_04172_amd import rbfl
from paper_2508_04172_amd import workloads as wl

from test_gpu_parity import CASES, both, column_scale, gpu_eval, gpu_interp

pytestmark = pytest.mark.gpu

SLICES = 7      # the split form's digit count until rbfl_autotune picks one


def _prepared(name, form):
    cfg, art, h = both(name)
    h.prepare(form)
    return cfg, art, h


@pytest.mark.parametrize("name", list(CASES))
def test_split_interpolant(name):
    cfg, art, h = _prepared(name, rbfl.FORM_SPLIT)
    qd = wl.queries(cfg, n=min(cfg.n_queries, 2000))
    Ys = gpu_interp(h, qd, cfg.t_trig, rbfl.FORM_SPLIT)
    Yd = gpu_interp(h, qd, cfg.t_trig, rbfl.FORM_FP64)
    Yo = lk.rbf_eval(art, qd.x)
    col_scale = column_scale(art)
    basis = np.concatenate([su.gaussian_kernel(qd.x, art.x_nodes, art.eps), su.poly_matrix(qd.x, art.degree)], 1)
    amp = (np.abs(basis) @ np.abs(art.W)).max(axis=0) / col_scale
    # worst case of the split arithmetic with the kernels' power-of-two scales:
    # a weight column's 2^e strictly above its largest |W| (e from frexp; 1 for
    # an all-zero column), a proposal's the smallest power of two at or above
    # max(1, max_d |x_d|)^3
    wmax = np.abs(art.W).max(axis=0)
    s_c = np.where(wmax > 0, np.ldexp(1.0, np.frexp(wmax)[1]), 1.0)
    cube = np.maximum(1.0, np.abs(qd.x).max(axis=1)) ** 3
    mant, ex = np.frexp(cube)
    s_q = np.ldexp(1.0, np.where(mant == 0.5, ex - 1, ex))
    assert np.all(s_q >= np.abs(basis).max(axis=1))
    split_bound = (SLICES + 3) * 254.0 ** (-SLICES) * basis.shape[1] * s_q.max() * s_c / col_scale
    bar = np.maximum(1e-6, 1e-13 * amp) + split_bound
    err = np.abs(Ys - Yo).max(axis=0) / col_scale
    vs64 = np.abs(Ys - Yd).max(axis=0) / col_scale
    print(f"[mixed] {name} split: max column-relative error vs oracle {err.max():.3e}, "
          f"vs the FP64 form {vs64.max():.3e}", flush=True)
    assert np.all(err <= bar), f"column {int(np.argmax(err / bar))}: {err.max():.3e}"
    assert np.all(np.abs(Ys - Yd).max(axis=0) <= split_bound * col_scale + 1e-15 * amp * col_scale)


@pytest.mark.parametrize("name", list(CASES))
def test_split_lnl(name):
    cfg, art, h = _prepared(name, rbfl.FORM_SPLIT)
    n = min(cfg.n_queries, 3000)
    idx, jit = wl.node_jitter(n, cfg.n_nodes)
    qd = wl.queries(cfg, n=n)
    for label, qg, qo in (("uniform", qd, qd),
                          ("near nodes", qd.near_nodes(h.nodes(), idx, jit), qd.near_nodes(art.x_nodes, idx, jit))):
        lg = gpu_eval(h, qg, cfg.t_trig, rbfl.FORM_SPLIT)
        lo = lk.meshfree_lnl(art, *lk.query_params(art, qo))
        fin = np.isfinite(lo)
        assert np.array_equal(fin, np.isfinite(lg))
        d = np.abs(lg[fin] - lo[fin])
        print(f"[mixed] {name} split {label}: {fin.sum()} valid, max |dlnL| {d.max():.3e}, "
              f"median {np.median(d):.3e}", flush=True)
        assert d.max() <= 1e-3


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_reported(name):
    cfg, art, h = _prepared(name, rbfl.FORM_FP32)
    qd = wl.queries(cfg, n=min(cfg.n_queries, 3000))
    lg = gpu_eval(h, qd, cfg.t_trig, rbfl.FORM_FP32)
    lo = lk.meshfree_lnl(art, *lk.query_params(art, qd))
    fin = np.isfinite(lo)
    assert np.array_equal(fin, np.isinf(lg) == False)  # noqa: E712
    assert not np.isnan(lg).any()
    d = np.abs(lg[fin] - lo[fin])
    q = np.quantile(d, [0.5, 0.9, 0.99, 1.0])
    print(f"[mixed] {name} fp32: |dlnL| median {q[0]:.3e}, 90% {q[1]:.3e}, 99% {q[2]:.3e}, max {q[3]:.3e}",
          flush=True)


@pytest.mark.parametrize("name", list(CASES))
def test_bf16_reported(name):
    """The BF16 form: runs, keeps the FP64 domain flags, stays finite where they
    are set; its error distribution is reported."""
    cfg, art, h = _prepared(name, rbfl.FORM_BF16)
    qd = wl.queries(cfg, n=min(cfg.n_queries, 3000))
    lg = gpu_eval(h, qd, cfg.t_trig, rbfl.FORM_BF16)
    lo = lk.meshfree_lnl(art, *lk.query_params(art, qd))
    fin = np.isfinite(lo)
    assert np.array_equal(fin, np.isinf(lg) == False)  # noqa: E712
    assert not np.isnan(lg).any()
    d = np.abs(lg[fin] - lo[fin])
    q = np.quantile(d, [0.5, 0.9, 0.99, 1.0])
    print(f"[mixed] {name} bf16: |dlnL| median {q[0]:.3e}, 90% {q[1]:.3e}, 99% {q[2]:.3e}, max {q[3]:.3e}",
          flush=True)


@pytest.mark.parametrize("name", list(CASES))
def test_split_fused_epilogue(name):
    """ln L finished inside the split contraction (rbfl_fuse_epilogue bit 1):
    the tile's outputs are the values the default order stores, weighted in
    place, so ln L agrees with the default split order to rounding (summation
    order only), keeps its domain flags and stays within 1e-3 of the oracle."""
    cfg, art, h = _prepared(name, rbfl.FORM_SPLIT)
    n = min(cfg.n_queries, 3000)
    idx, jit = wl.node_jitter(n, cfg.n_nodes, seed=23)
    qd = wl.queries(cfg, n=n, seed=23)
    qg = qd.near_nodes(h.nodes(), idx, jit)
    ref = gpu_eval(h, qg, cfg.t_trig, rbfl.FORM_SPLIT)
    h.fuse_epilogue(False, split=True)
    try:
        assert h.split_order()["fused_epilogue"]
        lg = gpu_eval(h, qg, cfg.t_trig, rbfl.FORM_SPLIT)
        l64 = gpu_eval(h, qg, cfg.t_trig, rbfl.FORM_FP64)     # the FP64 form keeps its own order
    finally:
        h.fuse_epilogue(False)
    assert not h.split_order()["fused_epilogue"]
    lo = lk.meshfree_lnl(art, *lk.query_params(art, qd.near_nodes(art.x_nodes, idx, jit)))
    fin = np.isfinite(lo)
    assert np.array_equal(np.isfinite(ref), np.isfinite(lg)) and np.array_equal(np.isnan(ref), np.isnan(lg))
    assert np.array_equal(fin, np.isfinite(lg)) and np.array_equal(fin, np.isfinite(l64))
    d = np.abs(lg[fin] - lo[fin])
    dr = np.abs(lg[fin] - ref[fin]).max()
    print(f"[mixed] {name} split fused epilogue: {fin.sum()} valid, max |dlnL| vs oracle {d.max():.3e}, "
          f"vs the default order {dr:.3e}", flush=True)
    assert d.max() <= 1e-3
    assert dr <= 1e-9 * max(1.0, np.abs(ref[fin]).max())


def test_split_order_autotuned():
    """With more than 4096 tuning proposals (and a work space that holds
    them) rbfl_autotune of the split form times both evaluation orders and
    keeps the fused one only if 1% faster; the evaluation it leaves in place
    matches the oracle."""
    torch = pytest.importorskip("torch")
    cfg, art, h = _prepared("small_multi", rbfl.FORM_SPLIT)
    n = 8192
    h.reserve(n)
    idx, jit = wl.node_jitter(n, cfg.n_nodes, seed=31)
    qd = wl.queries(cfg, n=n, seed=31)
    p = torch.from_numpy(np.ascontiguousarray(rbfl.params_soa(h, qd.near_nodes(h.nodes(), idx, jit),
                                                              cfg.t_trig))).cuda()
    h.autotune(p.data_ptr(), n, rbfl.FORM_SPLIT, torch.cuda.current_stream().cuda_stream)
    o = h.split_order()
    print(f"[mixed] split order: separate epilogue {o['ms']:.4f} ms, fused {o['fused_epilogue_ms']:.4f} ms, "
          f"fused kept {o['fused_epilogue']}", flush=True)
    assert o["ms"] > 0 and o["fused_epilogue_ms"] > 0
    assert o["fused_epilogue"] == (o["fused_epilogue_ms"] < 0.99 * o["ms"])
    sub = np.arange(0, n, 7)
    lg = gpu_eval(h, qd.near_nodes(h.nodes(), idx, jit).subset(sub), cfg.t_trig, rbfl.FORM_SPLIT)
    lo = lk.meshfree_lnl(art, *lk.query_params(art, qd.near_nodes(art.x_nodes, idx, jit).subset(sub)))
    fin = np.isfinite(lo)
    assert np.array_equal(fin, np.isfinite(lg))
    assert np.abs(lg[fin] - lo[fin]).max() <= 1e-3
    h.fuse_epilogue(False)


def test_split_tolerance_per_handle():
    """rbfl_set_split_tol: a looser bar never keeps more digits than the
    default one on the same proposals, the kept count is within the bar it
    was tuned to, ln L stays within 1e-3 of the oracle, and bars outside
    (0, 1e-3] are refused."""
    torch = pytest.importorskip("torch")
    cfg, art, h = _prepared("small_multi", rbfl.FORM_SPLIT)
    n = 3000
    idx, jit = wl.node_jitter(n, cfg.n_nodes, seed=41)
    qd = wl.queries(cfg, n=n, seed=41)
    qg = qd.near_nodes(h.nodes(), idx, jit)
    p = torch.from_numpy(np.ascontiguousarray(rbfl.params_soa(h, qg, cfg.t_trig))).cuda()
    sp = torch.cuda.current_stream().cuda_stream
    chosen = {}
    try:
        for tol in (rbfl.SPLIT_TOL, 1e-3):
            h.set_split_tol(tol)
            tune = h.autotune(p.data_ptr(), n, rbfl.FORM_SPLIT, sp)
            v = tune["variant"]
            assert tune["max_dlnl_vs_fp64"][v] <= tol
            assert h.split_state()["within_tol"]
            chosen[tol] = tune["slices"]
            lg = gpu_eval(h, qg, cfg.t_trig, rbfl.FORM_SPLIT)
            lo = lk.meshfree_lnl(art, *lk.query_params(art, qd.near_nodes(art.x_nodes, idx, jit)))
            fin = np.isfinite(lo)
            assert np.array_equal(fin, np.isfinite(lg))
            assert np.abs(lg[fin] - lo[fin]).max() <= 1e-3
        print(f"[mixed] split digits kept at bar 1e-4: {chosen[rbfl.SPLIT_TOL]}, at 1e-3: {chosen[1e-3]}", flush=True)
        assert chosen[1e-3] <= chosen[rbfl.SPLIT_TOL]
        lib = rbfl.load()
        for bad in (0.0, -1e-4, 2e-3, float("nan")):
            assert lib.rbfl_set_split_tol(h._h, bad) == rbfl.E_INVALID_ARG
    finally:
        h.set_split_tol(rbfl.SPLIT_TOL)


def test_split_chunked_matches_single_pass():
    """Batches above the work-space capacity give the same split-form results
    as one pass (the digit buffer is re-filled per chunk)."""
    cfg, art, h = _prepared("small_multi", rbfl.FORM_SPLIT)
    qd = wl.queries(cfg, n=70000, seed=9)
    l1 = gpu_eval(h, qd, cfg.t_trig, rbfl.FORM_SPLIT)
    idx = np.arange(0, 70000, 997)
    l2 = gpu_eval(h, qd.subset(idx), cfg.t_trig, rbfl.FORM_SPLIT)
    ok = np.isfinite(l2)
    assert np.array_equal(np.isfinite(l1[idx]), ok)
    assert np.array_equal(l1[idx][ok], l2[ok])


@pytest.mark.parametrize("name", list(CASES))
def test_split_autotuned_slices(name):
    """The autotuner's digit count: within 1e-4 of the FP64 form on its own
    proposals, within 1e-3 of the oracle on a fresh seeded set."""
    cfg, art, h = _prepared(name, rbfl.FORM_SPLIT)
    torch = pytest.importorskip("torch")
    n = min(cfg.n_queries, 3000)
    idx, jit = wl.node_jitter(n, cfg.n_nodes, seed=17)
    qd = wl.queries(cfg, n=n, seed=5)
    p = torch.from_numpy(np.ascontiguousarray(rbfl.params_soa(h, qd.near_nodes(h.nodes(), idx, jit),
                                                              cfg.t_trig))).cuda()
    tune = h.autotune(p.data_ptr(), n, rbfl.FORM_SPLIT, torch.cuda.current_stream().cuda_stream)
    errs = tune["max_dlnl_vs_fp64"]
    print(f"[mixed] {name} split autotune: S = {tune['slices']}, max |dlnL| vs FP64 per variant "
          f"{['%.1e' % e for e in errs]}, ms {['%.3f' % m for m in tune['ms']]}", flush=True)
    assert errs[tune["variant"]] <= rbfl.SPLIT_TOL
    # 7 and 8 digits (variants 2, 3) sit within a few units of FP64 rounding
    assert errs[2] <= rbfl.SPLIT_TOL and errs[3] <= rbfl.SPLIT_TOL
    qd2 = wl.queries(cfg, n=n, seed=11)
    lg = gpu_eval(h, qd2, cfg.t_trig, rbfl.FORM_SPLIT)
    lo = lk.meshfree_lnl(art, *lk.query_params(art, qd2))
    fin = np.isfinite(lo)
    assert np.array_equal(fin, np.isfinite(lg))
    d = np.abs(lg[fin] - lo[fin])
    print(f"[mixed] {name} split S = {tune['slices']} on fresh proposals: max |dlnL| {d.max():.3e}", flush=True)
    assert d.max() <= 1e-3
