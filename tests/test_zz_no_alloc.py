"""rbfl_eval_static (the FP64 online stage with the library's fixed device
work-space array, for callers that cannot allocate) against rbfl_eval on the
same proposals: bit-identical ln L and NaN counts, on two calls in a row, the
second with fewer proposals (the array keeps the first call's contents), each
spanning several chunks and a ragged last chunk."""
import numpy as np
import pytest

from full_size import handle
from paper_2508_04172_amd import rbfl
from paper_2508_04172_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def both_entry_points(h, params):
    torch = _torch()
    p = torch.from_numpy(np.ascontiguousarray(params)).cuda()
    n = params.shape[1]
    sp = torch.cuda.current_stream().cuda_stream
    a = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
    b = torch.full((n,), -7.0, dtype=torch.float64, device="cuda")
    h.eval(p.data_ptr(), n, a.data_ptr(), rbfl.FORM_FP64, sp)
    torch.cuda.synchronize()
    nan_a = h.nan_count()
    h.eval_static(p.data_ptr(), n, b.data_ptr(), sp)
    torch.cuda.synchronize()
    nan_b = h.nan_count()
    return a.cpu().numpy(), b.cpu().numpy(), nan_a, nan_b


@pytest.mark.timeout(600)
def test_eval_static_equals_eval_on_two_calls():
    cfg, h = handle("cfg2")
    sz = h.sizes()
    rows = (sz["N"] + sz["M"] + 31) // 32 * 32
    kp = (sz["K"] + 127) // 128 * 128
    chunk = (rbfl.STATIC_SCRATCH_BYTES // (8 * (rows + kp))) // 8 * 8
    for call, n in enumerate((3 * chunk + 1237, chunk + 5)):
        idx, jit = wl.node_jitter(n, cfg.n_nodes, seed=31 + call)
        params = rbfl.params_soa(h, wl.queries(cfg, n=n, seed=37 + call).near_nodes(h.nodes(), idx, jit),
                                 cfg.t_trig)
        params[5, 11] = np.nan                     # one NaN proposal per call
        a, b, nan_a, nan_b = both_entry_points(h, params)
        print(f"[no-alloc] call {call}: {n} proposals in chunks of {chunk}, {np.isfinite(a).sum()} finite ln L",
              flush=True)
        assert np.isfinite(a).sum() > n // 4
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), f"call {call}: ln L differs"
        assert nan_a == nan_b == 1


@pytest.mark.timeout(600)
def test_eval_static_equals_eval_time_banded():
    """The same on a handle with time-banded antenna patterns (4 bands, 12
    output blocks): the banded epilogue behind both entry points."""
    cfg = wl.SMALL_BANDED
    h = rbfl.Handle.from_config(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg))
    sz = h.sizes()
    rows = (sz["N"] + sz["M"] + 31) // 32 * 32
    kp = (sz["K"] + 127) // 128 * 128
    chunk = (rbfl.STATIC_SCRATCH_BYTES // (8 * (rows + kp))) // 8 * 8
    for call, n in enumerate((3 * chunk + 1237, chunk + 5)):
        idx, jit = wl.node_jitter(n, cfg.n_nodes, seed=41 + call)
        params = rbfl.params_soa(h, wl.queries(cfg, n=n, seed=43 + call).near_nodes(h.nodes(), idx, jit),
                                 cfg.t_trig)
        params[5, 11] = np.nan
        a, b, nan_a, nan_b = both_entry_points(h, params)
        assert np.isfinite(a).sum() > n // 4
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), f"banded call {call}: ln L differs"
        assert nan_a == nan_b == 1
    h.close()


def test_eval_static_rejects_bad_arguments():
    cfg, h = handle("cfg2")
    lib = rbfl.load()
    assert lib.rbfl_eval_static(None, None, 0, None, None) == rbfl.E_INVALID_ARG
    assert lib.rbfl_eval_static(h.ptr, None, 10, None, None) == rbfl.E_INVALID_ARG
