"""ctypes binding of the rbfl C ABI (include/rbfl.h).

Argument marshalling only: every step of the start-up and online stages runs
in the HIP library.  Device buffers are passed as raw pointers (e.g.
``tensor.data_ptr()``) and streams as HIP stream handles (under ROCm,
``torch.cuda.current_stream().cuda_stream``).  Loading fails loudly if the
library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbfl.so")

ABI_VERSION = 7
MAX_MODES = 5
MAX_DET = 4
MAX_BANDS = 16
MAX_BLOCKS = 64

OK, E_INVALID_ARG, E_OUT_OF_MEMORY, E_DEVICE, E_NUMERICAL, E_UNSUPPORTED, E_STATE = range(7)
FORM_FP64, FORM_FP32, FORM_BF16, FORM_SPLIT, FORM_SURROGATE = range(5)
FLAG_CENTER_NODE, FLAG_SQUEEZE, FLAG_OPTIMISE_CENTRE = 0x1, 0x2, 0x4

Q_SIZES, Q_FRAME, Q_D_REF, Q_NODES, Q_NODE_PHYS, Q_WEIGHTS, Q_BASIS, Q_NODE_VALUES, Q_SINGULAR, Q_COND, \
    Q_TIMING, Q_Z_NODES, Q_KERNEL_STATS, Q_TUNE, Q_SURROGATE, Q_SPLIT_ERR, Q_F_REF, Q_SQUEEZE, Q_CENTRE, \
    Q_PIPELINE, Q_SURROGATE_NET, Q_SPLIT_STATE, Q_NAN_COUNT, Q_SURROGATE_BASE, Q_EPS, Q_BANDS, \
    Q_SPLIT_ORDER = range(27)
SPLIT_TOL = 1e-4
STATIC_SCRATCH_BYTES = 128 << 20

EXPORTED = ("rbfl_last_error", "rbfl_build", "rbfl_build_many", "rbfl_brute", "rbfl_exact_parts", "rbfl_eval", "rbfl_interp", "rbfl_prepare", "rbfl_reserve",
            "rbfl_query", "rbfl_autotune", "rbfl_variants", "rbfl_set_variant", "rbfl_pipeline",
            "rbfl_fuse_epilogue", "rbfl_set_split_tol",
            "rbfl_profile", "rbfl_plan_create", "rbfl_plan_launch",
            "rbfl_plan_query", "rbfl_plan_set_variant", "rbfl_plan_destroy", "rbfl_eval_ragged", "rbfl_surrogate_train", "rbfl_surrogate_force",
            "rbfl_mlp_create", "rbfl_mlp_forward", "rbfl_mlp_loss_grad", "rbfl_mlp_adam", "rbfl_mlp_get",
            "rbfl_mlp_destroy", "rbfl_sampler_create", "rbfl_sampler_run", "rbfl_sampler_smc", "rbfl_sampler_query",
            "rbfl_sampler_destroy", "rbfl_prior_weights", "rbfl_save", "rbfl_load", "rbfl_eval_static",
            "rbfl_destroy")
SAMPLER_PRIOR_ONLY = 0x1
PLAN_GRAPH, PLAN_AUTOTUNE, PLAN_SPLIT = 0x1, 0x2, 0x4


class BuildSpec(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32),
        ("n_det", C.c_int32),
        ("n_modes", C.c_int32),
        ("modes", (C.c_int32 * 2) * MAX_MODES),
        ("fs", C.c_double),
        ("seg_len", C.c_double),
        ("f_low", C.c_double),
        ("psd_scale", C.c_double),
        ("psd", C.POINTER(C.c_double)),
        ("data_fd", C.POINTER(C.c_double)),
        ("noise_white", C.POINTER(C.c_double)),
        ("inj_phys", C.c_double * 4),
        ("inj_ext", C.c_double * 5),
        ("inj_snr", C.c_double),
        ("d_ref", C.c_double),
        ("det_geom", C.POINTER(C.c_double)),
        ("center_phys", C.c_double * 4),
        ("match", C.c_double),
        ("metric", C.POINTER(C.c_double)),
        ("t_trig", C.c_double),
        ("half_window", C.c_double),
        ("n_nodes", C.c_int32),
        ("q", C.c_int32),
        ("eps", C.c_double),
        ("poly_degree", C.c_int32),
        ("chi_max", C.c_double),
        ("flags", C.c_uint32),
        ("f_ref", C.c_double),
        ("earth_rate", C.c_double),
        ("n_bands", C.c_int32),
    ]


class SamplerSpec(C.Structure):
    _fields_ = [
        ("walkers", C.c_int32),
        ("form", C.c_int32),
        ("seed", C.c_uint64),
        ("t_lo", C.c_double),
        ("t_hi", C.c_double),
        ("d_lo", C.c_double),
        ("d_hi", C.c_double),
        ("d_exp", C.c_double),
        ("gamma", C.c_double),
        ("p_jump", C.c_double),
        ("flags", C.c_uint32),
        ("anneal_steps", C.c_int64),
        ("beta0", C.c_double),
    ]


class TrainSpec(C.Structure):
    _fields_ = [
        ("hidden", C.c_int32),
        ("batch", C.c_int32),
        ("epochs", C.c_int32),
        ("lr", C.c_double),
        ("beta1", C.c_double),
        ("beta2", C.c_double),
        ("adam_eps", C.c_double),
        ("init_normals", C.POINTER(C.c_double)),
        ("train_params", C.c_void_p),
        ("n_train", C.c_int64),
        ("holdout_params", C.c_void_p),
        ("n_holdout", C.c_int64),
        ("threshold", C.c_double),
        ("base_degree", C.c_int32),
    ]


def mlp_param_count(n_in: int, hidden: int, n_out: int) -> int:
    return hidden * n_in + hidden + hidden * hidden + hidden + n_out * hidden + n_out


class RbflError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rbfl status {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load librbfl.so (built in-tree by ``python -m paper_2508_04172_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2508_04172_amd.build`")
    # PyTorch ships its own HIP runtime (same soname, loaded by path).  Loading
    # it first lets this library bind to that runtime instead of pulling in a
    # second copy, which would leave torch without a usable device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    lib.rbfl_last_error.restype = C.c_char_p
    lib.rbfl_last_error.argtypes = []
    lib.rbfl_build.restype = C.c_int32
    lib.rbfl_build.argtypes = [C.POINTER(BuildSpec), C.c_void_p, C.POINTER(C.c_void_p)]
    lib.rbfl_build_many.restype = C.c_int32
    lib.rbfl_build_many.argtypes = [C.POINTER(BuildSpec), C.c_int32, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]
    lib.rbfl_brute.restype = C.c_int32
    lib.rbfl_brute.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
    lib.rbfl_exact_parts.restype = C.c_int32
    lib.rbfl_exact_parts.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
    lib.rbfl_eval.restype = C.c_int32
    lib.rbfl_eval.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p]
    lib.rbfl_interp.restype = C.c_int32
    lib.rbfl_interp.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p]
    lib.rbfl_prepare.restype = C.c_int32
    lib.rbfl_prepare.argtypes = [C.c_void_p, C.c_int32]
    lib.rbfl_reserve.restype = C.c_int32
    lib.rbfl_reserve.argtypes = [C.c_void_p, C.c_int64]
    lib.rbfl_query.restype = C.c_int32
    lib.rbfl_query.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t]
    lib.rbfl_autotune.restype = C.c_int32
    lib.rbfl_autotune.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]
    lib.rbfl_variants.restype = C.c_int32
    lib.rbfl_variants.argtypes = [C.c_int32]
    lib.rbfl_set_variant.restype = C.c_int32
    lib.rbfl_set_variant.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
    lib.rbfl_fuse_epilogue.restype = C.c_int32
    lib.rbfl_fuse_epilogue.argtypes = [C.c_void_p, C.c_int32]
    lib.rbfl_set_split_tol.restype = C.c_int32
    lib.rbfl_set_split_tol.argtypes = [C.c_void_p, C.c_double]
    lib.rbfl_pipeline.restype = C.c_int32
    lib.rbfl_pipeline.argtypes = [C.c_void_p, C.c_int32]
    lib.rbfl_profile.restype = C.c_int32
    lib.rbfl_profile.argtypes = [C.c_void_p, C.c_int32]
    lib.rbfl_plan_create.restype = C.c_int32
    lib.rbfl_plan_create.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_int64), C.c_void_p,
                                     C.c_void_p, C.c_uint32, C.c_void_p, C.POINTER(C.c_void_p)]
    lib.rbfl_plan_launch.restype = C.c_int32
    lib.rbfl_plan_launch.argtypes = [C.c_void_p, C.c_void_p]
    lib.rbfl_plan_query.restype = C.c_int32
    lib.rbfl_plan_query.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    lib.rbfl_plan_set_variant.restype = C.c_int32
    lib.rbfl_plan_set_variant.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]
    lib.rbfl_plan_destroy.restype = C.c_int32
    lib.rbfl_plan_destroy.argtypes = [C.c_void_p]
    lib.rbfl_eval_ragged.restype = C.c_int32
    lib.rbfl_eval_ragged.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_int64), C.c_void_p,
                                     C.c_void_p, C.c_void_p]
    lib.rbfl_surrogate_train.restype = C.c_int32
    lib.rbfl_surrogate_train.argtypes = [C.c_void_p, C.POINTER(TrainSpec), C.c_void_p]
    lib.rbfl_surrogate_force.restype = C.c_int32
    lib.rbfl_surrogate_force.argtypes = [C.c_void_p, C.c_int32]
    lib.rbfl_mlp_create.restype = C.c_int32
    lib.rbfl_mlp_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_void_p)]
    lib.rbfl_mlp_forward.restype = C.c_int32
    lib.rbfl_mlp_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
    lib.rbfl_mlp_loss_grad.restype = C.c_int32
    lib.rbfl_mlp_loss_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_double),
                                       C.c_void_p]
    lib.rbfl_mlp_adam.restype = C.c_int32
    lib.rbfl_mlp_adam.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_void_p]
    lib.rbfl_mlp_get.restype = C.c_int32
    lib.rbfl_mlp_get.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t]
    lib.rbfl_mlp_destroy.restype = C.c_int32
    lib.rbfl_mlp_destroy.argtypes = [C.c_void_p]
    lib.rbfl_sampler_create.restype = C.c_int32
    lib.rbfl_sampler_create.argtypes = [C.c_void_p, C.POINTER(SamplerSpec), C.c_void_p, C.c_void_p,
                                        C.POINTER(C.c_void_p)]
    lib.rbfl_sampler_run.restype = C.c_int32
    lib.rbfl_sampler_run.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p]
    lib.rbfl_sampler_smc.restype = C.c_int32
    lib.rbfl_sampler_smc.argtypes = [C.c_void_p, C.c_double, C.c_int32, C.c_int32, C.c_void_p,
                                     C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    lib.rbfl_sampler_query.restype = C.c_int32
    lib.rbfl_sampler_query.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t]
    lib.rbfl_sampler_destroy.restype = C.c_int32
    lib.rbfl_sampler_destroy.argtypes = [C.c_void_p]
    lib.rbfl_prior_weights.restype = C.c_int32
    lib.rbfl_prior_weights.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.POINTER(C.c_double),
                                       C.c_double, C.c_void_p, C.POINTER(C.c_double), C.c_void_p]
    lib.rbfl_eval_static.restype = C.c_int32
    lib.rbfl_eval_static.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
    lib.rbfl_save.restype = C.c_int32
    lib.rbfl_save.argtypes = [C.c_void_p, C.c_char_p]
    lib.rbfl_load.restype = C.c_int32
    lib.rbfl_load.argtypes = [C.c_char_p, C.c_void_p, C.POINTER(C.c_void_p)]
    lib.rbfl_destroy.restype = C.c_int32
    lib.rbfl_destroy.argtypes = [C.c_void_p]
    _lib = lib
    return lib


def _check(code: int):
    if code != OK:
        raise RbflError(code, load().rbfl_last_error().decode())


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return C.POINTER(C.c_double)()
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def spec_from_config(cfg, white: Optional[np.ndarray], inj_ext, metric: Optional[np.ndarray] = None,
                     keep: Optional[list] = None) -> BuildSpec:
    """Marshal a workload configuration into the C spec.  `keep` receives the
    numpy arrays whose memory the spec points to (they must outlive the call)."""
    s = BuildSpec()
    s.abi_version = ABI_VERSION
    s.n_det = cfg.n_det
    s.n_modes = len(cfg.modes)
    for a, (l, m) in enumerate(cfg.modes):
        s.modes[a][0] = l
        s.modes[a][1] = m
    s.fs, s.seg_len, s.f_low = cfg.fs, cfg.seg_len, cfg.f_low
    s.psd_scale = cfg.psd_scale
    geom = np.ascontiguousarray(np.array(cfg.sites, dtype=np.float64))
    w = None if white is None else np.ascontiguousarray(white, dtype=np.float64)
    met = None if metric is None else np.ascontiguousarray(metric, dtype=np.float64)
    if keep is not None:
        keep.extend([geom, w, met])
    s.det_geom = _dptr(geom)
    s.noise_white = _dptr(w)
    s.psd = C.POINTER(C.c_double)()
    s.data_fd = C.POINTER(C.c_double)()
    s.metric = _dptr(met)
    for i in range(4):
        s.inj_phys[i] = cfg.inj_phys[i]
        s.center_phys[i] = cfg.seed_phys[i]
    for i in range(5):
        s.inj_ext[i] = float(inj_ext[i])
    s.inj_snr = cfg.inj_snr
    s.d_ref = 0.0
    s.match = cfg.match
    s.t_trig = cfg.t_trig
    s.half_window = cfg.half_window
    s.n_nodes = cfg.n_nodes
    s.q = cfg.q
    s.eps = cfg.eps
    s.poly_degree = cfg.poly_degree
    s.chi_max = cfg.chi_max
    s.flags = ((FLAG_CENTER_NODE if cfg.center_node else 0) | (FLAG_SQUEEZE if cfg.squeeze else 0)
               | (FLAG_OPTIMISE_CENTRE if getattr(cfg, "optimise_centre", False) else 0))
    s.f_ref = cfg.f_ref
    s.earth_rate = getattr(cfg, "earth_rate", 0.0)
    s.n_bands = getattr(cfg, "n_bands", 1)
    return s


class Handle:
    """Owns one rbfl handle (start-up artefacts resident on the GPU)."""

    def __init__(self, ptr: C.c_void_p):
        self._h = ptr

    @classmethod
    def build(cls, spec: BuildSpec, stream: int = 0) -> "Handle":
        lib = load()
        h = C.c_void_p()
        _check(lib.rbfl_build(C.byref(spec), C.c_void_p(stream), C.byref(h)))
        return cls(h)

    @classmethod
    def from_config(cls, cfg, white, inj_ext, metric=None, stream: int = 0) -> "Handle":
        keep = []
        spec = spec_from_config(cfg, white, inj_ext, metric, keep)
        return cls.build(spec, stream)

    @classmethod
    def build_many(cls, specs, n_threads: int = 4, stream: int = 0) -> list:
        """Handles of several start-ups at once (rbfl_build_many): their SVDs
        share batched calls on `stream`, the other stages run on n_threads
        host threads."""
        lib = load()
        n = len(specs)
        arr = (BuildSpec * n)(*specs)
        hs = (C.c_void_p * n)()
        _check(lib.rbfl_build_many(arr, n, n_threads, C.c_void_p(stream), hs))
        return [cls(C.c_void_p(hs[i])) for i in range(n)]

    @classmethod
    def from_configs(cls, items, n_threads: int = 4, stream: int = 0) -> list:
        """build_many over (cfg, white, inj_ext) triples."""
        keep = []
        specs = [spec_from_config(cfg, white, inj, None, keep) for cfg, white, inj in items]
        return cls.build_many(specs, n_threads, stream)

    @classmethod
    def load(cls, path: str, stream: int = 0) -> "Handle":
        """A handle restored from a file written by save() (rbfl_load)."""
        lib = load()
        h = C.c_void_p()
        _check(lib.rbfl_load(os.fsencode(path), C.c_void_p(stream), C.byref(h)))
        return cls(h)

    def save(self, path: str):
        """Writes the handle's start-up artefacts to `path` (rbfl_save)."""
        _check(load().rbfl_save(self._h, os.fsencode(path)))

    def nan_count(self) -> int:
        """NaN ln L values of the last rbfl_eval call (RBFL_Q_NAN_COUNT)."""
        return int(self._query(Q_NAN_COUNT, 1, np.int64)[0])

    def split_state(self) -> dict:
        """Whether the split form's digit count was autotuned and met the tuner's bar (RBFL_Q_SPLIT_STATE)."""
        v = self._query(Q_SPLIT_STATE, 3)
        return {"tuned": bool(v[0]), "within_tol": bool(v[1]), "slices": int(v[2])}

    def split_order(self) -> dict:
        """Whether the split form finishes ln L inside its contraction, and the autotuner's ms per
        evaluation with the separate epilogue and in that order (RBFL_Q_SPLIT_ORDER)."""
        v = self._query(Q_SPLIT_ORDER, 3)
        return {"fused_epilogue": bool(v[0]), "ms": float(v[1]), "fused_epilogue_ms": float(v[2])}

    def close(self):
        if self._h is not None and self._h.value:
            _check(load().rbfl_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ptr(self) -> int:
        return self._h.value

    def brute(self, params_ptr: int, n: int, lnl_ptr: int, stream: int = 0):
        """Exact ln L without the interpolant (rbfl_brute)."""
        _check(load().rbfl_brute(self._h, C.c_void_p(params_ptr), n, C.c_void_p(lnl_ptr), C.c_void_p(stream)))

    def exact_parts(self, params_ptr: int, n: int, out_ptr: int, stream: int = 0):
        """ln L from exact outputs at the proposals, [2][n] (rbfl_exact_parts)."""
        _check(load().rbfl_exact_parts(self._h, C.c_void_p(params_ptr), n, C.c_void_p(out_ptr), C.c_void_p(stream)))

    def eval(self, params_ptr: int, n: int, lnl_ptr: int, form: int = FORM_FP64, stream: int = 0):
        _check(load().rbfl_eval(self._h, C.c_void_p(params_ptr), n, C.c_void_p(lnl_ptr), form,
                                C.c_void_p(stream)))

    def eval_static(self, params_ptr: int, n: int, lnl_ptr: int, stream: int = 0):
        """FP64 ln L with the library's fixed work-space array, no allocation (rbfl_eval_static)."""
        _check(load().rbfl_eval_static(self._h, C.c_void_p(params_ptr), n, C.c_void_p(lnl_ptr),
                                       C.c_void_p(stream)))

    def interp(self, params_ptr: int, n: int, out_ptr: int, form: int = FORM_FP64, stream: int = 0):
        _check(load().rbfl_interp(self._h, C.c_void_p(params_ptr), n, C.c_void_p(out_ptr), form,
                                  C.c_void_p(stream)))

    def prepare(self, form: int):
        _check(load().rbfl_prepare(self._h, form))

    def reserve(self, n: int):
        _check(load().rbfl_reserve(self._h, n))

    def _query(self, what: int, shape, dtype=np.float64) -> np.ndarray:
        out = np.zeros(shape, dtype=dtype)
        _check(load().rbfl_query(self._h, what, out.ctypes.data_as(C.c_void_p), out.nbytes))
        return out

    def sizes(self) -> dict:
        v = self._query(Q_SIZES, 8, np.int64)
        return dict(zip(("N", "M", "K", "q", "T", "n_det", "n_modes", "half_w"), (int(x) for x in v)))

    def frame(self) -> dict:
        v = self._query(Q_FRAME, 44)
        return {"theta_c": v[0:4], "vecs": v[4:20].reshape(4, 4), "lam": v[20:24], "semi": v[24:28],
                "metric": v[28:44].reshape(4, 4)}

    def centre(self) -> dict:
        """The centre used and the network-SNR optimisation's result (RBFL_Q_CENTRE)."""
        v = self._query(Q_CENTRE, 8)
        return {"phys": v[0:4], "iota": float(v[4]), "phi": float(v[5]), "snr_seed": float(v[6]),
                "snr_opt": float(v[7])}

    def squeeze(self) -> tuple:
        """(factor applied to the longest semi-axis, true match at its new tip)."""
        v = self._query(Q_SQUEEZE, 2)
        return float(v[0]), float(v[1])

    def f_ref(self) -> float:
        return float(self._query(Q_F_REF, 1)[0])

    def d_ref(self) -> float:
        return float(self._query(Q_D_REF, 1)[0])

    def nodes(self) -> np.ndarray:
        return self._query(Q_NODES, (self.sizes()["N"], 4))

    def node_phys(self) -> np.ndarray:
        return self._query(Q_NODE_PHYS, (self.sizes()["N"], 4))

    def weights(self) -> np.ndarray:
        s = self.sizes()
        return self._query(Q_WEIGHTS, (s["N"] + s["M"], s["K"]))

    def basis(self) -> np.ndarray:
        s = self.sizes()
        v = self._query(Q_BASIS, (self.n_blocks(), s["n_modes"], s["T"], s["q"], 2))
        return v[..., 0] + 1j * v[..., 1]

    def node_values(self) -> np.ndarray:
        s = self.sizes()
        return self._query(Q_NODE_VALUES, (s["N"], s["K"]))

    def singular(self) -> np.ndarray:
        s = self.sizes()
        return self._query(Q_SINGULAR, (self.n_blocks(), s["n_modes"], min(s["N"], s["T"])))

    def z_nodes(self) -> np.ndarray:
        s = self.sizes()
        v = self._query(Q_Z_NODES, (self.n_blocks(), s["n_modes"], s["N"], s["T"], 2))
        return v[..., 0] + 1j * v[..., 1]

    def cond(self) -> float:
        return float(self._query(Q_COND, 1)[0])

    def eps(self) -> float:
        """The interpolants' Gaussian shape parameter (RBFL_Q_EPS; chosen by the library when the spec's is 0)."""
        return float(self._query(Q_EPS, 1)[0])

    def bands(self):
        """Time bands of the antenna patterns (RBFL_Q_BANDS): (bin edges [B + 1]
        int64, band times [B][n_modes]), or None for frozen patterns (B = 1)."""
        n_modes = self.sizes()["n_modes"]
        v = self._query(Q_BANDS, 2 + (MAX_BANDS + 1) + MAX_BANDS * MAX_MODES)
        B = int(v[0])
        if B == 1:
            return None
        return v[2:B + 3].astype(np.int64), v[B + 3:B + 3 + B * n_modes].reshape(B, n_modes).copy()

    def n_blocks(self) -> int:
        """Blocks of interpolated outputs: detectors, or (detector, band) pairs."""
        return int(self._query(Q_BANDS, 2 + (MAX_BANDS + 1) + MAX_BANDS * MAX_MODES)[1])

    def exports(self) -> dict:
        """Every artefact the online stage evaluates with, as host arrays (the
        keyword arguments of an evaluation-parity check): frame, nodes, RBF
        weights, SVD basis, window half-width, reference distance and frequency."""
        fr = self.frame()
        return {"theta_c": fr["theta_c"], "metric_g": fr["metric"], "vecs": fr["vecs"], "lam": fr["lam"],
                "semi": fr["semi"], "x_nodes": self.nodes(), "phys_nodes": self.node_phys(), "W": self.weights(),
                "basis": self.basis(), "half_w": self.sizes()["half_w"], "d_ref": self.d_ref(),
                "f_ref": self.f_ref(), "eps": self.eps(), "cond": self.cond(), "singular": self.singular(),
                "node_values": self.node_values(), "bands": self.bands()}

    def timing(self) -> np.ndarray:
        return self._query(Q_TIMING, 8)

    def autotune(self, params_ptr: int, n: int, form: int = FORM_FP64, stream: int = 0) -> dict:
        _check(load().rbfl_autotune(self._h, C.c_void_p(params_ptr), n, form, C.c_void_p(stream)))
        v = self._query(Q_TUNE, 36).reshape(4, 9)
        out = {"variant": int(v[form, 0]), "ms": [float(x) for x in v[form, 1:] if x > 0]}
        if form == FORM_SPLIT:
            out["slices"] = split_slices(out["variant"])
            out["max_dlnl_vs_fp64"] = [float(x) for x in self._query(Q_SPLIT_ERR, 8)]
        return out

    def surrogate_train(self, init_normals: np.ndarray, train_ptr: int, n_train: int, holdout_ptr: int,
                        n_holdout: int, hidden: int = 256, batch: int = 1024, epochs: int = 20, lr: float = 1e-3,
                        beta1: float = 0.9, beta2: float = 0.999, adam_eps: float = 1e-8,
                        threshold: float = 1e-3, stream: int = 0, base_degree: int = 0) -> dict:
        z = np.ascontiguousarray(init_normals, dtype=np.float64)
        sp = TrainSpec(hidden, batch, epochs, lr, beta1, beta2, adam_eps, _dptr(z), C.c_void_p(train_ptr), n_train,
                       C.c_void_p(holdout_ptr), n_holdout, threshold, base_degree)
        _check(load().rbfl_surrogate_train(self._h, C.byref(sp), C.c_void_p(stream)))
        return self.surrogate_stats()

    def surrogate_force(self, on: bool):
        _check(load().rbfl_surrogate_force(self._h, 1 if on else 0))

    def surrogate_stats(self) -> dict:
        v = self._query(Q_SURROGATE, 8)
        return {"accepted": bool(v[0]), "holdout_max_dlnl": float(v[1]), "holdout_median_dlnl": float(v[2]),
                "first_loss": float(v[3]), "last_loss": float(v[4]), "epochs": int(v[5]),
                "train_s": float(v[6]), "n_train": int(v[7])}

    def surrogate_net(self, hidden: int):
        """The trained surrogate (RBFL_Q_SURROGATE_NET): FP32 parameter vector
        for 4 -> hidden -> hidden -> K, and the per-column mean and standard
        deviation of its outputs."""
        K = self.sizes()["K"]
        n = mlp_param_count(4, hidden, K)
        v = self._query(Q_SURROGATE_NET, n + 2 * K, np.float32)
        return v[:n].copy(), v[n:n + K].copy(), v[n + K:].copy()

    def surrogate_base(self) -> dict:
        """The residual form's FP64 base (RBFL_Q_SURROGATE_BASE): degree, per-axis mean m and deviation s
        of the training proposals' unit-ball coordinates, coefficients [nbase][K] (None without a base)."""
        K = self.sizes()["K"]
        v = np.zeros(10 + 35 * K)               # room for the largest base (35 monomials of degree <= 3)
        _check(load().rbfl_query(self._h, Q_SURROGATE_BASE, v.ctypes.data_as(C.c_void_p), v.nbytes))
        nbase = int(v[1])
        return {"degree": int(v[0]), "nbase": nbase, "m": v[2:6].copy(), "s": v[6:10].copy(),
                "B": v[10:10 + nbase * K].reshape(nbase, K).copy() if nbase else None}

    def set_variant(self, form: int, variant: int):
        """Pins the contraction tile variant of `form` (rbfl_set_variant)."""
        _check(load().rbfl_set_variant(self._h, form, variant))

    def set_pipeline(self, chunks: int):
        """Chunks per FP64 evaluation (1 = serial order); the autotuner sets it."""
        _check(load().rbfl_pipeline(self._h, chunks))

    def set_split_tol(self, tol: float):
        """The split autotune's bar against the FP64 form (rbfl_set_split_tol; default SPLIT_TOL)."""
        _check(load().rbfl_set_split_tol(self._h, float(tol)))

    def fuse_epilogue(self, on: bool, split: bool = False):
        """ln L finished inside the FP64 contraction (`on`) and inside the split contraction
        (`split`) (rbfl_fuse_epilogue; sets both); the autotuner sets them."""
        _check(load().rbfl_fuse_epilogue(self._h, (1 if on else 0) | (2 if split else 0)))

    def pipeline(self) -> dict:
        """The FP64 evaluation order in use and the autotuner's ms per evaluation (RBFL_Q_PIPELINE):
        chunks per call, ms at 1, 2, 4, 8 chunks, ln L inside the contraction and its ms."""
        v = self._query(Q_PIPELINE, 7)
        return {"chunks": int(v[0]), "ms": {d: float(x) for d, x in zip((1, 2, 4, 8), v[1:5]) if x > 0},
                "fused_epilogue": bool(v[5]), "fused_epilogue_ms": float(v[6])}

    def profile(self, on: bool):
        _check(load().rbfl_profile(self._h, 1 if on else 0))

    def kernel_stats(self) -> dict:
        v = self._query(Q_KERNEL_STATS, 9)
        return {"contract_ms": v[0], "contract_launches": int(v[1]), "contract_n": int(v[2]),
                "epilogue_ms": v[3], "epilogue_launches": int(v[4]), "epilogue_n": int(v[5]),
                "rows_ms": v[6], "rows_launches": int(v[7]), "rows_n": int(v[8])}


def variants(form: int) -> int:
    """Number of contraction tile variants of `form` (rbfl_variants)."""
    v = load().rbfl_variants(form)
    if v < 0:
        raise ValueError(f"no tile variants for form {form}")
    return v


def split_slices(variant: int) -> int:
    """Digit count S of a split-form contraction variant."""
    return 5 + variant


class Plan:
    """A multi-event batch plan (rbfl_plan_*): fixed events, proposal counts and
    device buffers; launch() replays it (as a HIP graph with PLAN_GRAPH)."""

    def __init__(self, handles, counts, params_ptr: int, lnl_ptr: int, flags: int = PLAN_GRAPH | PLAN_AUTOTUNE,
                 stream: int = 0):
        self._handles = list(handles)          # keep the events alive as long as the plan
        arr = (C.c_void_p * len(handles))(*[h.ptr for h in handles])
        cnt = (C.c_int64 * len(counts))(*[int(x) for x in counts])
        p = C.c_void_p()
        _check(load().rbfl_plan_create(arr, len(handles), cnt, C.c_void_p(params_ptr), C.c_void_p(lnl_ptr), flags,
                                       C.c_void_p(stream), C.byref(p)))
        self._p = p

    def launch(self, stream: int = 0):
        _check(load().rbfl_plan_launch(self._p, C.c_void_p(stream)))

    def set_variant(self, variant: int, stream: int = 0):
        """Pins the FP64 tile variant (rbfl_plan_set_variant)."""
        _check(load().rbfl_plan_set_variant(self._p, variant, C.c_void_p(stream)))

    def info(self) -> dict:
        v = np.zeros(16)
        _check(load().rbfl_plan_query(self._p, v.ctypes.data_as(C.c_void_p), v.nbytes))
        out = {"variant": int(v[0]), "items": int(v[1]), "grid": int(v[2]), "proposals": int(v[3]),
               "tune_ms": [float(x) for x in v[4:12] if x > 0]}
        if v[12]:
            out.update({"form": "split", "slices_min": int(v[13]), "slices_max": int(v[14]),
                        "within_split_tol": None if v[15] < 0 else bool(v[15])})
        return out

    def close(self):
        if self._p is not None and self._p.value:
            _check(load().rbfl_plan_destroy(self._p))
        self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The library's surrogate network on its own (rbfl_mlp_*), FP32 on the device."""

    def __init__(self, n_in: int, hidden: int, n_out: int, normals: np.ndarray):
        z = np.ascontiguousarray(normals, dtype=np.float64)
        assert z.size == mlp_param_count(n_in, hidden, n_out)
        p = C.c_void_p()
        _check(load().rbfl_mlp_create(n_in, hidden, n_out, _dptr(z), C.byref(p)))
        self._p = p
        self.n_params = z.size

    def forward(self, x_ptr: int, B: int, y_ptr: int, stream: int = 0):
        _check(load().rbfl_mlp_forward(self._p, C.c_void_p(x_ptr), B, C.c_void_p(y_ptr), C.c_void_p(stream)))

    def loss_grad(self, x_ptr: int, t_ptr: int, B: int, stream: int = 0) -> float:
        l = C.c_double()
        _check(load().rbfl_mlp_loss_grad(self._p, C.c_void_p(x_ptr), C.c_void_p(t_ptr), B, C.byref(l),
                                         C.c_void_p(stream)))
        return l.value

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream: int = 0):
        _check(load().rbfl_mlp_adam(self._p, lr, beta1, beta2, eps, C.c_void_p(stream)))

    def get(self, what: int) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(load().rbfl_mlp_get(self._p, what, out.ctypes.data_as(C.c_void_p), out.nbytes))
        return out

    def close(self):
        if self._p is not None and self._p.value:
            _check(load().rbfl_mlp_destroy(self._p))
        self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sampler:
    """Ensemble sampler driving a handle's online stage (rbfl_sampler_*)."""

    def __init__(self, handle: "Handle", walkers: int, t_range, d_range, seed: int = 1, form: int = FORM_FP64,
                 d_exp: float = 0.0, gamma: float = 0.0, p_jump: float = 0.1, prior_only: bool = False,
                 init_ptr: int = 0, anneal_steps: int = 0, beta0: float = 1.0, stream: int = 0):
        spec = SamplerSpec(walkers=walkers, form=form, seed=seed, t_lo=t_range[0], t_hi=t_range[1],
                           d_lo=d_range[0], d_hi=d_range[1], d_exp=d_exp, gamma=gamma, p_jump=p_jump,
                           flags=SAMPLER_PRIOR_ONLY if prior_only else 0, anneal_steps=anneal_steps,
                           beta0=beta0)
        self.walkers = walkers
        self._handle = handle          # the handle must outlive the sampler
        self._s = C.c_void_p()
        _check(load().rbfl_sampler_create(handle.ptr, C.byref(spec), C.c_void_p(init_ptr or None),
                                          C.c_void_p(stream), C.byref(self._s)))

    def run(self, steps: int, thin: int = 1, chain_ptr: int = 0, slots: int = 0, stream: int = 0):
        _check(load().rbfl_sampler_run(self._s, steps, thin, C.c_void_p(chain_ptr or None), slots,
                                       C.c_void_p(stream)))

    def smc(self, ess_frac: float = 0.5, moves: int = 10, max_stages: int = 200, stream: int = 0):
        """Tempered SMC start; returns (log evidence, stages, final beta)."""
        lz, st, b = C.c_double(0.0), C.c_int32(0), C.c_double(0.0)
        _check(load().rbfl_sampler_smc(self._s, ess_frac, moves, max_stages, C.c_void_p(stream), C.byref(lz),
                                       C.byref(st), C.byref(b)))
        return lz.value, st.value, b.value

    def walkers_state(self) -> np.ndarray:
        out = np.empty((12, self.walkers))
        _check(load().rbfl_sampler_query(self._s, 0, out.ctypes.data_as(C.c_void_p), out.nbytes))
        return out

    def accepted(self) -> np.ndarray:
        out = np.empty(self.walkers)
        _check(load().rbfl_sampler_query(self._s, 1, out.ctypes.data_as(C.c_void_p), out.nbytes))
        return out

    def stats(self) -> tuple:
        out = np.empty(2)
        _check(load().rbfl_sampler_query(self._s, 2, out.ctypes.data_as(C.c_void_p), out.nbytes))
        return int(out[0]), float(out[1])

    def close(self):
        if self._s is not None and self._s.value:
            _check(load().rbfl_sampler_destroy(self._s))
        self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def prior_weights(handle: "Handle", params_ptr: int, ld: int, n: int, box, d_exp: float, logw_ptr: int,
                  stream: int = 0, want_n_eff: bool = True):
    """Log importance weights to a prior uniform in (m1, m2, chi1, chi2) within
    box (rbfl_prior_weights); returns N_eff when asked."""
    b = (C.c_double * 8)(*[float(v) for v in box])
    ne = C.c_double(0.0)
    _check(load().rbfl_prior_weights(handle.ptr, C.c_void_p(params_ptr), ld, n, b, d_exp, C.c_void_p(logw_ptr),
                                     C.byref(ne) if want_n_eff else None, C.c_void_p(stream)))
    return ne.value if want_n_eff else None


def eval_ragged(handles, counts, params_ptr: int, lnl_ptr: int, stream: int = 0):
    arr = (C.c_void_p * len(handles))(*[h.ptr for h in handles])
    cnt = (C.c_int64 * len(counts))(*[int(x) for x in counts])
    _check(load().rbfl_eval_ragged(arr, len(handles), cnt, C.c_void_p(params_ptr), C.c_void_p(lnl_ptr),
                                   C.c_void_p(stream)))


def params_soa(handle: Handle, qd, t_trig: float) -> np.ndarray:
    """[11][n] parameter array in the paper's coordinates for a normalised
    query draw, using this handle's own semi-axes and reference distance."""
    semi = handle.frame()["semi"]
    n = len(qd)
    p = np.empty((11, n))
    p[0:4] = (qd.x * semi[None, :]).T
    p[4:9] = qd.ext.T
    p[9] = t_trig + qd.dt
    p[10] = handle.d_ref() * qd.dist_ratio
    return p
