"""Full-size handles shared by the GPU test modules of one pytest process, so
that each large start-up runs once: the 3-detector five-mode workload
(N = 800), the single-detector cubic-tail workload (N = 1500, M = 35) and the
third-generation workload (N = 3000, K = 2475)."""
import time

import numpy as np

from paper_2508_04172_amd import rbfl
from paper_2508_04172_amd import workloads as wl

CONFIGS = {"cfg2": wl.CFG2, "cfg3": wl.CFG3, "cfg5": wl.CFG5}
_handles = {}


def handle(name):
    """(config, handle) of a full-size workload, built on first use."""
    if name not in _handles:
        cfg = CONFIGS[name]
        print(f"[full] GPU start-up {cfg.name}", flush=True)
        t0 = time.time()
        h = rbfl.Handle.from_config(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg))
        print(f"[full] {cfg.name}: start-up {time.time() - t0:.1f} s, stages {np.round(h.timing()[:6], 2)}, "
              f"sizes {h.sizes()}, cond {h.cond():.2e}", flush=True)
        _handles[name] = (cfg, h)
    return _handles[name]
