"""Benchmark: ln L evaluations per second of the meshfree likelihood on one GPU.

One step = one pass of the whole online stage (query ingest, kernel rows,
MFMA contraction, spline/reconstruction, extrinsic combination) over a batch
of 1e6 seeded proposals of the 3-detector, 5-mode workload (N = 800 nodes,
q = 40, K = 1275 interpolated reals per proposal), with the proposals
already resident in HBM.  Prints one JSON line.

Also reported: the reduced-precision forms' throughput and their max |d ln L|
against the FP64 oracle on a seeded sample, the dominant kernel's roofline
(its HIP-event duration per launch), and the oracle's own throughput on the
host cores (baseline only).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ln L evals/s at |dlnL|<=1e-3 vs FP64 oracle: plain vs mixed/batched/surrogate"
PEAK_FP64 = 78.6e12     # dense FP64 MFMA, MI355X
PEAK_FP32 = 157.3e12    # dense FP32 MFMA, MI355X
PEAK_BF16 = 2.5e15      # dense bf16 MFMA, MI355X
PEAK_HBM = 8.0e12       # HBM3E, MI355X
PEAK_INT8 = 5.0e15      # dense int8 MFMA, MI355X


def roof(achieved, peak, unit="TFLOP/s", bound="mfma", **extra):
    """Roofline object of one form's dominant kernel: achieved and peak in
    units of 1e12 per second, and their ratio."""
    return dict({"bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": unit,
                 "frac": achieved / peak}, **extra)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


PROFILE = os.path.join(ROOT, "profiles", "k_gemm_fp64_cfg2_hlv_5mode.md")


def gemm_source_hash() -> str:
    """Hash of what fixes the FP64 GEMM's memory traffic: its source file and
    the row and column padding of the library."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2508_04172_amd", "csrc")
    h = hashlib.sha256(open(os.path.join(csrc, "contract_fp64.hip"), "rb").read())
    consts = open(os.path.join(csrc, "rbfl_internal.h")).read()
    for name in ("kRowChunk", "kColTile"):
        h.update(re.search(rf"constexpr int {name} = (\d+);", consts).group(0).encode())
    return h.hexdigest()[:16]


def recorded_traffic(variant: int, per_launch_n: float):
    """HBM bytes per launch of k_gemm_fp64 (FETCH_SIZE and WRITE_SIZE, each
    scaled by the copy-kernel calibration) from the committed profile summary,
    for this source and tile variant, scaled to the average launch; None when
    the kernel has changed since the counters were taken."""
    if not os.path.exists(PROFILE):
        return None
    src = gemm_source_hash()
    for line in open(PROFILE):
        if not line.startswith("traffic-record:"):
            continue
        kv = dict(f.split("=", 1) for f in line.split()[1:])
        if kv.get("kernel") == "k_gemm_fp64" and kv.get("source") == src and int(kv["variant"]) == variant:
            return float(kv["bytes"]) * per_launch_n / float(kv["proposals"])
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--queries", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=200000)
    ap.add_argument("--check-sample", type=int, default=2000)
    ap.add_argument("--ragged-build-threads", type=int, default=4,
                    help="host threads (one stream each) building the multi-event batch's handles")
    ap.add_argument("--ragged-events", type=int, default=64,
                    help="events in the multi-event batch form (0 = skip)")
    ap.add_argument("--surrogate-train", type=int, default=200000,
                    help="training proposals for the surrogate form (0 = skip)")
    ap.add_argument("--surrogate-epochs", type=int, default=20)
    ap.add_argument("--third-generation-surrogate", type=int, default=200000,
                    help="training proposals for the surrogate on the third-generation workload (0 = skip)")
    ap.add_argument("--no-third-generation", action="store_true",
                    help="skip the FP64 and surrogate forms on the third-generation workload (2048 s at 4096 Hz, "
                         "N=3000, K=2475, 1e6 proposals per pass)")
    ap.add_argument("--no-rotating", action="store_true",
                    help="skip the third-generation workload on a rotating Earth (sidereal rate): patterns "
                         "frozen at t_c against 16 time bands, error against the exact rotating-Earth ln L")
    ap.add_argument("--rotating-bands", type=int, default=16)
    ap.add_argument("--no-mixed-cfg3", action="store_true",
                    help="skip every arithmetic form on the 10 Hz single-detector cubic-tail workload "
                         "(N=1500, M=35, q=60, 4e6 proposals)")
    ap.add_argument("--method-error", action="store_true",
                    help="also report the method's error against the exact ln L (rbfl_brute) at matches "
                         "0.90/0.95/0.97/0.99 on the single-detector workload (1e4 proposals each) and on "
                         "the 3-detector workload, with the exact path's throughput")
    ap.add_argument("--sampler", action="store_true",
                    help="also run a GPU-resident parameter estimation on the 3-detector workload: "
                         "differential-evolution ensemble driving the FP64 online stage, then prior reweighting")
    ap.add_argument("--sampler-walkers", type=int, default=65536)
    ap.add_argument("--sampler-steps", type=int, default=200)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one elementwise 512 MiB copy kernel (known bytes, for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is a design "
              "note only", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2508_04172_amd import rbfl
    from paper_2508_04172_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    cfg = wl.CFG2
    n = args.queries or cfg.n_queries
    white = wl.white_noise(cfg)
    inj = wl.injection_extrinsics(cfg)

    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")     # 512 MiB
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)       # one elementwise kernel: 512 MiB read, 512 MiB written
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 512 MiB read + 512 MiB written")
    log("GPU start-up (rbfl_build)")
    t0 = time.time()
    h = rbfl.Handle.from_config(cfg, white, inj)
    build_s = time.time() - t0
    sz = h.sizes()
    log(f"start-up {build_s:.2f} s, sizes {sz}, cond {h.cond():.3e}")

    idx, jit = wl.node_jitter(n, cfg.n_nodes)
    qd = wl.queries(cfg, n=n)
    q_gpu = qd.near_nodes(h.nodes(), idx, jit)
    params = torch.from_numpy(np.ascontiguousarray(rbfl.params_soa(h, q_gpu, cfg.t_trig))).cuda()
    lnl = torch.empty(n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    # one chunk per step: the work space for 1e6 proposals (Y 10 GB, basis rows
    # 6.7 GB for this workload) fits easily in 288 GB of HBM, and one launch
    # per stage avoids the gaps and tails of sixteen smaller ones
    h.reserve(min(n, 1 << 20))
    tune = {}
    for name, form in (("fp64", rbfl.FORM_FP64), ("fp32", rbfl.FORM_FP32), ("bf16", rbfl.FORM_BF16),
                       ("split", rbfl.FORM_SPLIT)):
        if form != rbfl.FORM_FP64:
            h.prepare(form)
        tune[name] = h.autotune(params.data_ptr(), n, form, sp)
        log(f"autotune {name}: variant {tune[name]['variant']}, ms per launch {tune[name]['ms']}")
        if form == rbfl.FORM_FP64:
            tune["fp64_pipeline"] = h.pipeline()
            log(f"autotune fp64 pipeline: {tune['fp64_pipeline']}")
        if form == rbfl.FORM_SPLIT:
            tune["split_order"] = h.split_order()
            log(f"autotune split order: {tune['split_order']}")

    def run_form(form, steps, warmup):
        for _ in range(warmup):
            h.eval(params.data_ptr(), n, lnl.data_ptr(), form, sp)
        torch.cuda.synchronize()
        h.profile(True)
        t = time.perf_counter()
        for _ in range(steps):
            h.eval(params.data_ptr(), n, lnl.data_ptr(), form, sp)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        h.profile(False)
        ks = h.kernel_stats()
        return wall, ks, lnl.cpu().numpy()

    log(f"timing FP64 form: {args.warmup} warmup + {args.steps} steps of {n} proposals")
    wall, ks, l64 = run_form(rbfl.FORM_FP64, args.steps, args.warmup)
    ms_per_step = wall / args.steps * 1e3
    value = n * args.steps / wall
    NM, K = sz["N"] + sz["M"], sz["K"]
    flop_per_query = 2.0 * NM * K
    per_launch_n = ks["contract_n"] / max(1, ks["contract_launches"])
    contract_ms = ks["contract_ms"] / max(1, ks["contract_launches"])
    achieved = flop_per_query * per_launch_n / (contract_ms * 1e-3)
    rows_ms = ks["rows_ms"] / max(1, ks["rows_launches"])
    epi_ms = ks["epilogue_ms"] / max(1, ks["epilogue_launches"])
    # basis-row stage: writes 8 bytes per padded row per proposal, reads 32 bytes of coordinates
    rows_padded = (NM + 15) // 16 * 16      # the rows kernel writes N + M rounded up to 16-row groups
    rows_bytes = (8.0 * rows_padded + 32.0) * per_launch_n
    fp64_variant = tune["fp64"]["variant"]
    fused = fp64_variant == len(tune["fp64"]["ms"]) - 1    # the last FP64 variant is the fused kernel
    log(f"FP64: {value:.4e} evals/s, {ms_per_step:.2f} ms/step; rows {rows_ms:.3f} ms/launch, contraction "
        f"{contract_ms:.3f} ms/launch ({achieved / 1e12:.2f} TFLOP/s), epilogue {epi_ms:.3f} ms/launch")

    forms = {"fp64": {"evals_per_s": value, "ms_per_step": ms_per_step, "variant": fp64_variant,
                      "contract_ms_per_launch": contract_ms, "contract_tflops": achieved / 1e12,
                      "rows_ms_per_launch": rows_ms,
                      "rows_gbs": rows_bytes / (rows_ms * 1e-3) / 1e9 if rows_ms > 0 else None,
                      "epilogue_ms_per_launch": epi_ms}}
    outs = {"fp64": l64}
    # the split form twice: with the tuner's default bar (within RBFL_SPLIT_TOL =
    # 1e-4 of the FP64 form on the tuning proposals, a tenth of the 1e-3 target)
    # and with half the target as the bar (fewer digits where these proposals allow)
    for name, form in (("fp32", rbfl.FORM_FP32), ("bf16", rbfl.FORM_BF16), ("split", rbfl.FORM_SPLIT),
                       ("split_tol_5e-4", rbfl.FORM_SPLIT)):
        if name == "split_tol_5e-4":
            h.set_split_tol(5e-4)
            tune[name] = h.autotune(params.data_ptr(), n, form, sp)
            tune[name + "_order"] = h.split_order()
            log(f"autotune {name}: variant {tune[name]['variant']}, ms per launch {tune[name]['ms']}, "
                f"order {tune[name + '_order']}")
        w2, ks2, lf = run_form(form, max(3, args.steps // 2), 1)
        v2 = n * max(3, args.steps // 2) / w2
        c2 = ks2["contract_ms"] / max(1, ks2["contract_launches"])
        ach = flop_per_query * per_launch_n / (c2 * 1e-3)
        forms[name] = {"evals_per_s": v2, "ms_per_step": w2 / max(3, args.steps // 2) * 1e3,
                       "contract_ms_per_launch": c2, "contract_tflops": ach / 1e12}
        if form == rbfl.FORM_FP32:
            forms[name]["roofline"] = roof(ach, PEAK_FP32, kernel="k_contract_fp32")
        elif form == rbfl.FORM_BF16:
            # reads (N+M) bf16 row entries and writes K FP64 outputs per proposal: at
            # 2 (N+M) K / (2 (N+M) + 8 K) flop per byte it sits below the bf16 ridge
            # (2.5e15 / 8e12 = 312 flop/B), so HBM bounds it
            bytes_launch = per_launch_n * (2.0 * NM + 8.0 * K) + 2.0 * NM * K
            gbs = bytes_launch / (c2 * 1e-3)
            forms[name]["roofline"] = {"bound": "hbm", "achieved": gbs / 1e9, "peak": PEAK_HBM / 1e9,
                                       "unit": "GB/s", "frac": gbs / PEAK_HBM, "kernel": "k_bf16_contract",
                                       "bytes_per_launch": bytes_launch,
                                       "mfma_tflops": ach / 1e12, "mfma_frac": ach / PEAK_BF16}
        if form == rbfl.FORM_SPLIT:
            # int8 products actually issued: one per slice pair i + j < S
            S = tune[name]["slices"]
            pairs = S * (S + 1) // 2
            tops = pairs * flop_per_query * per_launch_n / (c2 * 1e-3)
            fused = tune[name + "_order"]["fused_epilogue"]
            forms[name].update({"slices": S, "int8_tops": tops / 1e12, "int8_frac": tops / PEAK_INT8,
                                "tuner_tol": 5e-4 if name == "split_tol_5e-4" else rbfl.SPLIT_TOL,
                                "max_dlnl_vs_fp64_per_slice_count": tune[name]["max_dlnl_vs_fp64"][:4],
                                "order": tune[name + "_order"],
                                "roofline": roof(tops, PEAK_INT8, unit="TOP/s",
                                                 kernel="k_split_lnl (ln L inside the contraction; int8 products "
                                                        "issued)" if fused else
                                                 "k_split_contract (int8 products issued)")})
        outs[name] = lf
        log(f"{name}: {v2:.4e} evals/s, contraction {c2:.3f} ms/launch")
    h.set_split_tol(rbfl.SPLIT_TOL)

    if args.surrogate_train > 0:
        forms["surrogate"] = bench_surrogate(args, np, torch, rbfl, wl, cfg, h, params, lnl, l64,
                                             args.surrogate_train, args.surrogate_epochs, max(3, args.steps // 2))
    if args.ragged_events > 0:
        forms["ragged"] = bench_ragged(args, np, torch, rbfl, wl)

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg.name, "form": "plain FP64", "proposals_per_step": n,
                   "pipeline_chunks": tune["fp64_pipeline"]["chunks"],
                   "n_det": cfg.n_det, "modes": len(cfg.modes), "nodes": cfg.n_nodes, "q": cfg.q,
                   "K": K, "poly_degree": cfg.poly_degree, "eps": cfg.eps, "fs": cfg.fs,
                   "seg_len": cfg.seg_len, "f_low": cfg.f_low, "startup_s": round(build_s, 3)},
        "roofline": {"bound": "mfma", "kernel": "k_contract_fp64 (fused rows)" if fused else "k_gemm_fp64",
                     "achieved": achieved / 1e12,
                     "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64,
                     "traffic": None if fused else recorded_traffic(fp64_variant, per_launch_n),
                     "flop_per_launch": flop_per_query * per_launch_n,
                     "launch_ms": contract_ms},
        "forms": forms,
        "autotune": tune,
    }

    # accuracy of every form against the FP64 oracle on a seeded sample, and
    # the oracle's own throughput on the host cores
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_info
        from oracle import likelihood as lk
        from oracle import startup as su
        log("oracle start-up on the host")
        t = time.perf_counter()
        art = su.startup(cfg, white, inj)
        oracle_startup_s = time.perf_counter() - t
        log(f"oracle start-up {oracle_startup_s:.1f} s (rbfl_build {build_s:.2f} s)")
        rng = np.random.default_rng(321)
        m = min(args.cpu_sample, n)
        sample = np.sort(rng.choice(n, m, replace=False))
        q_cpu = qd.subset(sample).near_nodes(art.x_nodes, idx[sample], jit[sample])
        args_cpu = lk.query_params(art, q_cpu)
        log(f"oracle ln L on {m} sampled proposals")
        t = time.perf_counter()
        lo = lk.meshfree_lnl(art, *args_cpu)
        cpu_s = time.perf_counter() - t
        info = threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] or [1])
        blas = "; ".join(f"{i.get('internal_api')} {i.get('version')} ({os.path.basename(i.get('filepath', ''))}, "
                         f"{i.get('num_threads')} threads)" for i in info if i.get("user_api") == "blas")
        # one thread: a smaller seeded part of the same sample (same per-proposal work)
        m1 = min(m, max(2000, m // 10))
        from threadpoolctl import threadpool_limits
        sub1 = qd.subset(sample[:m1]).near_nodes(art.x_nodes, idx[sample[:m1]], jit[sample[:m1]])
        with threadpool_limits(limits=1):
            t = time.perf_counter()
            lk.meshfree_lnl(art, *lk.query_params(art, sub1))
            cpu1_s = time.perf_counter() - t
        result["cpu_baseline"] = {"value": m / cpu_s, "unit": "evals/s", "cores": int(threads),
                                  "kind": "oracle",
                                  "sample": f"{m} of the {n} proposals (seeded), FP64 numpy/BLAS, "
                                            f"{cpu_s:.1f} s; host os.cpu_count()={os.cpu_count()}",
                                  "single_thread_value": m1 / cpu1_s,
                                  "single_thread_sample": f"the first {m1} of that sample, {cpu1_s:.1f} s, BLAS "
                                                          "limited to 1 thread",
                                  "blas": blas,
                                  "startup_s": round(oracle_startup_s, 1),
                                  "startup_note": "the oracle's start-up (data, frame, nodes, FFT overlap series, "
                                                  "SVD, RBF solve) on the same host; rbfl_build took "
                                                  f"{build_s:.2f} s on the GPU"}
        log(f"oracle: {m / cpu_s:.4e} evals/s on {threads} threads, {m1 / cpu1_s:.4e} on one ({blas})")
        fin = np.isfinite(lo)
        for name, l in outs.items():
            lg = l[sample]
            agree = bool(np.array_equal(fin, np.isfinite(lg)))
            d = np.abs(lg[fin] - lo[fin]) if fin.any() else np.array([np.inf])
            forms[name].update({"max_dlnl": float(d.max()), "p99_dlnl": float(np.quantile(d, 0.99)),
                                "median_dlnl": float(np.median(d)), "domain_agrees": agree,
                                "meets_1e-3": bool(agree and d.max() <= 1e-3)})
        result["config"]["valid_fraction"] = float(fin.mean())
    if args.sampler:
        result["sampler"] = bench_sampler(args, np, torch, rbfl, wl, cfg)
    if args.method_error:
        result["method_error"] = bench_method_error(np, torch, rbfl, wl, h, cfg, qd, idx, jit)
    if not args.no_third_generation:
        result["third_generation"] = bench_third_generation(args, np, torch, rbfl, wl)
    if not args.no_mixed_cfg3:
        result["mixed_cfg3"] = bench_mixed(args, np, torch, rbfl, wl, wl.CFG3)
    if not args.no_rotating:
        result["rotating"] = bench_rotating(args, np, torch, rbfl, wl)
    print(json.dumps(result), flush=True)


def bench_surrogate(args, np, torch, rbfl, wl, cfg, h, params, lnl, l64, n_train, epochs, steps):
    """Surrogate form: MLP 4 -> 256 -> 256 -> K trained by the library's own
    kernels on proposals whose targets the FP64 interpolant computes; checked on
    1e4 held-out proposals at |d ln L| <= 1e-3 (fallback to the interpolant
    otherwise).  The network path's throughput is reported either way, and the
    network's own kernels (the three FP32 MFMA layers, HIP events) against the
    FP32 matrix-core peak."""
    n = params.shape[1]
    K = h.sizes()["K"]
    hidden = 256
    z = wl.mlp_normals(rbfl.mlp_param_count(4, hidden, K))

    def dev(m, seed):
        idx, jit = wl.node_jitter(m, cfg.n_nodes, seed=seed)
        qd = wl.queries(cfg, n=m, seed=seed).near_nodes(h.nodes(), idx, jit)
        return torch.from_numpy(np.ascontiguousarray(rbfl.params_soa(h, qd, cfg.t_trig))).cuda()

    tr = dev(n_train, 5)
    ho = dev(10000, 6)
    log(f"surrogate: training on {n_train} proposals, {epochs} epochs")
    st = h.surrogate_train(z, tr.data_ptr(), n_train, ho.data_ptr(), 10000, hidden=hidden,
                           batch=1024, epochs=epochs, lr=1e-3, threshold=1e-3)
    del tr, ho
    log(f"surrogate: {st}")
    h.surrogate_force(True)
    sp = torch.cuda.current_stream().cuda_stream
    h.eval(params.data_ptr(), n, lnl.data_ptr(), rbfl.FORM_SURROGATE, sp)
    torch.cuda.synchronize()
    h.profile(True)
    t = time.perf_counter()
    for _ in range(steps):
        h.eval(params.data_ptr(), n, lnl.data_ptr(), rbfl.FORM_SURROGATE, sp)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    h.profile(False)
    ks = h.kernel_stats()
    ls = lnl.cpu().numpy()
    h.surrogate_force(False)
    fin = np.isfinite(l64) & np.isfinite(ls)
    d = np.abs(ls[fin] - l64[fin])
    flop = 2.0 * (4 * hidden + hidden * hidden + hidden * K)
    res = {"network_evals_per_s": n * steps / wall, "network_ms_per_step": wall / steps * 1e3,
           "accepted": st["accepted"], "holdout_max_dlnl": st["holdout_max_dlnl"],
           "holdout_median_dlnl": st["holdout_median_dlnl"], "train_s": st["train_s"],
           "n_train": st["n_train"], "epochs": st["epochs"], "first_loss": st["first_loss"],
           "last_loss": st["last_loss"], "max_dlnl_vs_fp64_gpu_all": float(d.max()),
           "median_dlnl_vs_fp64_gpu_all": float(np.median(d)), "network_flop_per_eval": flop,
           "note": "the surrogate form evaluates the FP64 interpolant unless accepted"}
    net_ms = ks["contract_ms"] / max(1, ks["contract_launches"])
    if net_ms > 0:
        ach = flop * ks["contract_n"] / max(1, ks["contract_launches"]) / (net_ms * 1e-3)
        res.update({"network_ms_per_launch": net_ms, "epilogue_ms_per_launch":
                    ks["epilogue_ms"] / max(1, ks["epilogue_launches"]),
                    "roofline": roof(ach, PEAK_FP32, kernel="k_gemm_f32 + k_gemm_f32_nt (MLP layers)")})
    log(f"surrogate: network path {res['network_evals_per_s']:.4e} evals/s, accepted={st['accepted']}")
    return res


def bench_sampler(args, np, torch, rbfl, wl, cfg0):
    """Parameter estimation on the GPU (sampling in Delta e, Sec. II D) for the
    3-detector workload, start-up from an offset seed with the SNR-optimised
    centre and the squeezed ellipsoid: W walkers from the prior
    (t_c within the workload's span, d_L uniform in [d_ref / 2, 2 d_ref]), a
    tempered sequential Monte Carlo start (effective size 1/2 per stage, 10
    differential-evolution moves per stage) up to the full likelihood, then
    `steps` more moves of which every 10th state is kept; every proposal
    through the FP64 online stage; the samples reweighted to Table I's
    component-mass and spin box (N_eff).  Wall-clock of each phase, ln L
    evaluations/s, acceptance, log evidence, posterior medians."""
    stream = torch.cuda.current_stream().cuda_stream
    # the start-up as the paper runs it: a seed template off the injection
    # (inside the match ellipsoid, as a bank's best match would be), the
    # network-SNR optimised centre, the squeezed ellipsoid
    cfg = cfg0.with_(name=cfg0.name + "_optimised_squeezed", squeeze=True, optimise_centre=True,
                     centre_offset=(0.002, 0.0, 0.01, 0.0))
    t0 = time.perf_counter()
    h = rbfl.Handle.from_config(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg))
    t_build = time.perf_counter() - t0
    centre = h.centre()
    W, steps = args.sampler_walkers, args.sampler_steps
    thin = 10
    slots = steps // thin
    t0 = time.perf_counter()
    s = rbfl.Sampler(h, W, (cfg.t_trig - cfg.tc_span, cfg.t_trig + cfg.tc_span), (0.5 * h.d_ref(), 2.0 * h.d_ref()),
                     seed=7, p_jump=0.1, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log_z, stages, beta = s.smc(ess_frac=0.5, moves=10, max_stages=200, stream=stream)
    n_smc, _ = s.stats()
    t2 = time.perf_counter()
    chain = torch.empty((12, slots, W), dtype=torch.float64, device="cuda")
    s.run(steps, thin=thin, chain_ptr=chain.data_ptr(), slots=slots, stream=stream)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    n_done, acc = s.stats()
    s.close()
    logw = torch.empty(slots * W, dtype=torch.float64, device="cuda")
    box = (5.0, 20.0, 1.0, 3.0, -0.998, 0.998, -0.05, 0.05)
    n_eff = rbfl.prior_weights(h, chain.data_ptr(), slots * W, slots * W, box, 0.0, logw.data_ptr(), stream=stream)
    t4 = time.perf_counter()
    C = chain.cpu().numpy().reshape(12, -1)
    inj = wl.injection_extrinsics(cfg)
    p = torch.zeros((11, 1), dtype=torch.float64)
    p[4:9, 0] = torch.from_numpy(np.asarray(inj))
    p[9, 0] = cfg.t_trig
    p[10, 0] = h.d_ref()
    pg = p.cuda()
    li = torch.empty(1, dtype=torch.float64, device="cuda")
    h.eval(pg.data_ptr(), 1, li.data_ptr(), rbfl.FORM_FP64, stream)
    torch.cuda.synchronize()
    out = {"workload": cfg.name, "walkers": W, "start_up_s": t_build, "start_up_stages_s": list(h.timing()[:6]),
           "seed_phys": list(cfg.seed_phys), "centre_phys": [float(v) for v in centre["phys"]],
           "centre_snr_seed": centre["snr_seed"], "centre_snr_opt": centre["snr_opt"],
           "squeeze_factor": h.squeeze()[0], "smc_stages": stages, "smc_steps": n_smc,
           "final_beta": beta, "log_evidence": log_z, "sampling_steps": n_done - n_smc, "thin": thin,
           "kept_samples": int(slots * W), "evals": int(W * n_done + W),
           "create_s": t1 - t0, "smc_s": t2 - t1, "sampling_s": t3 - t2, "reweight_s": t4 - t3,
           "pe_wall_s": t4 - t0, "evals_per_s": W * n_done / (t3 - t1), "acceptance_overall": acc,
           "n_eff_table1_box": n_eff, "lnl_at_injection": float(li.cpu()[0]),
           "median_lnl": float(np.median(C[11])), "max_lnl": float(np.max(C[11])),
           "median_abs_dt_ms": float(np.median(np.abs(C[9] - cfg.t_trig)) * 1e3),
           "median_d_over_dref": float(np.median(C[10]) / h.d_ref()),
           "median_iota": float(np.median(C[7])), "iota_injected": float(inj[3])}
    log(f"sampler: {out}")
    return out


def bench_method_error(np, torch, rbfl, wl, h2, cfg2, qd2, idx2, jit2):
    """The meshfree approximation against the exact ln L on the same GPU: the
    single-detector (2,2) workload at four ellipsoid matches, unsqueezed and
    squeezed, with 1e4 proposals uniform in the ball and the extrinsic
    parameters at their injected values (the paper's Fig. 3 protocol), and
    the 3-detector workload on 2e3 of the bench's proposals.  The error is split with
    rbfl_exact_parts into the RBF interpolation (meshfree vs exact outputs on
    the time basis), the basis truncation (basis vs raw window samples) and
    the sub-sample spline (samples vs exact); with the exact path's
    throughput (one workgroup per proposal, direct band sums)."""
    sp = torch.cuda.current_stream().cuda_stream
    out = {"protocol": "|dlnL| quantiles over proposals where the meshfree ln L is finite; "
                       "parts: rbf = |meshfree - exact outputs on the basis|, truncation = |basis - raw samples|, "
                       "spline = |raw samples - exact|"}

    def q4(v):
        return {k: float(x) for k, x in zip(("median", "p90", "p99", "max"), np.quantile(v, [0.5, 0.9, 0.99, 1.0]))}

    def compare(h, params, n):
        p = torch.from_numpy(np.ascontiguousarray(params)).cuda()
        lm = torch.empty(n, dtype=torch.float64, device="cuda")
        lb = torch.empty(n, dtype=torch.float64, device="cuda")
        parts = torch.empty((2, n), dtype=torch.float64, device="cuda")
        h.eval(p.data_ptr(), n, lm.data_ptr(), rbfl.FORM_FP64, sp)
        h.brute(p.data_ptr(), n, lb.data_ptr(), sp)
        torch.cuda.synchronize()
        t = time.perf_counter()
        h.brute(p.data_ptr(), n, lb.data_ptr(), sp)
        torch.cuda.synchronize()
        brute_s = time.perf_counter() - t
        h.exact_parts(p.data_ptr(), n, parts.data_ptr(), sp)
        torch.cuda.synchronize()
        a, b, pr = lm.cpu().numpy(), lb.cpu().numpy(), parts.cpu().numpy()
        fin = np.isfinite(a)
        if not fin.any():
            return {"valid": 0}
        return {"valid": int(fin.sum()), "total": q4(np.abs(a[fin] - b[fin])),
                "rbf": q4(np.abs(a[fin] - pr[0][fin])), "truncation": q4(np.abs(pr[0][fin] - pr[1][fin])),
                "spline": q4(np.abs(pr[1][fin] - b[fin])),
                "median_abs_lnl": float(np.median(np.abs(b[fin]))), "max_lnl": float(np.max(b[fin])),
                "exact_evals_per_s": n / brute_s}

    cases = {}
    # the paper's Fig. 3 protocol: intrinsic points uniform in the ellipsoid,
    # every extrinsic parameter (sky, polarisation, inclination, phase,
    # distance, t_c) at its injected value
    runs = [(m, sq, 200, 1.0) for sq in (False, True) for m in (0.90, 0.95, 0.97, 0.99)]
    runs.append((0.97, True, 800, 2.0))
    for match, squeeze, n_nodes, eps in runs:
        name = f"cfg1_match{match:.2f}" + ("_squeezed" if squeeze else "") + (f"_N{n_nodes}" if n_nodes != 200 else "")
        cfg = wl.CFG1.with_(name=name, match=match, squeeze=squeeze, n_nodes=n_nodes, eps=eps)
        inj = wl.injection_extrinsics(cfg)
        h = rbfl.Handle.from_config(cfg, wl.white_noise(cfg), inj)
        n = 10000
        qd = wl.queries(cfg, n=n)
        qd.dt[:] = 0.0
        qd.ext[:, 4] = inj[4]
        qd.dist_ratio[:] = 1.0
        cases[name] = compare(h, rbfl.params_soa(h, qd, cfg.t_trig), n)
        cases[name].update(squeeze_factor=h.squeeze()[0], n_nodes=n_nodes, eps=eps, cond=h.cond())
        log(f"method error {name}: {cases[name]}")
    n = 2000
    p2 = rbfl.params_soa(h2, qd2.near_nodes(h2.nodes(), idx2, jit2), cfg2.t_trig)[:, :n]
    cases[cfg2.name] = compare(h2, p2, n)
    log(f"method error {cfg2.name}: {cases[cfg2.name]}")
    cfg2s = cfg2.with_(name=cfg2.name + "_squeezed", squeeze=True)
    t0 = time.time()
    h2s = rbfl.Handle.from_config(cfg2s, wl.white_noise(cfg2s), wl.injection_extrinsics(cfg2s))
    log(f"squeezed start-up {time.time() - t0:.2f} s, factor {h2s.squeeze()}")
    p2s = rbfl.params_soa(h2s, qd2.near_nodes(h2s.nodes(), idx2, jit2), cfg2.t_trig)[:, :n]
    cases[cfg2s.name] = compare(h2s, p2s, n)
    cases[cfg2s.name]["squeeze_factor"] = h2s.squeeze()[0]
    log(f"method error {cfg2s.name}: {cases[cfg2s.name]}")
    out["cases"] = cases
    return out


def bench_third_generation(args, np, torch, rbfl, wl):
    """The FP64 form on the third-generation workload: start-up time, then
    1e6 near-node proposals per pass in one launch per stage (autotuned tile
    and evaluation order), with the contraction's HIP-event time."""
    cfg = wl.CFG5
    n = 1_000_000
    log(f"third generation {cfg.name}: GPU start-up")
    t0 = time.time()
    h = rbfl.Handle.from_config(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg))
    build_s = time.time() - t0
    sz = h.sizes()
    log(f"third generation: start-up {build_s:.1f} s, sizes {sz}")
    idx, jit = wl.node_jitter(n, cfg.n_nodes)
    qd = wl.queries(cfg, n=n)
    params = torch.from_numpy(np.ascontiguousarray(rbfl.params_soa(h, qd.near_nodes(h.nodes(), idx, jit),
                                                                   cfg.t_trig))).cuda()
    lnl = torch.empty(n, dtype=torch.float64, device="cuda")
    sp = torch.cuda.current_stream().cuda_stream
    h.reserve(n)
    tune = h.autotune(params.data_ptr(), n, rbfl.FORM_FP64, sp)
    order = h.pipeline()
    log(f"third generation: tile {tune['variant']}, order {order}")
    h.eval(params.data_ptr(), n, lnl.data_ptr(), rbfl.FORM_FP64, sp)
    torch.cuda.synchronize()
    reps = 3
    h.profile(True)
    t = time.perf_counter()
    for _ in range(reps):
        h.eval(params.data_ptr(), n, lnl.data_ptr(), rbfl.FORM_FP64, sp)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / reps
    h.profile(False)
    ks = h.kernel_stats()
    flop = 2.0 * (sz["N"] + sz["M"]) * sz["K"]
    c_ms = ks["contract_ms"] / max(1, ks["contract_launches"])
    per = ks["contract_n"] / max(1, ks["contract_launches"])
    tflops = flop * per / (c_ms * 1e-3) / 1e12
    fin = lnl.isfinite()
    out = {"workload": cfg.name, "proposals_per_pass": n, "N": sz["N"], "M": sz["M"], "K": sz["K"], "q": sz["q"],
           "startup_s": round(build_s, 1), "evals_per_s": n / wall, "ms_per_pass": wall * 1e3,
           "tile_variant": tune["variant"], "order": order, "contract_ms_per_launch": c_ms,
           "contract_tflops": tflops, "contract_frac_of_fp64_peak": tflops * 1e12 / PEAK_FP64,
           "rows_ms_per_launch": ks["rows_ms"] / max(1, ks["rows_launches"]),
           "epilogue_ms_per_launch": ks["epilogue_ms"] / max(1, ks["epilogue_launches"]),
           "valid_fraction": float(fin.double().mean()), "any_nan": bool(lnl.isnan().any()),
           "roofline": roof(tflops * 1e12, PEAK_FP64, kernel="k_gemm_lnl_fp64" if order["fused_epilogue"]
                            else "k_gemm_fp64")}
    log(f"third generation: {n / wall:.4e} evals/s, contraction {c_ms:.2f} ms ({tflops:.2f} TFLOP/s)")
    l64 = lnl.cpu().numpy()
    if not args.no_cpu_baseline:
        from oracle import likelihood as lk
        from oracle import startup as su
        art = su.artefacts_from_exports(cfg, wl.injection_extrinsics(cfg), **h.exports())
        m = 2000
        sample = np.sort(np.random.default_rng(321).choice(n, m, replace=False))
        pe = params[:, sample].cpu().numpy()
        lo = lk.meshfree_lnl(art, pe[0:4].T.copy(), pe[4:9].T.copy(), pe[9].copy(), pe[10].copy())
        fin = np.isfinite(lo)
        agree = bool(np.array_equal(fin, np.isfinite(l64[sample])))
        d = np.abs(l64[sample][fin] - lo[fin])
        out.update({"max_dlnl": float(d.max()), "median_dlnl": float(np.median(d)), "domain_agrees": agree,
                    "meets_1e-3": bool(agree and d.max() <= 1e-3),
                    "check_sample": f"{m} seeded proposals of the pass; oracle online stage on the handle's "
                                    "exported artefacts"})
        log(f"third generation: max |dlnL| vs oracle {d.max():.3e}")
    # the split form on this workload: digit count and evaluation order tuned on
    # the pass (within RBFL_SPLIT_TOL of the FP64 form), then timed like it
    h.prepare(rbfl.FORM_SPLIT)
    tune_s = h.autotune(params.data_ptr(), n, rbfl.FORM_SPLIT, sp)
    h.eval(params.data_ptr(), n, lnl.data_ptr(), rbfl.FORM_SPLIT, sp)
    torch.cuda.synchronize()
    h.profile(True)
    t = time.perf_counter()
    for _ in range(reps):
        h.eval(params.data_ptr(), n, lnl.data_ptr(), rbfl.FORM_SPLIT, sp)
    torch.cuda.synchronize()
    wall_s = (time.perf_counter() - t) / reps
    h.profile(False)
    ks = h.kernel_stats()
    c_s = ks["contract_ms"] / max(1, ks["contract_launches"])
    S = tune_s["slices"]
    tops = S * (S + 1) / 2 * flop * per / (c_s * 1e-3)
    ls = lnl.cpu().numpy()
    order_s = h.split_order()
    out["split"] = {"evals_per_s": n / wall_s, "ms_per_pass": wall_s * 1e3, "slices": S,
                    "max_dlnl_vs_fp64_per_slice_count": tune_s["max_dlnl_vs_fp64"][:4], "order": order_s,
                    "contract_ms_per_launch": c_s, "speedup_vs_fp64": wall / wall_s,
                    "roofline": roof(tops, PEAK_INT8, unit="TOP/s",
                                     kernel="k_split_lnl (ln L inside the contraction; int8 products issued)"
                                     if order_s["fused_epilogue"] else "k_split_contract (int8 products issued)")}
    if not args.no_cpu_baseline:
        fin_s = np.isfinite(ls[sample])
        d = np.abs(ls[sample][fin] - lo[fin])
        out["split"].update({"max_dlnl": float(d.max()), "median_dlnl": float(np.median(d)),
                             "domain_agrees": bool(np.array_equal(fin, fin_s)),
                             "meets_1e-3": bool(np.array_equal(fin, fin_s) and d.max() <= 1e-3)})
    log(f"third generation split: S = {S}, {n / wall_s:.4e} evals/s ({wall / wall_s:.2f}x FP64), "
        f"contraction {c_s:.2f} ms, order {order_s}")
    if args.third_generation_surrogate > 0:
        out["surrogate"] = bench_surrogate(args, np, torch, rbfl, wl, cfg, h, params, lnl, l64,
                                           args.third_generation_surrogate, 10, reps)
    h.close()
    return out


def bench_rotating(args, np, torch, rbfl, wl):
    """Third-generation workload on a rotating Earth (sidereal rate; the
    injection synthesised with every mode's antenna factor and delay at its
    own stationary-phase time).  Two handles on the same data: antenna
    patterns frozen at t_c (Sec. II B) and B time bands.  Per handle: start-up
    time, FP64 evals/s on 2e5 near-node proposals with the contraction's
    roofline, and the error against the exact rotating-Earth ln L
    (rbfl_brute) at 256 nodes with the injection's sky, polarisation and
    inclination (drawn phase, distance and t_c).  The banded handle's ln L is
    also checked against the oracle's banded online stage on its exported
    artefacts (500 proposals)."""
    base = wl.CFG5_ROTATING
    n, n_err = 200_000, 256
    sp = torch.cuda.current_stream().cuda_stream
    out = {"workload": base.name, "earth_rate": base.earth_rate, "proposals_per_pass": n,
           "error_sample": f"{n_err} nodes (seeded), injection sky/polarisation/inclination, phase, distance "
                           "and t_c drawn about the injection"}
    exact = None
    for label, nb in (("frozen", 1), (f"bands_{args.rotating_bands}", args.rotating_bands)):
        cfg = base.with_(name=f"{base.name}_b{nb}", n_bands=nb)
        log(f"rotating: start-up with {nb} band(s)")
        t0 = time.time()
        h = rbfl.Handle.from_config(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg))
        build_s = time.time() - t0
        sz = h.sizes()
        idx, jit = wl.node_jitter(n, cfg.n_nodes)
        params = torch.from_numpy(np.ascontiguousarray(rbfl.params_soa(
            h, wl.queries(cfg, n=n).near_nodes(h.nodes(), idx, jit), cfg.t_trig))).cuda()
        lnl = torch.empty(n, dtype=torch.float64, device="cuda")
        h.reserve(65536)
        h.eval(params.data_ptr(), n, lnl.data_ptr(), rbfl.FORM_FP64, sp)
        torch.cuda.synchronize()
        reps = 3
        h.profile(True)
        t = time.perf_counter()
        for _ in range(reps):
            h.eval(params.data_ptr(), n, lnl.data_ptr(), rbfl.FORM_FP64, sp)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / reps
        h.profile(False)
        ks = h.kernel_stats()
        c_ms = ks["contract_ms"] / max(1, ks["contract_launches"])
        per = ks["contract_n"] / max(1, ks["contract_launches"])
        tflops = 2.0 * (sz["N"] + sz["M"]) * sz["K"] * per / (c_ms * 1e-3) / 1e12
        # error against the exact rotating-Earth ln L at nodes
        ni = np.random.default_rng(3).integers(0, cfg.n_nodes, n_err)
        qe = wl.queries(cfg.with_(random_sky=False), n=n_err, seed=77, clustered=0.05).near_nodes(
            h.nodes(), ni, np.zeros((n_err, 4)))
        pe = torch.from_numpy(np.ascontiguousarray(rbfl.params_soa(h, qe, cfg.t_trig))).cuda()
        le = torch.empty(n_err, dtype=torch.float64, device="cuda")
        h.eval(pe.data_ptr(), n_err, le.data_ptr(), rbfl.FORM_FP64, sp)
        if exact is None:
            ex = torch.empty(n_err, dtype=torch.float64, device="cuda")
            h.brute(pe.data_ptr(), n_err, ex.data_ptr(), sp)
            torch.cuda.synchronize()
            exact = ex.cpu().numpy()
        torch.cuda.synchronize()
        l_err = le.cpu().numpy()
        fin = np.isfinite(l_err) & np.isfinite(exact)
        e = np.abs(l_err[fin] - exact[fin])
        f = {"n_bands": nb, "K": sz["K"], "startup_s": round(build_s, 1), "evals_per_s": n / wall,
             "ms_per_pass": wall * 1e3, "contract_ms_per_launch": c_ms, "contract_tflops": tflops,
             "roofline": roof(tflops * 1e12, PEAK_FP64, kernel="k_gemm_fp64"),
             "vs_exact_rotating": {"n": int(fin.sum()), "median": float(np.median(e)),
                                   "p90": float(np.quantile(e, 0.9)), "max": float(e.max()),
                                   "max_abs_lnl": float(np.abs(exact[fin]).max())}}
        log(f"rotating {label}: start-up {build_s:.1f} s, {n / wall:.4e} evals/s, vs exact median "
            f"{np.median(e):.3e} max {e.max():.3e}")
        if nb > 1 and not args.no_cpu_baseline:
            from oracle import likelihood as lk
            from oracle import startup as su
            art = su.artefacts_from_exports(cfg, wl.injection_extrinsics(cfg), **h.exports())
            m = 500
            sample = np.sort(np.random.default_rng(321).choice(n, m, replace=False))
            ps = params[:, sample].cpu().numpy()
            lg = lnl.cpu().numpy()[sample]
            lo = lk.meshfree_lnl(art, ps[0:4].T.copy(), ps[4:9].T.copy(), ps[9].copy(), ps[10].copy())
            okf = np.isfinite(lo)
            agree = bool(np.array_equal(okf, np.isfinite(lg)))
            d = np.abs(lg[okf] - lo[okf])
            f.update({"max_dlnl_vs_oracle": float(d.max()), "domain_agrees": agree,
                      "meets_1e-3": bool(agree and d.max() <= 1e-3),
                      "check_sample": f"{m} seeded proposals of the pass; oracle banded online stage on the "
                                      "handle's exported artefacts"})
            log(f"rotating {label}: max |dlnL| vs oracle {d.max():.3e}")
        out[label] = f
        h.close()
    return out


def bench_mixed(args, np, torch, rbfl, wl, cfg):
    """Every arithmetic form on the single-detector cubic-tail workload
    (N = 1500, M = 35, q = 60, the precision-split configuration): throughput
    of a pass over its 4e6 proposals (near the nodes), each form's contraction
    against its own peak (HIP events on the launch stream), and max |d ln L|
    against the oracle's online stage run on the handle's exported artefacts
    for a seeded sample of the pass."""
    n = cfg.n_queries
    log(f"mixed {cfg.name}: GPU start-up")
    t0 = time.time()
    h = rbfl.Handle.from_config(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg))
    build_s = time.time() - t0
    sz = h.sizes()
    idx, jit = wl.node_jitter(n, cfg.n_nodes)
    qd = wl.queries(cfg, n=n)
    host = np.ascontiguousarray(rbfl.params_soa(h, qd.near_nodes(h.nodes(), idx, jit), cfg.t_trig))
    params = torch.from_numpy(host).cuda()
    lnl = torch.empty(n, dtype=torch.float64, device="cuda")
    sp = torch.cuda.current_stream().cuda_stream
    h.reserve(65536)
    NM, K = sz["N"] + sz["M"], sz["K"]
    flop = 2.0 * NM * K
    out = {"workload": cfg.name, "proposals": n, "N": sz["N"], "M": sz["M"], "K": K, "q": sz["q"],
           "startup_s": round(build_s, 3), "cond": h.cond(), "forms": {}}
    res = {}
    for name, form in (("fp64", rbfl.FORM_FP64), ("split", rbfl.FORM_SPLIT), ("fp32", rbfl.FORM_FP32),
                       ("bf16", rbfl.FORM_BF16)):
        if form != rbfl.FORM_FP64:
            h.prepare(form)
        tune = h.autotune(params.data_ptr(), n, form, sp)
        h.eval(params.data_ptr(), n, lnl.data_ptr(), form, sp)
        torch.cuda.synchronize()
        reps = 3
        h.profile(True)
        t = time.perf_counter()
        for _ in range(reps):
            h.eval(params.data_ptr(), n, lnl.data_ptr(), form, sp)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / reps
        h.profile(False)
        ks = h.kernel_stats()
        res[name] = lnl.cpu().numpy()
        c_ms = ks["contract_ms"] / max(1, ks["contract_launches"])
        per = ks["contract_n"] / max(1, ks["contract_launches"])
        f = {"evals_per_s": n / wall, "ms_per_pass": wall * 1e3, "contract_ms_per_launch": c_ms,
             "contract_tflops_equiv": flop * per / (c_ms * 1e-3) / 1e12 if c_ms > 0 else None}
        if form == rbfl.FORM_FP64:
            f["order"] = h.pipeline()
            fused = f["order"]["fused_epilogue"]
            f["roofline"] = roof(flop * per / (c_ms * 1e-3), PEAK_FP64,
                                 kernel="k_gemm_lnl_fp64 (ln L inside the contraction)" if fused else "k_gemm_fp64")
        elif form == rbfl.FORM_SPLIT:
            S = tune["slices"]
            f["slices"] = S
            f["split_state"] = h.split_state()
            f["order"] = h.split_order()
            f["max_dlnl_vs_fp64_per_slice_count"] = tune["max_dlnl_vs_fp64"][:4]
            fused = f["order"]["fused_epilogue"]
            f["roofline"] = roof(S * (S + 1) / 2 * flop * per / (c_ms * 1e-3), PEAK_INT8, unit="TOP/s",
                                 kernel="k_split_lnl (ln L inside the contraction; int8 products issued)" if fused
                                 else "k_split_contract (int8 products issued)")
        elif form == rbfl.FORM_FP32:
            f["roofline"] = roof(flop * per / (c_ms * 1e-3), PEAK_FP32, kernel="k_contract_fp32")
        else:
            f["roofline"] = roof(flop * per / (c_ms * 1e-3), PEAK_BF16, kernel="k_bf16_contract")
        out["forms"][name] = f
        log(f"mixed {cfg.name} {name}: {n / wall:.4e} evals/s, contraction {c_ms:.3f} ms/launch")
    if not args.no_cpu_baseline:
        from oracle import likelihood as lk
        from oracle import startup as su
        art = su.artefacts_from_exports(cfg, wl.injection_extrinsics(cfg), **h.exports())
        m = min(20000, n)
        sample = np.sort(np.random.default_rng(321).choice(n, m, replace=False))
        pe = host[:, sample]
        lo = lk.meshfree_lnl(art, pe[0:4].T.copy(), pe[4:9].T.copy(), pe[9].copy(), pe[10].copy())
        fin = np.isfinite(lo)
        out["check_sample"] = f"{m} seeded proposals of the pass; oracle online stage on the handle's exported artefacts"
        out["valid_fraction"] = float(fin.mean())
        for name, l in res.items():
            lg = l[sample]
            agree = bool(np.array_equal(fin, np.isfinite(lg)))
            d = np.abs(lg[fin] - lo[fin]) if fin.any() else np.array([np.inf])
            out["forms"][name].update({"max_dlnl": float(d.max()), "p99_dlnl": float(np.quantile(d, 0.99)),
                                       "median_dlnl": float(np.median(d)), "domain_agrees": agree,
                                       "meets_1e-3": bool(agree and d.max() <= 1e-3)})
            log(f"mixed {cfg.name} {name}: max |dlnL| {d.max():.3e}")
    h.close()
    return out


def bench_ragged(args, np, torch, rbfl, wl):
    """Multi-event form: seeded events (durations log-uniform in 8-512 s,
    200-1500 nodes, q 20-60, 1-5 modes, 3 detectors), 1024 walkers each, one
    captured plan launch per sampler step, in the FP64 form and in the split
    form (digit counts tuned per event), against one rbfl_eval per event; the
    oracle's online stage on each event's exported artefacts checks a seeded
    sample of every event's proposals."""
    evs = wl.ragged_events(args.ragged_events)
    walkers = 1024
    n_thr = max(1, args.ragged_build_threads)
    log(f"ragged: building {len(evs)} events with rbfl_build_many ({n_thr} host threads, one batched SVD call)")
    t0 = time.time()
    # the stages before and after the SVD run on n_thr host threads (one
    # stream each); the events' SVDs share one batched call on this stream
    items = [(cfg, wl.white_noise(cfg), wl.injection_extrinsics(cfg)) for cfg in evs]
    hs = rbfl.Handle.from_configs(items, n_threads=n_thr, stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    per_event = np.sum([h.timing()[[0, 1, 2, 4]] for h in hs], axis=0)
    svd_s = float(hs[0].timing()[3])
    stages = {"data": per_event[0], "frame_nodes": per_event[1], "series": per_event[2], "svd_batched": svd_s,
              "rbf_solve": per_event[3]}
    log(f"ragged: start-up {build_s:.1f} s; stages (summed over the events, the batched SVD once) "
        f"{ {k: round(float(v), 1) for k, v in stages.items()} }")
    cols = []
    for cfg, h in zip(evs, hs):
        idx, jit = wl.node_jitter(walkers, cfg.n_nodes, seed=cfg.query_seed)
        qd = wl.queries(cfg, n=walkers).near_nodes(h.nodes(), idx, jit)
        cols.append(rbfl.params_soa(h, qd, cfg.t_trig))
    params = np.ascontiguousarray(np.concatenate(cols, axis=1))
    total = params.shape[1]
    p = torch.from_numpy(params).cuda()
    sp = torch.cuda.current_stream().cuda_stream
    flops = sum(2.0 * (h.sizes()["N"] + h.sizes()["M"]) * h.sizes()["K"] * walkers for h in hs)
    steps = max(5, args.steps)

    def timed(plan):
        for _ in range(2):
            plan.launch(sp)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            plan.launch(sp)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    res = {"events": len(hs), "walkers_per_event": walkers, "startup_s": round(build_s, 2),
           "startup_threads": n_thr,
           "startup_stage_s": {k: round(float(v), 2) for k, v in stages.items()}}
    out = {}
    for form, flags in (("fp64", rbfl.PLAN_GRAPH | rbfl.PLAN_AUTOTUNE),
                        ("split", rbfl.PLAN_GRAPH | rbfl.PLAN_AUTOTUNE | rbfl.PLAN_SPLIT)):
        o = torch.empty(total, dtype=torch.float64, device="cuda")
        log(f"ragged {form}: plan (tuning)")
        plan = rbfl.Plan(hs, [walkers] * len(hs), p.data_ptr(), o.data_ptr(), flags, sp)
        wall = timed(plan)
        info = plan.info()
        plan.close()
        out[form] = o.cpu().numpy()
        r = {"evals_per_s": total / wall, "ms_per_step": wall * 1e3, "plan": info,
             "contract_tflops_equiv_incl_epilogue": flops / wall / 1e12}
        if form == "fp64":
            r["roofline"] = roof(flops / wall, PEAK_FP64,
                                 kernel="k_ragged_rows_fp64 + k_ragged_gemm_fp64 + k_ragged_epilogue (whole plan launch)")
        res[form] = r
        log(f"ragged {form}: {total / wall:.4e} evals/s, {info}")
    # int8 products of the split plan at the chosen digit counts: per event S(S+1)/2 digit pairs
    # (the tuner's choice is reported as the range; the products are counted at the largest S)
    smax = res["split"]["plan"].get("slices_max", 7)
    ops = sum(smax * (smax + 1) / 2 * 2.0 * (h.sizes()["N"] + h.sizes()["M"]) * h.sizes()["K"] * walkers for h in hs)
    res["split"]["roofline"] = roof(ops / (res["split"]["ms_per_step"] * 1e-3), PEAK_INT8, unit="TOP/s",
                                    kernel="k_ragged_split_rows + k_ragged_split_contract + k_ragged_epilogue "
                                           "(whole plan launch; int8 products at the largest digit count)")
    # the same work as one rbfl_eval per event
    sub = [p[:, i * walkers:(i + 1) * walkers].contiguous() for i in range(len(hs))]
    outs = [torch.empty(walkers, dtype=torch.float64, device="cuda") for _ in hs]
    for h, q, o in zip(hs, sub, outs):
        h.eval(q.data_ptr(), walkers, o.data_ptr(), rbfl.FORM_FP64, sp)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        for h, q, o in zip(hs, sub, outs):
            h.eval(q.data_ptr(), walkers, o.data_ptr(), rbfl.FORM_FP64, sp)
    torch.cuda.synchronize()
    wall_loop = (time.perf_counter() - t) / steps
    le = torch.cat(outs).cpu().numpy()
    fin = np.isfinite(le)
    res["per_event_loop_evals_per_s"] = total / wall_loop
    res["valid_fraction"] = float(fin.mean())
    for form in ("fp64", "split"):
        lr = out[form]
        agree = bool(np.array_equal(fin, np.isfinite(lr)))
        res[form]["domain_agrees_with_per_event"] = agree
        res[form]["max_abs_diff_vs_per_event_fp64"] = float(np.abs(lr[fin] - le[fin]).max()) if fin.any() else 0.0
    if not args.no_cpu_baseline:
        from oracle import likelihood as lk
        from oracle import startup as su
        per = 64
        rng = np.random.default_rng(77)
        worst = {"fp64": 0.0, "split": 0.0}
        agree = {"fp64": True, "split": True}
        for e, (cfg, h) in enumerate(zip(evs, hs)):
            art = su.artefacts_from_exports(cfg, wl.injection_extrinsics(cfg), **h.exports())
            idx = e * walkers + np.sort(rng.choice(walkers, per, replace=False))
            pe = params[:, idx]
            lo = lk.meshfree_lnl(art, pe[0:4].T.copy(), pe[4:9].T.copy(), pe[9].copy(), pe[10].copy())
            f = np.isfinite(lo)
            for form in ("fp64", "split"):
                lg = out[form][idx]
                agree[form] &= bool(np.array_equal(f, np.isfinite(lg)))
                if f.any():
                    worst[form] = max(worst[form], float(np.abs(lg[f] - lo[f]).max()))
        for form in ("fp64", "split"):
            res[form].update({"max_dlnl": worst[form], "domain_agrees": agree[form],
                              "meets_1e-3": bool(agree[form] and worst[form] <= 1e-3)})
        res["check_sample"] = f"{per} seeded proposals per event ({per * len(hs)} in all), oracle online stage on " \
                              "each event's exported artefacts"
        log(f"ragged: max |dlnL| vs oracle fp64 {worst['fp64']:.3e}, split {worst['split']:.3e}")
    for h in hs:
        h.close()
    return res


if __name__ == "__main__":
    main()
