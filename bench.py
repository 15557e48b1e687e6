"""Benchmark of the online fault-tolerant GEMM on one MI355X.

A step is one call of the whole hot path: ``ftgemm_run`` on the FP32 square
workload M = N = K = 8192, A, B, C ~ N(0, 1) (seeded, synthetic), alpha = 1,
beta = 1, online detect + correct with the automatic configuration.  Inputs
are resident in HBM before timing starts.  Prints one JSON line:

  value        FT-GEMM throughput, TFLOP/s over the algorithmic 2 M N K
  plain_*      the same kernel family with fault tolerance compiled out
  roofline     MFMA-bound: achieved TFLOP/s of the FT kernel against the FP32
               dense matrix peak of MI355X (157.3 TFLOP/s)
  injection    bit flips in accumulator lanes at 10 / 100 / 1000 faults per
               second of GEMM time: detected / corrected / missed / false
               positives, classified from the thresholds the kernel logged
  cpu_baseline the FP64 CPU oracle timed on a bounded sample of the workload

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2516.6
PEAK_FP8_MFMA_TFLOPS = 5033.2
PEAK_FP64_TFLOPS = 78.6      # FP64 vector FMA and FP64 matrix cores alike on MI355X
METRIC = "FT-GEMM TFLOP/s & %MFMA peak vs plain GEMM (same GPU), overhead %, detect/correct rate"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--size", type=int, default=8192)
    p.add_argument("--workload", choices=("square", "batched", "irregular", "ablation"), default="square",
                   help="square: the headline FP32 8192^3 (default); batched: 1024 uneven FP32/BF16 "
                        "problems in one persistent launch vs a loop of launches; irregular: tall-skinny, "
                        "small-K and odd shapes, autotuned vs fixed configuration; ablation: fused online "
                        "ABFT against the same checks run as separate launches (FP32 8192^3, beta = 0)")
    p.add_argument("--dtype", choices=("f32", "bf16", "fp8", "f64"), default="f32",
                   help="f32: the FP32 square workload (beta = 1); bf16: A, B heavy-tailed N(0,1) "
                        "rounded to bfloat16, beta = 0 (profiling of the BF16 kernel); fp8: the same "
                        "operands scaled per tensor to E4M3, alpha = the product of the two scales; f64: the binary64 "
                        "path (ftgemm_run_f64), N(0,1) operands, beta = 1")
    p.add_argument("--skip-cpu", action="store_true", help="do not time the CPU oracle")
    p.add_argument("--skip-injection", action="store_true", help="do not run the injection-rate sweep")
    p.add_argument("--plain-only", action="store_true", help="time only the FT-off kernel (profiling)")
    p.add_argument("--ft-only", action="store_true", help="time only the FT kernel (profiling)")
    p.add_argument("--probe", action="store_true",
                   help="one FT launch, one plain launch and one 1 GiB elementwise copy, then exit "
                        "(for hardware-counter runs: the copy calibrates FETCH_SIZE / WRITE_SIZE)")
    return p.parse_args()


def timed(fn, steps: int, warmup: int, stream) -> float:
    """Average milliseconds per call over `steps` calls, HIP events recorded on
    the stream the library launches on."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def classify(log_entries, events, c):
    """Classify applied faults from the residual thresholds the kernel logged
    at the first check after each fault (beta = tau / c)."""
    out = dict(injected=0, must=0, must_corrected=0, benign=0, benign_flagged=0, grey=0, grey_corrected=0,
               false_positive=0)
    corrected_at = {(int(e["tile_m"]), int(e["tile_n"]), int(e["kstep"]), int(e["row"]), int(e["col"]))
                    for e in events if int(e["kind"]) == 1}
    flagged_tiles = {(int(e["tile_m"]), int(e["tile_n"]), int(e["kstep"])) for e in events}
    fault_keys = set()
    for f in log_entries:
        out["injected"] += 1
        key = (int(f["tile_m"]), int(f["tile_n"]), int(f["check_step"]), int(f["row"]), int(f["col"]))
        fault_keys.add(key[:3])
        d = float(f["new_v"]) - float(f["old_v"])
        tr, tcol = float(f["tau_row"]), float(f["tau_col"])
        slack = 1e-3
        if not np.isfinite(f["new_v"]) or (abs(d) > tr * (1 + 1 / c) * (1 + slack) and
                                           abs(d) > tcol * (1 + 1 / c) * (1 + slack)):
            out["must"] += 1
            out["must_corrected"] += key in corrected_at
        elif abs(d) < tr * (1 - 1 / c) * (1 - slack) and abs(d) < tcol * (1 - 1 / c) * (1 - slack):
            out["benign"] += 1
            out["benign_flagged"] += key[:3] in flagged_tiles
        else:
            out["grey"] += 1
            out["grey_corrected"] += key in corrected_at
    out["false_positive"] = sum(1 for k in flagged_tiles if k not in fault_keys)
    out["missed"] = out["must"] - out["must_corrected"]
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); output tiles are independent, "
              "so several GPUs would each run this same kernel on their share", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2305_01024_amd import ftgemm as F
    from paper_2305_01024_amd import workloads as W

    assert torch.cuda.is_available(), "no GPU"
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "irregular":
        return bench_irregular(args)
    if args.workload == "ablation":
        return bench_ablation(args)
    if args.dtype == "f64":
        return bench_f64(args)
    N = args.size
    m = n = k = N
    lowp = args.dtype in ("bf16", "fp8")
    alpha = 1.0
    log(f"generating {args.dtype} inputs {m}x{n}x{k}")
    if lowp:
        A = W.heavy_tailed((m, k), 4, W.STREAM_A)
        B = W.heavy_tailed((k, n), 4, W.STREAM_B)
        if args.dtype == "bf16":
            (Ac, _), (Bc, _) = W.quantize_bf16(A), W.quantize_bf16(B)
            dA = torch.from_numpy(np.ascontiguousarray(Ac.T).view(np.int16)).cuda()
            dB = torch.from_numpy(np.ascontiguousarray(Bc.T).view(np.int16)).cuda()
        else:
            (Ac, sa), (Bc, sb) = W.quantize_e4m3(A), W.quantize_e4m3(B)
            dA = torch.from_numpy(np.ascontiguousarray(Ac.T)).cuda()
            dB = torch.from_numpy(np.ascontiguousarray(Bc.T)).cuda()
            alpha = sa * sb
        C0 = np.zeros((m, n), np.float32, order="F")
        beta = 0.0
    else:
        A = W.normal((m, k), 2, W.STREAM_A)
        B = W.normal((k, n), 2, W.STREAM_B)
        C0 = W.normal((m, n), 2, W.STREAM_C)
        dA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
        dB = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
        beta = 1.0
    dC0 = torch.from_numpy(np.ascontiguousarray(C0.T)).cuda()
    dC = dC0.clone()
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    dtype = {"f32": F.F32, "bf16": F.BF16, "fp8": F.F8E4M3}[args.dtype]
    peak = {"f32": PEAK_FP32_MFMA_TFLOPS, "bf16": PEAK_BF16_MFMA_TFLOPS, "fp8": PEAK_FP8_MFMA_TFLOPS}[args.dtype]
    h = F.ftgemm_create(dtype, 0)
    cfg = F.ftgemm_select_config(dtype, m, n, k)
    flop = 2.0 * m * n * k

    def call(level, report=None):
        return F.ftgemm_run(h, m, n, k, alpha, dA.data_ptr(), m, dB.data_ptr(), k, beta, dC.data_ptr(), m,
                            level, 0.0, sh, report)

    if args.probe:
        torch.cuda.synchronize()
        call(F.FT_CORRECT)
        torch.cuda.synchronize()
        call(F.FT_OFF)
        torch.cuda.synchronize()
        src = torch.ones(1 << 28, device="cuda")        # 1 GiB read, 1 GiB written
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        F.ftgemm_destroy(h)
        print(json.dumps({"probe": True, "dtype": args.dtype, "copy_bytes": src.numel() * 4, "m": m, "n": n,
                          "k": k, "source_sha256": kernel_source_hash(args.dtype)}), flush=True)
        return

    # a checked run first: the clean production path must raise no event
    rep = F.ReportBuffer(64)
    st = call(F.FT_CORRECT, rep)
    assert st == F.OK and rep.report.n_events == 0, (st, rep.report.n_events)

    ms_ft = ms_plain = None
    if not args.plain_only:
        log(f"timing FT kernel: {args.steps} steps after {args.warmup} warmup")
        ms_ft = timed(lambda: call(F.FT_CORRECT), args.steps, args.warmup, stream)
    if not args.ft_only:
        log("timing plain kernel")
        ms_plain = timed(lambda: call(F.FT_OFF), args.steps, args.warmup, stream)
    tf_ft = flop / (ms_ft * 1e-3) / 1e12 if ms_ft else None
    tf_plain = flop / (ms_plain * 1e-3) / 1e12 if ms_plain else None

    # the other levels on the same inputs: detect-only (one check per tile at
    # the end, the offline scheme), and both levels with recompute of tainted
    # tiles (clean: the extra launch finds an empty queue)
    levels = None
    if ms_ft and ms_plain:
        levels = {}
        for name, lvl in (("detect_only", F.FT_DETECT), ("detect_only_recompute", F.FT_DETECT | F.FT_RECOMPUTE),
                          ("online_recompute", F.FT_CORRECT | F.FT_RECOMPUTE)):
            t = timed(lambda: call(lvl), args.steps, args.warmup, stream)
            levels[name] = {"ms": round(t, 4), "overhead_pct": round(100.0 * (t / ms_plain - 1.0), 3)}
        # recovery: 8 tiles with two faults in one check interval (uncorrectable
        # online), recomputed by the second launch
        sites = np.zeros(8, dtype=F.FAULT_DTYPE)
        for q in range(8):
            sites[q] = (q, q, 1, 3, 5, W.KIND_ADD, 1e3, 0)
        two = np.sort(np.concatenate([sites, sites]), order=["tile_m", "tile_n", "kstep"])
        two["kstep"][1::2] = 2
        two["row"][1::2] = 40
        two["col"][1::2] = 50
        F.ftgemm_set_injection(h, two)
        t = timed(lambda: call(F.FT_CORRECT | F.FT_RECOMPUTE), 3, 1, stream)
        rep = F.ReportBuffer(64)
        st = call(F.FT_CORRECT | F.FT_RECOMPUTE, rep)
        F.ftgemm_set_injection(h, None)
        levels["online_recompute_8_uncorrectable_tiles"] = {
            "ms": round(t, 4), "status": int(st), "uncorrectable": int(rep.report.uncorrectable),
            "recomputed": int(rep.report.recomputed), "recompute_failed": int(rep.report.recompute_failed)}
        log(f"levels: {levels}")

    # fault injection at a rate per second of GEMM time (bits 0..30, and the
    # exponent bits 23..30 alone)
    injection = None
    if not args.skip_injection and ms_ft and not lowp:
        injection = injection_sweep(h, call, cfg, m, n, k, ms_ft, stream, args)

    # section 5.5: online against offline (detect-only + recompute) ABFT under
    # the paper's error model, at 2048^3, 4096^3 and this size
    online_offline = None
    if not args.skip_injection and ms_ft and ms_plain and not lowp and levels:
        online_offline = {}
        for size in sorted({2048, 4096, N}):
            if size == N:
                online_offline[str(size)] = online_vs_offline(h, call, cfg, size, ms_plain, levels["detect_only"]["ms"],
                                                              ms_ft, stream, args)
            else:
                online_offline[str(size)] = online_vs_offline_at(size, stream, args)
            log(f"online vs offline {size}: {online_offline[str(size)]}")

    cpu = None
    if not args.skip_cpu and not lowp:
        cpu = cpu_baseline(A, B, C0, cfg)

    F.ftgemm_destroy(h)
    ms = ms_ft if ms_ft else ms_plain
    tf = tf_ft if tf_ft else tf_plain
    kname = f"ftgemm_{args.dtype}_kernel<{cfg.m_tile},{cfg.n_tile},{cfg.k_step}>"
    traffic, traffic_src = measured_traffic(args.dtype, N) if ms_ft else (None, None)
    if args.dtype == "bf16":
        workload = f"bf16 square FT-GEMM M=N=K={N}, A,B~N(0,1) with 1% x100, bf16 RNE, alpha=1, beta=0, " \
                   f"online detect+correct"
    elif args.dtype == "fp8":
        workload = f"fp8-e4m3 square FT-GEMM M=N=K={N}, A,B~N(0,1) with 1% x100, per-tensor power-of-two " \
                   f"scale to E4M3 (RNE, saturating), alpha=scale_A*scale_B, beta=0, online detect+correct"
    else:
        workload = f"fp32 square FT-GEMM M=N=K={N}, A,B,C~N(0,1), alpha=1, beta=1, online detect+correct"
    out = {
        "metric": METRIC,
        "value": round(tf, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": workload, "m": m, "n": n, "k": k,
                   "tile": [cfg.m_tile, cfg.n_tile], "k_step": cfg.k_step,
                   "check_interval": cfg.check_interval},
        "ft_tflops": round(tf_ft, 3) if tf_ft else None,
        "plain_tflops": round(tf_plain, 3) if tf_plain else None,
        "ft_overhead_pct": round(100.0 * (ms_ft / ms_plain - 1.0), 3) if (ms_ft and ms_plain) else None,
        "mfma_frac_ft": round(tf_ft / peak, 4) if tf_ft else None,
        "mfma_frac_plain": round(tf_plain / peak, 4) if tf_plain else None,
        "roofline": {"bound": "mfma", "achieved": round(tf, 3), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(tf / peak, 4), "traffic": traffic,
                     "traffic_unit": "bytes per launch (HBM fetch + write, calibrated)",
                     "traffic_source": traffic_src,
                     "mfma_busy": measured_mfma_busy(args.dtype, N) if ms_ft else None,
                     "kernel": kname + (" FT=2" if ms_ft else " FT=0")},
        "levels": levels,
        "injection": injection,
        "online_vs_offline": online_offline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def _line(metric_value, ms, unit, dtype, config, extra, args, higher=True):
    out = {"metric": METRIC, "value": round(metric_value, 3), "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": higher, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_f64(args):
    """The binary64 path at size^3 (default 8192^3): N(0,1) A, B, C in HBM,
    alpha = 1, beta = 1; online FT (a check every 256 k), detect-only and
    plain launches timed with HIP events on the launch stream; one +1e3 fault
    per tile at a seeded k-step, row and column in a separate run, all of
    which must be corrected.  The kernel runs on the FP64 matrix cores
    (16x16x4 instruction), so the roofline is their dense peak."""
    import torch

    from paper_2305_01024_amd import ftgemm as F
    from paper_2305_01024_amd import workloads as W

    N = args.size
    m = n = k = N
    stream = torch.cuda.current_stream()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2305_01024 + 64)
    dA = torch.randn(k, m, device="cuda", dtype=torch.float64, generator=gen)
    dB = torch.randn(n, k, device="cuda", dtype=torch.float64, generator=gen)
    dC = torch.randn(n, m, device="cuda", dtype=torch.float64, generator=gen)
    h = F.ftgemm_create(F.F64, 0)

    def call(level=F.FT_CORRECT, report=None):
        return F.ftgemm_run_f64(h, m, n, k, 1.0, dA.data_ptr(), m, dB.data_ptr(), k, 1.0, dC.data_ptr(), m, level,
                                0.0, stream.cuda_stream, report)
    rep = F.ReportBuffer(16)
    assert call(report=rep) == F.OK and rep.report.n_events == 0
    cfg = rep.report.config.as_tuple()
    ms_ft = timed(call, args.steps, args.warmup, stream)
    ms_det = timed(lambda: call(F.FT_DETECT), args.steps, args.warmup, stream)
    ms_plain = timed(lambda: call(F.FT_OFF), args.steps, args.warmup, stream)
    flop = 2.0 * m * n * k
    tf = flop / (ms_ft * 1e-3) / 1e12
    ntm, ntn, nk = -(-m // cfg[0]), -(-n // cfg[1]), -(-k // cfg[2])
    g = W.rng(64, W.STREAM_SITES)
    sites = np.zeros(ntm * ntn, dtype=F.FAULT_DTYPE)
    for q in range(ntm * ntn):
        sites[q] = (q // ntn, q % ntn, int(g.integers(0, nk)), int(g.integers(0, min(cfg[0], m - (q // ntn) * cfg[0]))),
                    int(g.integers(0, min(cfg[1], n - (q % ntn) * cfg[1]))), W.KIND_ADD, 1e3, 0)
    F.ftgemm_set_injection(h, sites)
    rep = F.ReportBuffer(len(sites) + 16)
    st = call(report=rep)
    F.ftgemm_set_injection(h, None)
    inj = {"injected": len(sites), "corrected": int(rep.report.corrected),
           "uncorrectable": int(rep.report.uncorrectable), "status": int(st)}
    F.ftgemm_destroy(h)
    out = {"ft_tflops": round(tf, 3), "plain_tflops": round(flop / ms_plain / 1e9, 3),
           "detect_only_tflops": round(flop / ms_det / 1e9, 3),
           "ft_overhead_pct": round(100 * (ms_ft / ms_plain - 1), 2),
           "detect_only_overhead_pct": round(100 * (ms_det / ms_plain - 1), 2),
           "injection_one_per_tile": inj,
           "roofline": {"bound": "mfma", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(tf / PEAK_FP64_TFLOPS, 4), "traffic": None},
           "cpu_baseline": None}
    log(f"f64: {out}")
    _line(tf, ms_ft, "TFLOP/s", "f64",
          {"workload": f"fp64 square FT-GEMM M=N=K={N}, A,B,C~N(0,1), alpha=1, beta=1, online detect+correct",
           "m": m, "n": n, "k": k, "tile": list(cfg[:2]), "k_step": cfg[2], "check_interval": cfg[3]}, out, args)


def bench_batched(args):
    """1024 FT-GEMMs, M, N, K log-uniform in [32, 2048] (seeded), FP32 or BF16
    by a seeded coin: one persistent launch replayed from a HIP graph, the
    same launch eagerly, and a loop of one ftgemm_run per problem.  One
    additive 1e3 fault per 50 problems in a separate injected run."""
    import torch

    from paper_2305_01024_amd import ftgemm as F
    from paper_2305_01024_amd import workloads as W

    shapes = W.batched_problems(1024, 32, 2048, 5)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2305_01024 + 500)
    probs = F.make_problems(len(shapes))
    keep = []
    flop = 0.0
    t_peak = 0.0   # the batch's time at the dense peak of each problem's operand type, seconds
    for p, b in enumerate(shapes):
        A = torch.randn(b.k, b.m, device="cuda", generator=gen)        # column-major m x k
        B = torch.randn(b.n, b.k, device="cuda", generator=gen)        # column-major k x n
        C = torch.zeros(b.n, b.m, device="cuda")
        if b.dtype == "bf16":
            A = A.to(torch.bfloat16).view(torch.int16)
            B = B.to(torch.bfloat16).view(torch.int16)
        keep.append((A, B, C))
        q = probs[p]
        q["dtype"] = F.BF16 if b.dtype == "bf16" else F.F32
        q["m"], q["n"], q["k"] = b.m, b.n, b.k
        q["lda"], q["ldb"], q["ldc"] = b.m, b.k, b.m
        q["alpha"], q["beta"], q["scale_a"], q["scale_b"] = 1.0, 0.0, 1.0, 1.0
        q["A"], q["B"], q["C"] = A.data_ptr(), B.data_ptr(), C.data_ptr()
        flop += 2.0 * b.m * b.n * b.k
        t_peak += 2.0 * b.m * b.n * b.k / ((PEAK_BF16_MFMA_TFLOPS if b.dtype == "bf16" else PEAK_FP32_MFMA_TFLOPS) * 1e12)
    stream = torch.cuda.current_stream()
    h = F.ftgemm_create(F.F32, 0)
    hb = F.ftgemm_create(F.BF16, 0)
    rates = F.ftgemm_tune_batched(h, stream.cuda_stream)
    log(f"batched: {len(shapes)} problems, {flop / 1e12:.3f} TFLOP; variant rates {rates}")
    rep = F.ReportBuffer(64)
    st = F.ftgemm_batched(h, probs, F.FT_CORRECT, 0.0, stream.cuda_stream, rep)
    assert st == F.OK and rep.report.n_events == 0

    def batched():
        F.ftgemm_batched(h, probs, F.FT_CORRECT, 0.0, stream.cuda_stream)

    def loop():
        for p, b in enumerate(shapes):
            hh = hb if b.dtype == "bf16" else h
            A, B, C = keep[p]
            F.ftgemm_run(hh, b.m, b.n, b.k, 1.0, A.data_ptr(), b.m, B.data_ptr(), b.k, 0.0, C.data_ptr(), b.m,
                         F.FT_CORRECT, 0.0, stream.cuda_stream, None)

    ms_eager = timed(batched, args.steps, args.warmup, stream)
    ms_loop = timed(loop, max(1, args.steps // 4), 1, stream)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        batched()                      # same problem list: the cached plan
    stream.wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        F.ftgemm_batched(h, probs, F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream)
    ms_graph = timed(graph.replay, args.steps, args.warmup, stream)
    # injection: one additive fault per 50 problems
    g = W.rng(5, W.STREAM_SITES)
    chosen = sorted(g.choice(len(shapes), size=len(shapes) // 50, replace=False).tolist())
    sites = []
    for p in chosen:
        b = shapes[p]
        c = F.ftgemm_batched_config(h, p).as_tuple()
        s_ = W.fault_sites(g, b.m, b.n, b.k, c[0], c[1], c[2], c[3], 1, payload=1e3)
        s_["problem"] = p
        sites.append(s_)
    sites = np.concatenate(sites)
    sites = sites[np.lexsort((sites["kstep"], sites["tile_n"], sites["tile_m"], sites["problem"]))]
    F.ftgemm_set_injection(h, sites)
    rep = F.ReportBuffer(4096)
    F.ftgemm_batched(h, probs, F.FT_CORRECT, 0.0, stream.cuda_stream, rep)
    flog = F.ftgemm_get_injection_log(h)
    F.ftgemm_set_injection(h, None)
    corrected = {(int(e["problem"]), int(e["tile_m"]), int(e["tile_n"]), int(e["row"]), int(e["col"]))
                 for e in rep.events if int(e["kind"]) == F.EV_CORRECTED}
    hit = sum((int(x["problem"]), int(x["tile_m"]), int(x["tile_n"]), int(x["row"]), int(x["col"])) in corrected
              for x in flog)
    F.ftgemm_destroy(h)
    F.ftgemm_destroy(hb)
    tf = flop / (ms_graph * 1e-3) / 1e12
    _line(tf, ms_graph, "TFLOP/s", "f32+bf16",
          {"workload": "batched FT-GEMM: 1024 problems, M,N,K log-uniform [32,2048], FP32/BF16 by a fair coin, "
                       "alpha=1, beta=0, online detect+correct, one persistent launch replayed from a HIP graph",
           "problems": len(shapes), "tflop": round(flop / 1e12, 4)},
          {"eager_batched_ms": round(ms_eager, 4), "loop_of_launches_ms": round(ms_loop, 4),
           "graph_vs_loop_speedup": round(ms_loop / ms_graph, 3),
           "variant_rates_mac_per_s": [float(r) for r in rates],
           "injection": {"injected": int(len(flog)), "corrected_at_site": int(hit),
                         "events": int(rep.report.n_events), "uncorrectable": int(rep.report.uncorrectable)},
           # the mix's peak: its FLOPs over the time they take at each problem's dense MFMA peak
           "roofline": {"bound": "mfma", "achieved": round(tf, 3), "peak": round(flop / t_peak / 1e12, 1),
                        "unit": "TFLOP/s", "frac": round(tf / (flop / t_peak / 1e12), 4), "traffic": None,
                        "peak_note": "FP32 and BF16 dense MFMA peaks weighted by each problem's FLOPs"},
           "cpu_baseline": None}, args)


def bench_irregular(args):
    """The irregular FP32 shapes, U[-1,1], beta = 0: the configuration the
    autotuner picks (check at most every 256 k) against the fixed 256 x 256 x
    32, g = 8 one; then 100 exponent-bit flips per second of GEMM time."""
    import torch

    from paper_2305_01024_amd import ftgemm as F
    from paper_2305_01024_amd import workloads as W

    stream = torch.cuda.current_stream()
    h = F.ftgemm_create(F.F32, 0)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2305_01024 + 300)
    rows = []
    total_flop = total_ms = 0.0
    for (m, n, k) in W.irregular_shapes(3):
        A = torch.rand(k, m, device="cuda", generator=gen) * 2 - 1
        B = torch.rand(n, k, device="cuda", generator=gen) * 2 - 1
        C = torch.zeros(n, m, device="cuda")

        def call(level=F.FT_CORRECT):
            F.ftgemm_run(h, m, n, k, 1.0, A.data_ptr(), m, B.data_ptr(), k, 0.0, C.data_ptr(), m, level, 0.0,
                         stream.cuda_stream, None)
        F.ftgemm_set_config(h, (256, 256, 32, 8))
        ms_fixed = timed(call, args.steps, args.warmup, stream)
        F.ftgemm_set_config(h, None)
        cfg = F.ftgemm_tune(h, m, n, k, F.FT_CORRECT, 256, stream.cuda_stream).as_tuple()
        ms_tuned = timed(call, args.steps, args.warmup, stream)
        ms_plain = timed(lambda: call(F.FT_OFF), args.steps, args.warmup, stream)
        flop = 2.0 * m * n * k
        g = W.rng(3, W.STREAM_SITES)
        counts, _ = W.rate_schedule(g, 100, ms_tuned * 1e-3, 4)
        # above_threshold: applied faults whose logged residual at the first
        # check after them exceeds its threshold (the others are below what
        # the check can see: benign by construction)
        inj = dict(injected=0, above_threshold=0, corrected=0, events=0)
        for c_l in counts:
            sites = W.fault_sites(g, m, n, k, cfg[0], cfg[1], cfg[2], cfg[3], int(c_l), kind=W.KIND_XOR,
                                  bits=range(23, 31))
            F.ftgemm_set_injection(h, sites if len(sites) else None)
            rep = F.ReportBuffer(1024)
            F.ftgemm_run(h, m, n, k, 1.0, A.data_ptr(), m, B.data_ptr(), k, 0.0, C.data_ptr(), m, F.FT_CORRECT,
                         0.0, stream.cuda_stream, rep)
            flog = F.ftgemm_get_injection_log(h) if len(sites) else []
            inj["injected"] += len(sites)
            inj["above_threshold"] += sum(1 for f in flog if not (abs(f["r_row"]) <= f["tau_row"] and
                                                                   abs(f["r_col"]) <= f["tau_col"]))
            inj["corrected"] += int(rep.report.corrected)
            inj["events"] += int(rep.report.n_events)
        F.ftgemm_set_injection(h, None)
        rows.append({"shape": [m, n, k], "tuned_config": list(cfg), "tuned_tflops": round(flop / ms_tuned / 1e9, 2),
                     "fixed_tflops": round(flop / ms_fixed / 1e9, 2), "plain_tflops": round(flop / ms_plain / 1e9, 2),
                     "injection_100_per_s": inj})
        log(f"irregular {m}x{n}x{k}: {rows[-1]}")
        total_flop += flop
        total_ms += ms_tuned
    F.ftgemm_destroy(h)
    _line(total_flop / (total_ms * 1e-3) / 1e12, total_ms, "TFLOP/s", "f32",
          {"workload": "FP32 irregular FT-GEMM shapes (65536,256,4096), (256,65536,4096), (16384,16384,64), "
                       "(3001,1999,4097), U[-1,1], beta=0, autotuned configuration, one call per shape per step"},
          {"shapes": rows,
           "roofline": {"bound": "mfma", "achieved": round(total_flop / (total_ms * 1e-3) / 1e12, 3),
                        "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(total_flop / (total_ms * 1e-3) / 1e12 / PEAK_FP32_MFMA_TFLOPS, 4),
                        "traffic": None},
           "cpu_baseline": None}, args)


def bench_ablation(args):
    """Fused against non-fused ABFT on the same inputs (FP32 N(0,1), alpha = 1,
    beta = 0, 256 x 256 check tiles, a check every 256 k): the plain kernel,
    the fused online kernel, and ftgemm_run_nonfused (the same checks as
    separate launches around the plain kernel on 256-k chunks).  Then the
    check granularity on one compute tile (128 x 128, four wavefronts): plain,
    threadblock-level checks (128 x 128 check tiles) and warp-level checks
    (one 64 x 64 check tile per wavefront)."""
    import torch

    from paper_2305_01024_amd import ftgemm as F
    from paper_2305_01024_amd import workloads as W

    N = args.size
    m = n = k = N
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2305_01024 + 600)
    dA = torch.randn(k, m, device="cuda", generator=gen)
    dB = torch.randn(n, k, device="cuda", generator=gen)
    dC = torch.zeros(n, m, device="cuda")
    h = F.ftgemm_create(F.F32, 0)
    flop = 2.0 * m * n * k

    def fused(level=F.FT_CORRECT, report=None):
        return F.ftgemm_run(h, m, n, k, 1.0, dA.data_ptr(), m, dB.data_ptr(), k, 0.0, dC.data_ptr(), m, level,
                            0.0, sh, report)

    def nonfused(report=None):
        return F.ftgemm_run_nonfused(h, m, n, k, dA.data_ptr(), m, dB.data_ptr(), k, dC.data_ptr(), m, 256,
                                     stream=sh, report=report)

    for fn in (fused, nonfused):   # clean runs raise no event
        rep = F.ReportBuffer(16)
        assert fn(report=rep) == F.OK and rep.report.n_events == 0
    # the best plain kernel for the non-fused chunk shape (m, n, 256)
    chunk_cfg = F.ftgemm_tune(h, m, n, 256, F.FT_OFF, 256, sh).as_tuple()
    log(f"non-fused chunk GEMM configuration {chunk_cfg}; timing plain, fused, non-fused")
    ms_plain = timed(lambda: fused(F.FT_OFF), args.steps, args.warmup, stream)
    ms_fused = timed(fused, args.steps, args.warmup, stream)
    ms_nonfused = timed(nonfused, args.steps, args.warmup, stream)
    # one additive fault per tile in a seeded chunk: both paths must correct every one
    g = W.rng(6, W.STREAM_SITES)
    ntm = ntn = N // 256
    sites = np.zeros(ntm * ntn, dtype=F.FAULT_DTYPE)
    for q in range(ntm * ntn):
        sites[q] = (q // ntn, q % ntn, int(g.integers(0, N // 256)), int(g.integers(0, 256)),
                    int(g.integers(0, 256)), W.KIND_ADD, 1e4, 0)
    inj = {}
    for name, fn, kstep_scale in (("fused", fused, 8), ("nonfused", nonfused, 1)):
        s2 = sites.copy()
        s2["kstep"] = s2["kstep"] * kstep_scale   # fused sites are in 32-k steps, non-fused in 256-k chunks
        F.ftgemm_set_injection(h, s2)
        rep = F.ReportBuffer(ntm * ntn + 16)
        st = fn(report=rep)
        F.ftgemm_set_injection(h, None)
        inj[name] = {"injected": len(s2), "corrected": int(rep.report.corrected), "status": int(st),
                     "uncorrectable": int(rep.report.uncorrectable)}
    gran = bench_granularity(h, m, n, k, fused, args, stream)
    F.ftgemm_destroy(h)
    out = {"plain_ms": round(ms_plain, 4), "fused_ms": round(ms_fused, 4), "nonfused_ms": round(ms_nonfused, 4),
           "fused_overhead_pct": round(100 * (ms_fused / ms_plain - 1), 2),
           "nonfused_overhead_pct": round(100 * (ms_nonfused / ms_plain - 1), 2),
           "fused_speedup_over_nonfused_pct": round(100 * (ms_nonfused / ms_fused - 1), 2),
           "plain_tflops": round(flop / ms_plain / 1e9, 2), "nonfused_tflops": round(flop / ms_nonfused / 1e9, 2),
           "nonfused_chunk_config": list(chunk_cfg),
           "injection_one_per_tile": inj, "check_granularity": gran, "roofline": None, "cpu_baseline": None}
    log(f"ablation: {out}")
    _line(flop / (ms_fused * 1e-3) / 1e12, ms_fused, "TFLOP/s", "f32",
          {"workload": f"FP32 {N}^3 N(0,1), alpha=1, beta=0: fused online ABFT vs the same checks as separate "
                       f"launches around the plain kernel on 256-k chunks"}, out, args)


def bench_granularity(h, m, n, k, fused, args, stream):
    """Threadblock-level against warp-level checks on the 128 x 128 compute
    tile (2 x 2 wavefronts): times, and one +1e4 fault in each of the four
    wavefront tiles of 1024 seeded compute tiles, all four at the same k-step.
    Warp-level checks correct every fault; threadblock-level checks see four
    in one check interval of one tile and can only report them."""
    from paper_2305_01024_amd import ftgemm as F
    from paper_2305_01024_amd import workloads as W
    tile = (128, 128, 32, 8, 128, 128)
    wave = (128, 128, 32, 8, 64, 64)
    ms = {}
    for name, cfg, level in (("plain", tile, F.FT_OFF), ("threadblock", tile, F.FT_CORRECT),
                             ("wavefront", wave, F.FT_CORRECT)):
        F.ftgemm_set_config(h, cfg)
        ms[name] = timed(lambda: fused(level), args.steps, args.warmup, stream)
    g = W.rng(7, W.STREAM_SITES)
    ntm, ntn, nk = m // 128, n // 128, k // 32
    pick = g.choice(ntm * ntn, size=min(1024, ntm * ntn), replace=False)
    wsites = np.zeros(4 * len(pick), dtype=F.FAULT_DTYPE)
    q = 0
    for t in sorted(int(x) for x in pick):
        tm, tn, ks = t // ntn, t % ntn, int(g.integers(0, nk))
        for a in range(2):
            for b in range(2):
                wsites[q] = (2 * tm + a, 2 * tn + b, ks, int(g.integers(0, 64)), int(g.integers(0, 64)),
                             W.KIND_ADD, 1e4, 0)
                q += 1
    tsites = wsites.copy()   # the same elements in compute-tile coordinates
    tsites["tile_m"], tsites["tile_n"] = wsites["tile_m"] // 2, wsites["tile_n"] // 2
    tsites["row"] = wsites["row"] + 64 * (wsites["tile_m"] % 2)
    tsites["col"] = wsites["col"] + 64 * (wsites["tile_n"] % 2)
    wsites = wsites[np.lexsort((wsites["kstep"], wsites["tile_n"], wsites["tile_m"]))]
    tsites = tsites[np.lexsort((tsites["kstep"], tsites["tile_n"], tsites["tile_m"]))]
    inj = {}
    for name, cfg, sites in (("threadblock", tile, tsites), ("wavefront", wave, wsites)):
        F.ftgemm_set_config(h, cfg)
        F.ftgemm_set_injection(h, sites)
        rep = F.ReportBuffer(len(sites) + 16)
        st = fused(F.FT_CORRECT, rep)
        F.ftgemm_set_injection(h, None)
        inj[name] = {"injected": len(sites), "corrected": int(rep.report.corrected),
                     "uncorrectable": int(rep.report.uncorrectable), "status": int(st)}
    F.ftgemm_set_config(h, None)
    flop = 2.0 * m * n * k
    out = {"compute_tile": [128, 128], "check_every_k": 256,
           "ms": {x: round(v, 4) for x, v in ms.items()},
           "tflops": {x: round(flop / v / 1e9, 2) for x, v in ms.items()},
           "overhead_pct": {x: round(100 * (ms[x] / ms["plain"] - 1), 2) for x in ("threadblock", "wavefront")},
           "injection_four_per_compute_tile_same_step": inj}
    log(f"check granularity: {out}")
    return out


KERNEL_SOURCES = {
    "f32": ("ftgemm_fp32.hip", "ftgemm_fp32.hpp", "ftgemm_abft.hpp", "ftgemm_internal.h"),
    "bf16": ("ftgemm_bf16.hip", "ftgemm_bf16.hpp", "ftgemm_abft.hpp", "ftgemm_internal.h"),
    "fp8": ("ftgemm_fp8.hip", "ftgemm_fp8.hpp", "ftgemm_abft.hpp", "ftgemm_internal.h"),
}


def _flip_bit(old_v, new_v) -> int:
    """Bit position a logged XOR fault flipped (from the two FP32 values)."""
    x = int(np.float32(old_v).view(np.uint32)) ^ int(np.float32(new_v).view(np.uint32))
    return x.bit_length() - 1 if x else -1


def injection_sweep(h, call, cfg, m, n, k, ms_ft, stream, args, launches=50):
    """Bit flips in accumulator lanes at 10 / 100 / 1000 faults per second of
    GEMM time (the injection experiment of section 5.3, at this GPU's speed):
    for each rate, round(rate * t * launches) faults spread over `launches`
    launches of the injection build, at most one per tile and check interval,
    at uniform (k-step, row, column, bit).  Two bit sets: bits 0..30 (the
    workload's fault model, where most flips of low mantissa bits lie inside
    the rounding bound and are benign) and the exponent bits 23..30 alone (so
    that must-detect faults occur, and the detect and correct rates are
    measured, at every rate).  Counts per class and per bit position.  The
    correction cost is the time per launch against the injection build with
    a site that never hits (same kernel, same instrumentation, no fault);
    the instrumentation cost is that build against the production kernel."""
    from paper_2305_01024_amd import ftgemm as F
    from paper_2305_01024_amd import workloads as W

    never = np.zeros(1, dtype=F.FAULT_DTYPE)
    never[0] = (0, 0, 0, 0, 0, W.KIND_ADD, 1.0, 1)     # problem 1: no tile of this call matches it
    F.ftgemm_set_injection(h, never)
    ms_inj_clean = timed(lambda: call(F.FT_CORRECT), args.steps, args.warmup, stream)
    out = {"launches_per_rate": launches, "ms_injection_build_no_fault": round(ms_inj_clean, 4),
           "instrumentation_overhead_pct": round(100.0 * (ms_inj_clean / ms_ft - 1.0), 3)}
    fields = ("injected", "must", "must_corrected", "benign", "benign_flagged", "grey", "grey_corrected")
    for bits_name, bits in (("bits_0_30", range(0, 31)), ("bits_23_30", range(23, 31))):
        g = W.rng(2, W.STREAM_SITES)
        res = {}
        for rate in (10, 100, 1000):
            counts, total = W.rate_schedule(g, rate, ms_ft * 1e-3, launches)
            agg = None
            by_bit = {}
            t_inj = []
            for c_l in counts:
                sites = W.fault_sites(g, m, n, k, cfg.m_tile, cfg.n_tile, cfg.k_step, cfg.check_interval,
                                      int(c_l), kind=W.KIND_XOR, bits=bits) if c_l else never
                F.ftgemm_set_injection(h, sites)
                t_inj.append(timed(lambda: call(F.FT_CORRECT), 1, 0, stream))
                rep = F.ReportBuffer(4096)
                call(F.FT_CORRECT, rep)
                flog = F.ftgemm_get_injection_log(h) if c_l else np.zeros(0, F.FAULT_LOG_DTYPE)
                cl = classify(flog, rep.events, rep.report.tol_used)
                agg = cl if agg is None else {kk: agg[kk] + cl[kk] for kk in agg}
                for q in range(len(flog)):
                    b = _flip_bit(flog[q]["old_v"], flog[q]["new_v"])
                    one = classify(flog[q:q + 1], rep.events, rep.report.tol_used)
                    row = by_bit.setdefault(str(b), [0] * len(fields))
                    for q, name in enumerate(fields):
                        row[q] += one[name]
            agg["by_bit"] = {"fields": list(fields), **{b: by_bit[b] for b in sorted(by_bit, key=int)}}
            agg["ms_per_step"] = round(float(np.mean(t_inj)), 4)
            agg["correction_overhead_pct"] = round(100.0 * (agg["ms_per_step"] / ms_inj_clean - 1.0), 3)
            res[f"{rate}/s"] = agg
            log(f"injection {bits_name} {rate}/s: { {kk: v for kk, v in agg.items() if kk != 'by_bit'} }")
        out[bits_name] = res
    F.ftgemm_set_injection(h, None)
    return out


def _offline_model(tiles, t_plain, t_det, t_online, t_retry_extra, q, gamma0=1.0 / 256):
    """Section 5.5's model: every tile accumulation fails with probability
    gamma0, so a whole run fails with gamma = 1 - (1 - gamma0)^tiles; the
    offline (detect-only) scheme restarts the whole product on a failure and
    needs (1 - gamma) / (1 - 2 gamma) runs in expectation (no finite
    expectation for gamma >= 1/2), the online scheme one.  Also the
    tile-level recompute built here (only the flagged tiles run again):
    expected extra time of its retry launch, measured with q flagged tiles
    (q = tiles * gamma0 rounded, at least one).  The crossover gamma0* is
    where the offline expectation equals the online time."""
    gamma = 1.0 - (1.0 - gamma0) ** tiles
    runs = (1.0 - gamma) / (1.0 - 2.0 * gamma) if gamma < 0.5 else None
    r = t_online / t_det
    gamma_star = (r - 1.0) / (2.0 * r - 1.0)
    gamma0_star = 1.0 - (1.0 - gamma_star) ** (1.0 / tiles)
    return {"tiles": int(tiles), "gamma0": gamma0, "gamma": round(gamma, 6),
            "offline_expected_runs": round(runs, 4) if runs is not None else "unbounded (gamma >= 1/2)",
            "ms_plain": round(t_plain, 4), "ms_detect_only": round(t_det, 4), "ms_online": round(t_online, 4),
            "ms_offline_expected": round(t_det * runs, 4) if runs is not None else None,
            "ms_detect_only_tile_recompute_expected": round(t_det + t_retry_extra, 4),
            "tile_recompute_measured_with_flagged_tiles": int(q),
            "online_overhead_pct": round(100.0 * (t_online / t_plain - 1.0), 3),
            "detect_only_overhead_pct": round(100.0 * (t_det / t_plain - 1.0), 3),
            "crossover_gamma0": float(f"{gamma0_star:.3e}")}


def _retry_extra(h, call, cfg, N, q, stream, args):
    """Extra time of the recompute launch with q flagged tiles at the
    detect-only level: the injection build with q must-detect faults (one per
    tile) and recompute on, against the same build with a fault that never hits."""
    from paper_2305_01024_amd import ftgemm as F
    from paper_2305_01024_amd import workloads as W

    never = np.zeros(1, dtype=F.FAULT_DTYPE)
    never[0] = (0, 0, 0, 0, 0, W.KIND_ADD, 1.0, 1)
    F.ftgemm_set_injection(h, never)
    t0 = timed(lambda: call(F.FT_DETECT | F.FT_RECOMPUTE), 5, 1, stream)
    ntm, ntn = -(-N // cfg.m_tile), -(-N // cfg.n_tile)
    g = W.rng(55, W.STREAM_SITES)
    pick = np.sort(g.choice(ntm * ntn, size=q, replace=False))
    sites = np.zeros(q, dtype=F.FAULT_DTYPE)
    for x, t in enumerate(pick):
        sites[x] = (t // ntn, t % ntn, 0, 1, 2, W.KIND_ADD, 1e6, 0)
    F.ftgemm_set_injection(h, sites)
    t1 = timed(lambda: call(F.FT_DETECT | F.FT_RECOMPUTE), 5, 1, stream)
    rep = F.ReportBuffer(64)
    call(F.FT_DETECT | F.FT_RECOMPUTE, rep)
    F.ftgemm_set_injection(h, None)
    assert rep.report.recomputed == q and rep.report.recompute_failed == 0, (rep.report.recomputed, q)
    return max(0.0, t1 - t0)


def online_vs_offline(h, call, cfg, N, ms_plain, ms_det, ms_online, stream, args, gamma0=1.0 / 256):
    tiles = -(-N // cfg.m_tile) * -(-N // cfg.n_tile)
    q = max(1, int(round(tiles * gamma0)))
    extra = _retry_extra(h, call, cfg, N, q, stream, args)
    return _offline_model(tiles, ms_plain, ms_det, ms_online, extra, q, gamma0)


def online_vs_offline_at(N, stream, args, gamma0=1.0 / 256):
    """online_vs_offline on the FP32 square workload at N^3 (N(0,1), beta = 1)."""
    import torch

    from paper_2305_01024_amd import ftgemm as F
    from paper_2305_01024_amd import workloads as W

    dA = torch.from_numpy(np.ascontiguousarray(W.normal((N, N), 2, W.STREAM_A).T)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(W.normal((N, N), 2, W.STREAM_B).T)).cuda()
    dC = torch.from_numpy(np.ascontiguousarray(W.normal((N, N), 2, W.STREAM_C).T)).cuda()
    h = F.ftgemm_create(F.F32, 0)
    sh = stream.cuda_stream

    def call(level, report=None):
        return F.ftgemm_run(h, N, N, N, 1.0, dA.data_ptr(), N, dB.data_ptr(), N, 1.0, dC.data_ptr(), N, level, 0.0,
                            sh, report)
    try:
        cfg = F.ftgemm_select_config(F.F32, N, N, N)
        t_plain = timed(lambda: call(F.FT_OFF), args.steps, args.warmup, stream)
        t_det = timed(lambda: call(F.FT_DETECT), args.steps, args.warmup, stream)
        t_onl = timed(lambda: call(F.FT_CORRECT), args.steps, args.warmup, stream)
        return online_vs_offline(h, call, cfg, N, t_plain, t_det, t_onl, stream, args, gamma0)
    finally:
        F.ftgemm_destroy(h)


def kernel_source_hash(dtype: str) -> str:
    """sha256 over the device sources of the kernel the bench times."""
    import hashlib
    hsh = hashlib.sha256()
    for name in KERNEL_SOURCES[dtype]:
        with open(os.path.join(ROOT, "paper_2305_01024_amd", "csrc", name), "rb") as f:
            hsh.update(f.read())
    return hsh.hexdigest()


def measured_traffic(dtype: str, size: int):
    """HBM bytes per launch of the FT kernel from the committed hardware-counter
    summary (FETCH_SIZE and WRITE_SIZE passes, each scaled by what the counter
    reads for an elementwise copy of known size), or None when there is none
    for this workload or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"ftgemm_{dtype}_{size}_hbm_traffic.md")
    if not os.path.exists(path):
        return None, None
    text = open(path).read()
    blk = text.split("```json", 1)[1].split("```", 1)[0] if "```json" in text else None
    if blk is None:
        return None, None
    rec = json.loads(blk)
    if rec.get("source_sha256") != kernel_source_hash(dtype):
        return None, os.path.relpath(path, ROOT) + " (stale: kernel sources changed)"
    kib = 1024.0
    fetch = rec["ft_fetch_kib"] * kib * rec["copy_bytes_read"] / (rec["copy_fetch_kib"] * kib)
    write = rec["ft_write_kib"] * kib * rec["copy_bytes_written"] / (rec["copy_write_kib"] * kib)
    return int(round(fetch + write)), os.path.relpath(path, ROOT)


def measured_mfma_busy(dtype: str, size: int):
    """Matrix-core busy fraction of the FT and plain kernels from the committed
    hardware-counter summary (SQ_VALU_MFMA_BUSY_CYCLES per SIMD over the
    kernel's GPU-active cycles, and the clock those cycles imply), or None when
    there is none for this workload or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"ftgemm_{dtype}_{size}_mfma_util.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if "```json" not in text:
        return None
    rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    src = os.path.relpath(path, ROOT)
    if rec.get("source_sha256") != kernel_source_hash(dtype):
        return {"ft_pct": None, "plain_pct": None, "source": src + " (stale: kernel sources changed)"}
    return {"ft_pct": rec["ft_mfma_busy_pct"], "plain_pct": rec["plain_mfma_busy_pct"],
            "ft_clock_ghz": rec["ft_clock_ghz"], "plain_clock_ghz": rec["plain_clock_ghz"], "source": src}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, B, C0, cfg, target_s: float = 12.0, single_s: float = 5.0):
    """The FP64 oracle replay (online ABFT, same tile decomposition and
    checks) on a bounded sample of the workload's output tiles, distinct tiles
    drawn by a seeded permutation, scaled to TFLOP/s: once on every host
    thread, once on one thread."""
    from oracle import oracle as O
    from paper_2305_01024_amd import workloads as W

    m, k = A.shape
    n = B.shape[1]
    rc = O.ReplayConfig(mc=cfg.m_tile, nc=cfg.n_tile, ku=cfg.k_step, g=cfg.check_interval)
    ntm, ntn = -(-m // cfg.m_tile), -(-n // cfg.n_tile)
    order = np.random.default_rng(W.seed(2, 5)).permutation(ntm * ntn)
    A64 = np.asfortranarray(A, dtype=np.float64)
    B64 = np.asfortranarray(B, dtype=np.float64)
    C64 = np.asfortranarray(C0, dtype=np.float64)

    def sample(count):
        tiles = [(int(t) % ntm, int(t) // ntm) for t in order[:count]]
        t0 = time.perf_counter()
        O.replay(A64, B64, rc, C0=C64, alpha=1.0, beta=1.0, tiles=tiles)
        return time.perf_counter() - t0, tiles

    def leg(threads, budget):
        O.set_threads(threads)
        dt, tiles = sample(threads)
        count = min(ntm * ntn, max(threads, int(threads * budget / max(dt, 1e-3))))
        if count > threads:
            dt, tiles = sample(count)
        flop = 2.0 * cfg.m_tile * cfg.n_tile * k * len(tiles)
        return flop / dt / 1e12, len(tiles), dt

    threads = O.threads()
    log(f"cpu baseline: oracle replay on sampled tiles, {threads} threads, then 1")
    try:
        v_all, n_all, dt_all = leg(threads, target_s)
        v_one, n_one, dt_one = leg(1, single_s)
    finally:
        O.set_threads(threads)
    desc = f"({cfg.m_tile}x{cfg.n_tile}, full K={k}, distinct tiles of a seeded permutation of all {ntm * ntn})"
    return {"value": round(v_all, 6), "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_all} output tiles {desc} replayed in FP64 with online checks, {dt_all:.1f} s",
            "single_core": {"value": round(v_one, 6), "unit": "TFLOP/s", "cores": 1,
                            "sample": f"{n_one} output tiles, {dt_one:.1f} s"},
            "cpu_model": _cpu_model()}


if __name__ == "__main__":
    main()
