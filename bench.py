"""Benchmark of the block-sparse x dense SpMM on one MI355X.

Default (the driver's contract): one step = one static SpMM Y = W X at the
static-sweep point m = k = 8192, n = 4096, b = 16, density 1/16, FP16 inputs
and output with FP32 accumulation (uniformly random blocks, N(0,1) values).
Inputs are resident in HBM before timing. W untimed warmup steps, then K timed
steps between device synchronisations; HIP events on the launch stream give
the average kernel time. Printed as one JSON line with the roofline of the
kernel, the dense FP16 GEMM of the same shape on the same GPU, and the FP64
oracle timed on the host cores over a bounded column sample.

Other modes print their own JSON lines:
  --mode sweep      the static sweep (m = k = 8192, n in {256, 1024, 4096},
                    b in {1, 4, 8, 16, 32}, densities 1/128..1/4, b = 16 up to
                    d = 1) next to dense FP16, and the crossover densities
  --mode dynamic    1000 dynamic calls, m = k = 4096, n = 512, b = 16, d_max 1/8
  --mode precision  m = k = 16384, n = 2048, b in {16, 32}, BF16 and FP8 weights
  --mode small      the small FP32 case (m = k = 1024, n = 64), two kernels
  --mode table3     static and dynamic against dense at m = k = 4096, d = 1/16
  --mode serve      the 8-layer serving loop against one request at a time
  --mode group      one grouped launch of 16 products against 16 launches
  --mode skew       power-law and concentrated patterns, rows split or not
  --mode train      forward, data gradient and weight gradient of one layer
  --mode ell        blocked-ELL plans, explicit padding, b = 16/32/64
  --mode grid       the paper's sweep grid best over n and its power-law fit
  --mode copy       a 256 MiB device copy (counter calibration)
  --mode peaks      measured HBM bandwidth (copy, read) and dense FP16/BF16 GEMM rate
  --mode dispatch   the speedup model's sparse-or-dense choice against measurement
  --mode point      one static product (--point m,k,n,b,1/d,w,x,y), for profiling
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective TFLOP/s (nonzero FLOPs) and speedup vs dense FP16 GEMM; serve p50/p99"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f16": 2500.0, "bf16": 2500.0, "fp8": 2500.0, "f32": 157.3}
# The dominant kernel of the default step and the committed counter summary of it.
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2303_16999_amd", "csrc", f) for f in ("spmm_row.h", "spmm_row.hip")]
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "spmm_row_f16_b16_m8192_n4096_d16_traffic.md")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # untimed launches before each timed region: the GPU's clocks reach their
    # steady state only after tens of milliseconds of work (5 warm-up launches
    # of the headline SpMM measured 125 us per launch, 200 measured 114 us)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--mode", default="headline",
                    choices=["headline", "sweep", "dynamic", "precision", "copy", "serve", "group", "table3", "small",
                             "skew", "train", "grid", "ell", "peaks", "dispatch", "point"])
    ap.add_argument("--requests", type=int, default=2000, help="serve mode: measured requests per run")
    ap.add_argument("--rho", default="0.5,0.8", help="serve mode: offered load as fractions of the saturated rate")
    ap.add_argument("--rate-base", type=float, default=0.0,
                    help="serve mode: requests/s that rho multiplies instead of the measured saturated rate")
    ap.add_argument("--max-tokens", default="4096,16384,0",
                    help="serve mode: per-step token budgets of the continuous path (0 = none)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense FP16 comparator")
    ap.add_argument("--out", default=None, help="also append JSON lines to this file")
    ap.add_argument("--calls", type=int, default=1000, help="dynamic mode: number of calls")
    ap.add_argument("--dyn-n", type=int, default=512, help="dynamic mode: columns of X")
    ap.add_argument("--sweep-b", default="1,4,8,16,32", help="sweep mode: block sizes")
    ap.add_argument("--sweep-n", default="256,1024,4096", help="sweep mode: column counts")
    ap.add_argument("--point", default="8192,8192,4096,16,16,f16,f16,f16",
                    help="point mode: m,k,n,b,1/density,w,x,y of one static product")
    ap.add_argument("--grid-m", default="256,512,1024,2048,4096,8192", help="grid mode: feature sizes m = k")
    ap.add_argument("--grid-n", default="4,16,64,256,1024,4096,16384,65536", help="grid mode: batch sizes n")
    return ap.parse_args()


def emit(rec, out=None):
    line = json.dumps(rec)
    print(line, flush=True)
    if out:
        with open(out, "a") as fh:
            fh.write(line + "\n")


# ------------------------------------------------------------------ workloads

class StaticProblem:
    """Seeded static SpMM on the device: pattern s, values s+1, X s+2."""

    def __init__(self, m, k, n, b, d, w="f16", x=None, y=None, seed=0, scaled=False, mask=None):
        import torch
        from paper_2303_16999_amd import spmm, synth
        x = x or ("f16" if w == "fp8" else w)
        y = y or x
        self.m, self.k, self.n, self.b, self.d, self.w, self.x, self.y = m, k, n, b, d, w, x, y
        self.seed = seed
        mb, kb = -(-m // b), -(-k // b)
        self.mask = synth.block_mask(mb, kb, d, seed) if mask is None else mask
        self.rows, self.cols = synth.mask_coo(self.mask)
        self.nnzb = len(self.rows)
        vals = synth.scaled_block_values(self.nnzb, b, seed + 1) if scaled else synth.normal((self.nnzb, b, b), seed + 1)
        self.scales_store = None
        if w == "fp8":
            self.vals_store, self.scales_store = synth.quantize_e4m3fn_blocks(vals)
        else:
            self.vals_store = synth.to_storage(vals, w)
        self.vals_raw = vals
        X = synth.normal((k, n), seed + 2)
        self.X_store = synth.to_storage(X, x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.plan = spmm.StaticPlan(m, k, b, self.mask, w, x, y, n_hint=n)
        torch.cuda.synchronize()
        self.plan_ms = (time.perf_counter() - t0) * 1e3
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).view(torch.bfloat16) if a.dtype == np.uint16 \
            else torch.from_numpy(np.ascontiguousarray(a))
        self.values_dev = t(self.vals_store).cuda()
        self.scales_dev = t(self.scales_store).cuda() if self.scales_store is not None else None
        self.X = t(self.X_store).cuda()
        self.Y = torch.empty((m, n), dtype=spmm.torch_dtype(spmm.DTYPE_CODES[y]), device="cuda")
        self.plan.set_values(self.values_dev, self.scales_dev)
        torch.cuda.synchronize()

    def step(self):
        self.plan.run(self.X, self.Y)

    def flops(self):
        return 2.0 * self.n * self.nnzb * self.b * self.b  # full blocks at every benchmark shape

    def alg_bytes(self):
        eb = {"f32": 4, "f16": 2, "bf16": 2, "fp8": 1}
        B = eb[self.x] * self.k * self.n + eb[self.y] * self.m * self.n
        B += eb[self.w] * self.nnzb * self.b * self.b + 4 * self.nnzb + 4 * (-(-self.m // self.b) + 1)
        if self.w == "fp8":
            B += 4 * self.nnzb
        return float(B)


def plan_build_warm_ms(prob, reps=3):
    """Median host time of building the same static plan again (the first plan
    of a process also pays the runtime's one-time initialisation)."""
    import torch
    from paper_2303_16999_amd import spmm
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = spmm.StaticPlan(prob.m, prob.k, prob.b, prob.mask, prob.w, prob.x, prob.y, n_hint=prob.n)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
        plan.close()
    return float(np.median(ts))


def time_steps(step, steps, warmup):
    """Average ms per step with events on the current (launch) stream."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def launch_percentiles(step, reps):
    """p10/p50/p90 in ms of single back-to-back launches, one event pair each."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for i in range(reps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    t = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(reps)])
    return {"p10": round(float(np.percentile(t, 10)), 5), "p50": round(float(np.percentile(t, 50)), 5),
            "p90": round(float(np.percentile(t, 90)), 5)}


def time_cold(step, reps, flush):
    """Median ms of single steps with L2 and the Infinity Cache flushed between them."""
    import torch
    ts = []
    for _ in range(reps):
        flush.add_(1.0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        step()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def dense_fp16(m, k, n, steps, warmup, useful_flops):
    import torch
    g = torch.Generator(device="cuda").manual_seed(1234)
    A = torch.randn((m, k), device="cuda", dtype=torch.float16, generator=g)
    B = torch.randn((k, n), device="cuda", dtype=torch.float16, generator=g)
    C = torch.empty((m, n), device="cuda", dtype=torch.float16)
    ms = time_steps(lambda: torch.matmul(A, B, out=C), steps, warmup)
    del A, B, C
    return {"ms": ms, "tflops_useful": useful_flops / (ms * 1e-3) / 1e12,
            "tflops_dense": 2.0 * m * k * n / (ms * 1e-3) / 1e12}


def dense_gemm(m, k, n, steps, warmup, dt):
    """ms of the dense GEMM (m x k) @ (k x n) in dtype dt on the GPU (FP32 without TF32)."""
    import torch
    if dt == "f16":
        return dense_fp16(m, k, n, steps, warmup, 1.0)["ms"]
    torch.backends.cuda.matmul.allow_tf32 = False
    g = torch.Generator(device="cuda").manual_seed(1234)
    A = torch.randn((m, k), device="cuda", dtype=torch.float32, generator=g)
    B = torch.randn((k, n), device="cuda", dtype=torch.float32, generator=g)
    C = torch.empty((m, n), device="cuda", dtype=torch.float32)
    ms = time_steps(lambda: torch.matmul(A, B, out=C), steps, warmup)
    del A, B, C
    return ms


def cpu_baseline(prob, target_s=10.0):
    """The FP64 oracle (blockwise form) on a bounded column sample of the same workload."""
    from oracle import spmm_ref as O
    from paper_2303_16999_amd import synth
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas_threads = 1
    cores = len(os.sched_getaffinity(0))
    vals64 = synth.storage_to_f64(prob.vals_store, prob.w) if prob.w != "fp8" else None
    if vals64 is None:
        from oracle import fp8_ref
        vals64 = fp8_ref.dequantize_blocks(prob.vals_store, prob.scales_store)
    X64 = synth.storage_to_f64(prob.X_store, prob.x)
    cols = 64
    while True:
        sel = np.arange(cols)
        t0 = time.perf_counter()
        O.spmm_blockwise_columns(prob.m, prob.k, prob.b, prob.rows, prob.cols, vals64, X64, sel)
        dt = time.perf_counter() - t0
        if dt >= target_s / 4 or cols >= prob.n:
            break
        cols = min(prob.n, cols * 4)
    times = [dt]
    while sum(times) < target_s and len(times) < 5:  # repeat a short sample, report the median
        t0 = time.perf_counter()
        O.spmm_blockwise_columns(prob.m, prob.k, prob.b, prob.rows, prob.cols, vals64, X64, np.arange(cols))
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    fl = 2.0 * cols * prob.nnzb * prob.b * prob.b
    return {"value": fl / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores), "blas_threads": int(blas_threads),
            "kind": "oracle",
            "sample": "FP64 blockwise oracle on the first %d of %d columns of X (exact by column separability), "
                      "median of %d runs, %.2f s each" % (cols, prob.n, len(times), dt)}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    src_hash = kernel_source_hash()
    fields = {}
    for line in open(TRAFFIC_SUMMARY):
        if ":" in line and line.strip().startswith("- "):
            key, val = line.strip()[2:].split(":", 1)
            fields[key.strip()] = val.strip()
    if fields.get("kernel_source_sha256_16") != src_hash:
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ------------------------------------------------------------------ modes

def mode_headline(args):
    import torch
    prob = StaticProblem(8192, 8192, 4096, 16, 1 / 16, "f16", seed=0)
    flops, bytes_ = prob.flops(), prob.alg_bytes()
    dn = None
    if not args.no_dense:
        # the dense comparator runs first: its few hundred milliseconds of GEMMs
        # also bring the GPU's clocks to their steady state before the sparse timing
        dn = dense_fp16(8192, 8192, 4096, args.steps, args.warmup, flops)
    ms = time_steps(prob.step, args.steps, args.warmup)
    tflops = flops / (ms * 1e-3) / 1e12
    achieved = bytes_ / (ms * 1e-3) / 1e9
    flush = torch.empty(512 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
    cold_ms = time_cold(prob.step, 10, flush)
    del flush
    warm = launch_percentiles(prob.step, 50)
    rec = {
        "metric": METRIC, "value": round(tflops, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f16", "data": "synthetic",
        "config": {"workload": "static block-sparse SpMM, m=k=8192, n=4096, b=16, density 1/16, FP16 in/out, "
                               "FP32 accumulate (a point of the static sweep)",
                   "m": 8192, "k": 8192, "n": 4096, "b": 16, "density": 1 / 16, "nnz_blocks": prob.nnzb},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profile()},
        "mfma_frac": round(tflops / MFMA_PEAK_TFLOPS["f16"], 4),
        "cold_ms": round(cold_ms, 5),
        "cold_tflops": round(flops / (cold_ms * 1e-3) / 1e12, 3),
        "cold_frac": round(bytes_ / (cold_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "warm_ms_percentiles": warm,
        "plan_build_ms": round(prob.plan_ms, 3),
        "plan_build_ms_warm": round(plan_build_warm_ms(prob), 3),
        "kernel_source_sha256_16": kernel_source_hash(),
        "variant": prob.plan.variant_for(4096),
        "kernel": variant_kernel(prob.plan.variant_for(4096), 16),
    }
    if dn is not None:
        rec["dense_fp16"] = {k: round(v, 4) for k, v in dn.items()}
        rec["speedup_vs_dense"] = round(dn["ms"] / ms, 3)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(prob)
    emit(rec, args.out)


def mode_sweep(args):
    import torch
    dense_cache = {}
    flush = torch.empty(512 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
    points = []
    for n in [int(v) for v in args.sweep_n.split(",")]:
        for b in [int(v) for v in args.sweep_b.split(",")]:
            # b = 16 continues to d = 1/2 and 1 to locate its crossover with dense
            for dd in (128, 64, 32, 16, 8, 4) + ((2, 1) if b == 16 else ()):
                prob = StaticProblem(8192, 8192, n, b, 1.0 / dd, "f16", seed=0)
                ms = time_steps(prob.step, args.steps, args.warmup)
                cold = time_cold(prob.step, 5, flush)
                fl = prob.flops()
                if n not in dense_cache:
                    dense_cache[n] = dense_fp16(8192, 8192, n, args.steps, args.warmup, 1.0)["ms"]
                rec = {"mode": "sweep", "m": 8192, "k": 8192, "n": n, "b": b, "density": 1.0 / dd,
                       "nnz_blocks": prob.nnzb, "ms": round(ms, 5), "cold_ms": round(cold, 5),
                       "tflops": round(fl / (ms * 1e-3) / 1e12, 3),
                       "hbm_gbs": round(prob.alg_bytes() / (ms * 1e-3) / 1e9, 1),
                       "hbm_frac": round(prob.alg_bytes() / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "mfma_frac": round(fl / (ms * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS["f16"], 4),
                       "hbm_frac_cold": round(prob.alg_bytes() / (cold * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "plan_build_ms": round(prob.plan_ms, 3),
                       "dense_ms": round(dense_cache[n], 5), "speedup_vs_dense": round(dense_cache[n] / ms, 3)}
                emit(rec, args.out)
                points.append(rec)
                del prob
                torch.cuda.empty_cache()
    for n in sorted({p["n"] for p in points}):
        for b in sorted({p["b"] for p in points}):
            pts = sorted((p["density"], p["speedup_vs_dense"]) for p in points if p["n"] == n and p["b"] == b)
            if pts:
                emit({"mode": "crossover", "n": n, "b": b, "crossover_density": crossover_density(pts)}, args.out)


def crossover_density(pts):
    """Density at which the sparse/dense speedup falls to 1, interpolated
    linearly in (log d, log speedup) between the bracketing measured points;
    a string bound when every measured point is on one side."""
    for (d0, s0), (d1, s1) in zip(pts, pts[1:]):
        if s0 >= 1.0 > s1:
            t = math.log(s0) / (math.log(s0) - math.log(s1))
            return round(math.exp(math.log(d0) + t * (math.log(d1) - math.log(d0))), 5)
    if all(s >= 1.0 for _, s in pts):
        return "above %g" % pts[-1][0]
    if all(s < 1.0 for _, s in pts):
        return "below %g" % pts[0][0]
    return None


def variant_kernel(variant, b):
    """The kernel a static run of a row-kernel plan launches for a variant code."""
    if variant == 0:
        return "the rule's choice"
    form = variant >> 8
    if b >= 16:
        return {2: "k_spmm_row_pp", 4: "k_spmm_row (every block row split)"}.get(form, "k_spmm_row")
    if form == 2:
        return "k_spmm_b1_lds" if b == 1 else "k_spmm_small_lds"
    return "k_spmm_small"


def mode_point(args):
    """One static product (--point m,k,n,b,1/d,w,x,y), tuned on its first run
    like any plan, then timed: for profiling a single configuration."""
    m, k, n, b, dinv = (int(v) for v in args.point.split(",")[:5])
    w, x, y = args.point.split(",")[5:8]
    prob = StaticProblem(m, k, n, b, 1.0 / dinv, w, x=x, y=y, seed=0, scaled=(w == "fp8"))
    ms = time_steps(prob.step, args.steps, args.warmup)
    v = prob.plan.variant_for(n)
    emit({"mode": "point", "m": m, "k": k, "n": n, "b": b, "density": 1.0 / dinv, "w": w, "x": x, "y": y,
          "variant": v, "kernel": variant_kernel(v, b), "ms": round(ms, 5),
          "tflops": round(prob.flops() / (ms * 1e-3) / 1e12, 3),
          "alg_gbs": round(prob.alg_bytes() / (ms * 1e-3) / 1e9, 1)}, args.out)


def mode_precision(args):
    import torch
    from oracle import fp8_ref
    from oracle import spmm_ref as O
    from paper_2303_16999_amd import synth
    for b in (16, 32):
        for w, y in (("bf16", "bf16"), ("bf16", "f32"), ("fp8", "bf16"), ("fp8", "f32")):
            prob = StaticProblem(16384, 16384, 2048, b, 1 / 16, w, x="bf16", y=y, seed=0, scaled=True)
            ms = time_steps(prob.step, args.steps, args.warmup)
            cols = np.sort(np.random.default_rng(7).choice(2048, 64, replace=False))
            X64 = synth.storage_to_f64(prob.X_store, "bf16")
            v64 = fp8_ref.dequantize_blocks(prob.vals_store, prob.scales_store) if w == "fp8" \
                else synth.storage_to_f64(prob.vals_store, w)
            ref = O.spmm_blockwise_columns(prob.m, prob.k, b, prob.rows, prob.cols, v64, X64, cols)
            Yd = prob.Y.float().cpu().numpy().astype(np.float64)[:, cols]
            rec = {"mode": "precision", "b": b, "w": w, "x": "bf16", "y": y, "ms": round(ms, 5),
                   "tflops": round(prob.flops() / (ms * 1e-3) / 1e12, 3), "rel_fro_vs_oracle": O.rel_fro(Yd, ref)}
            if w == "fp8":
                raw = O.spmm_blockwise_columns(prob.m, prob.k, b, prob.rows, prob.cols,
                                               prob.vals_raw.astype(np.float64), X64, cols)
                rec["fp8_quantisation_rel_fro"] = O.rel_fro(ref, raw)
            emit(rec, args.out)
            del prob
            torch.cuda.empty_cache()


def mode_dynamic(args):
    """Dynamic mode: m = k = 4096, n = 512 (--dyn-n), b = 16, max density 1/8;
    every call brings a fresh pattern (nnz uniform in [max/2, max]) and fresh
    FP16 values. All call inputs are uploaded before timing; per-call HIP
    events, and the same calls replayed from a captured HIP graph."""
    import torch
    from paper_2303_16999_amd import spmm, synth
    m = k = 4096
    n, b = args.dyn_n, 16
    mb = kb = m // b
    max_nnz = mb * kb // 8
    calls = args.calls
    seed = 0
    g = torch.Generator(device="cuda")
    rows_d = torch.empty((calls, max_nnz), dtype=torch.int32, device="cuda")
    cols_d = torch.empty((calls, max_nnz), dtype=torch.int32, device="cuda")
    vals_d = torch.empty((calls, max_nnz, b, b), dtype=torch.float16, device="cuda")
    nnz_d = torch.empty((calls, 1), dtype=torch.int32, device="cuda")
    nnz_h = np.zeros(calls, np.int64)
    patterns = []
    for i in range(calls):
        r = synth.rng(seed + 3 + i)
        nnz = int(r.integers(max_nnz // 2, max_nnz + 1))
        flat = r.choice(mb * kb, size=nnz, replace=False)
        rr, cc = (flat // kb).astype(np.int32), (flat % kb).astype(np.int32)
        rows_d[i, :nnz] = torch.from_numpy(rr).cuda()
        cols_d[i, :nnz] = torch.from_numpy(cc).cuda()
        g.manual_seed(seed + 3 + i)
        vals_d[i, :nnz] = torch.randn((nnz, b, b), generator=g, device="cuda", dtype=torch.float32).half()
        nnz_d[i, 0] = nnz
        nnz_h[i] = nnz
        if i < 32:
            patterns.append((rr, cc))
    X = torch.from_numpy(synth.to_storage(synth.normal((k, n), seed + 2), "f16")).cuda()
    Y = torch.empty((m, n), dtype=torch.float16, device="cuda")
    status = torch.zeros((calls, 1), dtype=torch.int32, device="cuda")
    h = spmm.DynamicHandle(m, k, b, max_nnz, "f16", n_hint=n)
    call = lambda i: h.run(nnz_d[i], rows_d[i], cols_d[i], vals_d[i], X, Y, status[i])
    for i in range(min(args.warmup, calls)):
        call(i)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(calls + 1)]
    ev[0].record()
    for i in range(calls):
        call(i)
        ev[i + 1].record()
    torch.cuda.synchronize()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(calls)])
    assert int(status.max().item()) == 0, "a dynamic call reported an error"
    flops = 2.0 * nnz_h * b * b * n
    # static path on the same patterns (plans built outside timing)
    st_ms, dy_ms = [], []
    for i, (rr, cc) in enumerate(patterns):
        M = np.zeros((mb, kb), np.uint8)
        M[rr, cc] = 1
        order = np.lexsort((cc, rr))
        plan = spmm.StaticPlan(m, k, b, M, "f16", n_hint=n)
        plan.set_values(vals_d[i, : len(rr)][torch.from_numpy(order).cuda()].contiguous())
        st_ms.append(time_steps(lambda: plan.run(X, Y), 10, 2))
        dy_ms.append(time_steps(lambda: call(i), 10, 2))
        plan.close()
    # the same calls captured in one HIP graph (each call's block count is on
    # the device, so the captured calls take their new patterns on every
    # replay): device time per call without the host's launch work. Every
    # replay follows eager work and is checked against the eager result.
    G = min(64, calls)
    call(G - 1)
    torch.cuda.synchronize()
    Y_ref = Y.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for i in range(G):
            call(i)
    g_ms = []
    for _ in range(6):
        Y.fill_(float("nan"))
        status[:G].fill_(-1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        graph.replay()
        e1.record()
        torch.cuda.synchronize()
        assert int(status[:G].max().item()) == 0 and int(status[:G].min().item()) == 0, "a replayed call failed"
        assert torch.equal(Y, Y_ref), "a graph replay differs from the eager call"
        g_ms.append(e0.elapsed_time(e1) / G)
    del graph
    # end to end: each call's COO and values come from pinned host memory over PCIe first
    ne = min(32, calls)
    rows_h = torch.empty((ne, max_nnz), dtype=torch.int32, pin_memory=True)
    cols_h = torch.empty((ne, max_nnz), dtype=torch.int32, pin_memory=True)
    vals_h = torch.empty((ne, max_nnz, b, b), dtype=torch.float16, pin_memory=True)
    nnz_hh = torch.empty((ne, 1), dtype=torch.int32, pin_memory=True)
    rows_h.copy_(rows_d[:ne])
    cols_h.copy_(cols_d[:ne])
    vals_h.copy_(vals_d[:ne])
    nnz_hh.copy_(nnz_d[:ne])
    r_st, c_st, v_st, n_st = (torch.empty_like(rows_d[0]), torch.empty_like(cols_d[0]), torch.empty_like(vals_d[0]),
                              torch.empty_like(nnz_d[0]))

    def call_e2e(i):
        j = i % ne
        q = int(nnz_h[j])  # only the call's own entries cross PCIe
        n_st.copy_(nnz_hh[j], non_blocking=True)
        r_st[:q].copy_(rows_h[j, :q], non_blocking=True)
        c_st[:q].copy_(cols_h[j, :q], non_blocking=True)
        v_st[:q].copy_(vals_h[j, :q], non_blocking=True)
        h.run(n_st, r_st, c_st, v_st, X, Y, status[0])

    reps = 4 * ne
    for i in range(4):
        call_e2e(i)
    torch.cuda.synchronize()
    ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev2[0].record()
    for i in range(reps):
        call_e2e(i)
        ev2[i + 1].record()
    torch.cuda.synchronize()
    per2 = np.array([ev2[i].elapsed_time(ev2[i + 1]) for i in range(reps)])
    assert int(status[0].item()) == 0
    e2e_flops = np.array([2.0 * nnz_h[i % ne] * b * b * n for i in range(reps)])
    e2e_bytes = np.array([float(nnz_h[i % ne]) * (8 + 2 * b * b) + 4 for i in range(reps)])
    dn = dense_fp16(m, k, n, 20, 5, 1.0)
    rec = {"mode": "dynamic", "m": m, "k": k, "n": n, "b": b, "max_density": 1 / 8, "calls": calls,
           "e2e_ms_mean": round(float(per2.mean()), 5), "e2e_ms_p50": round(float(np.percentile(per2, 50)), 5),
           "e2e_ms_p99": round(float(np.percentile(per2, 99)), 5),
           "e2e_tflops": round(float(e2e_flops.sum() / (per2.sum() * 1e-3) / 1e12), 3),
           "e2e_h2d_gbs": round(float(e2e_bytes.sum() / (per2.sum() * 1e-3) / 1e9), 2),
           "call_ms_mean": round(float(per.mean()), 5), "call_ms_p50": round(float(np.percentile(per, 50)), 5),
           "call_ms_p99": round(float(np.percentile(per, 99)), 5),
           "graph_call_ms": round(float(np.median(g_ms)), 5), "graph_calls": G,
           "tflops": round(float(flops.sum() / (per.sum() * 1e-3) / 1e12), 3),
           "static_ms_mean_same_patterns": round(float(np.mean(st_ms)), 5),
           "dynamic_ms_mean_same_patterns": round(float(np.mean(dy_ms)), 5),
           "dynamic_over_static_throughput": round(float(np.mean(st_ms) / np.mean(dy_ms)), 3),
           "dense_fp16_ms": round(dn["ms"], 5), "dynamic_speedup_vs_dense": round(dn["ms"] / float(per.mean()), 3),
           "static_speedup_vs_dense": round(dn["ms"] / float(np.mean(st_ms)), 3)}
    emit(rec, args.out)


def mlp_plans(layers=8, d_in=4096, d_hid=16384, b=16, d=1 / 16, seed=0):
    """The serving model: `layers` x (W1 d_hid x d_in, ReLU, W2 d_in x d_hid), FP16
    block-sparse weights resident on the device, scaled so activations stay O(1)."""
    import torch
    from paper_2303_16999_amd import spmm, synth
    plans, dims, relu = [], [d_in], []
    for l in range(2 * layers):
        k, m = (d_in, d_hid) if l % 2 == 0 else (d_hid, d_in)
        mask = synth.block_mask(m // b, k // b, d, seed + 2 * l)
        nnz = int(mask.sum())
        scale = (1.0 if l % 2 == 0 else math.sqrt(2.0)) / math.sqrt(k * d)
        g = torch.Generator(device="cuda").manual_seed(seed + 2 * l + 1)
        vals = (torch.randn((nnz, b, b), generator=g, device="cuda", dtype=torch.float32) * scale).half()
        plan = spmm.StaticPlan(m, k, b, mask, "f16", n_hint=256)
        plan.set_values(vals)
        plans.append(plan)
        dims.append(m)
        relu.append(1 if l % 2 == 0 else 0)
    torch.cuda.synchronize()
    return plans, dims, relu


def pretune(plans, dims, max_n=2048):
    """Runs the autotuner on every plan for each n class 1 .. max_n, so grouped
    launches and the serving loop (which look up tuned variants but never
    measure) run on measured tile choices."""
    import torch
    n = 1
    while n <= max_n:
        for l, p in enumerate(plans):
            X = torch.randn((dims[l], -(-n // 8) * 8), device="cuda").half()
            Y = torch.empty((dims[l + 1], -(-n // 8) * 8), device="cuda", dtype=torch.float16)
            p.autotune(X, Y, n=n)
        n *= 2
    torch.cuda.synchronize()


def run_trace(srv, arrivals, ns, x_host, y_hosts, t_start=None):
    """Open-loop driver: submit request i at arrivals[i] (seconds from start), poll
    completions; returns the completion records in id order."""
    from paper_2303_16999_amd import spmm
    done = {}
    t0 = spmm.clock() if t_start is None else t_start
    nreq = len(ns)
    i = 0
    while len(done) < nreq:
        now = spmm.clock() - t0
        while i < nreq and arrivals[i] <= now:
            n = int(ns[i])
            srv.submit(i, n, _view(x_host, n), _view(y_hosts[i % len(y_hosts)], n))
            i += 1
        for d in srv.poll():
            done[d["id"]] = d
        if i < nreq:
            wait = arrivals[i] - (spmm.clock() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.0005))
        else:
            time.sleep(0.0002)
    return [done[j] for j in range(nreq)], t0


def _view(buf, n, rows=4096):
    """[rows x n8] view (n8 = n rounded up to a multiple of 8: the device layout)
    over the front of a flat pinned host buffer."""
    n8 = -(-n // 8) * 8
    return buf[: rows * n8].view(rows, n8)


def mode_serve(args):
    """Serving: 8-layer sparse MLP (4096 -> 16384 -> 4096 per layer, b = 16,
    density 1/16, FP16 weights resident, tile variants tuned per n class),
    Poisson arrivals, n ~ log-uniform [1, 2048]; continuous batching through
    grouped launches against the plain one-request-at-a-time path on the same
    trace."""
    import torch
    from paper_2303_16999_amd import spmm, synth
    plans, dims, relu = mlp_plans()
    pretune(plans, dims)
    flop_per_token = sum(2.0 * dims[l] * dims[l + 1] / 16 for l in range(len(dims) - 1))
    # pinned host buffers in the device layout, so request copies are plain DMA
    x_host = torch.empty(4096 * 2048, dtype=torch.float16, pin_memory=True)
    x_host.copy_(torch.from_numpy(synth.to_storage(synth.normal((4096 * 2048,), 7), "f16")))
    y_hosts = [torch.zeros(4096 * 2048, dtype=torch.float16, pin_memory=True) for _ in range(8)]
    budget = 32768 * (4096 + 16384) * 2  # 32,768 tokens of activations in flight
    warm = 200
    nmeas = args.requests

    def make_server(mode, max_tokens=0):
        return spmm.Server(plans, dims, relu=relu, mem_budget_bytes=budget, max_active=256, mode=mode,
                           max_tokens=max_tokens)

    # accuracy: the two paths agree bit for bit on a sample of requests
    sample_n = [1, 7, 64, 300, 2048]
    outs = {}
    for mode in (spmm.SERVE_CONTINUOUS, spmm.SERVE_PLAIN):
        srv = make_server(mode)
        ys = [torch.zeros((4096, -(-n // 8) * 8), dtype=torch.float16, pin_memory=True) for n in sample_n]
        for i, n in enumerate(sample_n):
            srv.submit(i, n, _view(x_host, n), ys[i])
        srv.drain()
        srv.poll()
        srv.close()
        outs[mode] = [y[:, :n].clone() for y, n in zip(ys, sample_n)]
    same = all(torch.equal(a, b) for a, b in zip(outs[spmm.SERVE_CONTINUOUS], outs[spmm.SERVE_PLAIN]))
    finite = all(torch.isfinite(y.float()).all().item() for y in outs[spmm.SERVE_CONTINUOUS])

    # saturated rates: every request arrives at once
    _, n_sat = synth.serving_trace(600, 1.0, seed=11)
    token_caps = [int(v) for v in args.max_tokens.split(",")]
    sat = {}
    for mode, name, cap in [(spmm.SERVE_CONTINUOUS, "continuous", c) for c in token_caps] + [(spmm.SERVE_PLAIN, "plain", 0)]:
        srv = make_server(mode, cap)
        t0 = spmm.clock()
        recs, _ = run_trace(srv, np.zeros(len(n_sat)), n_sat, x_host, y_hosts, t0)
        t_sat = max(r["done_s"] for r in recs) - t0
        st = srv.stats()
        srv.close()
        sat[(name, cap)] = len(n_sat) / t_sat
        emit({"mode": "serve_saturation", "path": name, "max_tokens": cap, "requests": len(n_sat),
              "tokens": int(n_sat.sum()), "seconds": round(t_sat, 4), "req_per_s": round(len(n_sat) / t_sat, 2),
              "tokens_per_s": round(n_sat.sum() / t_sat, 1),
              "effective_tflops": round(n_sat.sum() * flop_per_token / t_sat / 1e12, 3),
              "steps": st["steps"], "problems_per_step": round(st["problems_run"] / max(1, st["steps"]), 2),
              "paths_bitwise_equal": bool(same), "outputs_finite": bool(finite)}, args.out)
    mu_max = max(v for (name, cap), v in sat.items() if name == "continuous")
    if args.rate_base > 0:  # a fixed base rate, so that runs offer the same load
        mu_max = args.rate_base

    for rho in [float(v) for v in args.rho.split(",")]:
        arrivals, ns = synth.serving_trace(warm + nmeas, rho * mu_max, seed=12)
        runs = [(spmm.SERVE_CONTINUOUS, "continuous", c) for c in token_caps] + [(spmm.SERVE_PLAIN, "plain", 0)]
        for mode, name, cap in runs:
            srv = make_server(mode, cap)
            recs, t0 = run_trace(srv, arrivals, ns, x_host, y_hosts)
            st = srv.stats()
            srv.close()
            meas = recs[warm:]
            lat = np.array([r["done_s"] - r["submit_s"] for r in meas]) * 1e3
            t_first = min(r["submit_s"] for r in meas)
            t_last = max(r["done_s"] for r in meas)
            toks = sum(r["n"] for r in meas)
            emit({"mode": "serve", "path": name, "max_tokens": cap, "rho": rho,
                  "rate_req_per_s": round(rho * mu_max, 2), "requests": len(meas), "tokens": int(toks),
                  "tokens_per_s": round(toks / (t_last - t_first), 1),
                  "req_per_s": round(len(meas) / (t_last - t_first), 2),
                  "effective_tflops": round(toks * flop_per_token / (t_last - t_first) / 1e12, 3),
                  "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
                  "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
                  "latency_ms_mean": round(float(lat.mean()), 3),
                  "steps": st["steps"], "peak_active": st["peak_active"],
                  "peak_pool_mib": round(st["peak_pool_bytes"] / 2**20, 1)}, args.out)
    for p in plans:
        p.close()
    torch.cuda.synchronize()


def mode_group(args):
    """The 16 serving matrices (tile variants tuned per n class) with n_i ~
    log-uniform [1, 2048]: one grouped launch in each of its two forms (one workgroup per unit, launched directly;
    persistent workgroups walking the units on a static per-XCD schedule) against 16
    separate launches."""
    import torch
    from paper_2303_16999_amd import spmm, synth
    plans, dims, relu = mlp_plans()
    pretune(plans, dims)
    g = synth.rng(21)
    for trial in range(3):
        ns = [int(v) for v in np.clip(np.floor(np.exp(g.uniform(0, math.log(2049), size=16))), 1, 2048)]
        Xs = [torch.randn((dims[l], ns[l] + (-ns[l]) % 8), device="cuda").half() for l in range(16)]
        Ys = [torch.empty((dims[l + 1], ns[l] + (-ns[l]) % 8), device="cuda", dtype=torch.float16) for l in range(16)]
        grp = spmm.Group(16)

        def grouped():
            grp.run(plans, Xs, Ys, ns=ns, relu=relu)

        def separate():
            for l in range(16):
                plans[l].run(Xs[l], Ys[l], n=ns[l])

        form = os.environ.get("SPMM_GROUP_PERSIST")
        os.environ["SPMM_GROUP_PERSIST"] = "0"
        ms_g = time_steps(grouped, args.steps * 5, args.warmup)
        os.environ["SPMM_GROUP_PERSIST"] = "1"
        ms_p = time_steps(grouped, args.steps * 5, args.warmup)
        if form is None:
            del os.environ["SPMM_GROUP_PERSIST"]
        else:
            os.environ["SPMM_GROUP_PERSIST"] = form
        ms_s = time_steps(separate, args.steps * 5, args.warmup)
        fl = sum(2.0 * dims[l] * dims[l + 1] / 16 * ns[l] for l in range(16))
        emit({"mode": "group", "n": ns, "grouped_ms": round(ms_g, 5), "persistent_ms": round(ms_p, 5),
              "separate_ms": round(ms_s, 5), "speedup": round(ms_s / ms_g, 3),
              "persistent_speedup": round(ms_s / ms_p, 3), "grouped_tflops": round(fl / (ms_g * 1e-3) / 1e12, 3),
              "persistent_tflops": round(fl / (ms_p * 1e-3) / 1e12, 3),
              "separate_tflops": round(fl / (ms_s * 1e-3) / 1e12, 3)}, args.out)
        grp.close()
    for p in plans:
        p.close()


def mode_table3(args):
    """Static and dynamic sparse against dense at m = k = 4096, d = 1/16,
    b in {1, 4, 16}, FP16 and FP32, best over n: the shape of the paper's
    static-vs-dynamic comparison (Table 3; dense of the same dtype). The
    dynamic call re-encodes the static pattern (COO in random order) on every
    call."""
    import torch
    from paper_2303_16999_amd import spmm
    m = k = 4096
    for dt, b in [("f16", 1), ("f16", 4), ("f16", 16), ("f32", 1), ("f32", 4), ("f32", 16)]:
        best = {"static": 0.0, "dynamic": 0.0}
        for n in (1024, 4096, 16384):
            prob = StaticProblem(m, k, n, b, 1 / 16, dt, seed=0)
            ms_s = time_steps(prob.step, args.steps, args.warmup)
            perm = np.random.default_rng(1).permutation(prob.nnzb)
            r = torch.from_numpy(prob.rows[perm].copy()).cuda()
            c = torch.from_numpy(prob.cols[perm].copy()).cuda()
            v = prob.values_dev[torch.from_numpy(perm).cuda()].contiguous()
            nnz = torch.tensor([prob.nnzb], dtype=torch.int32, device="cuda")
            status = torch.zeros(1, dtype=torch.int32, device="cuda")
            h = spmm.DynamicHandle(m, k, b, prob.nnzb, dt, n_hint=n)
            ms_d = time_steps(lambda: h.run(nnz, r, c, v, prob.X, prob.Y, status), args.steps, args.warmup)
            assert int(status.item()) == 0
            dn = dense_gemm(m, k, n, args.steps, args.warmup, dt)
            rec = {"mode": "table3", "dtype": dt, "m": m, "k": k, "n": n, "b": b, "density": 1 / 16,
                   "static_ms": round(ms_s, 5), "dynamic_ms": round(ms_d, 5), "dense_ms": round(dn, 5),
                   "static_over_dense": round(dn / ms_s, 3), "dynamic_over_dense": round(dn / ms_d, 3),
                   "static_tflops": round(prob.flops() / (ms_s * 1e-3) / 1e12, 3)}
            emit(rec, args.out)
            best["static"] = max(best["static"], rec["static_over_dense"])
            best["dynamic"] = max(best["dynamic"], rec["dynamic_over_dense"])
            del prob, h, v
            torch.cuda.empty_cache()
        emit({"mode": "table3_best_over_n", "dtype": dt, "b": b, "static_over_dense": best["static"],
              "dynamic_over_dense": best["dynamic"]}, args.out)


def mode_small(args):
    """The small FP32 case: m = k = 1024, n = 64, b = 16, density 1/16 (row-wise
    FP32 16x16x4 MFMA kernel): latency and error against the FP64 oracle; then
    FP32 at m = k = 8192, n = 1024, d = 1/16."""
    from oracle import spmm_ref as O
    import torch
    prob = StaticProblem(1024, 1024, 64, 16, 1 / 16, "f32", seed=0)
    ms = time_steps(prob.step, max(args.steps, 50), args.warmup)
    pct = launch_percentiles(prob.step, 50)
    prob.step()
    torch.cuda.synchronize()
    ref = O.spmm_blockwise(1024, 1024, 16, prob.rows, prob.cols, prob.vals_store.astype(np.float64),
                           prob.X_store.astype(np.float64))
    err = O.rel_fro(prob.Y.cpu().numpy().astype(np.float64), ref)
    emit({"mode": "small_fp32", "kernel": "row", "m": 1024, "k": 1024, "n": 64, "b": 16, "density": 1 / 16,
          "ms": round(ms, 5), "launch_ms_percentiles": pct,
          "tflops": round(prob.flops() / (ms * 1e-3) / 1e12, 3), "rel_fro_vs_oracle": err, "bound": 1e-5},
         args.out)
    big = StaticProblem(8192, 8192, 1024, 16, 1 / 16, "f32", seed=0)
    msb = time_steps(big.step, args.steps, args.warmup)
    emit({"mode": "fp32_large", "kernel": "row", "m": 8192, "k": 8192, "n": 1024, "b": 16, "density": 1 / 16,
          "ms": round(msb, 5), "tflops": round(big.flops() / (msb * 1e-3) / 1e12, 3),
          "mfma_fp32_frac": round(big.flops() / (msb * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS["f32"], 4)}, args.out)


def mode_skew(args):
    """Skewed patterns at m = k = 8192, n = 4096, b = 16, d = 1/16, FP16: the
    uniform pattern, power-law row lengths and all blocks in the fewest rows,
    with long rows split over a workgroup's waves and without."""
    import torch
    from paper_2303_16999_amd import synth
    mb = kb = 512
    masks = {"uniform": synth.block_mask(mb, kb, 1 / 16, 0),
             "power_law_1.2": synth.skewed_mask(mb, kb, 1 / 16, 1.2, 0),
             "concentrated": synth.concentrated_mask(mb, kb, 1 / 16, 0)}
    dn = dense_fp16(8192, 8192, 4096, args.steps, args.warmup, 1.0)["ms"]
    for name, mask in masks.items():
        for split in (True, False):
            if not split:
                os.environ["SPMM_SPLIT"] = "0"
            prob = StaticProblem(8192, 8192, 4096, 16, 1 / 16, "f16", seed=0, mask=mask)
            os.environ.pop("SPMM_SPLIT", None)
            ms = time_steps(prob.step, args.steps, args.warmup)
            rl = mask.sum(1)
            emit({"mode": "skew", "pattern": name, "split_long_rows": split,
                  "variant": prob.plan.variant_for(4096),
                  "split_rows": prob.plan.info()["num_split_rows"], "max_row_blocks": int(rl.max()),
                  "mean_row_blocks": float(rl.mean()), "ms": round(ms, 5),
                  "tflops": round(prob.flops() / (ms * 1e-3) / 1e12, 3), "dense_ms": round(dn, 5),
                  "speedup_vs_dense": round(dn / ms, 3)}, args.out)
            del prob
            torch.cuda.empty_cache()


def mode_train(args):
    """The three products of a training step of one block-sparse layer at
    m = k = 8192, n = 4096, FP16 (b = 16 at densities 1/16 and 1/4; b = 8, 4
    and 1 at 1/16): forward Y = (M o W) X, data gradient dX = (M o W)^T dY on
    the transposed plan, weight gradient dW = (dY X^T) o M (FP32 blocks), next
    to the three dense FP16 GEMMs of the same step."""
    import torch
    m = k = 8192
    n = 4096
    g = torch.Generator(device="cuda").manual_seed(77)
    A = torch.randn((m, k), device="cuda", dtype=torch.float16, generator=g)
    Xd = torch.randn((k, n), device="cuda", dtype=torch.float16, generator=g)
    dYd = torch.randn((m, n), device="cuda", dtype=torch.float16, generator=g)
    Yd, dXd, dWd = (torch.empty((m, n), device="cuda", dtype=torch.float16),
                    torch.empty((k, n), device="cuda", dtype=torch.float16),
                    torch.empty((m, k), device="cuda", dtype=torch.float16))
    dense = {"forward": time_steps(lambda: torch.matmul(A, Xd, out=Yd), args.steps, args.warmup),
             "data_grad": time_steps(lambda: torch.matmul(A.t(), dYd, out=dXd), args.steps, args.warmup),
             "weight_grad": time_steps(lambda: torch.matmul(dYd, Xd.t(), out=dWd), args.steps, args.warmup)}
    del A, Xd, dYd, Yd, dXd, dWd
    torch.cuda.empty_cache()
    for b, d in ((16, 1 / 16), (16, 1 / 4), (8, 1 / 16), (4, 1 / 16), (1, 1 / 16)):
        prob = StaticProblem(m, k, n, b, d, "f16", seed=0)
        dY = torch.randn((m, n), device="cuda", dtype=torch.float16, generator=g)
        dX = torch.empty((k, n), device="cuda", dtype=torch.float16)
        G = torch.empty((prob.nnzb, b, b), device="cuda", dtype=torch.float32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tp = prob.plan.transpose(n_hint=n)
        torch.cuda.synchronize()
        transpose_ms = (time.perf_counter() - t0) * 1e3
        steps = {"forward": prob.step, "data_grad": lambda: tp.run(dY, dX),
                 "weight_grad": lambda: prob.plan.sddmm(dY, prob.X, G)}
        flops = prob.flops()
        rec = {"mode": "train", "m": m, "k": k, "n": n, "b": b, "density": d, "nnz_blocks": prob.nnzb,
               "transpose_plan_ms": round(transpose_ms, 3)}
        total_s = total_d = 0.0
        for name, fn in steps.items():
            ms = time_steps(fn, args.steps, args.warmup)
            total_s += ms
            total_d += dense[name]
            rec[name] = {"ms": round(ms, 5), "tflops": round(flops / (ms * 1e-3) / 1e12, 3),
                         "dense_ms": round(dense[name], 5), "speedup_vs_dense": round(dense[name] / ms, 3)}
        # weight gradient: reads dY and X, writes the FP32 blocks
        wg_bytes = 2.0 * (m + k) * n + 4.0 * prob.nnzb * b * b
        rec["weight_grad"]["alg_gbs"] = round(wg_bytes / (rec["weight_grad"]["ms"] * 1e-3) / 1e9, 1)
        rec["step_ms"] = round(total_s, 5)
        rec["dense_step_ms"] = round(total_d, 5)
        rec["step_speedup_vs_dense"] = round(total_d / total_s, 3)
        emit(rec, args.out)
        del prob, tp, dY, dX, G
        torch.cuda.empty_cache()


def mode_dispatch(args):
    """Dense dispatch at m = k = 8192, n = 4096, FP16: for each (b, d) the
    speedup model's predicted sparse/dense ratio, the measured best sparse
    variant and the dense GEMM on the plan's dense copy (both through the
    autotuner), and the variant a plan with dense dispatch runs."""
    import torch
    from paper_2303_16999_amd import spmm
    m = k = 8192
    n = 4096
    for b, d in ((1, 1 / 16), (4, 1 / 16), (4, 1 / 4), (8, 1 / 16), (16, 1 / 16), (16, 1 / 4), (16, 1 / 2)):
        prob = StaticProblem(m, k, n, b, d, "f16", seed=0)
        plan = spmm.StaticPlan(m, k, b, prob.mask, "f16", n_hint=n, dense_dispatch=2)
        plan.set_values(prob.values_dev)
        ratio, _ = plan.dispatch()
        best, times = plan.autotune(prob.X, prob.Y, n=n)
        dense_ms = times.pop(3 * 256)
        sparse_v = min(times, key=times.get)
        rec = {"mode": "dispatch", "m": m, "k": k, "n": n, "b": b, "density": d,
               "model_ratio": round(ratio, 3), "model_picks": "dense" if ratio < 1 else "sparse",
               "sparse_best_ms": round(times[sparse_v], 5), "sparse_best_variant": sparse_v,
               "dense_ms": round(dense_ms, 5), "measured_ratio": round(dense_ms / times[sparse_v], 3),
               "tuner_picks": "dense" if best == 3 * 256 else "sparse"}
        emit(rec, args.out)
        plan.close()
        del prob
        torch.cuda.empty_cache()


def mode_grid(args):
    """The paper's static sweep grid (Table 1 of Section 4: m = k in 2^8..2^13,
    n in 2^2..2^16 by powers of 4, b in {1, 4, 8, 16}, d in {1/4 .. 1/32},
    FP16): static sparse and dense FP16 TFLOP/s (nonzero FLOPs), each best
    over n, their ratio per (m, b, d), and a power-law fit of the ratio
    (Section 5, "Will my application speed up?")."""
    import torch
    from paper_2303_16999_amd import spmm, synth
    from paper_2303_16999_amd import speedup_model
    ms_list = [int(v) for v in args.grid_m.split(",")]
    n_list = [int(v) for v in args.grid_n.split(",")]
    bs, ds = (1, 4, 8, 16), (4, 8, 16, 32)
    g = torch.Generator(device="cuda").manual_seed(11)
    results = []
    for m in ms_list:
        plans = {}
        for b in bs:
            for dd in ds:
                mb = -(-m // b)
                mask = synth.block_mask(mb, mb, 1.0 / dd, 0)
                plan = spmm.StaticPlan(m, m, b, mask, "f16", n_hint=1024)
                nnzb = plan.info()["nnzb"]
                vals = torch.randn((max(nnzb, 1), b, b), device="cuda", dtype=torch.float16, generator=g)
                plan.set_values(vals)
                plans[(b, dd)] = (plan, vals, 2.0 * nnzb * b * b)  # FLOPs per column of X
        best = {key: (0.0, None) for key in plans}
        best_dense = {dd: (0.0, None) for dd in ds}
        for n in n_list:
            if m * n * 2 * 3 > 6 * 2 ** 30:
                continue
            ld = -(-n // 8) * 8  # rows of X and Y start 16-byte aligned
            X = torch.randn((m, ld), device="cuda", dtype=torch.float16, generator=g)
            Y = torch.empty((m, ld), device="cuda", dtype=torch.float16)
            Xd = X[:, :n].contiguous()
            Yd = torch.empty((m, n), device="cuda", dtype=torch.float16)
            A = torch.randn((m, m), device="cuda", dtype=torch.float16, generator=g)
            steps = max(3, min(args.steps, int(2e9 / max(1, m * m * n))))
            tdense = time_steps(lambda: torch.matmul(A, Xd, out=Yd), steps, 2)
            for dd in ds:
                tf = 2.0 * m * m * n / dd / (tdense * 1e-3) / 1e12  # nonzero FLOPs of density 1/dd
                if tf > best_dense[dd][0]:
                    best_dense[dd] = (tf, n)
            for key, (plan, _, fpc) in plans.items():
                t = time_steps(lambda: plan.run(X, Y, n=n), steps, 2)
                tf = fpc * n / (t * 1e-3) / 1e12
                if tf > best[key][0]:
                    best[key] = (tf, n)
            del X, Y, Xd, Yd, A
            torch.cuda.empty_cache()
        for (b, dd), (tf, n_best) in sorted(best.items()):
            dtf, dn = best_dense[dd]
            rec = {"mode": "grid", "m": m, "k": m, "b": b, "density": 1.0 / dd, "sparse_tflops": round(tf, 3),
                   "sparse_best_n": n_best, "dense_tflops_nonzero": round(dtf, 3), "dense_best_n": dn,
                   "speedup": round(tf / dtf, 4) if dtf > 0 else None}
            emit(rec, args.out)
            results.append(rec)
        del plans
        torch.cuda.empty_cache()
    pts = [(r["m"], r["density"], r["b"], r["speedup"]) for r in results if r["speedup"]]
    fit = speedup_model.fit(pts)
    emit(dict({"mode": "grid_fit"}, **fit), args.out)


def mode_ell(args):
    """Blocked-ELL and large blocks at m = k = 8192, n = 4096, density 1/16,
    FP16: (1) the plan built from a blocked-ELL description against the one
    built from the mask (the same kernel), and the cost of materialising the
    ELL padding as explicit zero blocks (the padding the paper expects tensor
    cores to absorb, Section 5); (2) b = 16, 32 and 64 at equal density."""
    import torch
    from paper_2303_16999_amd import spmm, synth
    m = k = 8192
    n = 4096
    g = torch.Generator(device="cuda").manual_seed(21)
    X = torch.randn((k, n), device="cuda", dtype=torch.float16, generator=g)
    Y = torch.empty((m, n), device="cuda", dtype=torch.float16)
    dn = dense_fp16(m, k, n, args.steps, args.warmup, 1.0)["ms"]
    b = 16
    mb = kb = m // b
    mask = synth.block_mask(mb, kb, 1 / 16, 0)
    width = int(mask.sum(1).max())
    cols = synth.ell_from_mask(mask, width, 1)
    nnzb = int(mask.sum())
    vals = torch.randn((mb * width, b, b), device="cuda", dtype=torch.float16, generator=g)
    ell_plan = spmm.StaticPlan.from_ell(m, k, b, cols, "f16", n_hint=n)
    ell_plan.set_values_ell(vals)
    mask_plan = spmm.StaticPlan(m, k, b, mask, "f16", n_hint=n)
    mask_plan.set_values(torch.randn((nnzb, b, b), device="cuda", dtype=torch.float16, generator=g))
    # padding made explicit: every row filled to the ELL width with zero blocks in unused columns
    rng = np.random.default_rng(2)
    padded = mask.copy()
    for r in range(mb):
        free = np.nonzero(padded[r] == 0)[0]
        padded[r, rng.choice(free, width - int(mask[r].sum()), replace=False)] = 1
    pr, pc = np.nonzero(padded)
    pvals = torch.zeros((pr.size, b, b), device="cuda", dtype=torch.float16)
    keep = torch.from_numpy(mask[pr, pc].astype(bool)).cuda()
    pvals[keep] = torch.randn((nnzb, b, b), device="cuda", dtype=torch.float16, generator=g)
    pad_plan = spmm.StaticPlan(m, k, b, padded, "f16", n_hint=n)
    pad_plan.set_values(pvals)
    flops = 2.0 * nnzb * b * b * n
    for name, plan in (("mask", mask_plan), ("ell", ell_plan), ("ell_padded_explicit", pad_plan)):
        ms = time_steps(lambda: plan.run(X, Y), args.steps, args.warmup)
        emit({"mode": "ell", "plan": name, "m": m, "k": k, "n": n, "b": b, "density": 1 / 16, "ell_width": width,
              "blocks_run": int(pr.size) if name == "ell_padded_explicit" else nnzb, "nnz_blocks": nnzb,
              "ms": round(ms, 5), "tflops_nonzero": round(flops / (ms * 1e-3) / 1e12, 3),
              "dense_ms": round(dn, 5), "speedup_vs_dense": round(dn / ms, 3)}, args.out)
    del ell_plan, mask_plan, pad_plan, vals, pvals
    torch.cuda.empty_cache()
    for bb in (16, 32, 64):
        prob = StaticProblem(m, k, n, bb, 1 / 16, "f16", seed=0)
        ms = time_steps(prob.step, args.steps, args.warmup)
        emit({"mode": "block_size", "m": m, "k": k, "n": n, "b": bb, "density": 1 / 16, "nnz_blocks": prob.nnzb,
              "ms": round(ms, 5), "tflops": round(prob.flops() / (ms * 1e-3) / 1e12, 3),
              "dense_ms": round(dn, 5), "speedup_vs_dense": round(dn / ms, 3)}, args.out)
        del prob
        torch.cuda.empty_cache()


def mode_copy(args):
    """Plain copy of a known size, for calibrating the HBM byte counters."""
    import torch
    x = torch.ones(256 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    ms = time_steps(lambda: y.copy_(x), args.steps, args.warmup)
    emit({"mode": "copy", "bytes_read": x.numel() * 4, "bytes_written": y.numel() * 4, "ms": ms}, args.out)


def mode_peaks(args):
    """Measured peaks for the roofline: HBM bandwidth of a 1 GiB device copy
    (bytes read + written) and of a 2 GiB read-only reduction, and the dense
    FP16 / BF16 matrix-core rate of hipBLASLt GEMMs (torch.matmul) at
    8192 x 8192 x 8192. Library kernels, used only as yardsticks."""
    import torch
    n = 1024 * 1024 * 1024 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    ms = time_steps(lambda: y.copy_(x), args.steps, args.warmup)
    emit({"mode": "peaks", "what": "hbm_copy", "bytes": 2 * n * 4, "ms": round(ms, 4),
          "gbs": round(2 * n * 4 / (ms * 1e-3) / 1e9, 1), "datasheet_gbs": HBM_PEAK_GBS}, args.out)
    del y
    z = torch.ones(2 * n, dtype=torch.float32, device="cuda")
    out = torch.empty((), dtype=torch.float32, device="cuda")
    ms = time_steps(lambda: torch.sum(z, dim=0, out=out), args.steps, args.warmup)
    emit({"mode": "peaks", "what": "hbm_read", "bytes": 2 * n * 4, "ms": round(ms, 4),
          "gbs": round(2 * n * 4 / (ms * 1e-3) / 1e9, 1), "datasheet_gbs": HBM_PEAK_GBS}, args.out)
    del x, z
    torch.cuda.empty_cache()
    for dt, name in ((torch.float16, "f16"), (torch.bfloat16, "bf16")):
        m = 8192
        a = torch.randn((m, m), device="cuda").to(dt)
        b = torch.randn((m, m), device="cuda").to(dt)
        c = torch.empty((m, m), device="cuda", dtype=dt)
        ms = time_steps(lambda: torch.matmul(a, b, out=c), args.steps, args.warmup)
        emit({"mode": "peaks", "what": "gemm_" + name, "m": m, "n": m, "k": m, "ms": round(ms, 4),
              "tflops": round(2.0 * m ** 3 / (ms * 1e-3) / 1e12, 1),
              "datasheet_tflops": MFMA_PEAK_TFLOPS[name]}, args.out)
        del a, b, c
        torch.cuda.empty_cache()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2303_16999_amd import spmm
    spmm.lib()  # fails loudly if the HIP library is missing
    {"headline": mode_headline, "sweep": mode_sweep, "precision": mode_precision, "copy": mode_copy,
     "dynamic": mode_dynamic, "serve": mode_serve, "group": mode_group, "table3": mode_table3,
     "small": mode_small, "skew": mode_skew, "train": mode_train, "grid": mode_grid,
     "ell": mode_ell, "peaks": mode_peaks, "dispatch": mode_dispatch, "point": mode_point}[args.mode](args)


if __name__ == "__main__":
    main()
