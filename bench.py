#!/usr/bin/env python3
"""Benchmark: bracket + independence checks per second and time-to-closure on one MI355X.

One step = one complete closure (the whole bracket loop, full certification
unless --early-exit) of the workload's generators; the generator phase of each
step's handle runs before the timed region, so the inputs (and the first basis
elements) are resident in HBM when timing starts.

Default workload: two random traceless anti-Hermitian 16 x 16 matrices
(seed 2, Frobenius-normalised), tol 1e-10, FP64 decisions -- closure su(16),
dim 255, 32,385 brackets per step.

Prints ONE JSON line.  `roofline` describes the dominant kernel, timed live
with HIP events on the library's stream during the timed steps; `cpu_baseline`
times the CPU reference on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bracket+independence checks/sec and time-to-closure; mixed/batched vs FP64 plain, 1 GPU"

# MI355X published peaks
PEAK = {"hbm_GBps": 8000.0, "fp64_TF": 78.6, "fp32_TF": 157.3, "bf16_TF": 2500.0}


def workload(name: str):
    from paper_2506_01120_amd import workloads as W

    if name == "batch64":
        probs = W.batch_problems(tol=1e-8)
        return probs, 1e-8, ("64 independent problems: Ising n=3..7, XX+YY n=3..6, 29 random Pauli-string sets "
                             "on n=4..6 qubits, random pairs d=8..24 (seeds 1000+i)")
    if name == "su16":
        return W.rand_pair(16, seed=2), 1e-10, "random traceless anti-Hermitian pair d=16 seed 2 -> su(16)"
    if name == "ising3":
        return W.ising(3), 1e-10, "open transverse-field Ising chain n=3 d=8 -> so(6)"
    if name == "su32":
        return W.rand_pair(32, seed=3), 1e-8, "random traceless anti-Hermitian pair d=32 seed 3 -> su(32)"
    if name == "ising7":
        return W.ising(7), 1e-10, "open transverse-field Ising chain n=7 d=128 -> so(14)"
    if name == "sums5":
        return W.pauli_sums(5, 2, 3, 5), 1e-10, "two random 3-term Pauli sums on 5 qubits (seed 5), d=32"
    if name == "su64":
        return W.rand_pair(64, seed=5), 1e-8, "random traceless anti-Hermitian pair d=64 seed 5 -> su(64)"
    raise SystemExit(f"unknown workload {name}")


def run_steps(gens, tol, cfg, steps):
    import torch

    from paper_2506_01120_amd import BatchClosure, LieClosure

    if isinstance(gens, list):  # a batch of problems: one step = the whole batch
        batches = [BatchClosure([p.gens for p in gens], [p.tol for p in gens], **cfg) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in batches:
            b.run()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stats = [b.stats(-1) for b in batches]  # batch aggregate: counters summed, grouped-launch timers
        dims = [[b.dim(i) for i in range(b.n)] for b in batches]
        for b in batches:
            b.close()
        return t1 - t0, stats, dims
    handles = [LieClosure(gens, tol, **cfg) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for h in handles:
        h.run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = [h.stats() for h in handles]
    dims = [h.dim for h in handles]
    for h in handles:
        h.close()
    return t1 - t0, stats, dims


def roofline(stats, precision: str):
    """Dominant kernel class over the timed steps: algorithmic work / summed HIP-event time."""
    names = list(stats[0]["kernel_ms"].keys())
    ms = {k: sum(s["kernel_ms"][k] for s in stats) for k in names}
    fl = {k: sum(s["kernel_flops"][k] for s in stats) for k in names}
    by = {k: sum(s["kernel_bytes"][k] for s in stats) for k in names}
    n = {k: sum(s["kernel_launches"][k] for s in stats) for k in names}
    dom = max(names, key=lambda k: ms[k])
    t = ms[dom] / 1e3
    if t <= 0 or n[dom] == 0:
        return {"kernel": dom, "bound": "hbm", "achieved": 0.0, "peak": PEAK["hbm_GBps"], "unit": "GB/s",
                "frac": 0.0, "traffic": None, "note": "no timed kernel launches", "breakdown": {}}
    peak_tf = PEAK["fp64_TF"] if precision == "fp64" else PEAK["fp32_TF"] if precision == "fp32" else PEAK["bf16_TF"]
    intensity = fl[dom] / by[dom] if by[dom] else float("inf")
    ridge = peak_tf * 1e12 / (PEAK["hbm_GBps"] * 1e9)
    if fl[dom] > 0 and intensity >= ridge:
        achieved, peak, unit, bound = fl[dom] / t / 1e12, peak_tf, "TFLOP/s", "mfma"
    else:
        achieved, peak, unit, bound = by[dom] / t / 1e9, PEAK["hbm_GBps"], "GB/s", "hbm"
    def cls_roof(k):
        # each class against its own bound: the matrix-core peak of the arithmetic it runs in
        # (the screen's GEMMs in the screen precision, the screened bracket in FP32, everything
        # else in FP64) when it works at or above that ridge intensity, HBM otherwise
        tk = ms[k] / 1e3
        if tk <= 0:
            return {}
        cls_prec = precision if k in ("dot", "sub") else ("fp32" if k == "comm" and precision != "fp64" else "fp64")
        ptf = PEAK[cls_prec + "_TF"] if cls_prec != "bf16x3" else PEAK["bf16_TF"]
        if fl[k] > 0 and (not by[k] or fl[k] / by[k] >= ptf * 1e12 / (PEAK["hbm_GBps"] * 1e9)):
            return {"tflops": round(fl[k] / tk / 1e12, 3), "frac": round(fl[k] / tk / 1e12 / ptf, 4)}
        return {"gbps": round(by[k] / tk / 1e9, 2), "frac": round(by[k] / tk / 1e9 / PEAK["hbm_GBps"], 5)}

    breakdown = {k: {"ms": round(ms[k], 3), "launches": n[k], "avg_us": round(1e3 * ms[k] / n[k], 3) if n[k] else 0,
                     **cls_roof(k)}
                 for k in names if n[k]}
    return {"kernel": dom, "bound": bound, "achieved": round(achieved, 4), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 5), "traffic": None,
            "algorithmic_flops_per_launch": fl[dom] / n[dom], "algorithmic_bytes_per_launch": by[dom] / n[dom],
            "avg_launch_us": 1e6 * t / n[dom], "breakdown": breakdown}


# kernel class -> source file of its kernels (the traffic record is void once that file changes)
KERNEL_SOURCE = {
    "accept": "kernels_accept.hip",
    "verify": "kernels_gemm.hip",
    "dot": {"fp64": "kernels_gemm.hip", "fp32": "kernels_gemm.hip", "bf16x3": "kernels_bf16.hip"},
    "sub": {"fp64": "kernels_gemm.hip", "fp32": "kernels_gemm.hip", "bf16x3": "kernels_bf16.hip"},
    "comm": {"fp64": "kernels_f64.hip", "fp32": "kernels_screen.hip", "bf16x3": "kernels_screen.hip"},
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.txt")


def source_sha256(kernel: str, precision: str):
    import hashlib

    src = KERNEL_SOURCE.get(kernel)
    if isinstance(src, dict):
        src = src.get(precision)
    if not src:
        return None
    path = os.path.join(ROOT, "paper_2506_01120_amd", "csrc", src)
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel: str, workload: str, precision: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter record, if
    it was taken on this workload and the kernel's source is unchanged since; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    sha = source_sha256(kernel, precision)
    for line in open(TRAFFIC_FILE):
        f = dict(kv.split("=", 1) for kv in line.split() if "=" in kv)
        if (f.get("kernel") == kernel and f.get("workload") == workload and f.get("precision") == precision
                and f.get("source_sha256") == sha):
            return float(f["fetch_bytes_per_launch"]) + float(f["write_bytes_per_launch"])
    return None


def calibrate_copy(mib: int, copies: int = 5):
    """A plain device-to-device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters (run under rocprofv3 --pmc)."""
    import torch

    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(copies):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device-to-device copy", "bytes_per_copy": n, "copies": copies}))


def cpu_baseline(gens, tol, early_exit: bool, target_s: float = 10.0):
    """The CPU reference as it stands, single-threaded, on this host: whole closures until ~target_s."""
    from oracle import oracle as ref

    ref.load()
    done, cands, t = 0, 0, 0.0
    while t < target_s and done < 3:
        o = ref.Oracle(gens, tol)
        t0 = time.perf_counter()
        o.run(early_exit=early_exit)
        t += time.perf_counter() - t0
        cands += o.result().candidates
        done += 1
    return {"value": cands / t, "unit": "checks/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} complete closure(s) of the same workload, {cands} bracket checks, {t:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="su16")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--decide", default="screen", choices=["fp64", "strict", "screen"])
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--early-exit", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the saturated block size and GEMM tiles by timing them at init (before timing)")
    ap.add_argument("--tune-cache", default=None, help="text cache of autotuner choices")
    ap.add_argument("--gemm-tile", type=int, default=0,
                    help="screening GEMM workgroup tile of saturated blocks (1: 64x64, 2: 128x128); "
                         "0: autotuned or heuristic")
    ap.add_argument("--method", default="orthonormalization",
                    choices=["orthonormalization", "rank_svd", "matrix_inversion"],
                    help="rank_svd: the standard algorithm with an SVD rank test (comparison baseline); "
                         "matrix_inversion: the paper's Algorithm 2")
    ap.add_argument("--representation", default="dense", choices=["dense", "pauli"],
                    help="pauli: the sparse Pauli-sum representation (d = 2^n, FP64)")
    ap.add_argument("--raw-basis", action="store_true",
                    help="Algorithm 3: also keep the raw basis B and bracket raw elements (single problems)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-candidate-at-a-time FP64 comparison run")
    ap.add_argument("--tol", type=float, default=0.0, help="override the workload's tolerance")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device copy of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    gens, tol, desc = workload(args.workload)
    if args.tol > 0:
        tol = args.tol
        if isinstance(gens, list):
            for p in gens:
                p.tol = tol
    cfg = dict(precision=args.precision, decide=args.decide, block=args.block, early_exit=args.early_exit,
               autotune=args.autotune, tune_cache=args.tune_cache, raw_basis=args.raw_basis, method=args.method,
               representation=args.representation, gemm_tile=args.gemm_tile)
    if args.raw_basis and args.workload == "batch64":
        raise SystemExit("--raw-basis is for single problems")

    print(f"[bench] warmup {args.warmup} x {args.workload} {cfg}", file=sys.stderr, flush=True)
    if args.warmup:
        run_steps(gens, tol, cfg, args.warmup)
    print(f"[bench] timed {args.steps} steps", file=sys.stderr, flush=True)
    elapsed, stats0, dims = run_steps(gens, tol, cfg, args.steps)
    checks = sum(s["candidates"] for s in stats0)
    value = checks / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    # per-kernel HIP events need eager launches: a second timed pass of the same steps
    print(f"[bench] profiled {args.steps} steps (HIP events per kernel)", file=sys.stderr, flush=True)
    elapsed_p, stats, _ = run_steps(gens, tol, dict(cfg, profile=True), args.steps)
    roof = roofline(stats, args.precision)
    roof["profiled_ms_per_step"] = round(1e3 * elapsed_p / args.steps, 3)
    roof["traffic"] = measured_traffic(roof["kernel"], args.workload, args.precision)

    plain = None
    if not args.no_plain:
        plain_cfg = dict(cfg, precision="fp64", block=1, autotune=False, representation="dense")
        if isinstance(gens, list):
            # the batched workload's denominator: every problem on its own, one candidate at a time
            print("[bench] plain one-at-a-time FP64 comparison: each problem alone", file=sys.stderr, flush=True)
            pt, pc = 0.0, 0
            for p in gens:
                t, ps, _ = run_steps(p.gens, p.tol, plain_cfg, 1)
                pt += t
                pc += ps[0]["candidates"]
            plain = {"checks_per_s": pc / pt, "ms_per_step": 1e3 * pt, "form": "each problem alone, block 1, FP64"}
        else:
            print("[bench] plain one-at-a-time FP64 comparison step", file=sys.stderr, flush=True)
            pt, pstats, _ = run_steps(gens, tol, plain_cfg, 1)
            plain = {"checks_per_s": pstats[0]["candidates"] / pt, "ms_per_step": 1e3 * pt,
                     "form": "block 1, FP64"}

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] CPU reference baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(gens, tol, args.early_exit)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "checks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else ("f32+f64" if args.precision == "fp32" else "bf16x3+f64"),
        "data": "synthetic (seeded generators)",
        "config": {"workload": desc,
                   "d": (int(gens.shape[-1]) if not isinstance(gens, list) else "8..128"),
                   "n_gen": (int(gens.shape[0]) if not isinstance(gens, list) else "2..13"), "tol": tol,
                   "dim": (dims[0] if not isinstance(gens, list) else sum(dims[0])),
                   "checks_per_step": checks // args.steps, "precision": args.precision,
                   "decide": args.decide if args.precision != "fp64" else "fp64",
                   "block": stats0[0]["block"], "block_growth": stats0[0]["block_growth"],
                   "tile_dot": stats0[0]["tile_dot"], "tile_sub": stats0[0]["tile_sub"],
                   "autotuned": stats0[0]["autotuned"], "early_exit": bool(args.early_exit),
                   "representation": args.representation,
                   "algorithm": ("Algorithm 1, SVD rank test (baseline)" if args.method == "rank_svd" else
                                 "Algorithm 2, matrix inversion" if args.method == "matrix_inversion" else
                                 "Algorithm 3 (raw basis kept)" if args.raw_basis else "Algorithm 4 (dimension only)"),
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "plain_fp64": plain,
        "speedup_vs_plain_fp64": round(value / plain["checks_per_s"], 2) if plain else None,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
