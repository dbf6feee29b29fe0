#!/usr/bin/env python3
"""Benchmark: bracket + independence checks per second and time-to-closure on one MI355X.

One step = one complete closure (the whole bracket loop, full certification
unless --early-exit) of the workload's generators; the generator phase of each
step's handle runs before the timed region, so the inputs (and the first basis
elements) are resident in HBM when timing starts.  The time of one closure
including its init (allocation, generator phase) is reported beside it.

Default workload: the largest single-GPU configuration -- two random traceless
anti-Hermitian 64 x 64 matrices (seed 5, Frobenius-normalised), tol 1e-8, full
certification: closure su(64), dim 4095, 8,382,465 bracket checks per step,
screened in split BF16 on the matrix cores with every decision that keeps a
candidate taken in FP64 (certified screen), autotuned block size and tiles.

Prints ONE JSON line.  `roofline` describes the dominant kernel, timed live
with HIP events on the library's stream; `cpu_baseline` times the CPU
reference on a bounded sample of the same workload; `plain_fp64` and
`blocked_fp64` time the one-candidate-at-a-time and blocked FP64 GPU forms of
the same closure (extrapolated from a measured prefix when a full run would
take minutes).
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


def run_steps(gens, tol, cfg, steps, budget=0):
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
        h.run(budget or None)
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
    for k, b in breakdown.items():
        # a class above its peak means its algorithmic accounting is wrong, not a fast kernel
        if b.get("frac", 0) > 1.0:
            b["suspect"] = True
            print(f"[bench] WARNING: kernel class {k} reads {b['frac']:.2f} of its peak; its work accounting "
                  f"overstates the launches' work", file=sys.stderr, flush=True)
    return {"kernel": dom, "bound": bound, "achieved": round(achieved, 4), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 5), "traffic": None,
            "algorithmic_flops_per_launch": fl[dom] / n[dom], "algorithmic_bytes_per_launch": by[dom] / n[dom],
            "avg_launch_us": 1e6 * t / n[dom], "breakdown": breakdown}


# kernel class -> source file of its kernels (the traffic record is void once that file changes)
KERNEL_SOURCE = {
    "accept": "kernels_accept.hip",
    "verify": "kernels_gemm.hip",
    "dot": {"fp64": "kernels_gemm.hip", "fp32": "kernels_gemm.hip", "bf16x3": "kernels_bf16p.hip"},
    "sub": {"fp64": "kernels_gemm.hip", "fp32": "kernels_gemm.hip", "bf16x3": "kernels_bf16p.hip"},
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


def _oracle_work(d: int, n: float) -> float:
    """Flops the CPU reference spends on one candidate against n accepted elements: the two
    naive complex products of the bracket (16 d^3) and n Householder reflectors applied to a
    vector of d^2 complex entries (about 16 d^2 n)."""
    return 16.0 * d ** 3 + 16.0 * d * d * n


def cpu_sample(gens, tol, early_exit: bool, target_s: float) -> dict:
    """The CPU reference as it stands, single-threaded: whole closures (at most three) while
    they fit in about target_s, else a prefix of one closure in chunks of candidates."""
    from oracle import oracle as ref

    ref.load()
    d = int(gens.shape[-1])
    checks, t, work, complete, n_reached = 0, 0.0, 0.0, 0, 0
    while t < target_s and complete < 3:
        o = ref.Oracle(gens, tol)
        c_prev = 0
        chunk = 64 if d >= 48 else 256  # a chunk of about a second or less
        while t < target_s:
            n0 = o.dim
            t0 = time.perf_counter()
            o.run(early_exit=early_exit, budget=chunk)
            t += time.perf_counter() - t0
            c = o.candidates
            work += (c - c_prev) * _oracle_work(d, 0.5 * (n0 + o.dim))
            checks += c - c_prev
            c_prev = c
            n_reached = o.dim
            if o.done:
                break
        if not o.done:
            break
        complete += 1
    partial = complete == 0 or t >= target_s and not o.done
    return {"checks": checks, "seconds": t, "work": work, "complete": complete, "partial": bool(partial),
            "n_reached": n_reached}


def cpu_baseline(gens, tol, early_exit: bool, full_checks: int, dim: int, target_s: float = 15.0,
                 workers: int = 1, workload_name: str = "") -> dict:
    """Oracle throughput on this host.  workers = 1: this process.  workers > 1: that many
    single-threaded copies run concurrently as child processes (all-core throughput of
    independent closures; one closure is sequential).  When no closure completes inside the
    sample, the rate in flops of the flop model above is extrapolated to the whole closure."""
    import subprocess

    d = int(gens.shape[-1])
    if workers == 1:
        samples = [cpu_sample(gens, tol, early_exit, target_s)]
    else:
        cmd = [sys.executable, os.path.abspath(__file__), "--cpu-worker", "--workload", workload_name,
               "--cpu-target-s", str(target_s)] + (["--early-exit"] if early_exit else [])
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1")
        procs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True, env=env) for _ in range(workers)]
        samples = []
        for pr in procs:
            out, _ = pr.communicate()
            if pr.returncode != 0:
                raise RuntimeError(f"CPU worker failed with status {pr.returncode}")
            samples.append(json.loads(out.strip().splitlines()[-1]))
    checks = sum(x["checks"] for x in samples)
    secs = max(x["seconds"] for x in samples)
    if not any(x["partial"] for x in samples):
        value = sum(x["checks"] / x["seconds"] for x in samples)
        what = (f"{sum(x['complete'] for x in samples)} complete closure(s) of the same workload over "
                f"{len(samples)} process(es), {checks} bracket checks, {secs:.1f} s")
        return {"value": value, "unit": "checks/s", "cores": workers, "kind": "oracle", "sample": what,
                "extrapolated": False}
    rate = sum(x["work"] / x["seconds"] for x in samples)
    full_work = full_checks * _oracle_work(d, dim)
    value = full_checks / (full_work / rate)
    n_reached = min(x["n_reached"] for x in samples)
    what = (f"prefix of the same closure in {len(samples)} process(es): {checks} bracket checks in {secs:.1f} s, "
            f"basis grown to {n_reached} elements, {rate / 1e9:.2f} GFLOP/s of the oracle's flop model "
            f"16d^3 + 16d^2 N per check; extrapolated to all {full_checks} checks at N = {dim} "
            f"(an upper bound of the CPU rate: at N = {dim} each check streams {16 * d * d * dim / 1e6:.0f} MB "
            f"of reflectors)")
    return {"value": value, "unit": "checks/s", "cores": workers, "kind": "oracle", "sample": what,
            "extrapolated": True, "s_per_closure": full_work / rate}


def host_description() -> dict:
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    return {"cpu_model": model, "nproc": cores, "cpu_count": os.cpu_count()}


def gpu_form(gens, tol, cfg, full_checks: int, window_s: float = 2.0, chunk: int = 1024) -> dict:
    """Time another GPU form of the same closure: run it to completion when it finishes within
    about window_s past saturation, else through the growth phase (|V| reaching the ambient
    bound) plus a window of about window_s in the saturated phase, and extrapolate the rest of
    the closure at that window's rate (labelled)."""
    import torch

    from paper_2506_01120_amd import LieClosure

    h = LieClosure(gens, tol, **cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = False
    while not done:
        done = h.run(budget=chunk)
        st = h.stats()
        if st["dim"] >= st["ambient"]:
            break
    t_growth = time.perf_counter() - t0
    c_growth = st["candidates"]
    t1 = time.perf_counter()
    while not done and time.perf_counter() - t1 < window_s:
        done = h.run(budget=chunk)
    t_end = time.perf_counter()
    st = h.stats()
    h.close()
    c_end = st["candidates"]
    if done:
        return {"checks_per_s": c_end / (t_end - t0), "s_per_closure": t_end - t0, "extrapolated": False}
    rate = (c_end - c_growth) / (t_end - t1)
    total = (t_end - t0) + (full_checks - c_end) / rate
    return {"checks_per_s": full_checks / total, "s_per_closure": total, "extrapolated": True,
            "measured": f"{c_end} of {full_checks} checks in {t_end - t0:.2f} s (growth phase to |V| = "
                        f"{st['dim']}: {c_growth} checks in {t_growth:.2f} s; saturated window: "
                        f"{c_end - c_growth} checks in {t_end - t1:.2f} s)"}


def time_with_init(gens, tol, cfg) -> dict:
    """One closure including its init: handle creation (allocations, generator upload and phase;
    the autotuner's choice is already cached in the process) and the bracket loop."""
    import torch

    from paper_2506_01120_amd import BatchClosure, LieClosure

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if isinstance(gens, list):
        h = BatchClosure([p.gens for p in gens], [p.tol for p in gens], **cfg)
    else:
        h = LieClosure(gens, tol, **cfg)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    h.run()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    h.close()
    return {"init_ms": round(1e3 * (t1 - t0), 3), "run_ms": round(1e3 * (t2 - t1), 3),
            "total_ms": round(1e3 * (t2 - t0), 3)}


# Per-workload defaults of the screen precision: the benchmark configurations run the
# FP64 form at d = 8 and 16, split BF16 at d = 32 and 64, and FP32 for the batch.
DEFAULT_PRECISION = {"ising3": "fp64", "su16": "fp64", "su32": "bf16x3", "su64": "bf16x3", "batch64": "fp32",
                     "ising7": "fp64", "sums5": "fp64"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="su64")
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32", "bf16x3"],
                    help="screen precision (default: per workload, split BF16 for su64)")
    ap.add_argument("--decide", default="screen", choices=["fp64", "strict", "screen"])
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--early-exit", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="block size and GEMM tiles from the shape heuristics instead of timing them at init")
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
    ap.add_argument("--profiled-steps", type=int, default=3,
                    help="closures of the per-kernel HIP-event pass (at most --steps)")
    ap.add_argument("--budget", type=int, default=0,
                    help="profiling runs only: each step runs at most this many candidates (0: whole closures)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="concurrent single-threaded oracle processes of the all-core CPU figure (0: skip)")
    ap.add_argument("--cpu-target-s", type=float, default=15.0)
    ap.add_argument("--cpu-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain and blocked FP64 comparison runs")
    ap.add_argument("--tol", type=float, default=0.0, help="override the workload's tolerance")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device copy of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.cpu_worker:
        # child process of the all-core CPU figure: the oracle only, no GPU
        gens, tol, _ = workload(args.workload)
        print(json.dumps(cpu_sample(gens, args.tol or tol, args.early_exit, args.cpu_target_s)))
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
    precision = args.precision or DEFAULT_PRECISION.get(args.workload, "fp64")
    autotune = not args.no_autotune and args.block == 0 and args.method == "orthonormalization"
    cfg = dict(precision=precision, decide=args.decide, block=args.block, early_exit=args.early_exit,
               autotune=autotune, tune_cache=args.tune_cache, raw_basis=args.raw_basis, method=args.method,
               representation=args.representation, gemm_tile=args.gemm_tile)
    if args.raw_basis and args.workload == "batch64":
        raise SystemExit("--raw-basis is for single problems")
    is_batch = isinstance(gens, list)

    print(f"[bench] warmup {args.warmup} x {args.workload} {cfg}", file=sys.stderr, flush=True)
    if args.warmup:
        run_steps(gens, tol, cfg, args.warmup, args.budget)
    print(f"[bench] timed {args.steps} steps", file=sys.stderr, flush=True)
    elapsed, stats0, dims = run_steps(gens, tol, cfg, args.steps, args.budget)
    checks = sum(s["candidates"] for s in stats0)
    value = checks / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    full_checks = checks // args.steps
    # per-kernel HIP events need eager launches: a second pass of (some of) the same steps
    psteps = max(1, min(args.steps, args.profiled_steps))
    print(f"[bench] profiled {psteps} steps (HIP events per kernel)", file=sys.stderr, flush=True)
    elapsed_p, stats, _ = run_steps(gens, tol, dict(cfg, profile=True), psteps, args.budget)
    roof = roofline(stats, precision)
    roof["profiled_ms_per_step"] = round(1e3 * elapsed_p / psteps, 3)
    roof["profiled_steps"] = psteps
    roof["traffic"] = measured_traffic(roof["kernel"], args.workload, precision)
    print(f"[bench] one closure including init", file=sys.stderr, flush=True)
    with_init = time_with_init(gens, tol, cfg) if not args.budget else None

    plain = blocked = None
    if not args.no_plain and not args.budget:
        plain_cfg = dict(cfg, precision="fp64", block=1, autotune=False, representation="dense", gemm_tile=0)
        if is_batch:
            # the batched workload's denominator: every problem on its own, one candidate at a time
            print("[bench] plain one-at-a-time FP64 comparison: each problem alone", file=sys.stderr, flush=True)
            pt, pc = 0.0, 0
            for p in gens:
                t, ps, _ = run_steps(p.gens, p.tol, plain_cfg, 1)
                pt += t
                pc += ps[0]["candidates"]
            plain = {"checks_per_s": pc / pt, "s_per_closure": pt, "form": "each problem alone, block 1, FP64",
                     "extrapolated": False}
            print("[bench] blocked FP64 comparison: the batch in FP64", file=sys.stderr, flush=True)
            bt, bs, _ = run_steps(gens, tol, dict(cfg, precision="fp64", gemm_tile=0), 1)
            blocked = {"checks_per_s": bs[0]["candidates"] / bt, "s_per_closure": bt,
                       "form": "grouped batch, FP64 decisions and projections", "extrapolated": False}
        else:
            print("[bench] plain one-at-a-time FP64 comparison", file=sys.stderr, flush=True)
            plain = dict(gpu_form(gens, tol, plain_cfg, full_checks), form="block 1, FP64")
            print("[bench] blocked FP64 comparison", file=sys.stderr, flush=True)
            blocked = dict(gpu_form(gens, tol, dict(cfg, precision="fp64", gemm_tile=0), full_checks,
                                    chunk=16384), form="adaptive blocks, FP64, autotuned" if autotune else
                           "adaptive blocks, FP64")

    cpu = cpu_all = None
    host = host_description()
    if not args.no_cpu_baseline and not is_batch and not args.budget:
        print("[bench] CPU reference baseline (one thread)", file=sys.stderr, flush=True)
        dim0 = dims[0]
        cpu = cpu_baseline(gens, tol, args.early_exit, full_checks, dim0, args.cpu_target_s)
        cpu["host"] = host
        workers = min(args.cpu_workers, host["nproc"])
        if workers > 1:
            print(f"[bench] CPU reference, {workers} concurrent processes", file=sys.stderr, flush=True)
            cpu_all = cpu_baseline(gens, tol, args.early_exit, full_checks, dim0, args.cpu_target_s, workers,
                                   args.workload)

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
        "dtype": "f64" if precision == "fp64" else ("f32+f64" if precision == "fp32" else "bf16x3+f64"),
        "data": "synthetic (seeded generators)",
        "config": {"workload": desc,
                   "d": (int(gens.shape[-1]) if not is_batch else "8..128"),
                   "n_gen": (int(gens.shape[0]) if not is_batch else "2..13"), "tol": tol,
                   "dim": (dims[0] if not is_batch else sum(dims[0])),
                   "checks_per_step": full_checks, "precision": precision,
                   "decide": args.decide if precision != "fp64" else "fp64",
                   "block": stats0[0]["block"], "block_growth": stats0[0]["block_growth"],
                   "tile_dot": stats0[0]["tile_dot"], "tile_sub": stats0[0]["tile_sub"],
                   "autotuned": stats0[0]["autotuned"], "early_exit": bool(args.early_exit),
                   "budget_per_step": args.budget or None,
                   "representation": args.representation,
                   "algorithm": ("Algorithm 1, SVD rank test (baseline)" if args.method == "rank_svd" else
                                 "Algorithm 2, matrix inversion" if args.method == "matrix_inversion" else
                                 "Algorithm 3 (raw basis kept)" if args.raw_basis else "Algorithm 4 (dimension only)"),
                   "parallelism": "single GPU"},
        "time_to_closure_ms": round(ms_per_step, 3),
        "time_to_closure_with_init": with_init,
        "roofline": roof,
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_all,
        "plain_fp64": plain,
        "blocked_fp64": blocked,
        "speedup_vs_plain_fp64": round(value / plain["checks_per_s"], 2) if plain else None,
        "speedup_vs_blocked_fp64": round(value / blocked["checks_per_s"], 2) if blocked else None,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
