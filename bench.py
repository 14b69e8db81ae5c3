#!/usr/bin/env python3
"""Throughput of restarted sGMRES (k-truncated Arnoldi, sparse sign sketch) on one MI355X.

One step = one complete solve from x0 = 0 to relative residual 1e-10 of the
full-size workload: 2D convection-diffusion on a 1024 x 1024 grid
(n = 1,048,576, nnz = 5,238,784, beta = (50, 20)), b ~ N(0, 1) (seed 0),
d = 200, k = 4, s = 400, zeta = 8, FP64 throughout.  Inputs are resident in HBM
before the timed region.

Prints ONE JSON line with the metric plus:
  roofline      basis kernel (the dominant kernel): algorithmic HBM bytes per
                launch / average launch time, measured with HIP events on the
                solve's stream inside the timed region
  cpu_baseline  the CPU oracle timed on a bounded sample of the same workload on
                this host, scaled to solves/s
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sGMRES solves/s at rel. residual 1e-10 (n=1M, d=200); HBM GB/s vs peak"
HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E

# Basis-kernel HBM traffic per launch on the cd1024 workload, from rocprofv3
# FETCH_SIZE / WRITE_SIZE scaled by the copy calibration (summaries and commands
# in profiles/<kernel>_cd1024_hbm_counters.md).  Valid only for the kernel
# source it was measured on; any change to it makes the figure stale (null).
MEASURED_TRAFFIC = {
    # (kernel, workload, precision) -> sources the figure is tied to, their
    # hash, and FETCH_SIZE x 2 + WRITE_SIZE per launch
    ("arnoldi", "cd1024", "fp64"): {"files": ("arnoldi_kernel.hpp", "common.hpp"), "source_hash": "bf31ac0e39bb5c1c",
                                    "bytes_per_launch": 1.5814e+10},
    ("chebyshev", "cd1024", "fp64"): {"files": ("chebyshev.hip", "common.hpp"), "source_hash": "eb5be861a9705acd",
                                      "bytes_per_launch": 1.2882e+10},
    ("stream", "cd2048", "fp32"): {"files": ("stream_kernel.hpp", "common.hpp"), "source_hash": "96705d678d66f60c",
                                   "bytes_per_launch": 2.2215e+10},
}


def kernel_source_hash(files) -> str:
    import hashlib

    m = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2111_00113_amd", "csrc", f), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, precision: str):
    """Counter-measured bytes per launch of this kernel at this workload, or
    None when none were taken or the kernel's source has changed since."""
    e = MEASURED_TRAFFIC.get((kernel, workload, precision))
    if e is None or kernel_source_hash(e["files"]) != e["source_hash"]:
        return None
    return e["bytes_per_launch"]


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# bytes of one value of A and of one stored basis entry per precision mode
VAL_BYTES = {"fp64": 8.0, "fp32": 4.0, "bf16": 4.0}
BASIS_BYTES = {"fp64": 8.0, "fp32": 4.0, "bf16": 2.0}


def basis_launch_bytes(n: int, nnz: int, k: int, dc: float, prec: str = "fp64") -> float:
    """Algorithmic HBM bytes of one basis-kernel launch (dc Arnoldi steps).

    Per step: the CSR arrays (4 B index + the value per nonzero, 4 B per row),
    the k window columns read and b_{j+1} written: in FP64
    12 nnz + 4n + 8n(k+1); values and basis entries shrink with the precision."""
    vb, eb = VAL_BYTES[prec], BASIS_BYTES[prec]
    return dc * ((4.0 + vb) * nnz + 4.0 * n + eb * n * (k + 1))


def compulsory_launch_bytes(n: int, nnz: int, dc: float, prec: str = "fp64") -> float:
    """Bytes this kernel must move per launch when it reads A's column indices:
    it keeps the window and the row pointers on chip, so per step only the
    column indices and values, the gathered b_j and the written b_{j+1}; plus r
    read and b_1 written once.  (Slots that are a diagonal across a slice have
    their columns formed instead, so on banded operators it reads less.)"""
    vb, eb = VAL_BYTES[prec], BASIS_BYTES[prec]
    return dc * ((4.0 + vb) * nnz + eb * n) + eb * n * (dc - 1) + (8.0 + eb) * n + 4.0 * (n + 1)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_cycles_per_solve(workload: str):
    """Cycles the oracle's own restarted solve of this workload takes (stored
    by tests/golden/make_cd1024_oracle_solve.py, which calls only the oracle)."""
    path = os.path.join(ROOT, "tests", "golden", f"{workload}_oracle_solve.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return int(json.load(fh)["cycles"])


def cpu_baseline(A, f, p, cycles_per_solve: float, cycles_source: str, sample_cols: int) -> dict:
    """The CPU oracle timed on this host on a bounded sample of the workload,
    scaled to solves/s with the oracle's own cycle count.

    All cores (the threads this process may run on, at most 16): one complete
    cycle at full size (residual, d basis columns with their sketches, the
    sketched least squares, the combine).  One core: the residual, the first
    sample_cols basis columns of that cycle (scaled by d / sample_cols), the
    least squares and the combine.  The oracle's sums have a fixed order, so
    the thread count changes only its run time."""
    import numpy as np

    import oracle

    n = A.n
    d, k, s, zeta = p["d"], p["k"], p["s"], p["zeta"]
    try:
        cores = max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        cores = 1
    model = cpu_model()
    out = {"kind": "oracle", "unit": "solves/s", "cpu_model": model}
    # all cores: one full cycle (a one-cycle solve) at full size
    oracle.set_threads(cores)
    try:
        t0 = time.perf_counter()
        r0, _ = oracle.residual(A, f, np.zeros(n))
        t_res_all = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.sgmres_solve(A, f, d=d, k=k, s=s, zeta=zeta, seed=p["seed"], tol=0.0, restarts=0)
        t_one_all = time.perf_counter() - t0
    finally:
        oracle.set_threads(1)
    # a one-cycle solve evaluates |b|, two residuals and one cycle; a solve of
    # C cycles evaluates C + 1 residuals and C cycles
    per_solve_all = cycles_per_solve * (t_one_all - t_res_all) + t_res_all
    # one core: a bounded part of the same cycle
    t0 = time.perf_counter()
    r, _ = oracle.residual(A, f, np.zeros(n))
    t_res = time.perf_counter() - t0
    t0 = time.perf_counter()
    cyc = oracle.arnoldi_cycle(A, r, sample_cols, k, s, zeta, p["seed"], 0)
    t_basis = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    C = cyc["SAB"][:, :sample_cols]
    C = np.column_stack([C] + [rng.standard_normal((s, 1)) for _ in range(d - sample_cols)])
    t0 = time.perf_counter()
    oracle.sketched_lsq(C, cyc["g"])
    t_lsq = time.perf_counter() - t0
    Bd = rng.standard_normal((d, n))  # row q = basis column q (column-major n x d)
    y = rng.standard_normal(d)
    x = np.zeros(n)
    L = oracle.lib()
    t0 = time.perf_counter()
    L.oracle_basis_combine(n, d, Bd, y, x)
    t_comb = time.perf_counter() - t0
    per_solve_1 = cycles_per_solve * (t_res + t_basis * (d / sample_cols) + t_lsq + t_comb) + t_res
    out.update({
        "value": 1.0 / per_solve_all,
        "cores": cores,
        "s_per_solve": per_solve_all,
        "single_core": {"value": 1.0 / per_solve_1, "cores": 1, "s_per_solve": per_solve_1},
        "cycles_per_solve": cycles_per_solve,
        "sample": (f"{cores} threads: one full cycle at full size timed as a one-cycle oracle solve "
                   f"({t_one_all:.1f} s); 1 thread: one residual, {sample_cols} of {d} basis columns of cycle 0 "
                   f"(scaled by {d}/{sample_cols}), one {s}x{d} sketched least-squares solve and one {n}x{d} "
                   f"combine ({t_res + t_basis + t_lsq + t_comb:.1f} s); both scaled by {cycles_per_solve:g} "
                   f"cycles per solve ({cycles_source}); host CPU {model}"),
    })
    return out


def grad_bench(args, A, f, p, sg, torch, np) -> int:
    """Differentiable solve: L = |x(A, b) - x_t|^2, forward sGMRES on A, backward
    sGMRES on A^T plus the gradient on A's pattern; one step = forward + backward."""
    dev = "cuda:0"
    rp = torch.as_tensor(A.row_ptr, device=dev)
    ci = torch.as_tensor(A.col_idx, device=dev)
    val = torch.as_tensor(A.val, device=dev)
    bt = torch.as_tensor(f, device=dev)
    xt = torch.as_tensor(np.random.default_rng(1).standard_normal(A.n), device=dev)

    def step():
        v = val.clone().requires_grad_(True)
        b = bt.clone().requires_grad_(True)
        x = sg.sgmres_solve_diff(rp, ci, v, b, d=p["d"], k=p["k"], s=p["s"], seed=p["seed"], tol=p["tol"],
                                 restarts=p["restarts"])
        L = ((x - xt) ** 2).sum()
        L.backward()
        return float(L.detach())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        L = step()
        log(f"grad step {i}: L={L:.6e}")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    print(json.dumps({
        "metric": "differentiable sGMRES steps/s (forward solve + adjoint solve + dL/dA, dL/db)",
        "value": args.steps / el, "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: loss |x - x_t|^2, x_t ~ N(0,1) seed 1; forward and adjoint "
                               f"d={p['d']}, k={p['k']}, s={p['s']}, tol={p['tol']:g}"},
    }), flush=True)
    return 0


def batch_bench(args, sg, synth, torch, np) -> int:
    """Many independent systems in one launch per cycle (one workgroup per
    system), FP32 cycles with FP64 refinement, against FP64 sGMRES solving the
    same systems one at a time on the same GPU."""
    dev = "cuda:0"
    torch.cuda.set_device(0)
    d, k, s, tol, restarts = 100, 2, 200, 1e-10, 50
    log(f"generating {args.batch_count} systems")
    W = synth.batch_workload(args.batch_count if args.mode == "batch" else 0)
    systems = [(sg.DeviceCSR.from_host(A, dev), torch.as_tensor(b, device=dev),
                torch.zeros(A.n, dtype=torch.float64, device=dev)) for A, b in W]
    rows = sum(A.n for A, _ in W)
    nnz = sum(A.nnz for A, _ in W)
    log(f"generating the block of {args.block_rhs} right-hand sides")
    A1, B1 = synth.block_rhs_workload(1 << 20, args.block_rhs)
    dA1 = sg.DeviceCSR.from_host(A1, dev)
    block = [(dA1, torch.as_tensor(b, device=dev), torch.zeros(A1.n, dtype=torch.float64, device=dev)) for b in B1]
    del W, B1

    bpath = {"part-split": sg.PATH_PART_SPLIT, "multi": sg.PATH_MULTI}.get(args.path, 0)

    def batched(sysl, prec):
        for _, _, x in sysl:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, res = sg.sgmres_solve_batched(sysl, d, k, s, 0, tol, restarts, precision=prec, path=bpath,
                                          rows_per_thread=args.rows_per_thread)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if rc != sg.OK or max(r["relres"] for r in res) > tol:
            raise RuntimeError(f"batched solve ({prec}) did not converge")
        return el, res

    def one_at_a_time(sysl):
        for _, _, x in sysl:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cyc = 0
        for A, b, x in sysl:
            rc, info = sg.sgmres_solve(A, b, x, d, k, s, 0, tol, restarts)
            if rc != sg.OK:
                raise RuntimeError("single solve did not converge")
            cyc += info["cycles"]
        torch.cuda.synchronize()
        return time.perf_counter() - t0, cyc

    groups = (("many", systems), ("block", block)) if args.mode == "batch" else (("block", block),)
    for prec in ("fp32", "fp64"):  # warm-up (also times the workgroup shapes once)
        for _, sysl in groups:
            batched(sysl, prec)
    one_at_a_time(groups[0][1][:4])
    out = {}
    for name, sysl in groups:
        t32 = t64 = None
        for _ in range(args.steps):
            e32, r32 = batched(sysl, "fp32")
            e64, r64 = batched(sysl, "fp64")
            t32 = e32 if t32 is None else min(t32, e32)
            t64 = e64 if t64 is None else min(t64, e64)
        tseq, cseq = one_at_a_time(sysl)
        out[name] = dict(
            systems=len(sysl), fp32_batched_s=t32, fp64_batched_s=t64, fp64_one_at_a_time_s=tseq,
            fp32_batched_systems_per_s=len(sysl) / t32, fp64_batched_systems_per_s=len(sysl) / t64,
            fp64_one_at_a_time_systems_per_s=len(sysl) / tseq,
            speedup_fp32_batched_vs_fp64_one_at_a_time=tseq / t32,
            cycles_fp32=sum(r["cycles"] for r in r32), cycles_fp64=sum(r["cycles"] for r in r64),
            cycles_one_at_a_time=cseq, max_relres_fp32=max(r["relres"] for r in r32))
        log(f"{name}: {out[name]}")
    if args.mode == "block":
        b = out["block"]
        print(json.dumps({
            "metric": (f"block of {len(block)} right-hand sides sharing A, systems/s at rel. residual 1e-10 "
                       f"(n = 2^20 random sparse, d={d}, k={k}, s={s})"),
            "value": b["fp64_batched_systems_per_s"], "unit": "systems/s", "n_gpus": 1, "steps": args.steps,
            "warmup": 1, "ms_per_step": b["fp64_batched_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": (f"random_dominant(2^20, 6 off-diagonals, seed 2) with {len(block)} right-hand "
                                    f"sides default_rng(2); d={d}, k={k}, s={s}, zeta=8, tol=1e-10")},
            "rhs_block": b}), flush=True)
        return 0
    m = out["many"]
    # the line reports the FP64 batched solve (faster than FP32 cycles here: those
    # need a refinement cycle); whole-solve algorithmic bytes of its basis steps
    # (per step and system: (4 + 8) nnz + 4n + 8n(k + 1)) over its solve time
    algo = (12.0 * nnz + 4.0 * rows + 8.0 * rows * (k + 1)) * d * (m["cycles_fp64"] / len(systems))
    achieved = algo / m["fp64_batched_s"] / 1e9
    print(json.dumps({
        "metric": (f"batched sGMRES systems/s at rel. residual 1e-10 ({len(systems)} random sparse systems, "
                   f"n in [16384, 262144], d={d}, k={k}, s={s})"),
        "value": m["fp64_batched_systems_per_s"], "unit": "systems/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": m["fp64_batched_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"{len(systems)} systems random_dominant(n_i, 6 off-diagonals, seed [4, i]), "
                                f"n_i = default_rng(4).integers(16384, 262144), total rows {rows}, nnz {nnz}; "
                                f"block: n = 2^20 with {args.block_rhs} right-hand sides; d={d}, k={k}, s={s}, "
                                f"zeta=8, tol=1e-10"), "rows": rows, "nnz": nnz},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": None,
                     "kernel": ("batched_cycle_kernel" if bpath == sg.PATH_PART_SPLIT else "arnoldi_multi_kernel")
                     + " (whole solve: algorithmic basis bytes / solve time)"},
        "many_systems": m, "rhs_block": out["block"],
    }), flush=True)
    return 0


def cheb_launch_bytes(n: int, nnz: int, dc: float, prec: str = "fp64") -> float:
    """Algorithmic HBM bytes of one Chebyshev basis-kernel launch (dc steps).

    Per step: the CSR arrays (4 B index + the value per nonzero, 4 B per row),
    b_j gathered and b_{j+1} written (the two previous vectors stay in
    registers): in FP64 12 nnz + 4n + 16n."""
    vb, eb = VAL_BYTES[prec], BASIS_BYTES[prec]
    return dc * ((4.0 + vb) * nnz + 4.0 * n + 2.0 * eb * n)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed solves")
    ap.add_argument("--warmup", type=int, default=1, help="untimed solves")
    ap.add_argument("--workload", default="cd1024")
    ap.add_argument("--cpu-sample-cols", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--rows-per-thread", type=int, default=0)
    ap.add_argument("--spmv-mode", type=int, default=0, help="0 row per thread, 1 CSR-stream")
    ap.add_argument("--basis", default="arnoldi", choices=["arnoldi", "chebyshev"],
                    help="arnoldi: k-truncated Arnoldi (the method's default); chebyshev: Section 4.4 recurrence")
    ap.add_argument("--cheb-box", default="4,4,0", help="c,dx,dy of the spectral box for --basis chebyshev")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"],
                    help="basis cycles in FP64, FP32, or FP32 with a bfloat16 basis (FP64 refinement)")
    ap.add_argument("--mode", default="solve", choices=["solve", "grad", "batch", "block"],
                    help="solve: the sGMRES metric; grad: differentiable solve (forward + adjoint); "
                         "batch: many systems per launch against one-at-a-time FP64 solves; "
                         "block: only the block of right-hand sides of the batch workload")
    ap.add_argument("--batch-count", type=int, default=256, help="systems in the many-systems workload")
    ap.add_argument("--block-rhs", type=int, default=32, help="right-hand sides of the n = 2^20 block")
    ap.add_argument("--halo-off", action="store_true", help="truncated Arnoldi: three grid barriers per step")
    ap.add_argument("--path", default="auto", choices=["auto", "stream", "part-split", "multi"],
                    help="basis kernel for systems beyond the resident capacity (auto: streaming)")
    ap.add_argument("--stream-state", type=int, default=0, choices=[0, 1, 2],
                    help="streaming path: 0 auto, 1 m and w in registers, 2 in an HBM buffer")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 3 plain device-to-device copies of MIB MiB (counter calibration)")
    args = ap.parse_args()

    if args.calibrate_copy:
        import torch

        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "copies": 3}), flush=True)
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(row-block sharding across GPUs is a design, not code).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2111_00113_amd as sg
    import synth

    if args.mode in ("batch", "block"):
        return batch_bench(args, sg, synth, torch, np)

    log(f"building workload {args.workload}")
    A, f, p = synth.workload(args.workload)
    dev = "cuda:0"
    torch.cuda.set_device(0)
    dA = sg.DeviceCSR.from_host(A, dev)
    fb = torch.as_tensor(f, dtype=torch.float64, device=dev)
    x = torch.zeros(A.n, dtype=torch.float64, device=dev)
    d, k, s = p["d"], p["k"], p["s"]
    cheb = args.basis == "chebyshev"
    box = tuple(float(t) for t in args.cheb_box.split(",")) if cheb else None

    path = {"auto": 0, "stream": sg.PATH_STREAM, "part-split": sg.PATH_PART_SPLIT, "multi": 0}[args.path]

    def solve(profile: bool) -> dict:
        x.zero_()
        rc, info = sg.sgmres_solve(dA, fb, x, d, k, s, p["seed"], p["tol"], p["restarts"], zeta=p["zeta"],
                                   profile=profile, block_size=args.block_size,
                                   rows_per_thread=args.rows_per_thread, spmv_mode=args.spmv_mode, cheb_box=box,
                                   precision=args.precision, path=path, stream_state=args.stream_state,
                                   halo_off=args.halo_off)
        if rc != sg.OK:
            raise RuntimeError(f"solve did not converge: {info}")
        return info

    if args.mode == "grad":
        return grad_bench(args, A, f, p, sg, torch, np)

    for w in range(args.warmup):
        info = solve(False)
        log(f"warmup {w}: cycles={info['cycles']} relres={info['relres']:.3e}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    per_solve = []
    for i in range(args.steps):
        ti = time.perf_counter()
        infos.append(solve(True))
        torch.cuda.synchronize()
        per_solve.append(time.perf_counter() - ti)
        log(f"step {i}: cycles={infos[-1]['cycles']} relres={infos[-1]['relres']:.3e} "
            f"{per_solve[-1] * 1e3:.2f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    cycles = sum(i["cycles"] for i in infos)
    steps = sum(i["steps"] for i in infos)
    t_basis = sum(i["t_basis_ms"] for i in infos)
    t_lsq = sum(i["t_lsq_ms"] for i in infos)
    t_comb = sum(i["t_combine_ms"] for i in infos)
    t_res = sum(i["t_residual_ms"] for i in infos)
    t_sketch = sum(i["t_sketch_ms"] for i in infos)
    dc_avg = steps / cycles
    run_path = infos[-1]["path"]
    streaming = run_path == sg.PATH_STREAM
    # streaming path: the basis kernel alone (the sketch of the finished basis,
    # S A B = (S B) H and g = S r follow it as separate launches)
    launch_ms = (t_basis - t_sketch) / cycles
    pr = args.precision
    launch_bytes = (cheb_launch_bytes(A.n, A.nnz, dc_avg, pr) if cheb
                    else basis_launch_bytes(A.n, A.nnz, k, dc_avg, pr))
    resident = launch_ms > 0.0  # a basis kernel was timed (not the part-split path of large systems)
    if not resident:
        launch_ms = elapsed * 1e3 / cycles  # whole cycle: basis, least squares and combine
    achieved = launch_bytes / (launch_ms * 1e-3) / 1e9
    # x after the last timed solve: confirm the residual with an independent host SpMV
    xr = x.cpu().numpy()
    relres_host = float(np.linalg.norm(f - A.to_scipy() @ xr) / np.linalg.norm(f))

    out = {
        "metric": METRIC if not cheb else METRIC.replace("sGMRES", "sGMRES (Chebyshev basis)"),
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "median_ms_per_solve": float(np.median(per_solve)) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32 basis cycles, f64 refinement",
                  "bf16": "f32 arithmetic, bf16 basis, f64 refinement"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: "
                         + ("random sparse nonsymmetric, 7 nonzeros per row, diagonal dominance 1.2"
                            if args.workload.startswith("rd") else "2D convection-diffusion 5-point")
                         + f", n={A.n}, nnz={A.nnz}, "
                         f"d={d}, k={k}, s={s}, zeta={p['zeta']}, tol={p['tol']:g}, b~N(0,1) seed 0, x0=0"
                         + (f", Chebyshev basis box c,dx,dy={args.cheb_box}" if cheb else "")
                         + (f", {args.precision} basis cycles" if args.precision != "fp64" else "")),
            "basis": args.basis,
            "precision": args.precision,
            "n": A.n,
            "nnz": A.nnz,
            "d": d,
            "k": k,
            "s": s,
            "zeta": p["zeta"],
            "tol": p["tol"],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": (measured_traffic("stream" if streaming else args.basis, args.workload, args.precision)
                        if resident else None),
            "traffic_unit": "bytes per launch",
            "kernel": ("stream_kernel (streaming truncated Arnoldi)" if streaming else
                       ("chebyshev_kernel" if cheb else "arnoldi_kernel (spmv_truncarnoldi)")) if resident
                      else "batched_cycle_kernel as a batch of one (n above the resident capacity); "
                           "time per whole cycle",
            "bytes_per_launch": launch_bytes,
            "compulsory_bytes_per_launch": compulsory_launch_bytes(A.n, A.nnz, dc_avg, pr),
            "avg_launch_ms": launch_ms,
        },
        "cycles_per_solve": cycles / args.steps,
        "relres_final": infos[-1]["relres"],
        "relres_host_check": relres_host,
        "basis_phase_us_per_step": [round(sum(i["phase_us"][q] for i in infos) / max(steps, 1), 3)
                                    for q in range(8)],
        "gpu_ms_per_solve": {
            "basis": t_basis / args.steps,
            "sketch_of_basis": t_sketch / args.steps,
            "lsq": t_lsq / args.steps,
            "combine": t_comb / args.steps,
            "residual": t_res / args.steps,
        },
    }
    rf = out["roofline"]
    if streaming:
        # the same algorithmic bytes over the basis kernel plus the sketch of the
        # finished basis (the fused kernels' counterpart)
        both_ms = t_basis / cycles
        rf["sketch_ms_per_cycle"] = t_sketch / cycles
        rf["frac_basis_and_sketch"] = launch_bytes / (both_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS
    out["path"] = {1: "arnoldi 3-barrier", 2: "arnoldi halo", 3: "chebyshev", 4: "part-split",
                   5: "stream"}.get(run_path, str(run_path))
    out["launch"] = {"block": infos[-1]["launch_block"], "rows_per_thread": infos[-1]["launch_rows"],
                     "grid": infos[-1]["launch_grid"]}
    # the same launch time against two other byte counts, labelled: the bytes the
    # counters measured (when current for this kernel source) and the bytes this
    # kernel must move (window kept on chip, no row pointers)
    rf["frac_basis"] = "algorithmic bytes per launch (12 nnz + 4n + 8n(k+1) per step) / avg launch time"
    if rf["traffic"]:
        rf["frac_measured_traffic"] = rf["traffic"] / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS
    rf["frac_compulsory"] = rf["compulsory_bytes_per_launch"] / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS
    rf["target_frac"] = 0.60
    rf["gap_to_target"] = 0.60 - rf["frac"]
    if not args.no_cpu_baseline and not cheb and args.precision == "fp64":
        log("timing the CPU oracle on a bounded sample")
        oc = oracle_cycles_per_solve(args.workload)
        src = ("the oracle's own solve of this workload, tests/golden" if oc is not None
               else "no stored oracle solve for this workload: the GPU run's count")
        out["cpu_baseline"] = cpu_baseline(A, f, p, float(oc) if oc is not None else cycles / args.steps, src,
                                           args.cpu_sample_cols)
    print(json.dumps(out), flush=True)
    del dA, fb, x
    torch.cuda.synchronize()
    sg.sgmres_release_workspace()
    return 0


if __name__ == "__main__":
    _rc = main()
    if _rc:
        sys.exit(_rc)
