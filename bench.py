"""Benchmark of the demagnetizing-field hot path on one MI355X.

Workload (default): the thin-film LLG problem, 512 x 512 x 16 cells of 4 nm,
Ms = 8e5 A/m, A = 1.3e-11 J/m, alpha = 0.02, RK4 with dt = 1e-13 s, seeded
random unit m.  One step = one RK4 step = four H_d evaluations (x R2C, y FFT,
z FFT + N^.M^ + z IFFT, y IFFT, x C2R) and four fused exchange + LLG stage
updates, all in the library's HIP kernels, inputs resident in HBM.

value = H_d evaluations x cells / wall time of the timed steps (Gcells/s),
i.e. demag throughput inside the full RK4 step (the LLG kernels' time counts
against it).  The roofline object describes the dominant kernel, timed live
with HIP events around each of its launches in the timed region; its bytes are
the algorithmic bytes of that kernel (inputs read once, outputs written once,
zero padding never stored).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def geometry(n):
    nx, ny, nz = n
    N = [1 if v == 1 else 2 * v for v in n]
    D = [1 if v == 1 else v // 2 + 1 for v in N]
    return N, D


def stage_bytes(n):
    """Algorithmic HBM bytes of one launch of each stage kernel."""
    nx, ny, nz = n
    (Nx, Ny, Nz), (X1, Y1, Z1) = geometry(n)
    cells = nx * ny * nz
    f = 12 * cells                   # one FP32 3-vector field
    s1 = 3 * nz * X1 * ny * 8        # complex64 after x
    s2 = 3 * nz * X1 * Ny * 8        # complex64 after y (z padding never stored)
    k = 6 * Z1 * X1 * Y1 * 4         # packed real kernel
    return {
        "x_fwd": f + s1,
        "y_fwd": s1 + s2 if ny > 1 else 0,
        "z_conv": 2 * (s2 if ny > 1 else s1) + k,
        "y_inv": s2 + s1 if ny > 1 else 0,
        "x_inv": s1 + f,
        # RK4 stage update, averaged over the four stages: 48, 72, 72, 60 B/cell
        "llg": 63 * cells,
    }


def cpu_baseline(n, cell, budget_s=20.0):
    """The FP64 oracle's FFT convolution on this host (set-up excluded)."""
    import workloads as W
    from oracle import demag as odemag
    workers = os.cpu_count() or 1
    op = odemag.DemagFFT(n, cell, workers=workers)
    M = W.magnetisation(n, 0).astype(np.float64)
    op(M)  # warm-up
    times = []
    t_start = time.perf_counter()
    while len(times) < 3 and time.perf_counter() - t_start < budget_s:
        t0 = time.perf_counter()
        op(M)
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    cells = n[0] * n[1] * n[2]
    return {"value": cells / t / 1e9, "unit": "Gcells/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(times)} FP64 H_d evaluations of the {n[0]}x{n[1]}x{n[2]} mesh "
                      f"(scipy rfftn/irfftn, workers={workers}; tensor set-up excluded), "
                      f"median {t:.3f} s each"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2308_08447_amd as pkg
    import workloads as W
    from oracle import llg as ollg  # noqa: F401  (gamma constant only via W below)

    cfg = W.THIN_FILM
    n, cell = cfg["n"], cfg["cell"]
    cells = n[0] * n[1] * n[2]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    plan = pkg.demag_setup(n + cell, stream=stream)
    pkg.demag_autotune(plan, stream)
    variants = [pkg.demag_get_variant(plan, st) for st in range(5)]
    m0 = torch.from_numpy(W.unit_vectors((n[2], n[1], n[0]), seed=0)).to(dev)
    m = m0.clone()
    params = (cfg["Ms"], cfg["A"], cfg["alpha"], 2.21276e5, (0.0, 0.0, 0.0))

    for _ in range(args.warmup):
        pkg.llg_step(plan, m, params, cfg["dt"], 1, stream)
    torch.cuda.synchronize()
    nch = pkg.demag_get_chunks(plan)
    pkg.demag_timing_enable(plan, 4 * args.steps * nch)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pkg.llg_step(plan, m, params, cfg["dt"], 1, stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = pkg.demag_timing_read(plan)
    pkg.demag_timing_enable(plan, 0)

    # standalone demag_field throughput (not the headline; same stream, no events)
    M = (m0 * cfg["Ms"]).contiguous()
    H = torch.empty_like(M)
    for _ in range(3):
        pkg.demag_field(plan, M, H, stream)
    torch.cuda.synchronize()
    reps = 4 * args.steps
    t1 = time.perf_counter()
    for _ in range(reps):
        pkg.demag_field(plan, M, H, stream)
    torch.cuda.synchronize()
    t_field = (time.perf_counter() - t1) / reps
    pkg.demag_destroy(plan)

    ms_per_step = 1e3 * elapsed / args.steps
    value = 4 * cells * args.steps / elapsed / 1e9
    nbytes = stage_bytes(n)   # per H_d evaluation (per RK stage for "llg")
    evals = 4 * args.steps
    per_stage = {}
    for name, (tot_ms, cnt) in stages.items():
        if cnt:
            # the y/z stages run once per chunk: bytes per launch = bytes per evaluation / chunks
            per_launch = nbytes[name] * evals / cnt
            avg = tot_ms / cnt
            per_stage[name] = {"avg_us": round(1e3 * avg, 2), "launches": cnt,
                               "bytes_per_launch": int(per_launch),
                               "GB_per_s": round(per_launch / (avg * 1e-3) / 1e9, 1),
                               "us_per_eval": round(1e3 * tot_ms / evals, 2)}
    dom = max(per_stage, key=lambda k: per_stage[k]["avg_us"] * per_stage[k]["launches"])
    achieved = per_stage[dom]["GB_per_s"]
    b5 = sum(v for k, v in nbytes.items() if k != "llg")

    out = {
        "metric": "demag H_d evals: Gcells/s + % HBM roofline; serve p50/p99 latency",
        "value": round(value, 3),
        "unit": "Gcells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "mesh": list(n), "cell_m": list(cell),
                   "hd_evals_per_step": 4, "global_batch": 1, "parallelism": "none",
                   "stage_variants": variants, "yz_chunks": nch},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "stages": per_stage,
        "demag_field_gcells_per_s": round(cells / t_field / 1e9, 3),
        "demag_field_us": round(1e6 * t_field, 1),
        "demag_field_effective_frac": round(b5 / t_field / 1e9 / HBM_PEAK_GBS, 4),
        "llg_cell_steps_per_s": round(cells * args.steps / elapsed, 1),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, cell)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
