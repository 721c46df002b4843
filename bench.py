"""Benchmark of the demagnetizing-field hot path on one MI355X.

Workload (default): demag_field on the large film, 1024 x 1024 x 32 cells of
4 nm (the largest single-GPU configuration), Ms = 8e5 A/m, seeded random unit
M x Ms resident in HBM.  One step = one H_d evaluation of Eq. (1) as the
zero-padded FFT convolution (x R2C, the y and z transforms, the symmetric
tensor product and the inverse transforms), all in the library's HIP kernels.

value = cells / wall time per evaluation (Gcells/s) in FP32.  The roofline
object describes the dominant kernel, timed live with HIP events around each of
its launches on the launch stream; its bytes are the algorithmic bytes of that
kernel (inputs read once, outputs written once, zero padding never stored), and
its traffic is the HBM bytes per launch from stored rocprofv3 counter runs of
the same kernels.  Extra keys: the BF16x3 MFMA form on the same film; the
thin-film RK4 LLG block (512 x 512 x 16 cells, four H_d and four fused exchange
+ LLG stages per step, with the extrapolated-H_d and periodic variants); the
small configuration's latency (32 x 32 x 4, eager and graph-replayed); a short
serving sample; and the FP64 oracle timed on the host cores (cpu_baseline).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
       [--workload large_film|large_film_only|thin_film|atomistic|switching|field]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
ROOT = os.path.dirname(os.path.abspath(__file__))
# sources whose change invalidates a stored hardware-counter measurement
# kernel sources behind each form's stored counters (a change to one of them
# invalidates that form's traffic lines)
_SHARED_SOURCES = ("stage_common.h", "fft_lds.h", "mfma_dft.h", "engine.h")
KERNEL_SOURCES = {
    5: ["paper_2308_08447_amd/csrc/" + f
        for f in ("stages_x.hip", "stages_y.hip", "stages_z.hip") + _SHARED_SOURCES],
    3: ["paper_2308_08447_amd/csrc/" + f for f in ("stages_xz.hip", "dynamics.hip") + _SHARED_SOURCES],
}
COUNTERS = "profiles/counters_thin_film_512x512x16.md"
COUNTERS_LARGE = "profiles/counters_large_film_1024x1024x32.md"


def kernel_sources_sha256(form):
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[form]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_traffic(stage, counters=COUNTERS, form=3, launches_per_eval=1):
    """HBM bytes per launch of `stage` from the stored rocprofv3 counter runs
    (FETCH_SIZE x its copy-kernel calibration + WRITE_SIZE): the stage's bytes
    per evaluation divided by its launches per evaluation in this run (the y
    and z stages of a chunked plan split one evaluation's bytes over their
    chunks), or None when no measurement is stored or the form's kernel sources
    changed since it was taken."""
    path = os.path.join(ROOT, counters)
    if not os.path.exists(path):
        return None
    vals, sha = {}, None
    with open(path) as f:
        for line in f:
            p = line.split()
            if len(p) == 3 and p[0] == "traffic_bytes_per_eval":
                vals[p[1]] = float(p[2])
            elif len(p) == 2 and p[0] == "kernel_sources_sha256":
                sha = p[1]
    if sha != kernel_sources_sha256(form) or stage not in vals:
        return None
    return vals[stage] / launches_per_eval


def geometry(n, pbc=(False, False, False)):
    """Transform lengths (2n open, n periodic, 1 for n = 1) and folded sizes."""
    N = [v if (v == 1 or p) else 2 * v for v, p in zip(n, pbc)]
    D = [1 if v == 1 else v // 2 + 1 for v in N]
    return N, D


def stage_bytes(n, form=5, pbc=(False, False, False)):
    """Algorithmic HBM bytes of one evaluation of each stage (inputs read once,
    outputs written once, zero padding never stored), for the five-pass form
    (form 5) or the three-kernel thin-mesh form (form 3: x+z, y conv, z+x);
    pbc: periodic axes (unpadded transforms, five-pass form)."""
    nx, ny, nz = n
    (Nx, Ny, Nz), (X1, Y1, Z1) = geometry(n, pbc)
    cells = nx * ny * nz
    f = 12 * cells                   # one FP32 3-vector field
    k = 6 * Z1 * X1 * Y1 * 4         # packed real kernel
    # RK4 stage update, averaged over the four stages: 48, 72, 72, 60 B/cell
    llg = 63 * cells
    if form == 3:
        t = 3 * Nz * X1 * ny * 8     # all Nz transformed planes, ny rows, X1 columns
        return {"x_fwd": f + t, "z_conv": 2 * t + k, "x_inv": t + f, "llg": llg}
    s1 = 3 * nz * X1 * ny * 8        # complex64 after x
    s2 = 3 * nz * X1 * Ny * 8        # complex64 after y (z padding never stored)
    return {
        "x_fwd": f + s1,
        "y_fwd": s1 + s2 if ny > 1 else 0,
        "z_conv": 2 * (s2 if ny > 1 else s1) + k,
        "y_inv": s2 + s1 if ny > 1 else 0,
        "x_inv": s1 + f,
        "llg": llg,
    }


def cpu_baseline(n, cell, budget_s=20.0, one_thread=True):
    """The FP64 oracle's FFT convolution on this host (set-up excluded)."""
    import workloads as W
    from oracle import demag as odemag
    workers = os.cpu_count() or 1
    t_setup = time.perf_counter()
    op = odemag.DemagFFT(n, cell, workers=workers)
    t_setup = time.perf_counter() - t_setup
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
    # the same steps in FP32 (SciPy single-precision transforms), for a
    # like-for-like figure beside the FP32 GPU path
    op32 = op.to_float32()
    del op
    M32 = M.astype(np.float32)
    op32(M32)
    t0 = time.perf_counter()
    op32(M32)
    t32 = time.perf_counter() - t0
    del op32
    t1 = None
    if one_thread:  # one evaluation on a single thread, for a per-core figure
        op1 = odemag.DemagFFT(n, cell, workers=1)
        t0 = time.perf_counter()
        op1(M)
        t1 = time.perf_counter() - t0
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": cells / t / 1e9, "unit": "Gcells/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(times)} FP64 H_d evaluations of the {n[0]}x{n[1]}x{n[2]} mesh "
                      f"(scipy rfftn/irfftn, workers={workers}; tensor set-up excluded), "
                      f"median {t:.3f} s each",
            "setup_s": round(t_setup, 2),
            "fp32_scipy_gcells_per_s": round(cells / t32 / 1e9, 6),
            "one_thread_gcells_per_s": round(cells / t1 / 1e9, 6) if t1 else None, "cpu_model": model}


def serve_run(pkg, reqs, rate, budget, max_active, flags):
    """Runs one request mix through the server.  rate None = all submitted at
    once (closed loop); else Poisson arrivals of that rate (1/s).  Returns
    (wall seconds, latencies, stats)."""
    import threading
    import workloads as W
    srv = pkg.serve_open(budget, max_active, flags)
    ids = [None] * len(reqs)
    arrivals = (W.poisson_arrivals(len(reqs), rate, seed=17) if rate else np.zeros(len(reqs)))
    t0 = time.perf_counter()

    def submitter():
        for i, (n, alpha, steps, m0) in enumerate(reqs):
            wait = t0 + arrivals[i] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            ids[i] = pkg.serve_submit(srv, n + W.CELL_4NM, (W.MS, W.A_EX, alpha, 2.21276e5,
                                                            (0.0, 0.0, 0.0)), 1e-13, steps, m0)

    th = threading.Thread(target=submitter)
    th.start()
    lat = []
    try:
        for i, (n, alpha, steps, m0) in enumerate(reqs):
            while ids[i] is None:
                time.sleep(1e-4)
            lat.append(pkg.serve_wait(srv, ids[i], np.empty_like(m0)))
        th.join()
        wall = time.perf_counter() - t0
        stats = pkg.serve_get_stats(srv)
    finally:
        pkg.serve_close(srv)
    return wall, np.array(lat), stats


def serve_bench(pkg, count, steps, loads, budget=16 << 30, max_active=64, seed=2024):
    """Serving workload: `count` independent LLG relaxations, meshes drawn
    uniformly from {32..512}^2 x {1,2,4,8} (4 nm cells), alpha ~ U[0.01, 0.5],
    seeded random m, RK4 dt = 1e-13 s, `steps` steps each, HBM budget 16 GB."""
    import workloads as W
    mix = W.serve_requests(count, seed)
    reqs = [(n, a, steps, W.unit_vectors((n[2], n[1], n[0]), s % 1000003)) for n, a, s in mix]
    flags = pkg.SERVE_GRAPHS
    # plain FP32 form for comparison: the same requests one after another through
    # llg_step on one stream (a plan per request; N^ is shared per shape)
    import torch
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cell_steps = 0
    for k, (n, a, nsteps, m0) in enumerate(reqs):
        if k % 32 == 0:
            print(f"serve: sequential baseline, request {k} of {count}", file=sys.stderr, flush=True)
        plan = pkg.demag_setup(n + W.CELL_4NM, stream=stream)
        m = torch.from_numpy(m0).cuda()
        pkg.llg_step(plan, m, (W.MS, W.A_EX, a, 2.21276e5, (0.0, 0.0, 0.0)), 1e-13, nsteps, stream)
        m.cpu()
        pkg.demag_destroy(plan)
        cell_steps += n[0] * n[1] * n[2] * nsteps
    seq_wall = time.perf_counter() - t0
    # closed loop (everything queued at t = 0): saturated throughput
    print("serve: closed loop", file=sys.stderr, flush=True)
    wall, lat, st = serve_run(pkg, reqs, None, budget, max_active, flags)
    thr = count / wall
    out = {"requests": count, "steps_per_request": steps, "hbm_budget_GB": budget / 2**30,
           "max_active": max_active, "closed_loop_req_per_s": round(thr, 3),
           "closed_loop_cell_steps_per_s": round(st["cell_steps"] / wall, 1),
           "peak_GB": round(st["peak_bytes"] / 2**30, 2), "graph_captures": st["graph_captures"],
           "sequential_plain_req_per_s": round(count / seq_wall, 3),
           "sequential_plain_cell_steps_per_s": round(cell_steps / seq_wall, 1),
           "open_loop": []}
    for f in loads:
        print(f"serve: Poisson arrivals at {f} x the closed-loop rate", file=sys.stderr, flush=True)
        wall, lat, st = serve_run(pkg, reqs, f * thr, budget, max_active, flags)
        out["open_loop"].append({"load": f, "arrival_rate_per_s": round(f * thr, 3),
                                 "p50_s": round(float(np.percentile(lat, 50)), 4),
                                 "p99_s": round(float(np.percentile(lat, 99)), 4),
                                 "req_per_s": round(count / wall, 3),
                                 "cell_steps_per_s": round(st["cell_steps"] / wall, 1)})
    return out


def _stage_table(nbytes, stages, evals):
    per_stage = {}
    for name, (tot_ms, cnt) in stages.items():
        if cnt:
            per_launch = nbytes[name] * evals / cnt
            avg = tot_ms / cnt
            per_stage[name] = {"avg_us": round(1e3 * avg, 2), "launches": cnt,
                               "bytes_per_launch": int(per_launch),
                               "GB_per_s": round(per_launch / (avg * 1e-3) / 1e9, 1),
                               "us_per_eval": round(1e3 * tot_ms / evals, 2)}
    return per_stage


_LAST_VARIANTS = []  # tile variants the last _field_run's autotuning picked


def _field_run(pkg, n, cell, flags, M, H, args, stream, label):
    """Autotuned demag_field on one mesh: per-stage event timing over args.steps
    evaluations, then the same number untimed.  Returns (seconds per
    evaluation, per-stage table, chunk count)."""
    import torch
    print(f"{label}: set-up", file=sys.stderr, flush=True)
    plan = pkg.demag_setup(n + cell, flags, stream=stream)
    try:
        if args.variants or args.chunks:  # pinned schedule (profiler runs), else autotuned
            for st, v in enumerate(args.variants or []):
                pkg.demag_set_variant(plan, st, v)
            if args.chunks:
                pkg.demag_set_chunks(plan, args.chunks)
        else:
            pkg.demag_autotune(plan, stream)
        nch = pkg.demag_get_chunks(plan)
        form = pkg.demag_get_form(plan)
        _LAST_VARIANTS[:] = [pkg.demag_get_variant(plan, st) for st in range(5)]
        print(f"{label}: timing", file=sys.stderr, flush=True)
        for _ in range(args.warmup):
            pkg.demag_field(plan, M, H, stream)
        torch.cuda.synchronize()
        pkg.demag_timing_enable(plan, args.steps * nch)
        for _ in range(args.steps):
            pkg.demag_field(plan, M, H, stream)
        torch.cuda.synchronize()
        stages = pkg.demag_timing_read(plan)
        pkg.demag_timing_enable(plan, 0)
        t1 = time.perf_counter()
        for _ in range(args.steps):
            pkg.demag_field(plan, M, H, stream)
        torch.cuda.synchronize()
        t_field = (time.perf_counter() - t1) / args.steps
    finally:
        pkg.demag_destroy(plan)
    return t_field, _stage_table(stage_bytes(n, form), stages, args.steps), nch, form


def large_film_bench(pkg, args):
    """demag_field on 1024x1024x32 cells of 4 nm, seeded random unit M x Ms, in
    the FP32 form (the reported value) and in the two split-precision BF16 MFMA
    forms; the MFMA results are compared with the FP32 result."""
    import torch
    import workloads as W
    cfg = W.LARGE_FILM
    n, cell = cfg["n"], cfg["cell"]
    cells = n[0] * n[1] * n[2]
    stream = torch.cuda.current_stream()
    M = torch.from_numpy(W.magnetisation(n, 0)).cuda()
    H32 = torch.empty_like(M)
    H = torch.empty_like(M)
    b5 = sum(v for k, v in stage_bytes(n).items() if k != "llg")
    modes = {}
    for flags, name in ((0, "fp32"), (pkg.DEMAG_BF16X3_MFMA, "bf16x3_mfma")):
        t_field, per_stage, nch, form = _field_run(pkg, n, cell, flags, M, H32 if flags == 0 else H,
                                                   args, stream, f"large film {name}")
        entry = {"Gcells_per_s": round(cells / t_field / 1e9, 3), "ms_per_eval": round(1e3 * t_field, 4),
                 "form": "thin (x+z, y conv, z+x)" if form == 3 else "five-pass",
                 "stage_variants": list(_LAST_VARIANTS),
                 "effective_hbm_frac": round(b5 / t_field / 1e9 / HBM_PEAK_GBS, 4),
                 "yz_chunks": nch, "stages": per_stage}
        if flags:
            d = [float((H[a] - H32[a]).norm() / H32[a].norm()) for a in range(3)]
            entry["rel_l2_vs_fp32_per_field"] = [float("%.3e" % v) for v in d]
        modes[name] = entry
    fp = modes["fp32"]
    per_stage = fp["stages"]
    dom = max(per_stage, key=lambda k: per_stage[k]["avg_us"] * per_stage[k]["launches"])
    lpe = {k: per_stage[k]["launches"] / args.steps for k in per_stage}   # launches per evaluation
    tr = [counter_traffic(k, COUNTERS_LARGE, 5) for k in per_stage]         # per evaluation
    fp["counter_bytes_per_eval"] = int(sum(tr)) if all(t is not None for t in tr) else None
    out = {"metric": "demag H_d evals: Gcells/s + % HBM roofline; serve p50/p99 latency",
           "value": fp["Gcells_per_s"],
           "unit": "Gcells/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": fp["ms_per_eval"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": cfg["name"], "mesh": list(n), "cell_m": list(cell),
                      "form": fp["form"], "yz_chunks": fp["yz_chunks"]},
           "roofline": {"bound": "hbm", "kernel": dom, "achieved": per_stage[dom]["GB_per_s"],
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(per_stage[dom]["GB_per_s"] / HBM_PEAK_GBS, 4),
                        "traffic": counter_traffic(dom, COUNTERS_LARGE, 5, lpe[dom]),
                        "bytes_per_launch": per_stage[dom]["bytes_per_launch"]},
           "demag_field_bytes_b5": b5,
           "modes": modes}
    return out


def field_bench(pkg, args):
    """demag_field alone on an nx x ny x nz mesh of 4 nm cubes, seeded random unit
    M x Ms: per-stage event timing and wall time per evaluation (a short,
    self-contained command for profiler runs)."""
    import torch
    import workloads as W
    n = tuple(int(v) for v in args.mesh.split(","))
    cells = n[0] * n[1] * n[2]
    stream = torch.cuda.current_stream()
    M = torch.from_numpy(W.magnetisation(n, 0)).cuda()
    H = torch.empty_like(M)
    t_field, per_stage, nch, form = _field_run(pkg, n, W.CELL_4NM, 0, M, H, args, stream, f"field {n}")
    return {"workload": "field", "mesh": list(n), "Gcells_per_s": round(cells / t_field / 1e9, 3),
            "us_per_eval": round(1e6 * t_field, 1), "form": form, "yz_chunks": nch,
            "stage_variants": _LAST_VARIANTS, "stages": per_stage}


def atomistic_bench(pkg, args):
    """Heun steps of 1024x1024x256 spins (a = 0.4 nm, J = 1e-21 J, mu_s = 1 muB,
    alpha = 0.05, dt = 1e-15 s, T = 0), demag on 4^3-spin macrocells."""
    import torch
    import workloads as W
    cfg = W.ATOMISTIC
    n = cfg["n"]
    spins = n[0] * n[1] * n[2]
    stream = torch.cuda.current_stream()
    plan = pkg.atom_setup((n[0], n[1], n[2], cfg["a"], cfg["macro"]), stream=stream)
    S = torch.from_numpy(W.unit_vectors((n[2], n[1], n[0]), seed=0)).cuda()
    prm = (cfg["J"], cfg["mu_s"], cfg["alpha"], 2.21276e5, (0.0, 0.0, 0.0))
    pkg.atom_step(plan, S, prm, cfg["dt"], args.warmup, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pkg.atom_step(plan, S, prm, cfg["dt"], args.steps, stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    pkg.atom_destroy(plan)
    norm_err = float((S.norm(dim=0) - 1).abs().max())
    # algorithmic Heun step bytes: 2 macrocell averages (read S, read S_p: 12 B/spin
    # each), predictor (read S, write S_p: 24), corrector (read S and S_p, write S:
    # 36) = 84 B/spin; neighbour re-reads come from cache.  The kernels also store
    # and re-read the predictor slope (24 B/spin more, 108 moved in all).
    per_spin = 2 * 12 + 24 + 36
    ms = 1e3 * el / args.steps
    return {"metric": "atomistic spin-steps/s", "value": round(spins * args.steps / el / 1e9, 3),
            "unit": "Gspin-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": cfg["name"], "lattice": list(n), "macro": cfg["macro"]},
            "roofline": {"bound": "hbm", "kernel": "whole Heun step", "achieved":
                         round(per_spin * spins / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(per_spin * spins / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "traffic": None, "bytes_per_spin": per_spin,
                         "bytes_per_spin_moved_by_the_kernels": 108},
            "max_norm_error": norm_err}


def switching_bench(pkg, args):
    """The switching problem of the precision study (Sec. II, Fig. 2), 480x240x2
    cells of 5 nm: S state, then 1 ns under H = (-20, 1, 0) kA/m at the reference
    step (10 fs) and the coarser steps, <m> recorded every 400 fs on the device;
    the mean relative error of each coarse trajectory against the reference."""
    import torch
    import workloads as W
    from paper_2308_08447_amd import switching as sw
    cfg = W.SWITCHING
    n, cell = cfg["n"], cfg["cell"]
    cells = n[0] * n[1] * n[2]
    stream = torch.cuda.current_stream()
    plan = pkg.demag_setup(n + cell, stream=stream)
    try:
        pkg.demag_autotune(plan, stream)
        m = torch.empty((3, n[2], n[1], n[0]), dtype=torch.float32, device="cuda")
        print("switching: S state", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        prep_steps = sw.s_state(pkg, plan, m, cfg, stream)
        torch.cuda.synchronize()
        t_prep = time.perf_counter() - t0
        s0 = m.clone()
        ms = torch.empty(3, dtype=torch.float32, device="cuda")
        pkg.demag_field_mean(plan, s0, ms, stream)
        recs, runs = {}, {}
        for dt in (cfg["dt_ref"],) + tuple(cfg["dts"]):
            print(f"switching: 1 ns at dt = {dt * 1e15:.0f} fs", file=sys.stderr, flush=True)
            m.copy_(s0)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rec = sw.switch(pkg, plan, m, cfg, dt, stream)
            torch.cuda.synchronize()
            el = time.perf_counter() - t1
            steps = int(round(cfg["t_switch"] / dt))
            recs[dt] = rec.cpu().numpy().astype(np.float64)
            runs[dt] = {"steps": steps, "s": round(el, 3),
                        "ms_per_step": round(1e3 * el / steps, 4),
                        "gcells_per_s": round(4 * cells * steps / el / 1e9, 3)}
    finally:
        pkg.demag_destroy(plan)
    ref = recs[cfg["dt_ref"]]
    for dt in cfg["dts"]:
        runs[dt]["epsilon_vs_ref"] = float("%.3e" % sw.epsilon(recs[dt], ref))
    t = np.arange(len(ref)) * cfg["record_every"]
    cross = np.nonzero(ref[:, 0] < 0)[0]
    coarse = max(cfg["dts"])
    return {
        "metric": "switching problem: mean relative error vs the 10 fs reference; Gcells/s",
        "value": runs[coarse]["gcells_per_s"], "unit": "Gcells/s",
        "n_gpus": 1, "steps": runs[coarse]["steps"], "warmup": 0,
        "ms_per_step": runs[coarse]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": cfg["name"], "mesh": list(n), "cell_m": list(cell),
                   "alpha": cfg["alpha"], "H_switch_A_per_m": list(cfg["H_switch"]),
                   "s_state": {"ramp": f"{cfg['ramp_steps']} x {cfg['ramp_time'] * 1e12:.0f} ps from "
                                       f"{cfg['H_sat'] / 1e6:.0f} MA/m along [1,1,1]",
                               "relax_ps": cfg["relax_time"] * 1e12, "alpha": cfg["alpha_prep"],
                               "steps": prep_steps, "s": round(t_prep, 3),
                               "mean_m": [round(float(v), 5) for v in ms.cpu()]},
                   "record_every_fs": cfg["record_every"] * 1e15},
        "runs_fs": {f"{dt * 1e15:.0f}": runs[dt] for dt in runs},
        "reference": {"first_mx_below_zero_ps": round(float(t[cross[0]]) * 1e12, 1) if len(cross) else None,
                      "final_mean_m": [round(float(v), 5) for v in ref[-1]]},
    }


def thin_film_block(pkg, args):
    """The thin-film LLG workload, 512 x 512 x 16 cells of 4 nm, RK4 dt = 1e-13 s:
    RK4 steps (four H_d evaluations and four fused exchange + LLG stage updates
    each), timed once with per-stage events (the stage table) and once as one
    llg_step call without events (the step time: the stage events lengthen the
    gaps between kernels by about 0.07 ms per step at this size), the same steps with the
    extrapolated H_d, the film periodic in x and y, and demag_field alone."""
    import torch
    import workloads as W
    cfg = W.THIN_FILM
    n, cell = cfg["n"], cfg["cell"]
    cells = n[0] * n[1] * n[2]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    plan = pkg.demag_setup(n + cell, stream=stream)
    if args.variants or args.chunks:
        for st, v in enumerate(args.variants or []):
            pkg.demag_set_variant(plan, st, v)
        if args.chunks:
            pkg.demag_set_chunks(plan, args.chunks)
    else:
        pkg.demag_autotune(plan, stream)
    variants = [pkg.demag_get_variant(plan, st) for st in range(5)]
    form = pkg.demag_get_form(plan)
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
    elapsed_ev = time.perf_counter() - t0
    stages = pkg.demag_timing_read(plan)
    pkg.demag_timing_enable(plan, 0)

    m_plain = m.clone()
    # the step time itself: the same number of steps in one llg_step call (the
    # captured step replayed), with no stage events between the kernels, on a
    # copy of m (the graph is captured by the first call on that tensor)
    mc = m.clone()
    pkg.llg_step(plan, mc, params, cfg["dt"], 2, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pkg.llg_step(plan, mc, params, cfg["dt"], args.steps, stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    del mc

    # the same steps with one H_d per RK4 step (quartic extrapolation of H_d at
    # the sub-steps once five step-start fields exist): wall time and the
    # difference of the trajectory from the plain one
    plan_x = pkg.demag_setup(n + cell, pkg.DEMAG_EXTRAPOLATE_HD, stream=stream)
    mx = m0.clone()
    for _ in range(args.warmup):
        pkg.llg_step(plan_x, mx, params, cfg["dt"], 1, stream)
    torch.cuda.synchronize()
    tx0 = time.perf_counter()
    for _ in range(args.steps):
        pkg.llg_step(plan_x, mx, params, cfg["dt"], 1, stream)
    torch.cuda.synchronize()
    elapsed_x = time.perf_counter() - tx0
    pkg.demag_destroy(plan_x)
    inc_plain, inc_x = m_plain - m0, mx - m0
    extrap = {"ms_per_step": round(1e3 * elapsed_x / args.steps, 4), "hd_evals_per_step": 1,
              "speedup_vs_plain_rk4": round(elapsed / elapsed_x, 3),
              "rel_l2_of_increment_vs_plain": float("%.3e" % float((inc_x - inc_plain).norm() / inc_plain.norm())),
              "steps": args.warmup + args.steps,
              "note": "the first five steps evaluate every stage (history start-up)"}

    # periodic in x and y with 32 images per side: set-up time (FP64 image-sum
    # tensor), RK4 steps and per-stage H_d timing of the unpadded transforms
    pbc = (True, True, False)
    t_s = time.perf_counter()
    plan_p = pkg.demag_setup(n + cell, pkg.pbc_flags(*pbc, images=32), stream=stream)
    torch.cuda.synchronize()
    setup_p = time.perf_counter() - t_s
    mp = m0.clone()
    for _ in range(args.warmup):
        pkg.llg_step(plan_p, mp, params, cfg["dt"], 1, stream)
    torch.cuda.synchronize()
    pkg.demag_timing_enable(plan_p, 4 * args.steps * pkg.demag_get_chunks(plan_p))
    for _ in range(args.steps):
        pkg.llg_step(plan_p, mp, params, cfg["dt"], 1, stream)
    torch.cuda.synchronize()
    stages_p = pkg.demag_timing_read(plan_p)
    pkg.demag_timing_enable(plan_p, 0)
    pkg.llg_step(plan_p, mp, params, cfg["dt"], 2, stream)   # captures the step
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    pkg.llg_step(plan_p, mp, params, cfg["dt"], args.steps, stream)
    torch.cuda.synchronize()
    elapsed_p = time.perf_counter() - tp0
    pkg.demag_destroy(plan_p)
    per_stage_p = _stage_table(stage_bytes(n, 5, pbc), stages_p, 4 * args.steps)
    hd_p = sum(v["us_per_eval"] for k, v in per_stage_p.items() if k != "llg")
    periodic = {"axes": "xy", "images_per_side": 32,
                "setup_s": round(setup_p, 3),
                "ms_per_step": round(1e3 * elapsed_p / args.steps, 4),
                "gcells_per_s": round(4 * cells * args.steps / elapsed_p / 1e9, 3),
                "hd_us_per_eval": round(hd_p, 1),
                "stages": per_stage_p}

    # measured device-to-device copy bandwidth (read + write bytes / time)
    cp_src = torch.empty(256 * 2**20, dtype=torch.float32, device=dev)
    cp_dst = torch.empty_like(cp_src)
    cp_dst.copy_(cp_src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        cp_dst.copy_(cp_src)
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * cp_src.numel() * 4 / (time.perf_counter() - t0) / 1e9
    del cp_src, cp_dst

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
    nbytes = stage_bytes(n, form)   # per H_d evaluation (per RK stage for "llg")
    evals = 4 * args.steps
    per_stage = _stage_table(nbytes, stages, evals)
    dom = max(per_stage, key=lambda k: per_stage[k]["avg_us"] * per_stage[k]["launches"])
    achieved = per_stage[dom]["GB_per_s"]
    # the reference byte count is the five-pass one (B5), whichever form runs
    b5 = sum(v for k, v in stage_bytes(n, 5).items() if k != "llg")
    b_form = sum(v for k, v in nbytes.items() if k != "llg")
    # counter-measured HBM bytes of one evaluation (stored rocprofv3 runs of the
    # current kernels), to set against B5
    tr = [counter_traffic(k, COUNTERS, form) for k in nbytes if k != "llg"]   # per evaluation
    counter_eval = int(sum(tr)) if tr and all(v is not None for v in tr) else None

    out = {
        "metric": "demag H_d evals: Gcells/s + % HBM roofline (thin-film RK4 steps)",
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
                   "form": "thin (x+z, y conv, z+x)" if form == 3 else "five-pass",
                   "stage_variants": variants, "yz_chunks": nch},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": counter_traffic(dom, COUNTERS, form,
                                                per_stage[dom]["launches"] / evals),
                     "bytes_per_launch": per_stage[dom]["bytes_per_launch"]},
        "stages": per_stage,
        "ms_per_step_with_stage_events": round(1e3 * elapsed_ev / args.steps, 4),
        "demag_field_gcells_per_s": round(cells / t_field / 1e9, 3),
        "demag_field_us": round(1e6 * t_field, 1),
        "demag_field_effective_frac": round(b5 / t_field / 1e9 / HBM_PEAK_GBS, 4),
        "demag_field_bytes_b5": b5,
        "demag_field_bytes_this_form": b_form,
        "demag_field_counter_bytes": counter_eval,
        "measured_copy_GB_per_s": round(copy_gbs, 1),
        "demag_field_frac_of_copy": round(b5 / t_field / 1e9 / copy_gbs, 4),
        "llg_cell_steps_per_s": round(cells * args.steps / elapsed, 1),
        "llg_extrapolated_hd": extrap,
        "pbc_xy": periodic,
    }
    return out


def small_config_block(pkg):
    """The small configuration, 32 x 32 x 4 cells: latency per demag_field call,
    synchronous (call + synchronize) and pipelined (calls queued back to back),
    each as the median over repeated windows, eagerly and by replaying the call
    captured as a HIP graph.  Its 1.4 MB of traffic stays in the caches, so it
    has no HBM roofline."""
    import torch
    import workloads as W
    dev = torch.device("cuda:0")
    n1 = W.DEMAG_SMALL["n"]
    stream = torch.cuda.current_stream()
    plan1 = pkg.demag_setup(n1 + W.DEMAG_SMALL["cell"], stream=stream)
    M1 = torch.from_numpy(W.magnetisation(n1, 0)).to(dev)
    H1 = torch.empty_like(M1)
    try:
        for _ in range(20):
            pkg.demag_field(plan1, M1, H1, stream)
        torch.cuda.synchronize()
        H_eager = H1.clone()
        # one call captured as a graph on a capture stream (kernel launches only)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            pkg.demag_field(plan1, M1, H1, torch.cuda.current_stream())
        torch.cuda.synchronize()

        def windows(call, nwin=9, per=100):
            sync, pipe = [], []
            for _ in range(nwin):
                lat = []
                for _ in range(per):
                    t0 = time.perf_counter()
                    call()
                    torch.cuda.synchronize()
                    lat.append(time.perf_counter() - t0)
                sync.append(float(np.median(lat)))
                t0 = time.perf_counter()
                for _ in range(per):
                    call()
                torch.cuda.synchronize()
                pipe.append((time.perf_counter() - t0) / per)
            return sync, pipe

        s_e, p_e = windows(lambda: pkg.demag_field(plan1, M1, H1, stream))
        H1.zero_()
        s_g, p_g = windows(g.replay)
        torch.cuda.synchronize()
        graph_equal = bool(torch.equal(H1, H_eager))
        del g
    finally:
        pkg.demag_destroy(plan1)
    us = lambda v: round(1e6 * v, 1)
    return {"mesh": list(n1),
            "eager": {"sync_us_median": us(np.median(s_e)), "pipelined_us_median": us(np.median(p_e)),
                      "pipelined_us_windows": [us(v) for v in p_e]},
            "graph_replay": {"sync_us_median": us(np.median(s_g)), "pipelined_us_median": us(np.median(p_g)),
                             "pipelined_us_windows": [us(v) for v in p_g],
                             "bitwise_equal_to_eager": graph_equal},
            "windows": "9 windows of 100 calls each",
            "note": "cache-resident and launch-bound: no HBM roofline"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the short serving sample")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MB",
                    help="first run one plain device copy of MB megabytes (a known-size "
                         "reference for hardware byte counters)")
    ap.add_argument("--workload", default="large_film",
                    choices=("large_film", "large_film_only", "thin_film", "atomistic", "switching", "field",
                             "small"),
                    help="large_film (default): 1024x1024x32 demag_field (FP32 and BF16x3 MFMA), plus "
                         "the thin-film, small-configuration and serving blocks; large_film_only: "
                         "the large film alone; thin_film: 512x512x16 RK4 LLG as the main line; "
                         "atomistic: 1024x1024x256 spins, Heun, 4^3 macrocells; "
                         "switching: the 480x240x2 switching problem, 1 ns at 10-400 fs steps; "
                         "field: demag_field alone on --mesh (for profiler runs); small: the "
                         "32x32x4 latency block alone")
    ap.add_argument("--mesh", default="512,512,16",
                    help="field workload: cells nx,ny,nz (4 nm cubes)")
    ap.add_argument("--variants", type=lambda s: [int(v) for v in s.split(",")], default=None,
                    help="pin the tile variant of the five FFT stages (e.g. 1,1,1,1,1) instead "
                         "of autotuning")
    ap.add_argument("--chunks", type=int, default=0,
                    help="pin the number of chunks the y/z stages run in instead of autotuning")
    ap.add_argument("--serve-full", action="store_true",
                    help="only the full serving workload: 256 requests x 1000 RK4 steps, "
                         "Poisson loads 0.5/0.8/0.95 of the closed-loop throughput")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2308_08447_amd as pkg
    import workloads as W

    if args.copy_probe:
        src = torch.empty(args.copy_probe * 2**20 // 4, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.serve_full:
        res = serve_bench(pkg, 256, 1000, (0.5, 0.8, 0.95))
        print(json.dumps({"metric": "serve p50/p99 latency", "data": "synthetic",
                          "config": {"workload": "serving: 256 LLG relaxations, meshes "
                                     "{32..512}^2 x {1,2,4,8}, 1000 RK4 steps each"},
                          "serve": res}), flush=True)
        return

    if args.workload == "field":
        print(json.dumps(field_bench(pkg, args)), flush=True)
        return
    if args.workload == "small":
        print(json.dumps(small_config_block(pkg)), flush=True)
        return
    if args.workload == "atomistic":
        print(json.dumps(atomistic_bench(pkg, args)), flush=True)
        return
    if args.workload == "switching":
        print(json.dumps(switching_bench(pkg, args)), flush=True)
        return

    if args.workload == "thin_film":
        out = thin_film_block(pkg, args)
        out["small_config"] = small_config_block(pkg)
        if not args.no_serve:
            out["serve"] = serve_bench(pkg, 64, 100, (0.8,))
        if not args.no_cpu_baseline:
            cfg = W.THIN_FILM
            out["cpu_baseline"] = cpu_baseline(cfg["n"], cfg["cell"])
        print(json.dumps(out), flush=True)
        return

    # default: demag_field on the large film (1024 x 1024 x 32, the largest
    # single-GPU configuration), then the thin-film RK4 block, the small
    # configuration's latency and a short serving sample as extra keys
    out = large_film_bench(pkg, args)
    if args.workload == "large_film":  # not for large_film_only
        print("thin film: RK4 steps", file=sys.stderr, flush=True)
        out["thin_film"] = thin_film_block(pkg, args)
        print("small configuration: latency", file=sys.stderr, flush=True)
        out["small_config"] = small_config_block(pkg)
        if not args.no_serve:
            out["serve"] = serve_bench(pkg, 64, 100, (0.8,))
    if not args.no_cpu_baseline:
        cfg = W.LARGE_FILM
        print("cpu baseline: FP64 oracle on the large film", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg["n"], cfg["cell"], budget_s=30.0, one_thread=False)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
