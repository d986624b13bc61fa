"""Benchmark of the extruded column loop on one MI355X.

Workload (one step): FP64 residual assembly of the integral of f v on a
512 x 512 triangulated unit square (524,288 jittered triangles, RCM-ordered)
extruded to 100 layers of prisms -- once on P1 x P1 (CG, INC) and once on
DG0 x DG0 (WRITE) -- with inputs resident in HBM.  Prints one JSON line:
whole-step throughput in GB/s of algorithmic bytes, the roofline of the
dominant kernel, the measured STREAM triad, and the CPU oracle on a bounded
sample of the same workload.  Secondary figures (higher-order mass actions,
cubic forward vs fused forward+adjoint, batched vs individual launches) are
added unless --quick.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector
TUNED_TABLE = os.path.join(ROOT, "paper_1604_05937_amd", "tuned_mi355x.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed(torch, fn, reps):
    """min and mean time (ms) of fn over reps runs, HIP events on the current stream."""
    fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        fn()
        e1.record(s)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return min(ts), sum(ts) / len(ts)


def timed_flushed(torch, fn, reps, flush):
    """min and mean time (ms) of fn over reps runs, with the 256 MB
    Infinity Cache (MALL) and the L2s flushed before each run by writing
    `flush` (>= 1 GiB) outside the timed events."""
    fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ts = []
    for r in range(reps):
        flush.fill_(float(r))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        fn()
        e1.record(s)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return min(ts), sum(ts) / len(ts)


def stream_triad(torch, exm):
    n = 1 << 28   # 3 arrays of 2 GiB
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.rand(n, dtype=torch.float64, device="cuda")
    c = torch.rand(n, dtype=torch.float64, device="cuda")
    best = 0.0
    for block in (256, 512, 1024):
        for grid in (0, 4096, 16384):
            t, _ = timed(torch, lambda: exm.stream_triad(a, b, c, 3.0, block=block, grid=grid), 5)
            best = max(best, 24.0 * n / (t * 1e-3) / 1e9)
    del a, b, c
    torch.cuda.empty_cache()
    return best


def read_traffic(kernel_tag: str, src_hash: str, launch: dict):
    """HBM bytes per launch from the rocprofv3 counter summary of this kernel
    build and launch configuration (profiles/<tag>.md, a line
    'traffic: {json}'), else None."""
    p = os.path.join(ROOT, "profiles", f"{kernel_tag}.md")
    if not os.path.exists(p):
        return None
    m = re.search(r"^traffic:\s*(\{.*\})\s*$", open(p).read(), flags=re.M)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("source_hash") != src_hash or d.get("launch") != launch:
        return None   # counters were taken on another kernel build or launch configuration
    return d.get("bytes_per_launch")


def host_threads() -> int:
    """Host threads the all-core baseline uses: OMP_NUM_THREADS when set (the
    machine's CPU share), else the CPUs this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def host_cpu() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(), "cpus_allowed": len(os.sched_getaffinity(0))}


def cpu_baseline(base, lam, vc, f1_host, f0_host, budget_s: float, runs: int = 10, all_core_budget_s: float = 30.0):
    """The oracle (plain C) on the host, two ways:
    - one thread, on a bounded sample of the same workload (the first base
      cells of the RCM order, all layers, P1 and DG0), the per-prism time
      extrapolated to the whole step;
    - every host thread (host_threads()) over the whole step, P1 colour by
      colour of the oracle's own greedy colouring, DG0 split over the
      threads; the minimum of `runs` runs (fewer if they exceed
      all_core_budget_s), as the paper takes the minimum of ten."""
    import numpy as np

    import oracle
    t0 = time.time()
    num_x = oracle.number(base.counts, lam, oracle.delta_table("CG1", "CG1"), base.cell_vertex, base.cell_edge)
    num_0 = oracle.number(base.counts, lam, oracle.delta_table("DG0", "DG0"), base.cell_vertex, base.cell_edge)
    X = oracle.coordinate_field(num_x, vc)
    log(f"cpu baseline: oracle numbering {time.time() - t0:.1f}s")
    out1 = np.zeros(num_x.n_dofs)
    out0 = np.zeros(num_0.n_dofs)
    per = {}
    for name, num, f, out, space in (("P1", num_x, f1_host, out1, ("CG1", "CG1")),
                                     ("DG0", num_0, f0_host, out0, ("DG0", "DG0"))):
        n = 256
        while True:
            cells = np.arange(n)
            t = time.perf_counter()
            oracle.par_loop(oracle.FORM_MASS, space, num, num_x, X, [f], [out], write=(name == "DG0"), cells=cells)
            dt = time.perf_counter() - t
            if dt > budget_s / 8 or n >= base.n_cells:
                break
            n = min(base.n_cells, int(n * max(2.0, budget_s / 2 / max(dt, 1e-3))))
        per[name] = (dt / (n * lam), n)
        log(f"cpu baseline {name}: {n} cells x {lam} layers in {dt:.2f}s")
    threads = host_threads()
    colour, n_colours = oracle.greedy_colour(base.cell_vertex, base.n_vertices)
    times = []
    t_all = time.perf_counter()
    for r in range(runs):
        out1[:] = 0.0
        t = time.perf_counter()
        oracle.par_loop_threaded(oracle.FORM_MASS, ("CG1", "CG1"), num_x, num_x, X, [f1_host], [out1],
                                 threads=threads, colour=colour)
        oracle.par_loop_threaded(oracle.FORM_MASS, ("DG0", "DG0"), num_0, num_x, X, [f0_host], [out0],
                                 write=True, threads=threads)
        times.append(time.perf_counter() - t)
        if time.perf_counter() - t_all > all_core_budget_s:
            break
    log(f"cpu baseline all cores: {threads} threads, {n_colours} colours, {len(times)} runs, "
        f"min {min(times):.2f}s per step")
    return per, {"threads": threads, "n_colours": n_colours, "runs": len(times), "min_s": min(times),
                 "median_s": float(np.median(times))}


def cpu_baseline_json(per, allc, step_bytes: float, n_prisms: int, gpu_step_ms: float | None) -> dict:
    cpu_step_s = (per["P1"][0] + per["DG0"][0]) * n_prisms
    res = {
        "value": round(step_bytes / allc["min_s"] / 1e9, 4),
        "unit": "GB/s",
        "cores": allc["threads"],
        "kind": "oracle",
        "sample": f"the whole step (P1xP1 INC + DG0xDG0 WRITE oracle assembly, 512x512x100) on "
                  f"{allc['threads']} host threads, P1 colour by colour of the oracle's own greedy colouring "
                  f"({allc['n_colours']} colours), DG0 split over the threads; minimum of {allc['runs']} runs",
        "step_s": round(allc["min_s"], 3),
        "step_s_median": round(allc["median_s"], 3),
        "single_core": {
            "value": round(step_bytes / cpu_step_s / 1e9, 4),
            "unit": "GB/s",
            "cores": 1,
            "sample": f"P1xP1 and DG0xDG0 oracle assembly of the first {per['P1'][1]} and {per['DG0'][1]} base "
                      f"cells (RCM order) x 100 layers, one thread, one run, per-prism time extrapolated to the "
                      f"{n_prisms}-prism step",
            "step_s_extrapolated": round(cpu_step_s, 2),
        },
        "host_cpu": host_cpu(),
    }
    if gpu_step_ms:
        res["gpu_speedup"] = round(allc["min_s"] / (gpu_step_ms * 1e-3), 1)
        res["single_core"]["gpu_speedup"] = round(cpu_step_s / (gpu_step_ms * 1e-3), 1)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--quick", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", choices=["p1", "dg0", "triad", "batch", "cpu", "cubic", "fused"],
                    help="launch only this kernel, warmup + steps times, and print nothing (for rocprofv3)")
    ap.add_argument("--config", default=None,
                    help="with --only: the launch configuration as JSON (exm_loop_opts fields) instead of autotuning")
    ap.add_argument("--launch", default=None,
                    help='launch configurations as JSON {"p1": {...}, "dg0": {...}} instead of autotuning '
                         "(the figures of a previous run, for profiling the timed region alone)")
    ap.add_argument("--cpu-seconds", type=float, default=16.0)
    ap.add_argument("--tuned", default=TUNED_TABLE,
                    help="launch-configuration table (exm_autotune_save format) to take the P1 and DG0 launches "
                         "from; the library's autotuner runs when it is missing or with --retune")
    ap.add_argument("--preroll", type=float, default=1.0,
                    help="seconds of untimed steps before the warmup steps (clock ramp-up)")
    ap.add_argument("--retune", action="store_true", help="run the autotuner instead of reading --tuned")
    ap.add_argument("--save-tune", default=None, help="write the tuned table here after autotuning")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark line: layer sweep (P1 and DG0 RHS, autotuned) on the fixed "
                         "512x512 base and at a constant ~52.4M prisms, plus RCM against a random base ordering; "
                         "one JSON line per point")
    args = ap.parse_args()
    if args.only == "cpu":
        cpu_only(args)
        return
    if args.gpus != 1:
        print(f"bench.py: this library runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1604_05937_amd as exm
    from paper_1604_05937_amd import meshgen, workloads as W

    exm.load_library()
    torch.cuda.init()
    if args.sweep:
        sweep(torch, exm)
        return
    if args.only == "triad":
        # calibration kernel for the HBM counters: reads 16 n bytes, writes 8 n
        n = 1 << 26
        a = torch.empty(n, dtype=torch.float64, device="cuda")
        b = torch.rand(n, dtype=torch.float64, device="cuda")
        c = torch.rand(n, dtype=torch.float64, device="cuda")
        for _ in range(args.warmup + args.steps):
            exm.stream_triad(a, b, c, 3.0)
        torch.cuda.synchronize()
        log(f"done: triad n = {n}, {16 * n} bytes read and {8 * n} written per launch")
        return
    if args.only == "batch":
        # the 64-mesh batch, its tilings timed at creation, then warmup + steps graph replays
        items, bytes_p1, bytes_dg0 = batch_items(torch, exm, W, meshgen)
        B = exm.Batch(items)
        torch.cuda.synchronize()
        for _ in range(args.warmup + args.steps):
            B.launch()
        torch.cuda.synchronize()
        log(f"done: batch, tiles P1 {B.tiles('P1')} DG0 {B.tiles('DG0')}, algorithmic bytes per replay "
            f"P1 {bytes_p1} DG0 {bytes_dg0}")
        return
    if args.only in ("cubic", "fused"):
        # the cubic residual (or its fused residual + adjoint) on 256 x 256 x 50, autotuned
        e4 = W.extruded(256, 50)
        V = e4.Vx
        u = W.device_values(V.n_dofs, 31)
        f = W.device_values(V.n_dofs, 32)
        w = W.device_values(V.n_dofs, meshgen.SEED_COTAN)
        F, gu, gf = V.zeros(), V.zeros(), V.zeros()
        R, I = exm.EXM_READ, exm.EXM_INC
        if args.only == "cubic":
            k, fields = exm.EXM_K_CUBIC, [(u, V, R), (f, V, R), (F, V, I)]
        else:
            k, fields = exm.EXM_K_CUBIC_FUSED, [(u, V, R), (f, V, R), (w, V, R), (F, V, I), (gu, V, I), (gf, V, I)]
        cfg = json.loads(args.config) if args.config else exm.autotune(k, e4.mesh, e4.X, V, fields)
        torch.cuda.synchronize()
        for _ in range(args.warmup + args.steps):
            exm.par_loop(k, e4.mesh, e4.X, V, fields, **cfg)
        torch.cuda.synchronize()
        by = W.cubic_bytes(e4, args.only == "fused")["algorithmic"]
        log(f"done: {args.only} {cfg}, {by} algorithmic bytes and {W.cubic_flops(e4, args.only == 'fused')} "
            f"algorithmic FP64 operations per launch")
        return
    t0 = time.time()
    work = W.extruded(512, 100, keep_host_coords=not args.no_cpu)
    V1, V0 = work.space("P1"), work.space("DG0")
    f1_host = meshgen.uniform_values(V1.n_dofs, seed=meshgen.SEED_FIELD)
    f0_host = meshgen.uniform_values(V0.n_dofs, seed=meshgen.SEED_FIELD)
    f1 = torch.from_numpy(f1_host).to("cuda")
    f0 = torch.from_numpy(f0_host).to("cuda")
    b1 = V1.zeros()
    b0 = V0.zeros()
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    log(f"setup {setup_s:.1f}s: {work.base.n_cells} cells x {work.n_layers} layers, P1 {V1.n_dofs} DoFs, DG0 {V0.n_dofs} DoFs")

    by1 = W.mass_bytes(work, "P1")
    by0 = W.mass_bytes(work, "DG0")
    if args.only in ("p1", "dg0"):
        name, f, b = ("P1", f1, b1) if args.only == "p1" else ("DG0", f0, b0)
        if args.config:
            cfg = json.loads(args.config)
        else:
            cfg = exm.autotune(exm.EXM_K_MASS, work.mesh, work.X, work.Vx, W.mass_args(work, name, f, b))
        torch.cuda.synchronize()
        for _ in range(args.warmup + args.steps):
            W.run_mass(work, name, f, b, **cfg)
        torch.cuda.synchronize()
        log(f"done: {name} {cfg}, {(by1 if name == 'P1' else by0)['algorithmic']} algorithmic bytes per launch")
        return

    if args.launch:
        given = json.loads(args.launch)
        cfg1, cfg0 = given["p1"], given["dg0"]
        log(f"given launch configurations: P1 {cfg1}  DG0 {cfg0}")
    elif not args.retune and args.tuned and os.path.exists(args.tuned):
        # the stored table of tuned launches (the same launches the committed profiles trace)
        exm.autotune_load(args.tuned)
        cfg1 = exm.par_loop_config(exm.EXM_K_MASS, work.mesh, work.X, work.Vx, W.mass_args(work, "P1", f1, b1))
        cfg0 = exm.par_loop_config(exm.EXM_K_MASS, work.mesh, work.X, work.Vx, W.mass_args(work, "DG0", f0, b0))
        log(f"tuned table {os.path.relpath(args.tuned, ROOT)}: P1 {cfg1}  DG0 {cfg0}")
    else:
        # autotuned launch configurations (the library keeps them for later calls)
        t0 = time.time()
        cfg1 = exm.autotune(exm.EXM_K_MASS, work.mesh, work.X, work.Vx, W.mass_args(work, "P1", f1, b1))
        cfg0 = exm.autotune(exm.EXM_K_MASS, work.mesh, work.X, work.Vx, W.mass_args(work, "DG0", f0, b0))
        log(f"autotune {time.time() - t0:.1f}s: P1 {cfg1}  DG0 {cfg0}")
        if args.save_tune:
            exm.autotune_save(args.save_tune)

    k1 = lambda: W.run_mass(work, "P1", f1, b1, **cfg1)
    k2 = lambda: W.run_mass(work, "DG0", f0, b0, **cfg0)

    # ---- timed region: K steps of (P1 assembly, DG0 assembly) ----
    s = torch.cuda.current_stream()
    # pre-roll: the step repeated, untimed, for --preroll seconds, so that the
    # GPU clocks have reached their steady state before the warmup steps
    t_end = time.perf_counter() + args.preroll
    while time.perf_counter() < t_end:
        for _ in range(16):
            k1()
            k2()
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        k1()
        k2()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t_start = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(s)
        k1()
        ev[i][1].record(s)
        k2()
        ev[i][2].record(s)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_start) * 1e3
    t1 = [ev[i][0].elapsed_time(ev[i][1]) for i in range(args.steps)]
    t2 = [ev[i][1].elapsed_time(ev[i][2]) for i in range(args.steps)]
    step_ms = ev[0][0].elapsed_time(ev[-1][2]) / args.steps
    step_bytes = by1["algorithmic"] + by0["algorithmic"]
    value = step_bytes / (step_ms * 1e-3) / 1e9
    log(f"step {step_ms:.3f} ms (P1 {np.mean(t1):.3f}, DG0 {np.mean(t2):.3f}); wall {wall_ms / args.steps:.3f} ms/step")

    stream_gbs = stream_triad(torch, exm)
    log(f"STREAM triad {stream_gbs:.0f} GB/s")

    k1_gbs = by1["algorithmic"] / (np.mean(t1) * 1e-3) / 1e9
    k2_gbs = by0["algorithmic"] / (np.mean(t2) * 1e-3) / 1e9
    dominant = ("p1_rhs_512x512x100", by1, t1, k1_gbs, cfg1) if np.mean(t1) >= np.mean(t2) else \
               ("dg0_rhs_512x512x100", by0, t2, k2_gbs, cfg0)
    src_hash = W.source_hash()
    traffic = read_traffic(dominant[0], src_hash, dominant[4])
    roofline = {
        "kernel": dominant[0],
        "bound": "hbm",
        "achieved": round(dominant[3], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(dominant[3] / HBM_PEAK_GBS, 4),
        "frac_of_stream": round(dominant[3] / stream_gbs, 4),
        "traffic": traffic,
        "algorithmic_bytes_per_launch": dominant[1]["algorithmic"],
        "avg_launch_ms": round(float(np.mean(dominant[2])), 4),
        # the same time on the byte count that reads all three coordinate
        # components at every extruded vertex (the kernel reads z per level
        # and (x, y) once per vertical column)
        "full_coordinate_field": {
            "algorithmic_bytes_per_launch": dominant[1]["algorithmic_full_coords"],
            "achieved": round(dominant[1]["algorithmic_full_coords"] / (np.mean(dominant[2]) * 1e-3) / 1e9, 1),
            "frac": round(dominant[1]["algorithmic_full_coords"] / (np.mean(dominant[2]) * 1e-3) / 1e9
                          / HBM_PEAK_GBS, 4),
        },
    }

    result = {
        "metric": "extruded assembly GB/s & % HBM peak; batched+adjoint vs plain, same GPU",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "RHS assembly of integral f v, P1xP1 (INC) + DG0xDG0 (WRITE), 512x512 triangulated "
                        "square (524288 tris, jittered, RCM) x 100 layers, FP64",
            "n_prisms": work.n_prisms,
            "p1_dofs": V1.n_dofs,
            "dg0_dofs": V0.n_dofs,
            "launch_p1": cfg1,
            "launch_dg0": cfg0,
            "source_hash": src_hash,
        },
        "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
        "stream_triad_gbs": round(stream_gbs, 1),
        "pct_stream": round(100 * value / stream_gbs, 2),
        "kernels": {
            "p1_rhs": {"ms": round(float(np.mean(t1)), 4), "gbs": round(k1_gbs, 1),
                       "pct_stream": round(100 * k1_gbs / stream_gbs, 2),
                       "valuable_gbs_paper_def": round(by1["valuable"] / (np.mean(t1) * 1e-3) / 1e9, 1),
                       "dofs_per_s": V1.n_dofs / (np.mean(t1) * 1e-3)},
            "dg0_rhs": {"ms": round(float(np.mean(t2)), 4), "gbs": round(k2_gbs, 1),
                        "pct_stream": round(100 * k2_gbs / stream_gbs, 2),
                        "valuable_gbs_paper_def": round(by0["valuable"] / (np.mean(t2) * 1e-3) / 1e9, 1),
                        "dofs_per_s": V0.n_dofs / (np.mean(t2) * 1e-3)},
        },
        "roofline": roofline,
        "setup_s": round(setup_s, 2),
    }

    if not args.quick:
        try:
            result["secondary"] = add_roofline(secondary(torch, exm, W, meshgen), stream_gbs)
        except Exception as e:   # secondary figures never hide the main line
            log(f"secondary measurements failed: {e!r}")
            result["secondary"] = {"error": repr(e)}

    if not args.no_cpu:
        per, allc = cpu_baseline(work.base, work.n_layers, work.vc, f1_host, f0_host, args.cpu_seconds)
        result["cpu_baseline"] = cpu_baseline_json(per, allc, step_bytes, work.n_prisms, step_ms)
    print(json.dumps(result), flush=True)


def cpu_only(args):
    """The CPU baseline alone (no GPU): the oracle on the step's workload."""
    from paper_1604_05937_amd import meshgen, workloads as W
    base = meshgen.tri_square(512)
    lam = 100
    vc = meshgen.extruded_vertex_coords(base, lam)
    n1 = base.n_vertices * (lam + 1)
    n0 = base.n_cells * lam
    f1 = meshgen.uniform_values(n1, seed=meshgen.SEED_FIELD)
    f0 = meshgen.uniform_values(n0, seed=meshgen.SEED_FIELD)
    step_bytes = W.mass_bytes_counts(base, lam, "P1")["algorithmic"] + \
        W.mass_bytes_counts(base, lam, "DG0")["algorithmic"]
    per, allc = cpu_baseline(base, lam, vc, f1, f0, args.cpu_seconds)
    print(json.dumps({"cpu_baseline": cpu_baseline_json(per, allc, step_bytes, base.n_cells * lam, None)}),
          flush=True)


def sweep(torch, exm):
    """Throughput against the layer count (Section 4.2: the base-map load is
    amortised over the column) and against the base ordering."""
    import numpy as np

    from paper_1604_05937_amd import meshgen, workloads as W

    def point(n, lam, order):
        t0 = time.time()
        e = W.extruded(n, lam, order=order)
        res = {"base": f"{n}x{n}", "n_layers": lam, "order": order, "n_prisms": e.n_prisms}
        for name in ("P1", "DG0"):
            V = e.space(name)
            x = W.device_values(V.n_dofs, meshgen.SEED_FIELD)
            y = V.zeros()
            cfg = exm.autotune(exm.EXM_K_MASS, e.mesh, e.X, e.Vx, W.mass_args(e, name, x, y))
            t, _ = timed(torch, lambda: W.run_mass(e, name, x, y, **cfg), 10)
            b = W.mass_bytes(e, name)
            res[name.lower()] = {"ms": round(t, 4), "gbs": round(b["algorithmic"] / t / 1e6, 1),
                                 "dofs_per_s": round(V.n_dofs / t * 1e3), "launch": cfg}
            del x, y
        del e
        torch.cuda.empty_cache()
        res["setup_s"] = round(time.time() - t0, 1)
        print(json.dumps(res), flush=True)

    for lam in (1, 2, 5, 10, 20, 50, 100, 200):
        point(512, lam, "rcm")
    # constant work: about 52.4M prisms, the base shrinking as the layers grow
    for lam in (5, 10, 20, 50, 200):
        point(int(round(512 * np.sqrt(100.0 / lam))), lam, "rcm")
    for lam in (1, 10, 100):
        point(512, lam, "random")


def direct_shapes(exm, name):
    races = [exm.EXM_RACE_ATOMIC, exm.EXM_RACE_COLOUR] if name in exm.CONTINUOUS else [exm.EXM_RACE_ATOMIC]
    return [dict(schedule=exm.EXM_SCHED_DIRECT, race=r, cols_per_wave=c, waves_per_block=w)
            for r in races for c, w in ((1, 4), (2, 4), (3, 4), (4, 4), (1, 2), (2, 2), (4, 2))]


def add_roofline(tree, stream_gbs):
    """Every secondary figure with an algorithmic GB/s gets its fraction of the
    HBM peak and of the measured STREAM triad (these kernels are HBM-bound)."""
    if isinstance(tree, dict):
        out = {k: add_roofline(v, stream_gbs) for k, v in tree.items()}
        for key in ("gbs", "spmv_gbs", "assemble_gbs", "batched_gbs", "forward_gbs", "fused_gbs"):
            if isinstance(tree.get(key), (int, float)):
                out[key.replace("gbs", "frac_hbm")] = round(tree[key] / HBM_PEAK_GBS, 4)
                out[key.replace("gbs", "frac_stream")] = round(tree[key] / stream_gbs, 4)
        return out
    return tree


def secondary(torch, exm, W, meshgen):
    import numpy as np
    out = {}
    # the RHS on the paper's nine spaces ({CG1, DG0, DG1} horizontally x vertically), 256 x 256 x 64
    # (working sets of 30-900 MB, some inside the 256 MB MALL: each is also
    # timed with the caches flushed before every launch)
    e9 = W.extruded(256, 64)
    nine = {}
    flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    for name in ("P1", "CG1xDG0", "CG1xDG1", "DG0xCG1", "DG0", "DG0xDG1", "DG1xCG1", "DG1xDG0", "DG1"):
        V = e9.space(name)
        x = W.device_values(V.n_dofs, meshgen.SEED_FIELD)
        y = V.zeros()
        cfg = exm.autotune(exm.EXM_K_MASS, e9.mesh, e9.X, e9.Vx, W.mass_args(e9, name, x, y))
        t, _ = timed(torch, lambda: W.run_mass(e9, name, x, y, **cfg), 10)
        tf, _ = timed_flushed(torch, lambda: W.run_mass(e9, name, x, y, **cfg), 10, flush)
        b = W.mass_bytes(e9, name)
        nine[name] = {"ms": round(t, 4), "gbs": round(b["algorithmic"] / t / 1e6, 1),
                      "dofs_per_s": round(V.n_dofs / t * 1e3), "schedule": cfg["schedule"],
                      "working_set_mb": round(b["algorithmic"] / 1e6, 1),
                      "flushed": {"ms": round(tf, 4), "gbs": round(b["algorithmic"] / tf / 1e6, 1)}}
        del x, y
    del flush
    out["rhs_nine_spaces_256x256x64"] = nine
    log("nine spaces: " + ", ".join(f"{k} {v['gbs']:.0f}" for k, v in nine.items()))
    del e9
    # columns of different heights: 512 x 512 x 100 with the bottom of every
    # column following a smooth bump (meshgen.layer_ranges, "bathymetry"),
    # beside the uniform mesh of the same sizes, with the schedules both run
    var = {}
    for kind in (None, "bathymetry"):
        ev = W.extruded(512, 100, layer_kind=kind)
        for name in ("P1", "DG0"):
            V = ev.space(name)
            x = W.device_values(V.n_dofs, meshgen.SEED_FIELD)
            y = V.zeros()
            # the DIRECT shapes (the tuner's candidates on such a mesh), GATHER for P1, PIPELINED for both
            shapes = direct_shapes(exm, name)
            if name == "P1":
                shapes += [dict(schedule=exm.EXM_SCHED_GATHER, waves_per_block=w) for w in (1, 2, 4)]
            pipe_shapes = ((64, 16), (48, 16), (96, 8)) if name == "P1" else ((32, 32), (64, 16), (32, 16))
            shapes += [dict(schedule=exm.EXM_SCHED_PIPELINED, race=exm.EXM_RACE_ATOMIC, tile_cells=t, chunk_layers=c)
                       for (t, c) in pipe_shapes]
            b = W.mass_bytes(ev, name)
            for label, group in (("direct", [c for c in shapes if c["schedule"] == exm.EXM_SCHED_DIRECT]),
                                 ("gather", [c for c in shapes if c["schedule"] == exm.EXM_SCHED_GATHER]),
                                 ("pipelined", [c for c in shapes if c["schedule"] == exm.EXM_SCHED_PIPELINED])):
                if not group:
                    continue
                t, cfg = min(((timed(torch, lambda: W.run_mass(ev, name, x, y, **c), 10)[0], c) for c in group),
                             key=lambda tc: tc[0])
                var[f"{name}_{kind or 'uniform'}_{label}"] = {
                    "prisms": ev.n_prisms, "ms": round(t, 4), "gbs": round(b["algorithmic"] / t / 1e6, 1),
                    "prisms_per_s": round(ev.n_prisms / t * 1e3), "launch": cfg}
            del x, y
        del ev
    out["rhs_variable_layers_512x512x100"] = var
    log("variable layers: " + ", ".join(f"{k} {v['gbs']:.0f}" for k, v in var.items()))
    out["race_resolution"] = race_figures(torch, exm, W, meshgen)
    out["layers_constant_work"] = layer_points(torch, exm, W, meshgen)
    out["matrix_p1_512x512x100"] = matrix_figures(torch, exm, W, meshgen)
    # mixed-degree DG (a DoF count per entity): half the cells DG1, half DG0, 256 x 256 x 64
    em = W.extruded(256, 64)
    nd = meshgen.cell_degrees(em.base, frac_dg1=0.5)
    dofs = [np.zeros((em.base.n_vertices, 2), np.int32), None, np.stack([np.zeros_like(nd), nd], 1)]
    Vm = exm.Space.mixed(em.mesh, dofs, element=exm.EXM_ELEMENT_DGMIX)
    x = W.device_values(Vm.n_dofs, meshgen.SEED_FIELD)
    y = Vm.zeros()
    margs = [(x, Vm, exm.EXM_READ), (y, Vm, exm.EXM_WRITE)]
    cfg = exm.autotune(exm.EXM_K_MASS, em.mesh, em.X, em.Vx, margs)
    t, _ = timed(torch, lambda: exm.par_loop(exm.EXM_K_MASS, em.mesh, em.X, em.Vx, margs, **cfg), 10)
    flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    tf, _ = timed_flushed(torch, lambda: exm.par_loop(exm.EXM_K_MASS, em.mesh, em.X, em.Vx, margs, **cfg), 10, flush)
    del flush
    mbytes = 16 * Vm.n_dofs + W.coord_bytes(em) + 4 * (em.base.n_cells + 1) + 4 * int(nd.sum()) + 24 * em.base.n_cells
    out["mass_dg_mixed_degree_256x256x64"] = {"dofs": Vm.n_dofs, "ms": round(t, 4),
                                              "gbs": round(mbytes / t / 1e6, 1), "launch": cfg,
                                              "flushed": {"ms": round(tf, 4), "gbs": round(mbytes / tf / 1e6, 1)}}
    log(f"mixed-degree DG mass {t:.3f} ms")
    del x, y, Vm, em
    # horizontal facets (lambda + 1 per column), the jump form: DG0 on 512 x 512 x 100, DG1 on 256 x 256 x 64
    fac = {}
    for name, (nb, lam) in (("DG0", (512, 100)), ("DG1", (256, 64))):
        ef = W.extruded(nb, lam)
        V = ef.space(name)
        x = W.device_values(V.n_dofs, meshgen.SEED_FIELD)
        y = V.zeros()
        fargs = [(x, V, exm.EXM_READ), (y, V, exm.EXM_WRITE)]
        cfg = exm.autotune(exm.EXM_K_FACET_JUMP, ef.mesh, ef.X, ef.Vx, fargs)
        t, _ = timed(torch, lambda: exm.par_loop(exm.EXM_K_FACET_JUMP, ef.mesh, ef.X, ef.Vx, fargs, **cfg), 10)
        b = W.mass_bytes(ef, name)   # x read, y written, z, lists: the same streams as the mass action
        fac[f"{name}_{nb}x{nb}x{lam}"] = {"facets": ef.base.n_cells * (lam + 1), "ms": round(t, 4),
                                          "gbs": round(b["algorithmic"] / t / 1e6, 1), "launch": cfg}
        del x, y, ef
    out["facet_jump"] = fac
    log("facets: " + ", ".join(f"{k} {v['gbs']:.0f} GB/s" for k, v in fac.items()))
    # higher-order mass actions: 256 x 256 x 64, DG1 x DG1 and P2 x P2
    e3 = W.extruded(256, 64)
    for name in ("DG1", "P2"):
        V = e3.space(name)
        x = W.device_values(V.n_dofs, meshgen.SEED_FIELD)
        y = V.zeros()
        args_ = W.mass_args(e3, name, x, y)
        cfg = exm.autotune(exm.EXM_K_MASS, e3.mesh, e3.X, e3.Vx, args_)
        t, _ = timed(torch, lambda: W.run_mass(e3, name, x, y), 10)
        flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        tf, _ = timed_flushed(torch, lambda: W.run_mass(e3, name, x, y), 10, flush)
        del flush
        b = W.mass_bytes(e3, name)
        out[f"mass_{name.lower()}_256x256x64"] = {"ms": round(t, 4), "gbs": round(b["algorithmic"] / t / 1e6, 1),
                                                  "launch": cfg,
                                                  "flushed": {"ms": round(tf, 4),
                                                              "gbs": round(b["algorithmic"] / tf / 1e6, 1)}}
        log(f"mass {name}: {t:.3f} ms")
        del x, y
    del e3
    # cubic residual vs fused forward+adjoint: 256 x 256 x 50, P1 x P1
    e4 = W.extruded(256, 50)
    V = e4.Vx
    u = W.device_values(V.n_dofs, 31)
    f = W.device_values(V.n_dofs, 32)
    w = W.device_values(V.n_dofs, meshgen.SEED_COTAN)
    F, gu, gf = V.zeros(), V.zeros(), V.zeros()
    fw = [(u, V, exm.EXM_READ), (f, V, exm.EXM_READ), (F, V, exm.EXM_INC)]
    fu = [(u, V, exm.EXM_READ), (f, V, exm.EXM_READ), (w, V, exm.EXM_READ), (F, V, exm.EXM_INC),
          (gu, V, exm.EXM_INC), (gf, V, exm.EXM_INC)]
    c_fw = exm.autotune(exm.EXM_K_CUBIC, e4.mesh, e4.X, V, fw)
    c_fu = exm.autotune(exm.EXM_K_CUBIC_FUSED, e4.mesh, e4.X, V, fu)
    t_fw, t_fw_mean = timed(torch, lambda: W.run_cubic(e4, u, f, F), 10)
    t_fu, t_fu_mean = timed(torch, lambda: W.run_fused(e4, u, f, w, F, gu, gf), 10)
    # the working set (~160 / 240 MB) fits in the 256 MB MALL: also timed
    # with the caches flushed before every launch
    flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    tf_fw, tf_fw_mean = timed_flushed(torch, lambda: W.run_cubic(e4, u, f, F), 10, flush)
    tf_fu, tf_fu_mean = timed_flushed(torch, lambda: W.run_fused(e4, u, f, w, F, gu, gf), 10, flush)
    del flush
    fl_fw, fl_fu = W.cubic_flops(e4, False), W.cubic_flops(e4, True)
    out["cubic_256x256x50"] = {"forward_ms": round(t_fw, 4), "fused_fwd_adj_ms": round(t_fu, 4),
                               "fused_over_forward": round(t_fu / t_fw, 3),
                               "forward_mean_ms": round(t_fw_mean, 4), "fused_mean_ms": round(t_fu_mean, 4),
                               "flushed": {"forward_ms": round(tf_fw, 4), "fused_fwd_adj_ms": round(tf_fu, 4),
                                           "fused_over_forward": round(tf_fu / tf_fw, 3),
                                           "forward_mean_ms": round(tf_fw_mean, 4),
                                           "fused_mean_ms": round(tf_fu_mean, 4)},
                               "launch_forward": c_fw,
                               "launch_fused": c_fu,
                               "forward_tflops": round(fl_fw / t_fw / 1e9, 2),
                               "forward_frac_fp64_peak": round(fl_fw / t_fw / 1e9 / FP64_PEAK_TFLOPS, 4),
                               "fused_tflops": round(fl_fu / t_fu / 1e9, 2),
                               "fused_frac_fp64_peak": round(fl_fu / t_fu / 1e9 / FP64_PEAK_TFLOPS, 4),
                               "forward_gbs": round(W.cubic_bytes(e4, False)["algorithmic"] / t_fw / 1e6, 1),
                               "fused_gbs": round(W.cubic_bytes(e4, True)["algorithmic"] / t_fu / 1e6, 1)}
    log(f"cubic forward {t_fw:.3f} ms, fused {t_fu:.3f} ms; flushed {tf_fw:.3f} / {tf_fu:.3f} ms")
    del e4, u, f, w, F, gu, gf
    torch.cuda.empty_cache()
    out["batch"] = batch_vs_plain(torch, exm, W, meshgen)
    return out


def race_figures(torch, exm, W, meshgen):
    """The race resolutions of CG increments side by side, same run: K1 (P1
    RHS) on 512 x 512 x 100 and the P2 mass action on 256 x 256 x 64, each
    schedule under FP64 atomics, colouring and (P1) owner computes."""
    out = {}
    A, C, O = exm.EXM_RACE_ATOMIC, exm.EXM_RACE_COLOUR, exm.EXM_RACE_OWNER
    P, T, D, G = exm.EXM_SCHED_PIPELINED, exm.EXM_SCHED_TILED, exm.EXM_SCHED_DIRECT, exm.EXM_SCHED_GATHER
    for name, (nb, lam), cases in (
            ("P1", (512, 100), [("pipelined_atomic", dict(schedule=P, race=A, tile_cells=64, chunk_layers=16)),
                                ("pipelined_colour", dict(schedule=P, race=C, tile_cells=64, chunk_layers=16)),
                                ("pipelined_owner", dict(schedule=P, race=O, tile_cells=64, chunk_layers=16)),
                                ("direct_atomic", dict(schedule=D, race=A, cols_per_wave=1, waves_per_block=4)),
                                ("direct_colour", dict(schedule=D, race=C, cols_per_wave=1, waves_per_block=4)),
                                ("gather_owner", dict(schedule=G, waves_per_block=4))]),
            ("P2", (256, 64), [("pipelined_atomic", dict(schedule=P, race=A, tile_cells=32, chunk_layers=8)),
                               ("pipelined_colour", dict(schedule=P, race=C, tile_cells=32, chunk_layers=8)),
                               ("tiled_atomic", dict(schedule=T, race=A, tile_cells=8, cols_per_wave=1)),
                               ("tiled_colour", dict(schedule=T, race=C, tile_cells=8, cols_per_wave=1)),
                               ("direct_atomic", dict(schedule=D, race=A, cols_per_wave=1, waves_per_block=4)),
                               ("direct_colour", dict(schedule=D, race=C, cols_per_wave=1, waves_per_block=4))])):
        e = W.extruded(nb, lam)
        V = e.space(name)
        x = W.device_values(V.n_dofs, meshgen.SEED_FIELD)
        y = V.zeros()
        b = W.mass_bytes(e, name)
        res = {"colours_cells": e.mesh.colours()}
        for label, opts in cases:
            t, tm = timed(torch, lambda: W.run_mass(e, name, x, y, **opts), 10)
            res[label] = {"ms": round(t, 4), "mean_ms": round(tm, 4), "gbs": round(b["algorithmic"] / t / 1e6, 1),
                          "launch": exm.par_loop_config(exm.EXM_K_MASS, e.mesh, e.X, e.Vx,
                                                        W.mass_args(e, name, x, y), **opts)}
        res["owner"] = "P1 only: there is no owner plan over edges" if name == "P2" else "vertex tiles"
        out[f"{name}_{nb}x{nb}x{lam}"] = res
        log(f"races {name}: " + ", ".join(f"{k} {v['ms']:.3f}" for k, v in res.items() if isinstance(v, dict)))
        del x, y, e
        torch.cuda.empty_cache()
    return out


def layer_points(torch, exm, W, meshgen):
    """Throughput against the layer count at a constant ~52.4 M prisms (the
    base shrinking as the columns grow: n = 512 sqrt(100 / lambda)) and
    against a random base ordering at 100 layers, P1 and DG0 RHS, each the
    fastest of a fixed set of PIPELINED launches (the full sweep with the
    autotuner is ``bench.py --sweep``)."""
    import numpy as np
    out = {}
    A = exm.EXM_RACE_ATOMIC
    shapes = {"P1": [(64, 16), (64, 8), (128, 8), (256, 8)],
              "DG0": [(32, 32), (32, 16), (64, 16), (50, 20), (38, 26), (30, 34)]}
    for lam, order in ((20, "rcm"), (50, "rcm"), (200, "rcm"), (100, "random")):
        n = 512 if order == "random" else int(round(512 * np.sqrt(100.0 / lam)))
        t0 = time.time()
        e = W.extruded(n, lam, order=order)
        pt = {"base": f"{n}x{n}", "n_layers": lam, "order": order, "n_prisms": e.n_prisms}
        for name in ("P1", "DG0"):
            V = e.space(name)
            x = W.device_values(V.n_dofs, meshgen.SEED_FIELD)
            y = V.zeros()
            b = W.mass_bytes(e, name)
            best = min((timed(torch, lambda: W.run_mass(e, name, x, y, schedule=exm.EXM_SCHED_PIPELINED, race=A,
                                                       tile_cells=tc, chunk_layers=S), 10)[0], tc, S)
                       for tc, S in shapes[name])
            pt[name] = {"ms": round(best[0], 4), "gbs": round(b["algorithmic"] / best[0] / 1e6, 1),
                        "tile_cells": best[1], "chunk_layers": best[2]}
            del x, y
        pt["setup_s"] = round(time.time() - t0, 1)
        out[f"lambda{lam}_{order}"] = pt
        log(f"layer point {n}x{n}x{lam} {order}: P1 {pt['P1']['gbs']:.0f} GB/s, DG0 {pt['DG0']['gbs']:.0f} GB/s")
        del e
        torch.cuda.empty_cache()
    return out


def matrix_figures(torch, exm, W, meshgen):
    """Mass matrix and cubic Jacobian of P1 x P1 on 512 x 512 x 100 in the
    vertically aligned layout: assembly, product with the matrix, and the
    matrix-free action of the column loop beside it."""
    em = W.extruded(512, 100)
    V = em.Vx
    M = exm.Matrix(V)
    n = V.n_dofs
    t_asm, _ = timed(torch, lambda: M.assemble(exm.EXM_K_MASS, em.X, V), 5)
    x = W.device_values(n, meshgen.SEED_FIELD)
    y = V.zeros()
    t_mv, _ = timed(torch, lambda: M.spmv(x, y), 10)
    cfg = exm.autotune(exm.EXM_K_MASS, em.mesh, em.X, V, W.mass_args(em, "P1", x, y))
    t_mf, _ = timed(torch, lambda: W.run_mass(em, "P1", x, y, **cfg), 10)
    u = W.device_values(n, 31)
    t_jac, _ = timed(torch, lambda: M.assemble(exm.EXM_K_CUBIC_JAC, em.X, V, u=u), 3)
    n_classes = em.base.n_vertices
    stored = 8 * M.n_stored
    pattern = 4 * M.n_pattern + 12 * n_classes
    spmv_bytes = stored + pattern + 16 * n               # values, pattern, x, y
    csr_bytes = 12 * M.nnz + 8 * (n + 1) + 16 * n         # what a CSR product moves
    # values written once, coordinates, the contribution lists (cell, nodes: 8 B per element-matrix entry)
    asm_bytes = stored + W.coord_bytes(em) + 8 * 36 * em.base.n_cells + 8 * (M.n_pattern + 1)
    r = {"nnz": M.nnz, "stored_values": M.n_stored, "pattern": M.n_pattern,
         "assemble_mass_ms": round(t_asm, 3), "assemble_gbs": round(asm_bytes / t_asm / 1e6, 1),
         "assemble_cubic_jacobian_ms": round(t_jac, 3),
         "spmv_ms": round(t_mv, 4), "spmv_gbs": round(spmv_bytes / t_mv / 1e6, 1),
         "spmv_bytes_vs_csr": round(spmv_bytes / csr_bytes, 3),
         "matrix_free_ms": round(t_mf, 4), "matrix_free_launch": cfg}
    log(f"matrix: assemble {t_asm:.2f} ms, jacobian {t_jac:.2f} ms, spmv {t_mv:.3f} ms "
        f"({r['spmv_gbs']} GB/s), matrix-free {t_mf:.3f} ms")
    del M, x, y, u, em
    torch.cuda.empty_cache()
    return r


def batch_items(torch, exm, W, meshgen):
    """The batch workload: 64 meshes (half P1, half DG0), 8 fields and 8
    cotangents each, seeded; with the algorithmic bytes of one replay for
    the P1 and the DG0 items: 8 fields x (forward + adjoint), input read and
    output written once, z and (x, y) once, and the P1 fans (vertex offsets
    and neighbours) or the DG0 lists once."""
    gen = torch.Generator(device="cuda")
    gen.manual_seed(meshgen.SEED_BATCH)
    items = []
    by = {True: 0, False: 0}
    for it in meshgen.batch_meshes(n_meshes=64):
        mesh = exm.Mesh(it.mesh, it.n_layers)
        Vx = exm.Space(mesh, "P1")
        V = exm.Space(mesh, it.space) if it.space != "P1" else Vx
        X = exm.coordinate_field(Vx, meshgen.extruded_vertex_coords(it.mesh, it.n_layers))
        rnd = lambda: torch.rand(V.n_dofs, dtype=torch.float64, device="cuda", generator=gen) * 2 - 1
        items.append(dict(space=V, coord_space=Vx, coords=X, mesh=mesh, name=it.space,
                          f=[rnd() for _ in range(8)], b=[V.zeros() for _ in range(8)],
                          w=[rnd() for _ in range(8)], g=[V.zeros() for _ in range(8)]))
        n = V.n_dofs
        p1 = it.space == "P1"
        by[p1] += 16 * (8 * n + 8 * n) + 8 * Vx.n_dofs + 16 * it.mesh.n_vertices \
            + (4 * (it.mesh.n_vertices + 1) + 8 * it.mesh.n_edges if p1 else 28 * it.mesh.n_cells)
    return items, by[True], by[False]


def batch_vs_plain(torch, exm, W, meshgen):
    """64 meshes (half P1, half DG0), 8 fields each: the batched forward +
    adjoint graph against the 1024 individual launches, same GPU, with the
    library's default launch and with the fastest single-launch schedule of
    each space at these layer counts (PIPELINED for both: ATOMIC 64-cell tiles
    of 16-layer chunks for P1, 32-cell tiles for DG0)."""
    t0 = time.time()
    items, bytes_p1, bytes_dg0 = batch_items(torch, exm, W, meshgen)
    total_bytes = bytes_p1 + bytes_dg0
    log(f"batch setup {time.time() - t0:.1f}s")
    t0 = time.time()
    B = exm.Batch(items)
    log(f"batch create (autotuned, captured) {time.time() - t0:.1f}s, units/blocks {B.info()}, tiles P1 {B.tiles('P1')} DG0 {B.tiles('DG0')}")
    t_batch, _ = timed(torch, B.launch, 5)

    def plain(best):
        for d in items:
            if best:
                opts = dict(schedule=exm.EXM_SCHED_PIPELINED, race=exm.EXM_RACE_ATOMIC, tile_cells=64,
                            chunk_layers=16) if d["name"] == "P1" else \
                    dict(schedule=exm.EXM_SCHED_PIPELINED, tile_cells=32, chunk_layers=16)
            else:
                opts = {}
            for src, dst in ((d["f"], d["b"]), (d["w"], d["g"])):
                for x, y in zip(src, dst):
                    if d["name"] == "P1":
                        y.zero_()
                        acc = exm.EXM_INC
                    else:
                        acc = exm.EXM_WRITE
                    exm.par_loop(exm.EXM_K_MASS, d["mesh"], d["coords"], d["coord_space"],
                                 [(x, d["space"], exm.EXM_READ), (y, d["space"], acc)], **opts)
    t_plain, _ = timed(torch, lambda: plain(False), 3)
    t_best, _ = timed(torch, lambda: plain(True), 3)
    log(f"batch {t_batch:.3f} ms vs individual {t_plain:.3f} ms (default launch), {t_best:.3f} ms (best schedule)")
    res = {"meshes": len(items), "fields_per_mesh": 8, "batched_ms": round(t_batch, 3),
           "individual_launches_ms": round(t_plain, 3), "batched_speedup": round(t_plain / t_batch, 3),
           "individual_best_schedule_ms": round(t_best, 3), "batched_speedup_vs_best": round(t_best / t_batch, 3),
           "batched_gbs": round(total_bytes / t_batch / 1e6, 1), "tiles_p1": list(B.tiles("P1")),
           "tiles_dg0": list(B.tiles("DG0"))}
    del items, B
    torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    main()
