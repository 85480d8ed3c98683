"""Benchmark of the pair-yield hot path on one MI355X.

A step is one plain differential-evolution generation of the DE-generation workload
(64 pulses, 2x(8+8) cubic B-spline coefficients, T = 800, nt = 16384, peak |E| = 0.1,
64x64x16 momentum modes over px,py in [-2,2], pz in [-1,1], F = 0.8, CR = 0.9):
propose -> pulse synthesis -> per-mode evolution and projection -> yield -> selection, all
through one po_de_generation call of the C ABI on torch's current stream, inputs resident in
HBM.  Prints one JSON line.

The roofline object describes the per-mode evolution kernel (the dominant kernel): its
launches are bracketed by HIP events inside the library (po_timer_*), on the stream the kernel
runs on.  The CPU baseline runs the plain oracle (test infrastructure) on a bounded sample of
the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector: 256 CU x 128 FLOP/clk x 2.4 GHz
# Series variants of the evolution kernel: tan(sqrt x)/sqrt x of degree n for (omega dt)^2 <= x_n.
TAN_DEGREES = (6, 8, 10, 13, 19)
TAN_XMAX = (0.0099, 0.0337, 0.0735, 0.1558, 0.3552)


def flop_per_mode_step(degree):
    """FP64 operations of one mode-step of the tangent-form step (an FMA counts 2): q (2 adds),
    x = |q|^2 (2 FMA), the series of degree n (n FMA), T q (3 mul), and 1 - i T Q applied to two
    2x2 blocks (8 real components x 3 FMA)."""
    return 2 + 4 + 2 * degree + 3 + 48


def series_degree(A, edge, spec, grid, torch):
    """Series degree the evolution kernel selects for this table (the kernel's own bound), or None
    when the large-step path applies."""
    amax = float(torch.max(torch.sqrt((A ** 2).sum(-1))).item())
    amax = max(amax, float(torch.max(torch.sqrt((edge ** 2).sum(-1))).item()))
    pm = [max(abs(grid["lo"][d]), abs(grid["hi"][d])) for d in range(3)]
    dt = spec["T"] / spec["nt"]
    pr = math.hypot(pm[0], pm[1]) + amax
    xb = (pr * pr + 1.0 + pm[2] ** 2) * dt * dt * (1.0 + 1e-6)
    for n, x in zip(TAN_DEGREES, TAN_XMAX):
        if xb <= x:
            return n
    return None


def cpu_baseline(w, sample_modes):
    import numpy as np
    import oracle
    from paper_1704_08919_amd import workloads as W

    spec, grid, coeff = w["specs"][0], w["grids"][0], w["coeff"][0]
    p, _ = oracle.grid_points(grid)
    p = p[:sample_modes]
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    t0 = time.perf_counter()
    A, _, edge, _ = oracle.synth(spec, coeff, precision="d", with_E=False)
    f = oracle.evolve_points(A, edge, spec["T"] / spec["nt"], p, precision="d", nthreads=threads)
    dt = time.perf_counter() - t0
    assert np.all(np.isfinite(f))
    ms = sample_modes * spec["nt"]
    return {"value": ms / dt, "unit": "mode-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"pulse 0 of {w['name']}: synthesis + first {sample_modes} of {W.n_modes(grid)} modes, "
                      f"all {spec['nt']} steps ({ms:.3e} mode-steps, {dt:.1f} s, double build, OpenMP)"}


def uneven_batch(api, W, torch, uniform_rate, reps=3):
    """256 pulses of uneven nt and grids through one autotuned plan (persistent queue, HIP graph)."""
    w = W.uneven_batch(0)
    specs, grids = w["specs"], w["grids"]
    t0 = time.perf_counter()
    plan = api.Plan(specs, grids, config=None)
    tune_s = time.perf_counter() - t0
    coeff = torch.as_tensor(w["coeff"].ravel(), dtype=torch.float64, device="cuda")
    J = torch.empty(len(specs), dtype=torch.float64, device="cuda")
    plan.evaluate(coeff, J)  # captures the graph
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        plan.evaluate(coeff, J)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
    ms_total = W.mode_steps(specs, grids)
    rate = ms_total / (ms / 1e3)
    cfg = plan.config
    plan.close()
    return {"workload": w["name"], "mode_steps": ms_total, "ms_per_evaluation": ms, "mode_steps_per_s": rate,
            "plan": cfg, "autotune_s": tune_s, "rate_vs_uniform_batch": rate / uniform_rate,
            "timing": "HIP events on torch's current stream around graph replays"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-modes", type=int, default=65536)
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-batch plan measurement")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 512 MiB device copy first (reference for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU layout is a design "
              "note, not a build target", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1704_08919_amd import api
    from paper_1704_08919_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(64 * 2 ** 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = W.de_generation(args.seed)
    spec, grid = w["specs"][0], w["grids"][0]
    N = len(w["specs"])
    D = 4 * spec["n_s"]
    prm = api.de_params(N, D, spec["n_s"], F=w["F"], CR=w["CR"], seed=args.seed + 1)
    pop = torch.as_tensor(w["coeff"].reshape(N, D), dtype=torch.float64, device="cuda").contiguous()
    A, edge, _, _ = api.synth(w["specs"], pop)
    degree = series_degree(A, edge, spec, grid, torch)
    assert degree is not None, "workload left the tangent-series range"
    del A, edge
    fit, _ = api.evaluate(w["specs"], w["grids"], pop)
    trial = torch.empty_like(pop)
    tfit = torch.empty_like(fit)
    for g in range(args.warmup):
        api.po_de_generation(prm, g, spec, grid, pop, fit, trial, tfit)
    torch.cuda.synchronize()
    api.po_timer_read()
    api.po_timer_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in range(args.warmup, args.warmup + args.steps):
        api.po_de_generation(prm, g, spec, grid, pop, fit, trial, tfit)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.po_timer_enable(False)
    evolve_ms, calls = api.po_timer_read()
    elapsed = t1 - t0
    mode_steps = W.mode_steps(w["specs"], w["grids"])
    value = mode_steps * args.steps / elapsed
    ev_s = evolve_ms / 1e3 / max(calls, 1)
    fps = flop_per_mode_step(degree)
    achieved = fps * mode_steps / ev_s / 1e12
    best = float(fit.max().item())
    out = {
        "metric": "mode-steps/s (FP64)",
        "value": value,
        "unit": "mode-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "pulses": N, "modes_per_pulse": W.n_modes(grid), "nt": spec["nt"],
                   "mode_steps_per_step": mode_steps, "step": "one DE generation (propose, synthesis, evolution, "
                   "yield, select) via po_de_generation"},
        "de_generations_per_s": args.steps / elapsed,
        "evolve_ms_per_call": ev_s * 1e3,
        "evolve_mode_steps_per_s": mode_steps / ev_s,
        "best_J": best,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_evolve (per-mode evolution + projection)", "flop_per_mode_step": fps,
                     "series_degree": degree},
    }
    if not args.no_uneven:
        out["uneven_batch"] = uneven_batch(api, W, torch, mode_steps / ev_s)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_modes)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
