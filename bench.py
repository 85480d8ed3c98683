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
# FP64 operations of one mode-step (an FMA counts 2): q (2 adds), x (2 FMA), the two series of
# degree D (2 D FMA), S q (3 mul), and the rotation of two 2x2 blocks (8 outputs x (1 mul + 3 FMA)).
def flop_per_mode_step(degree):
    return 2 + 4 + 4 * degree + 3 + 56


def series_degree(A, edge, spec, grid, torch):
    """Series degree the evolution kernel selects for this table (same bound as the kernel)."""
    amax = float(torch.max(torch.sqrt((A ** 2).sum(-1))).item())
    amax = max(amax, float(torch.max(torch.sqrt((edge ** 2).sum(-1))).item()))
    pm = [max(abs(grid["lo"][d]), abs(grid["hi"][d])) for d in range(3)]
    dt = spec["T"] / spec["nt"]
    pr = math.hypot(pm[0], pm[1]) + amax
    xb = (pr * pr + 1.0 + pm[2] ** 2) * dt * dt * (1.0 + 1e-6)
    return 6 if xb <= 0.14 else 7


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-modes", type=int, default=4096)
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
    w = W.de_generation(args.seed)
    spec, grid = w["specs"][0], w["grids"][0]
    N = len(w["specs"])
    D = 4 * spec["n_s"]
    prm = api.de_params(N, D, spec["n_s"], F=w["F"], CR=w["CR"], seed=args.seed + 1)
    pop = torch.as_tensor(w["coeff"].reshape(N, D), dtype=torch.float64, device="cuda").contiguous()
    A, edge, _, _ = api.synth(w["specs"], pop)
    degree = series_degree(A, edge, spec, grid, torch)
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
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_modes)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
