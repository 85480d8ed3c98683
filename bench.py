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
# The fixed per-mode-step count of a degree-8 cos/sin step (C - i S Q on two blocks), kept beside
# the count of the step actually required for reference.
FIXED_FLOP_PER_MODE_STEP = 97
# FP64 operations of one mode-step per series variant of the evolution kernel (an FMA counts 2).
# tan(theta)/theta polynomial of degree n: q (2 adds), x = |q|^2 (2 FMA), the polynomial (n FMA), T q
# (3 mul), and 1 - i T Q on two 2x2 blocks (8 real components x 3 FMA) = 57 + 2n.
# cos/sin of degree 7 (large steps): q, x, two series (14 FMA), S q, and C - i S Q on two blocks
# (8 x (1 mul + 3 FMA)) = 93, plus 6 per angle halving (not counted: a lower bound).
FLOP_PER_MODE_STEP = {"tan4": 65, "tan5": 67, "tan6": 69, "tan7": 71, "tan8": 73, "tan9": 75, "tan10": 77,
                      "tan11": 79, "cossin7_halving": 93}
HERE_PROFILES = os.path.join(ROOT, "profiles")
# launch shape of the plans used by the surrogate sections (fixed, so no autotuning is timed)
PLAN = dict(threads=256, modes_per_lane=1, persistent=1)


EVOLVE_SOURCES = ("evolve.hip", "dirac.hpp", "tan_fit.hpp", "reduce.hpp", "common.hpp")


def code_lines(text):
    """The lines of a C++ source without // comments, trailing blanks and empty lines (the
    evolution sources hold no block comments and no '//' inside string literals)."""
    out = []
    for line in text.splitlines():
        code = line.split("//", 1)[0].rstrip()
        if code:
            out.append(code)
    return "\n".join(out) + "\n"


def evolve_sources_sha256():
    """Hash of the code (comments left out) the evolution kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for name in EVOLVE_SOURCES:
        with open(os.path.join(ROOT, "paper_1704_08919_amd", "csrc", name), encoding="utf-8") as fh:
            h.update(code_lines(fh.read()).encode())
    return h.hexdigest()


def fp64_counter_record():
    """Measured FP64 work of one evolution call (rocprof counters) from the committed record, if
    taken on the evolution kernel's sources as they are now (else None)."""
    path = os.path.join(HERE_PROFILES, "k_evolve_fp64_counters_de_generation.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
        sha = evolve_sources_sha256()
    except OSError:
        return None
    return rec if rec.get("evolve_sources_sha256") == sha else None


def hbm_traffic_record():
    """HBM bytes per evolution call from the committed counter summary, if it was taken on the
    evolution kernel's sources as they are now (else None)."""
    path = os.path.join(HERE_PROFILES, "k_evolve_hbm_traffic_de_generation.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
        sha = evolve_sources_sha256()
    except OSError:
        return None
    return rec if rec.get("evolve_sources_sha256") == sha else None


def cpu_extrapolations(threads, sample_modes):
    """The same oracle build on one pulse of the uneven batch (its largest), of the full
    surrogate-DE workload and of the surrogate training data, extrapolated to each workload's unit
    of work: the evolution of the first sample_modes modes for all steps, linearly in mode-steps
    (modes and pulses are independent), plus the pulse's synthesis times the number of pulses (in
    the uneven batch weighted by (nt / nt_sampled)^2: lines and steps both grow with T at fixed
    dt)."""
    import numpy as np
    import oracle
    from paper_1704_08919_amd import workloads as W

    ub = W.uneven_batch(0)
    k = max(range(len(ub["specs"])), key=lambda i: ub["specs"][i]["nt"] * W.n_modes(ub["grids"][i]))
    spec5, grid5 = W.surrogate_de_spec()
    spec4, grid4 = W.surrogate_data_spec()
    nt_k = ub["specs"][k]["nt"]
    cases = [(ub["name"], "one evaluation of the 256-pulse batch", ub["specs"][k], ub["grids"][k], ub["coeff"][k],
              W.mode_steps(ub["specs"], ub["grids"]), sum((s["nt"] / nt_k) ** 2 for s in ub["specs"]),
              f"pulse {k} (the largest)"),
             ("surrogate_de_full_pop512_128x128x32_nt32768", "one plain DE generation (512 pulses)", spec5, grid5,
              W.draw_coeff(0, 1, spec5["n_s"])[0], 512 * spec5["nt"] * W.n_modes(grid5), 512.0, "one pulse"),
             ("surrogate_data_100k_T400_nt4096_64x64x16", "the 100,000-pulse training set", spec4, grid4,
              W.draw_coeff(0, 1, spec4["n_s"])[0], 100000 * spec4["nt"] * W.n_modes(grid4), 100000.0, "one pulse")]
    out = []
    for name, unit, spec, grid, coeff, total, synth_scale, which in cases:
        p, _ = oracle.grid_points(grid)
        p = p[:sample_modes]
        t0 = time.perf_counter()
        A, _, edge, _ = oracle.synth(spec, coeff, precision="d_fast", with_E=False)
        t1 = time.perf_counter()
        f = oracle.evolve_points(A, edge, spec["T"] / spec["nt"], p, precision="d_fast", nthreads=threads)
        t2 = time.perf_counter()
        assert np.all(np.isfinite(f))
        rate = len(p) * spec["nt"] / (t2 - t1)
        out.append({"workload": name, "unit": unit, "mode_steps_per_unit": total, "evolution_mode_steps_per_s": rate,
                    "synthesis_s_sampled_pulse": t1 - t0,
                    "s_per_unit_extrapolated": total / rate + synth_scale * (t1 - t0),
                    "sample": f"{which}: synthesis, then the first {len(p)} of {W.n_modes(grid)} modes for all "
                              f"{spec['nt']} steps ({t2 - t1:.1f} s)"})
    return out


def cpu_baseline(w, sample_modes, sample_pulses):
    import numpy as np
    import oracle
    from paper_1704_08919_amd import workloads as W

    from oracle import build as oracle_build

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    ms, dt = 0, 0.0
    for i in range(sample_pulses):
        spec, grid, coeff = w["specs"][i], w["grids"][i], w["coeff"][i]
        p, _ = oracle.grid_points(grid)
        p = p[:sample_modes]
        t0 = time.perf_counter()
        A, _, edge, _ = oracle.synth(spec, coeff, precision="d_fast", with_E=False)
        f = oracle.evolve_points(A, edge, spec["T"] / spec["nt"], p, precision="d_fast", nthreads=threads)
        dt += time.perf_counter() - t0
        assert np.all(np.isfinite(f))
        ms += len(p) * spec["nt"]
    n_modes = W.n_modes(w["grids"][0])
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next(line.split(":", 1)[1].strip() for line in fh if line.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": ms / dt, "unit": "mode-steps/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu, "host_cpus": os.cpu_count(),
            "extrapolated": guarded(cpu_extrapolations, threads, max(1, sample_modes // 4)),
            "build_flags": " ".join(oracle_build.FAST_FLAGS),
            "sample": f"pulses 0..{sample_pulses - 1} of {w['name']}: synthesis + first "
                      f"{min(sample_modes, n_modes)} of {n_modes} modes each, all {w['specs'][0]['nt']} steps "
                      f"({ms:.3e} mode-steps, {dt:.1f} s, the oracle's double-precision 4x4 evolution, "
                      f"OpenMP over modes)"}


def guarded(fn, *a):
    """Optional sections report their failure instead of losing the whole line."""
    try:
        return fn(*a)
    except Exception as e:  # noqa: BLE001
        return {"error": f"{type(e).__name__}: {e}"}


def fma_probe(api, torch, waves=(4, 5, 6, 8), chains=(2, 4, 8), iters=4096):
    """FP64 FMA issue rate with exactly w waves per SIMD and c independent chains per lane (the
    ceiling the evolution kernel's FP64 rate is read against), as a fraction of the 78.6 TFLOP/s
    peak; HIP events on the stream the probe runs on (torch's current stream)."""
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    sink = torch.empty(n_cu * max(waves) * 256, dtype=torch.float64, device="cuda")
    rows = []
    for w in waves:
        for c in chains:
            api.po_probe_fp64_fma(w, c, 64, sink)  # warm-up
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            flop = api.po_probe_fp64_fma(w, c, iters, sink)
            e1.record()
            torch.cuda.synchronize()
            tf = flop / (e0.elapsed_time(e1) * 1e-3) / 1e12
            rows.append({"waves_per_simd": w, "chains": c, "tflops": tf, "frac_of_peak": tf / FP64_PEAK_TFLOPS})
    return {"what": "v_fma_f64 chains, exactly w waves per SIMD on every CU", "rows": rows,
            "best_frac_at_4_waves": max(r["frac_of_peak"] for r in rows if r["waves_per_simd"] == 4),
            "best_frac": max(r["frac_of_peak"] for r in rows)}


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


def surrogate_training(api, W, S, torch, n=100000, n_train=90000, epochs=20, seed=11):
    """Surrogate data and training: n (coefficients, J) pairs from the plain evaluator (T = 400,
    nt = 4096, 64x64x16 modes), network 32 -> 3 x 256 GELU -> 1 trained with Adam lr 1e-3, batch
    1024; held-out error in decades of J."""
    import numpy as np
    spec, grid = W.surrogate_data_spec()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, J = S.generate_dataset(spec, grid, n, seed=seed, batch=1024, plan_config=PLAN)
    gen_s = time.perf_counter() - t0
    net = api.MLP(32, 256, 3, max_batch=1024, seed=seed + 1)
    t1 = time.perf_counter()
    mean, std, loss = S.train(net, X, J, n_train, epochs=epochs, batch=1024, seed=seed + 2)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    steps = epochs * (n_train // 1024)
    pred = S.predict(net, X[n_train:], n - n_train).cpu().numpy().astype(np.float64) * std + mean
    truth = np.log10(np.maximum(J[n_train:, 0].cpu().numpy(), 1e-300))
    rmse = float(np.sqrt(np.mean((pred - truth) ** 2)))
    r2 = float(1.0 - np.mean((pred - truth) ** 2) / np.var(truth))
    net.close()
    flop_step = 3 * 2 * 1024 * (32 * 256 + 2 * 256 * 256 + 256)  # forward + backward GEMM work
    return {"workload": f"{n} pulses, T=400, nt=4096, 64x64x16 modes", "generate_s": gen_s,
            "generate_mode_steps_per_s": n * 4096 * 65536 / gen_s, "train_s": train_s, "train_steps": steps,
            "train_steps_per_s": steps / train_s, "train_tflops_bf16": flop_step * steps / train_s / 1e12,
            "final_train_loss": loss, "heldout": n - n_train, "heldout_rmse_log10J": rmse, "heldout_r2": r2,
            "log10J_mean": mean, "log10J_std": std}


def surrogate_de(api, W, S, torch, pop=512, generations=200, seed=0):
    """Surrogate-screened DE against plain DE and random screening, same seed and initial
    population, evaluator of the surrogate-data workload (T = 400, nt = 4096, 64x64x16 modes)."""
    spec, grid = W.surrogate_data_spec()
    plain = S.run_de(spec, grid, pop, generations, seed, mode="plain", plan_config=PLAN)
    target = 0.99 * plain["best_J"]
    out = {"workload": f"pop {pop}, T=400, nt=4096, 64x64x16 modes, top 10% evaluated, retrain every 20",
           "plain": {k: plain[k] for k in ("generations", "wall_s", "plain_evaluations", "best_J")},
           "target_J": target, "plain_time_to_target_s": S.time_to_reach(plain["history"], target)}
    for mode in ("surrogate", "random"):
        r = S.run_de(spec, grid, pop, 10 * generations, seed, mode=mode, time_limit=plain["wall_s"], target=target,
                     plan_config=PLAN)
        tt = S.time_to_reach(r["history"], target)
        out[mode] = {k: r[k] for k in ("generations", "wall_s", "plain_evaluations", "best_J", "train_s")}
        out[mode]["time_to_target_s"] = tt
        out[mode]["speedup_vs_plain_wall"] = plain["wall_s"] / tt if tt else None
    return out


def surrogate_de_full(api, W, S, torch, phase, generations, seed=0, target_J=None, plain_wall_s=None, run_in=None,
                      run_out=None, time_budget_s=None, surrogate_limit_s=None):
    """Surrogate-assisted DE at the full configuration (pop 512, 2x(8+8) coefficients, T = 800,
    nt = 32768, 128x128x32 modes), one phase per process (a plain generation takes ~10 s).

    phase "plain": plain DE up to `generations`, resumable: the state in run_in/plain_seed<seed>.npz
    (if present) is continued, at most time_budget_s seconds are run in this process, and the new
    state plus every trial and its J of the generations run here are written to run_out.
    phase "surrogate": the screened DE from the same seed and initial population until the best J
    reaches target_J (0.99 of the plain run's best) or surrogate_limit_s (default plain_wall_s)
    passes.  Before its clock starts it times one plain evaluation of the 512-pulse population on
    this GPU, so the plain run's wall time can be compared on the same device.  Prints progress
    every generation."""
    import numpy as np
    spec, grid = W.surrogate_de_spec()
    pop = 512
    per_gen = pop * W.n_modes(grid) * spec["nt"]
    out = {"workload": f"surrogate_de_full: pop {pop}, T=800, nt=32768, 128x128x32 modes, seed {seed}",
           "phase": phase, "mode_steps_per_plain_generation": per_gen}
    if phase == "plain":
        state_name = f"plain_seed{seed}.npz"
        resume = None
        if run_in and os.path.exists(os.path.join(run_in, state_name)):
            with np.load(os.path.join(run_in, state_name)) as z:
                resume = {k: z[k] for k in z.files}
        record = []
        r = S.run_de(spec, grid, pop, generations, seed, mode="plain", plan_config=PLAN, progress_every=1,
                     resume=resume, time_budget=time_budget_s, record=record)
        done = r["generations"]
        out.update({k: r[k] for k in ("generations", "wall_s", "plain_evaluations", "best_J")})
        out["generations_this_process"] = len(record)
        out["s_per_generation"] = r["wall_s"] / (done + 1)  # + the initial population
        out["mode_steps_per_s"] = per_gen * (done + 1) / r["wall_s"]
        out["complete"] = done >= generations
        if out["complete"]:
            out["target_J_next_phase"] = 0.99 * r["best_J"]
            out["plain_time_to_target_s"] = S.time_to_reach(r["history"], 0.99 * r["best_J"])
        if run_out:
            os.makedirs(run_out, exist_ok=True)
            np.savez(os.path.join(run_out, state_name), pop=r["final_pop"], fit=r["final_fit"],
                     generation=np.int64(done), evals=np.int64(r["plain_evaluations"]),
                     history=np.asarray(r["history"], dtype=np.float64), wall_s=np.float64(r["wall_s"]))
            if record:
                g0, g1 = record[0][0], record[-1][0]
                np.savez(os.path.join(run_out, f"plain_seed{seed}_trials_g{g0:03d}_{g1:03d}.npz"),
                         generation=np.asarray([g for g, _, _ in record], dtype=np.int64),
                         trials=np.stack([x for _, x, _ in record]).astype(np.float32),
                         J=np.stack([j for _, _, j in record]))
        hist = r["history"]
    else:
        ev = S.Evaluator(spec, grid, pop, PLAN)
        x = torch.as_tensor(W.draw_coeff(seed, pop, spec["n_s"]).reshape(pop, -1), dtype=torch.float64, device="cuda")
        ev(x)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        ev(x)
        torch.cuda.synchronize()
        out["plain_evaluation_512_s_this_gpu"] = time.perf_counter() - tc
        ev.close()
        limit = surrogate_limit_s if surrogate_limit_s else plain_wall_s
        r = S.run_de(spec, grid, pop, 10 * generations, seed, mode="surrogate", time_limit=limit,
                     target=target_J, plan_config=PLAN, progress_every=1)
        tt = S.time_to_reach(r["history"], target_J)
        out.update({k: r[k] for k in ("generations", "wall_s", "plain_evaluations", "best_J", "train_s")})
        out.update({"target_J": target_J, "plain_wall_s": plain_wall_s, "time_to_target_s": tt,
                    "speedup_vs_plain_wall": plain_wall_s / tt if tt else None})
        rc = r["rank_corr"]
        if rc:
            out["rank_corr_evaluated_trials"] = {"median": float(sorted(rc)[len(rc) // 2]),
                                                 "first_20_mean": sum(rc[:20]) / len(rc[:20]),
                                                 "last_20_mean": sum(rc[-20:]) / len(rc[-20:]),
                                                 "per_generation": [round(v, 3) for v in rc]}
        hist = r["history"]
    out["history_every_10"] = [list(h) for h in hist[::10]] + [list(hist[-1])]
    return out


def de_variants(api, W, torch, pop=64, generations=60, islands=4, migrate_every=5, seed=0):
    """Plain DE/rand/1/bin (F = 0.8, CR = 0.9, one population) against self-adaptive jDE on
    `islands` islands with ring migration every `migrate_every` generations (Sec. IV B), from the
    same initial population, on the surrogate-data evaluator (T = 400, nt = 4096, 64x64x16
    modes): best J per generation and generations per second, every step on the device."""
    spec, grid = W.surrogate_data_spec()
    D = 4 * spec["n_s"]
    x0 = W.draw_coeff(seed, pop, spec["n_s"]).reshape(pop, D)
    fit0, _ = api.evaluate([spec] * pop, [grid] * pop, x0)
    out = {"workload": f"pop {pop}, T=400, nt=4096, 64x64x16 modes, {generations} generations"}
    for name in ("plain", f"jde_islands{islands}"):
        P = torch.as_tensor(x0, dtype=torch.float64, device="cuda")
        fit = fit0.clone()
        trial, tfit = torch.empty_like(P), torch.empty_like(fit)
        best = []
        if name == "plain":
            prm = api.de_params(pop, D, spec["n_s"], F=0.8, CR=0.9, seed=seed + 1)
        else:
            prm = api.jde_params(pop, D, spec["n_s"], islands=islands, seed=seed + 1)
            fcr = torch.tensor([[0.8, 0.9]] * pop, dtype=torch.float64, device="cuda")
            tfcr = torch.empty_like(fcr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for g in range(generations):
            if name == "plain":
                api.po_de_generation(prm, g, spec, grid, P, fit, trial, tfit)
            else:
                api.po_jde_generation(prm, g, spec, grid, P, fit, fcr, trial, tfit, tfcr)
                if (g + 1) % migrate_every == 0:
                    api.po_island_migrate(prm, P, fit, fcr)
            best.append(float(fit.max().item()))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"generations_per_s": generations / dt, "best_J_first": best[0], "best_J_final": best[-1],
                     "best_J_every_10": best[9::10]}
    out["final_ratio_jde_over_plain"] = out[f"jde_islands{islands}"]["best_J_final"] / out["plain"]["best_J_final"]
    return out


def local_search(api, W, torch, starts=10, seed=0):
    """Multistart local search of Sec. IV A (BFGS + strong Wolfe on the augmented Lagrangian of
    the energy constraint, gradients from the discrete adjoint on the device): evaluations per
    start, J reached, and the cost of one gradient against one evaluation of J."""
    import numpy as np
    from paper_1704_08919_amd import localsearch as LS
    w = W.local_search(seed, starts=starts)
    specs, grids, c = w["specs"], w["grids"], w["coeff"]
    x0 = c.reshape(starts, -1)
    out = LS.run(specs, grids, x0, w["U_const"])
    res = out["results"]
    # cost of a gradient relative to an evaluation of J, same batch
    xs = np.stack([r["x"] for r in res])
    t = {}
    for name in ("J", "gradient"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            if name == "J":
                api.evaluate(specs, grids, xs)
            else:
                api.evaluate_gradient(specs, grids, xs)
        torch.cuda.synchronize()
        t[name] = (time.perf_counter() - t0) / 3
    ms = W.mode_steps(specs, grids)
    return {"workload": w["name"], "starts": starts, "wall_s": out["wall_s"],
            "evaluations_per_start": out["evaluations"].tolist(),
            "J_start": out["J_start"].tolist(), "J_final": [r["J"] for r in res],
            "constraint_violation_max": max(abs(r["U"] - w["U_const"]) / w["U_const"] for r in res),
            "outer_iterations": [r["outer"] for r in res], "bfgs_iterations": [r["iterations"] for r in res],
            "best_J": res[out["best"]]["J"], "J_eval_s": t["J"], "gradient_eval_s": t["gradient"],
            "gradient_over_J_cost": t["gradient"] / t["J"],
            "gradient_mode_steps_per_s": ms / t["gradient"]}


def cost_to_reach(rows, target):
    """Per method, the time per momentum point at which eps first reaches `target`: rows in
    increasing nt per method; log-log interpolation between the last row above the target and the
    first at or below it (that row's cost if the method's first usable row is already below).
    Unstable or unresolved rows (eps > 1) count as above the target and are not interpolated from;
    a method that never reaches the target is absent."""
    reach, prev = {}, {}
    for row in rows:
        m, us = row["method"], row["us_per_mode"]
        e = None if (row.get("unstable") or row.get("unresolved")) else row["eps"]
        if m not in reach and e is not None and e <= target:
            p = prev.get(m)
            if p is not None and p[1] is not None and p[1] > target:
                a = math.log(target / p[1]) / math.log(e / p[1])
                reach[m] = math.exp(math.log(p[0]) + a * (math.log(us) - math.log(p[0])))
            else:
                reach[m] = us
        prev[m] = (us, e)
    return reach


def solver_comparison(api, W, torch, n_p=512, nts=(5000, 10000, 20000, 50000, 100000, 200000, 500000, 1000000),
                      nt_exact=2_000_000, target=1e-3):
    """The paper's accuracy-versus-time comparison (Sec. V C) on the circular multimode pulse of its
    2-D study: error eps = int |f - f_exact| / int f_exact over the momentum sheet against the GPU
    time per momentum point, for the second-order Dirac step (exponential midpoint), the
    fourth-order Magnus step, the split-operator steps (Strang, second order, and its fourth-order
    triple-jump composition) and the kinetic equation with RK4; f_exact = fourth-order Magnus step
    at nt_exact.  A kinetic-equation row whose eps exceeds 1 (RK4 unstable for the fastest modes) is
    marked unstable, with eps null; a row of one of the unitary steps whose eps exceeds 1 keeps its
    eps and is marked unresolved (the step is too coarse for the fastest modes).  Only the solver
    call is timed (tables are built beforehand)."""
    w = W.circular_pulse(0, nt=nts[0], n_p=n_p)
    spec0, coeff, grid = w["specs"][0], w["coeff"], w["grids"][0]
    M = W.n_modes(grid)
    f = torch.empty(M, dtype=torch.float64, device="cuda")

    def prepare(method, nt):
        s = [dict(spec0, nt=nt)]
        if method == "dirac2":
            A, edge, _, _ = api.synth(s, coeff)
            return lambda: api.po_evolve_modes(s, [grid], A, edge, f=f)
        if method == "magnus4":
            _, _, Ag, edge, _ = api.field_samples(s, coeff, api.GAUSS2)
            return lambda: api.po_evolve_modes_m4(s, [grid], Ag, edge, f=f)
        if method == "split2":
            A, edge, _, _ = api.synth(s, coeff)
            return lambda: api.po_evolve_modes_split(s, [grid], 2, A, edge, f=f)
        if method == "split4":
            _, _, At, edge, _ = api.field_samples(s, coeff, api.SPLIT4_OFFSETS)
            return lambda: api.po_evolve_modes_split(s, [grid], 4, At, edge, f=f)
        E, Ed, A, _, _ = api.field_samples(s, coeff, api.QKE_OFFSETS, with_end=True)
        return lambda: api.po_qke_modes(s, [grid], E, Ed, A, f=f)

    def timed(method, nt):
        call = prepare(method, nt)
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        call()
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1)

    methods = ("dirac2", "magnus4", "split2", "split4", "qke")
    for method in methods:  # load code objects before timing
        timed(method, 1000)
    ms_exact = timed("magnus4", nt_exact)
    fe = f.clone()
    den = float(fe.sum().item())

    def eps():
        v = float((f - fe).abs().sum().item()) / den
        return v if math.isfinite(v) else None

    timed("dirac2", nt_exact)
    check = eps()
    rows = []
    for method in methods:
        for nt in nts:
            ms = timed(method, nt)
            e = eps()
            row = {"method": method, "nt": nt, "eps": e, "us_per_mode": ms * 1e3 / M,
                   "mode_steps_per_s": M * nt / (ms * 1e-3)}
            if e is None or e > 1.0:
                if method == "qke":
                    # RK4 outside its stability interval for the fastest modes: f grows without bound
                    row["eps"], row["unstable"] = None, True
                else:
                    # the unitary steps stay bounded; the step is too coarse for the fastest modes
                    row["unresolved"] = True
            rows.append(row)
    reach = cost_to_reach(rows, target)
    out = {"workload": w["name"], "modes": M, "nt_exact": nt_exact, "exact_ms": ms_exact,
           "exact_check_eps_dirac2": check, "target_eps": target, "rows": rows,
           "us_per_mode_to_target": reach}
    for m in ("magnus4", "split2", "split4", "qke"):
        if m in reach and "dirac2" in reach:
            out[f"{m}_over_dirac2_at_target"] = reach[m] / reach["dirac2"]
    if reach:
        out["cheapest_at_target"] = min(reach, key=reach.get)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-modes", type=int, default=65536)
    ap.add_argument("--cpu-sample-pulses", type=int, default=3)
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-batch plan measurement")
    ap.add_argument("--no-fma-probe", action="store_true", help="skip the FP64 FMA issue-rate probe")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate training and DE comparison")
    ap.add_argument("--no-de-variants", action="store_true", help="skip the plain DE versus jDE-on-islands run")
    ap.add_argument("--no-local-search", action="store_true", help="skip the multistart BFGS local search")
    ap.add_argument("--no-solvers", action="store_true",
                    help="skip the accuracy-versus-time comparison of the Dirac, Magnus and kinetic solvers")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 512 MiB device copy first (reference for HBM counter scaling)")
    ap.add_argument("--surrogate-de-full", choices=("plain", "surrogate"),
                    help="run only one phase of the full-configuration surrogate-DE comparison")
    ap.add_argument("--full-generations", type=int, default=80, help="plain-DE generations of that comparison")
    ap.add_argument("--target-J", type=float, help="surrogate phase: 0.99 x the plain phase's best J")
    ap.add_argument("--plain-wall-s", type=float, help="surrogate phase: the plain phase's wall time")
    ap.add_argument("--run-in", help="plain phase: directory holding the state to resume (plain_seed<seed>.npz)")
    ap.add_argument("--run-out", help="plain phase: directory for the new state and the recorded trials")
    ap.add_argument("--time-budget-s", type=float, help="plain phase: seconds of DE work in this process")
    ap.add_argument("--surrogate-limit-s", type=float,
                    help="surrogate phase: stop after this many seconds (default: the plain wall time)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1704_08919_amd import api
    from paper_1704_08919_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.surrogate_de_full:
        from paper_1704_08919_amd import surrogate as S
        if args.surrogate_de_full == "surrogate" and (args.target_J is None or args.plain_wall_s is None):
            ap.error("--surrogate-de-full surrogate needs --target-J and --plain-wall-s from the plain phase")
        print(json.dumps(surrogate_de_full(api, W, S, torch, args.surrogate_de_full, args.full_generations,
                                           args.seed, args.target_J, args.plain_wall_s, args.run_in, args.run_out,
                                           args.time_budget_s, args.surrogate_limit_s)), flush=True)
        return
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
    fit, _ = api.evaluate(w["specs"], w["grids"], pop)
    trial = torch.empty_like(pop)
    tfit = torch.empty_like(fit)
    for g in range(args.warmup):
        api.po_de_generation(prm, g, spec, grid, pop, fit, trial, tfit)
    torch.cuda.synchronize()
    api.po_timer_enable(True)
    api.po_timer_read()
    api.po_timer_mode_steps()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in range(args.warmup, args.warmup + args.steps):
        api.po_de_generation(prm, g, spec, grid, pop, fit, trial, tfit)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    evolve_ms, calls = api.po_timer_read()
    by_series = api.po_timer_mode_steps()
    api.po_timer_enable(False)
    elapsed = t1 - t0
    mode_steps = W.mode_steps(w["specs"], w["grids"])
    value = mode_steps * args.steps / elapsed
    ev_s = evolve_ms / 1e3 / max(calls, 1)
    counted = sum(by_series.values())
    assert counted == mode_steps * args.steps, (counted, mode_steps * args.steps)
    flops = sum(FLOP_PER_MODE_STEP[k] * v for k, v in by_series.items())
    achieved = flops / (evolve_ms / 1e3) / 1e12
    traffic = hbm_traffic_record()
    measured = fp64_counter_record()
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
                     "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": traffic["bytes_per_call"] if traffic else None,
                     "kernel": "k_evolve (per-mode evolution + projection)",
                     "flop_per_mode_step_avg": flops / counted, "mode_steps_by_series": by_series,
                     "flop_per_mode_step_measured": measured["flop_per_mode_step"] if measured else None,
                     "fp64_issue_frac": (measured["fp64_instr_per_mode_step"] * mode_steps / ev_s
                                         / (FP64_PEAK_TFLOPS * 1e12 / 2)) if measured else None,
                     "achieved_at_fixed_97_flop": FIXED_FLOP_PER_MODE_STEP * mode_steps / ev_s / 1e12},
    }
    if not args.no_fma_probe:
        out["fp64_fma_probe"] = guarded(fma_probe, api, torch)
    if not args.no_uneven:
        out["uneven_batch"] = guarded(uneven_batch, api, W, torch, mode_steps / ev_s)
    if not args.no_solvers:
        out["solver_comparison"] = guarded(solver_comparison, api, W, torch)
    if not args.no_de_variants:
        out["de_variants"] = guarded(de_variants, api, W, torch)
    if not args.no_local_search:
        out["local_search"] = guarded(local_search, api, W, torch)
    if not args.no_surrogate:
        from paper_1704_08919_amd import surrogate as S
        out["surrogate_training"] = guarded(surrogate_training, api, W, S, torch)
        out["surrogate_de"] = guarded(surrogate_de, api, W, S, torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_modes, args.cpu_sample_pulses)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
