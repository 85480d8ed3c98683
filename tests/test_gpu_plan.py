"""GPU tests of plans: persistent work-queue launches, launch-shape independence of the results,
HIP-graph capture and replay, autotuning and its cache, and the full-size uneven batch."""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1704_08919_amd import api  # noqa: E402
from paper_1704_08919_amd import workloads as W  # noqa: E402

from test_gpu_parity import assert_J, assert_modes, dev, host, say  # noqa: E402

CONFIGS = [dict(threads=256, modes_per_lane=1, persistent=0), dict(threads=256, modes_per_lane=1, persistent=1),
           dict(threads=256, modes_per_lane=2, persistent=1), dict(threads=128, modes_per_lane=2, persistent=1),
           dict(threads=64, modes_per_lane=1, persistent=1), dict(threads=64, modes_per_lane=2, persistent=1, workgroups=37)]


def small_uneven_batch(seed=0):
    r = W.rng(seed + 99)
    nts = [257, 1000, 2048, 640, 4096, 300, 1536, 900, 64, 2000, 1200, 3000]
    grids_all = [W.grid((17, 13, 3), (-1.3, -0.9, -0.7), (1.1, 1.4, 0.8)), W.sheet_grid(32, 32, 1.5),
                 W.box_grid(24, 24, 4), W.grid((5, 1, 1), (-0.5, 0.2, 0.0), (0.5, 0.2, 0.0))]
    specs, grids = [], []
    for i, nt in enumerate(nts):
        T = nt * 400.0 / 4096.0
        specs.append(W.pulse_spec(n_s=8, T=T, nt=nt, norm_value=float(r.uniform(0.05, 0.2))))
        grids.append(grids_all[i % len(grids_all)])
    return specs, grids, W.draw_coeff(seed, len(nts), 8)


def test_plans_match_default_launch_bitwise():
    specs, grids, coeff = small_uneven_batch()
    J0, f0 = api.evaluate(specs, grids, coeff, want_f=True)
    J0, f0 = host(J0), host(f0)
    dc = dev(coeff.ravel())
    for cfg in CONFIGS:
        say(f"plan config {cfg}")
        plan = api.Plan(specs, grids, config=cfg)
        got = plan.config
        assert got["threads"] == cfg["threads"] and got["modes_per_lane"] == cfg["modes_per_lane"]
        J = torch.empty(len(specs), dtype=torch.float64, device="cuda")
        f = torch.empty(api.n_modes(grids), dtype=torch.float64, device="cuda")
        plan.evaluate(dc, J, f)
        assert np.array_equal(host(J), J0), cfg
        assert np.array_equal(host(f), f0), cfg
        plan.close()


def test_plan_graph_replay_with_eager_work_between():
    specs, grids, coeff = small_uneven_batch(1)
    plan = api.Plan(specs, grids, config=dict(threads=128, modes_per_lane=1, persistent=1))
    dc = dev(coeff.ravel())
    J = torch.empty(len(specs), dtype=torch.float64, device="cuda")
    plan.evaluate(dc, J)
    first = host(J).copy()
    ref = host(api.evaluate(specs, grids, coeff)[0])
    assert np.array_equal(first, ref)
    for k in range(4):
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        J.zero_()
        plan.evaluate(dc, J)
        torch.cuda.synchronize()
        assert np.array_equal(host(J), first), k
        del junk
    # same pointers, new values: the replay reads the new coefficients
    coeff2 = W.draw_coeff(77, len(specs), 8)
    dc.copy_(dev(coeff2.ravel()))
    plan.evaluate(dc, J)
    assert np.array_equal(host(J), host(api.evaluate(specs, grids, coeff2)[0]))
    # new output pointer: recapture
    J2 = torch.empty_like(J)
    f2 = torch.empty(api.n_modes(grids), dtype=torch.float64, device="cuda")
    plan.evaluate(dc, J2, f2)
    assert np.array_equal(host(J2), host(J))
    plan.close()


def test_evolve_modes_with_plan_matches_default():
    specs, grids, coeff = small_uneven_batch(2)
    A, edge, _, _ = api.synth(specs, coeff)
    f0, J0 = api.evolve(specs, grids, A, edge)
    plan = api.Plan(specs, grids, config=dict(threads=64, modes_per_lane=2, persistent=1))
    f1 = torch.empty_like(f0)
    J1 = torch.empty_like(J0)
    api.po_evolve_modes(specs, grids, A, edge, f=f1, J=J1, plan=plan)
    assert np.array_equal(host(f1), host(f0)) and np.array_equal(host(J1), host(J0))
    # a plan made for other pulses is rejected on the host
    other = api.Plan(specs[:3], grids[:3], config=dict(threads=256, modes_per_lane=1, persistent=0))
    with pytest.raises(Exception, match="plan"):
        api.po_evolve_modes(specs, grids, A, edge, f=f1, J=J1, plan=other)
    plan.close()
    other.close()


def test_autotune_and_cache(tmp_path):
    specs, grids, coeff = small_uneven_batch(3)
    cache = str(tmp_path / "tune.txt")
    plan = api.Plan(specs, grids, config=None, cache_path=cache)
    cfg = plan.config
    say(f"autotuned {cfg}")
    assert cfg["threads"] in (64, 128, 256) and cfg["modes_per_lane"] in (1, 2) and cfg["persistent"] in (0, 1)
    with open(cache) as fh:
        lines = fh.read().strip().splitlines()
    assert len(lines) == 1 and "gfx950" in lines[0]
    plan2 = api.Plan(specs, grids, config=None, cache_path=cache)
    assert plan2.config["threads"] == cfg["threads"] and plan2.config["modes_per_lane"] == cfg["modes_per_lane"]
    with open(cache) as fh:
        assert len(fh.read().strip().splitlines()) == 1  # served from the cache, no new tuning entry
    J = torch.empty(len(specs), dtype=torch.float64, device="cuda")
    plan2.evaluate(dev(coeff.ravel()), J)
    assert np.array_equal(host(J), host(api.evaluate(specs, grids, coeff)[0]))
    plan.close()
    plan2.close()


@pytest.mark.timeout(600)
def test_uneven_batch_workload_full_size(orc):
    """256 pulses, nt from 4096 to 65536, grids 32^2 / 64^2x8 / 96^2x16, autotuned persistent plan;
    sampled modes against the oracle and J against the exact sum of f."""
    w = W.uneven_batch(0)
    specs, grids, coeff = w["specs"], w["grids"], w["coeff"]
    say(f"uneven batch: {W.mode_steps(specs, grids):.3e} mode-steps")
    plan = api.Plan(specs, grids, config=None)
    say(f"autotuned {plan.config}")
    J = torch.empty(len(specs), dtype=torch.float64, device="cuda")
    f = torch.empty(api.n_modes(grids), dtype=torch.float64, device="cuda")
    plan.evaluate(dev(coeff.ravel()), J, f)
    J, f = host(J), host(f)
    assert np.all(np.isfinite(f)) and np.all(f >= 0) and np.all(f <= 2)
    offs = np.concatenate([[0], np.cumsum([W.n_modes(g) for g in grids])])
    order = np.argsort([s["nt"] for s in specs])
    for pi in (int(order[0]), int(order[-1]), 100):
        s, g = specs[pi], grids[pi]
        Ar, _, er, _ = orc.synth(s, coeff[pi])
        M = W.n_modes(g)
        idx = W.sample_mode_indices(pi, M, 8)
        p, dv = orc.grid_points(g)
        fr = orc.evolve_points(Ar, er, s["T"] / s["nt"], p[idx])
        assert_modes(f[offs[pi] + idx], fr, s["nt"], f"uneven batch pulse {pi} (nt {s['nt']})")
    for pi in range(0, 256, 17):
        g = grids[pi]
        dv = np.prod([(g["hi"][d] - g["lo"][d]) / g["n"][d] for d in range(3)
                      if not (g["n"][d] == 1 and g["lo"][d] == g["hi"][d])])
        assert abs(J[pi] - dv * math.fsum(f[offs[pi]:offs[pi + 1]])) <= 1e-13 * J[pi]
    # one whole 96^2 x 16 pulse (the shortest of that grid) and one 32^2 sheet pulse against the
    # long-double oracle: every mode at the per-mode bar, J at relative 1e-8
    big = [i for i in range(256) if tuple(grids[i]["n"]) == (96, 96, 16)]
    sheet = [i for i in range(256) if tuple(grids[i]["n"]) == (32, 32, 1)]
    for pi in (min(big, key=lambda i: specs[i]["nt"]), max(sheet, key=lambda i: specs[i]["nt"])):
        s, g = specs[pi], grids[pi]
        say(f"uneven batch pulse {pi}: long-double oracle on all {W.n_modes(g)} modes (nt {s['nt']})")
        Jr, fr = orc.evaluate(s, g, coeff[pi], precision="ld", want_f=True)
        assert_modes(f[offs[pi]:offs[pi + 1]], fr, s["nt"], f"uneven batch pulse {pi}, every mode")
        assert_J(J[pi], Jr, f"uneven batch pulse {pi}")
    plan.close()
