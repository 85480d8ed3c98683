"""GPU parity of the yield gradient (discrete adjoint of the Dirac steps) and of the synthesis
adjoint against the oracle's fourth-order central differences (long double), through the C ABI.

Tolerance: |g_gpu - g_ref| <= 1e-6 |g_ref| + 1e-8 max|g_ref|.  The difference stencil's own error
is below 1e-10 relative for the smooth, moderate fields used (peak |E| ~ 0.1); the kernels
accumulate ~nt rounded terms per entry.  J from the gradient call agrees with po_evolve_modes to
1e-11 relative (exact cos/sin form against the tangent form of the same step)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1704_08919_amd import api  # noqa: E402
from paper_1704_08919_amd import workloads as W  # noqa: E402

from test_gpu_parity import dev, host, say  # noqa: E402


def assert_grad(g, gr, what):
    g, gr = np.asarray(g), np.asarray(gr)
    err = np.abs(g - gr)
    tol = 1e-6 * np.abs(gr) + 1e-8 * np.abs(gr).max()
    say(f"{what}: {g.size} entries, max |g| {np.abs(gr).max():.3g}, max err/tol {np.max(err / tol):.3g}")
    assert np.all(err <= tol), (what, np.nonzero(err > tol)[0][:8])


@pytest.mark.parametrize("case", ["tan_range", "angle_halving", "two_pulses_ragged", "short_tables"])
def test_yield_gradient_matches_differences(orc, case):
    w = W.single_pulse(0)
    specs = [dict(w["specs"][0], nt=2048)]
    grids = [W.sheet_grid(8, 8, 1.0)]
    coeffs = [w["coeff"][0]]
    if case == "angle_halving":
        specs = [dict(w["specs"][0], nt=256)]  # omega dt up to ~2: the halved cos/sin path
    elif case == "two_pulses_ragged":
        specs = [dict(w["specs"][0], nt=700), W.pulse_spec(n_s=8, T=300.0, nt=1000, norm_value=0.08)]
        grids = [W.grid((5, 3, 2), (-0.8, -0.6, -0.5), (0.7, 0.9, 0.4)), W.sheet_grid(6, 7, 0.9)]
        coeffs = [w["coeff"][0], W.draw_coeff(8, 1, 8)[0]]
    say(f"yield gradient case {case}")
    tabs = [orc.synth(sp, c) for sp, c in zip(specs, coeffs)]
    if case == "short_tables":
        # tables shorter than one reduction group (5 steps) and not a multiple of it (13 steps):
        # stretches of the nt = 2048 table at its step, with the neighbouring rows as edges
        full, dt = tabs[0], specs[0]["T"] / specs[0]["nt"]
        specs, tabs = [], []
        for n0, n in ((100, 5), (900, 13)):
            specs.append(dict(w["specs"][0], nt=n, T=n * dt))
            tabs.append((full[0][n0:n0 + n], None, np.stack([full[0][n0 - 1], full[0][n0 + n]]), 1.0))
        grids = [W.sheet_grid(8, 8, 1.0), W.grid((5, 3, 2), (-0.8, -0.6, -0.5), (0.7, 0.9, 0.4))]
    A = np.concatenate([t[0] for t in tabs])
    edge = np.stack([t[2] for t in tabs])
    gA = torch.empty(A.shape, dtype=torch.float64, device="cuda")
    ge = torch.empty((len(specs), 2, 2), dtype=torch.float64, device="cuda")
    J = torch.empty(len(specs), dtype=torch.float64, device="cuda")
    api.po_yield_gradient(specs, grids, dev(A), dev(edge), gA, J=J, gedge=ge)
    _, J2 = api.evolve(specs, grids, dev(A), dev(edge), want_f=False)
    gA, ge, J, J2 = host(gA), host(ge), host(J), host(J2)
    assert np.all(np.abs(J - J2) <= 1e-11 * np.abs(J2)), (J, J2)
    row = 0
    for i, sp in enumerate(specs):
        nt = sp["nt"]
        ent = np.unique(np.concatenate([W.sample_mode_indices(i, 2 * nt, 14), [0, 1, 2 * nt - 1],
                                        2 * nt + np.arange(4)]))
        gr = orc.grad_table_fd(tabs[i][0], tabs[i][2], sp["T"] / nt, grids[i], ent)
        gg = np.concatenate([gA[row:row + nt].ravel(), ge[i].ravel()])[ent]
        assert_grad(gg, gr, f"{case} pulse {i}")
        row += nt


@pytest.mark.parametrize("norm", [W.NORM_NONE, W.NORM_ENERGY])
def test_coefficient_gradient_matches_differences(orc, norm):
    spec = W.pulse_spec(n_s=4, order=4, T=100.0, nt=256, norm=norm, norm_value=0.8)
    grid = W.sheet_grid(4, 4, 0.8)
    c = W.draw_coeff(21, 1, 4)[0]
    c[:, 0, :] *= 0.15
    say(f"coefficient gradient norm={norm}")
    J, g, U, gU = (host(t) for t in api.evaluate_gradient([spec], [grid], c))
    # the lowest-frequency amplitude changes A most; 2^-18 puts the stencil error below 1e-7
    Jr, Ur, gr, gUr = orc.grad_coeff_fd(spec, grid, c.ravel(), h=2.0 ** -18)
    assert abs(J[0] - Jr) <= 1e-10 * Jr
    assert abs(U[0] - Ur) <= 1e-12 * Ur
    assert_grad(g, gr, f"dJ/dc norm={norm}")
    if norm == W.NORM_NONE:
        assert_grad(gU, gUr, "dU/dc")
    else:
        assert np.all(gU == 0.0)


def test_peak_normalisation_rejected():
    w = W.single_pulse(0)
    with pytest.raises(Exception, match="not differentiable"):
        api.evaluate_gradient(w["specs"], w["grids"], w["coeff"])


def test_gradient_full_size_directional_property():
    # local-search workload size: the directional difference of the GPU J along a random
    # direction matches the GPU gradient (a property that holds at any size)
    w = W.local_search(0, starts=4)
    specs, grids, c = w["specs"], w["grids"], w["coeff"]
    J, g, U, gU = api.evaluate_gradient(specs, grids, c)
    J0, _ = api.evaluate(specs, grids, c)
    assert torch.allclose(J, J0, rtol=1e-11, atol=0)
    v = W.rng(5).normal(size=c.shape)
    v /= np.linalg.norm(v.reshape(len(specs), -1), axis=1)[:, None, None, None]
    h = 1e-4
    Jp, _ = api.evaluate(specs, grids, c + h * v)
    Jm, _ = api.evaluate(specs, grids, c - h * v)
    Jp2, _ = api.evaluate(specs, grids, c + 2 * h * v)
    Jm2, _ = api.evaluate(specs, grids, c - 2 * h * v)
    fd = (8 * (host(Jp) - host(Jm)) - (host(Jp2) - host(Jm2))) / (12 * h)
    pred = (host(g).reshape(len(specs), -1) * v.reshape(len(specs), -1)).sum(1)
    say(f"directional derivative: fd {fd}, gradient {pred}")
    assert np.all(np.abs(fd - pred) <= 1e-6 * np.abs(pred) + 1e-9 * np.abs(host(g)).max())


def test_local_search_improves_and_meets_constraint():
    from paper_1704_08919_amd import localsearch as LS
    w = W.local_search(0, starts=3, nt=1024, n=(16, 16, 4))
    x0 = w["coeff"].reshape(3, -1)
    out = LS.run(w["specs"], w["grids"], x0, w["U_const"])
    amp = LS.amplitude_mask(8)
    for k, r in enumerate(out["results"]):
        say(f"start {k}: J {out['J_start'][k]:.6e} -> {r['J']:.6e}, U {r['U']:.9f}, outer {r['outer']}, "
            f"iterations {r['iterations']}, evaluations {out['evaluations'][k]}")
        assert abs(r["U"] - w["U_const"]) <= 1e-6 * w["U_const"]
        # stationarity on the constraint surface: dJ/dc parallel to dU/dc
        J, g, U, gU = (host(t) for t in api.evaluate_gradient(w["specs"][:1], w["grids"][:1], r["x"]))
        proj = g - (g @ gU) / (gU @ gU) * gU
        assert np.linalg.norm(proj) <= 1e-2 * np.linalg.norm(g)
    assert amp.sum() == 16
    # the best local maximum found beats every start
    assert max(r["J"] for r in out["results"]) > max(out["J_start"])
