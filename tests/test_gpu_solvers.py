"""GPU parity of the field sampler, the kinetic-equation solver (Sec. II B), the fourth-order
Magnus step and the split-operator steps (Strang and its fourth-order composition) against the CPU
oracle, through the C ABI.

Tolerances: samples |x_gpu - x_ref| <= 1e-12 max|x_ref| (E, A) and 1e-11 max|x_ref| (dE/dt).
Dirac and Magnus steps: per mode the bound of the Dirac path, |f_gpu - f_ref| <= 1e-9 f_ref +
2 sqrt(f_ref) d + d^2, d = 4 * 2^-53 * sqrt(nt) (reference = long-double oracle on the same tables).
Kinetic equation: the pair density reached during the pulse, F = max_t |1 - chi_1(t)|, is many
orders above the final f (the transient quasi-particle density), and every FP64 step rounds at
that scale, so f carries an absolute error ~ 2^-53 sqrt(nt) F whatever the formulation; the bound
is |f_gpu - f_ref| <= 1e-9 |f_ref| + 8 * 2^-53 * sqrt(nt) * F with f_ref and F from the oracle in
quadruple precision (a long-double f = 1 - chi_1 would itself carry ~ 2^-64 sqrt(nt)).  J: relative
1e-8.  An RK4 step that is unstable for a mode (large omega dt) is outside the parity cases: the
oracle and the kernel then both grow without bound.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1704_08919_amd import api  # noqa: E402
from paper_1704_08919_amd import workloads as W  # noqa: E402

from test_gpu_parity import assert_J, assert_modes, dev, host, ragged_grid, say  # noqa: E402


def assert_qke(f_gpu, f_ref, fmax, nt, what):
    """Kinetic-equation bound: 1e-9 |f_ref| + 8 * 2^-53 * sqrt(nt) * max_t |1 - chi_1(t)|."""
    f_gpu, f_ref = np.asarray(f_gpu), np.asarray(f_ref)
    tol = 1e-9 * np.abs(f_ref) + 8.0 * 2.0 ** -53 * math.sqrt(nt) * np.asarray(fmax)
    err = np.abs(f_gpu - f_ref)
    say(f"{what}: {f_ref.size} modes, f_ref in [{f_ref.min():.3g}, {f_ref.max():.3g}], transient up to "
        f"{np.max(fmax):.3g}, max err/tol {np.max(err / tol):.3g}, max rel err {np.max(err / np.abs(f_ref)):.3g}")
    bad = np.nonzero(~(err <= tol))[0]
    assert bad.size == 0, f"{what}: {bad.size} modes outside tolerance, first {bad[:5]}: {f_gpu[bad[:5]]} vs {f_ref[bad[:5]]}"


def _max_abs_err(a, b):
    return np.max(np.abs(np.asarray(a) - np.asarray(b)))


@pytest.mark.parametrize("case", ["qke_points", "gauss_nodes", "ragged_three_offsets"])
def test_field_samples_match_oracle(orc, case):
    if case == "qke_points":
        w = W.single_pulse(0)
        specs, coeff, offsets, end = w["specs"], w["coeff"], api.QKE_OFFSETS, True
    elif case == "gauss_nodes":
        w = W.circular_pulse(0, nt=8192)
        specs, coeff, offsets, end = w["specs"], w["coeff"], api.GAUSS2, False
    else:
        specs = [W.pulse_spec(n_s=6, order=3, T=300.0, nt=1000, norm=W.NORM_ENERGY, norm_value=2.5),
                 W.pulse_spec(n_s=8, T=400.0, nt=777, norm=W.NORM_PEAK, norm_value=0.2)]
        coeff = np.concatenate([W.draw_coeff(5, 1, 6).ravel(), W.draw_coeff(6, 1, 8).ravel()])
        offsets, end = (0.0, 0.37, 0.91), True
    say(f"field samples case {case}")
    E, Ed, A, edge, scale = (host(t) for t in api.field_samples(specs, coeff, offsets, with_end=end))
    row, coff = 0, 0
    for i, sp in enumerate(specs):
        c = np.asarray(coeff).ravel()[coff:coff + 4 * sp["n_s"]].reshape(2, 2, sp["n_s"])
        coff += 4 * sp["n_s"]
        rows = sp["nt"] * len(offsets) + (1 if end else 0)
        Er, Edr, Ar = orc.field_samples(sp, c, offsets, with_end=end)
        for name, g, r, tol in (("E", E, Er, 1e-12), ("dE/dt", Ed, Edr, 1e-11), ("A", A, Ar, 1e-12)):
            err = _max_abs_err(g[row:row + rows], r)
            say(f"  pulse {i} {name}: max err {err:.3g} of max {np.abs(r).max():.3g}")
            assert err <= tol * np.abs(r).max(), (i, name)
        _, _, edge_r, scale_r = orc.synth(sp, c)
        assert _max_abs_err(edge[i], edge_r) <= 1e-12 * max(np.abs(Ar).max(), 1e-300)
        assert abs(scale[i] - scale_r) <= 1e-13 * abs(scale_r)
        row += rows


def test_field_samples_agree_with_synthesis_tables():
    w = W.de_generation(0, pop=2)
    specs, coeff = w["specs"], w["coeff"]
    E, Ed, A, edge, scale = api.field_samples(specs, coeff, (0.5,))
    A2, edge2, scale2, E2 = api.synth(specs, coeff, want_E=True)
    a, a2 = host(A), host(A2)
    say(f"midpoint samples vs synthesis tables: max diff {_max_abs_err(a, a2):.3g}")
    assert _max_abs_err(a, a2) <= 1e-14 * np.abs(a2).max()
    assert _max_abs_err(host(E), host(E2)) <= 1e-14 * np.abs(host(E2)).max()
    assert np.array_equal(host(scale), host(scale2)) and np.array_equal(host(edge), host(edge2))


def _qke_tables(orc, spec, coeff):
    E, Ed, A = orc.field_samples(spec, coeff, api.QKE_OFFSETS, with_end=True)
    return E, Ed, A


@pytest.mark.parametrize("case", ["rotating_single_pulse", "linear_single_pulse", "rotating_ragged_grid"])
def test_qke_matches_oracle(orc, case):
    # nt large enough for RK4 to be stable on every mode; a multimode rotating field converges
    # slowly where E passes near zero (R ~ 1/|E|^2 there), so f may still be slightly negative:
    # the bound then uses |f_ref|
    w = W.single_pulse(0)
    spec, coeff = dict(w["specs"][0], nt=16384), w["coeff"][0].copy()
    grid, linear = W.sheet_grid(16, 16, 1.5), False
    if case == "linear_single_pulse":
        coeff[1, 0, :] = 0.0  # no y component
        linear = True
    elif case == "rotating_ragged_grid":
        spec = dict(spec, nt=8000)
        grid = ragged_grid()
    say(f"qke case {case}")
    E, Ed, A = _qke_tables(orc, spec, coeff)
    f, J = api.qke([spec], [grid], dev(E), dev(Ed), dev(A), linear=linear)
    f, J = host(f), host(J)
    p, _ = orc.grid_points(grid)
    fr, fm = orc.qke_tabulated(E, Ed, A, spec["T"] / spec["nt"], p, linear=linear, precision="q", with_fmax=True)
    assert_qke(f, fr, fm, spec["nt"], f"qke {case}")
    assert_J(J[0], orc.pair_yield(grid, fr), f"qke {case}")
    # J from the stored f equals the fused J bit for bit
    J2 = torch.empty(1, dtype=torch.float64, device="cuda")
    api.po_pair_yield([grid], dev(f), J2)
    assert host(J2)[0] == J[0]


def test_qke_analytic_circular_field(orc):
    # the analytic circular pulse of the oracle's kinetic-equation pin, on a 16x16 sheet
    T, A0, Om, nt = 120.0, 0.8, 0.35, 4096
    th = -T / 2 + np.arange(2 * nt + 1) * (T / nt) / 2
    k = np.pi / T
    s, c = np.sin(k * (th + T / 2)), np.cos(k * (th + T / 2))
    h, hd = s ** 4, 4 * s ** 3 * c * k
    hdd = (12 * s ** 2 * c ** 2 - 4 * s ** 4) * k * k
    cx, sx = np.cos(Om * th), np.sin(Om * th)
    A = A0 * np.stack([h * cx, h * sx], 1)
    E = -A0 * np.stack([hd * cx - h * Om * sx, hd * sx + h * Om * cx], 1)
    Ed = -A0 * np.stack([hdd * cx - 2 * hd * Om * sx - h * Om ** 2 * cx,
                         hdd * sx + 2 * hd * Om * cx - h * Om ** 2 * sx], 1)
    spec = W.pulse_spec(T=T, nt=nt)
    grid = W.sheet_grid(16, 16, 1.2)
    f, J = api.qke([spec], [grid], dev(E), dev(Ed), dev(A))
    p, _ = orc.grid_points(grid)
    fr, fm = orc.qke_tabulated(E, Ed, A, T / nt, p, precision="q", with_fmax=True)
    assert_qke(host(f), fr, fm, nt, "qke analytic circular")
    assert_J(host(J)[0], orc.pair_yield(grid, fr), "qke analytic circular")


def _gauss_tables(orc, spec, coeff):
    _, _, Ag = orc.field_samples(spec, coeff, api.GAUSS2)
    _, _, edge, _ = orc.synth(spec, coeff)
    return Ag.reshape(-1, 2, 2), edge


@pytest.mark.parametrize("case", ["tan_series", "angle_halving", "ragged_grid"])
def test_magnus4_matches_oracle(orc, case):
    w = W.single_pulse(0)
    spec, coeff, grid = dict(w["specs"][0], nt=1024), w["coeff"][0], W.sheet_grid(12, 12, 1.5)
    if case == "angle_halving":
        spec = dict(spec, nt=96)  # omega dt up to ~8: the cos/sin path with halvings
    elif case == "ragged_grid":
        spec = dict(spec, nt=700)
        grid = W.grid((7, 5, 3), (-1.3, -0.9, -0.7), (1.1, 1.4, 0.8))
    say(f"magnus4 case {case}")
    Ag, edge = _gauss_tables(orc, spec, coeff)
    f, J = api.evolve_m4([spec], [grid], dev(Ag), dev(edge))
    f, J = host(f), host(J)
    p, _ = orc.grid_points(grid)
    fr = orc.evolve4_points(Ag, edge, spec["T"] / spec["nt"], p)
    assert_modes(f, fr, spec["nt"], f"magnus4 {case}")
    assert_J(J[0], orc.pair_yield(grid, fr), f"magnus4 {case}")
    J2 = torch.empty(1, dtype=torch.float64, device="cuda")
    api.po_pair_yield([grid], dev(f), J2)
    assert host(J2)[0] == J[0]


def _split_tables(orc, spec, coeff, order):
    if order == 2:
        A, _, edge, _ = orc.synth(spec, coeff)
        return A, edge
    _, _, At = orc.field_samples(spec, coeff, api.SPLIT4_OFFSETS)
    _, _, edge, _ = orc.synth(spec, coeff)
    return At.reshape(-1, 3, 2), edge


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("case", ["tan_series", "angle_halving", "ragged_grid", "zero_field"])
def test_split_matches_oracle(orc, order, case):
    w = W.single_pulse(0)
    spec, coeff, grid = dict(w["specs"][0], nt=1024), w["coeff"][0], W.sheet_grid(12, 12, 1.5)
    if case == "angle_halving":
        spec = dict(spec, nt=96)  # |q| up to ~8: the cos/sin path with halvings
    elif case == "ragged_grid":
        spec = dict(spec, nt=700)
        grid = W.grid((7, 5, 3), (-1.3, -0.9, -0.7), (1.1, 1.4, 0.8))
    say(f"split order {order} case {case}")
    At, edge = _split_tables(orc, spec, coeff, order)
    if case == "zero_field":  # the constant-field splitting error, pinned in closed form on the CPU
        grid = W.grid((7, 5, 3), (-1.3, -0.9, -0.7), (1.1, 1.4, 0.8))
        At, edge = np.zeros_like(At) + 0.1, np.zeros_like(edge) + 0.1
    f, J = api.evolve_split([spec], [grid], order, dev(At), dev(edge))
    f, J = host(f), host(J)
    p, _ = orc.grid_points(grid)
    fr = orc.evolve_split_points(At, edge, spec["T"] / spec["nt"], p, order=order)
    assert_modes(f, fr, spec["nt"], f"split{order} {case}")
    assert_J(J[0], orc.pair_yield(grid, fr), f"split{order} {case}")
    J2 = torch.empty(1, dtype=torch.float64, device="cuda")
    api.po_pair_yield([grid], dev(f), J2)
    assert host(J2)[0] == J[0]


def test_three_solvers_agree_as_dt_shrinks():
    # Dirac (2nd order), Magnus (4th order) and the kinetic equation converge to one f; a field
    # along x, where the kinetic equation converges at its fourth order (no R term)
    w = W.single_pulse(1)
    spec, grid = w["specs"][0], W.sheet_grid(32, 32, 1.5)
    coeff = w["coeff"].copy()
    coeff[0, 1, 0, :] = 0.0
    nt = 32768
    s = [dict(spec, nt=nt)]
    A, edge, _, _ = api.synth(s, coeff)
    f2, _ = api.evolve(s, [grid], A, edge)
    _, _, Ag, edge4, _ = api.field_samples(s, coeff, api.GAUSS2)
    f4, _ = api.evolve_m4(s, [grid], Ag, edge4)
    E, Ed, Aq, _, _ = api.field_samples(s, coeff, api.QKE_OFFSETS, with_end=True)
    fq, _ = api.qke(s, [grid], E, Ed, Aq, linear=True)
    f2, f4, fq = host(f2), host(f4), host(fq)
    big = f4 > 1e-3 * f4.max()
    e2 = np.max(np.abs(f2 - f4)[big] / f4[big])
    eq = np.max(np.abs(fq - f4)[big] / f4[big])
    say(f"relative spread at nt={nt} over {big.sum()} modes: dirac2 vs magnus4 {e2:.3g}, qke vs magnus4 {eq:.3g}")
    assert e2 <= 1e-4 and eq <= 1e-5


def test_circular_pulse_full_size_sampled(orc):
    # the solver-comparison workload at full size (512x512 sheet) in the launch the benchmark
    # times, sampled modes against the oracle, for all three solvers at nt = 20000
    w = W.circular_pulse(0, nt=20000)
    s, coeff, grid = w["specs"], w["coeff"], w["grids"][0]
    idx = np.array([0, 77_777, 131_071, 131_328, 200_000, 262_143])
    p_all, _ = orc.grid_points(grid)
    p = p_all[idx]
    c0 = coeff[0]
    spec = s[0]
    # Dirac, second order
    A, edge, _, _ = api.synth(s, coeff)
    f2, J2 = api.evolve(s, [grid], A, edge)
    Ar, _, edge_r, _ = orc.synth(spec, c0)
    assert_modes(host(f2)[idx], orc.evolve_points(Ar, edge_r, spec["T"] / spec["nt"], p), spec["nt"],
                 "circular dirac2 sampled")
    # Magnus, fourth order
    _, _, Ag, edge4, _ = api.field_samples(s, coeff, api.GAUSS2)
    f4, J4 = api.evolve_m4(s, [grid], Ag, edge4)
    Agr, edge_r4 = _gauss_tables(orc, spec, c0)
    assert_modes(host(f4)[idx], orc.evolve4_points(Agr, edge_r4, spec["T"] / spec["nt"], p), spec["nt"],
                 "circular magnus4 sampled")
    # kinetic equation, on sampled modes whose largest 2 omega dt stays inside RK4's stability
    # interval on the imaginary axis (2 sqrt 2); faster modes grow without bound in both codes
    E, Ed, Aq, _, _ = api.field_samples(s, coeff, api.QKE_OFFSETS, with_end=True)
    fq, _ = api.qke(s, [grid], E, Ed, Aq)
    Er, Edr, Aqr = _qke_tables(orc, spec, c0)
    amax = np.hypot(Aqr[:, 0], Aqr[:, 1]).max()
    wmax = np.sqrt(1 + (np.hypot(p_all[:, 0], p_all[:, 1]) + amax) ** 2)
    stable = np.nonzero(2 * wmax * spec["T"] / spec["nt"] <= 2.5)[0]
    assert stable.size > 1000
    iq = stable[np.linspace(0, stable.size - 1, 6).astype(int)]
    fqr, fm = orc.qke_tabulated(Er, Edr, Aqr, spec["T"] / spec["nt"], p_all[iq], precision="q", with_fmax=True)
    assert_qke(host(fq)[iq], fqr, fm, spec["nt"], "circular qke sampled")
    # split-operator steps, second and fourth order
    fs, Js = {}, {}
    for order in (2, 4):
        if order == 2:
            At, edge_s, Atr, edge_sr = A, edge, Ar, edge_r
        else:
            _, _, At, edge_s, _ = api.field_samples(s, coeff, api.SPLIT4_OFFSETS)
            Atr, edge_sr = _split_tables(orc, spec, c0, 4)
        fs[order], Js[order] = api.evolve_split(s, [grid], order, At, edge_s)
        assert_modes(host(fs[order])[idx], orc.evolve_split_points(Atr, edge_sr, spec["T"] / spec["nt"], p, order=order),
                     spec["nt"], f"circular split{order} sampled")
    # every J is the exact sum of the kernel's own f
    for f, J, name in ((f2, J2, "dirac2"), (f4, J4, "magnus4"), (fs[2], Js[2], "split2"), (fs[4], Js[4], "split4")):
        fh = host(f)
        assert np.all(np.isfinite(fh)) and np.all(fh >= 0) and np.all(fh <= 2 + 1e-12)
        Jr = math.fsum(fh) * ((6.0 / 512) ** 2)
        assert abs(host(J)[0] - Jr) <= 1e-12 * Jr, name


def test_fp64_fma_probe_rate():
    # the issue-rate probe runs at every occupancy it supports and reports a rate within the
    # device's FP64 peak (78.6 TFLOP/s, with 5% for clock and timer slack)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    sink = torch.empty(n_cu * 8 * 256, dtype=torch.float64, device="cuda")
    for w in (3, 4, 8):
        api.po_probe_fp64_fma(w, 4, 16, sink)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        flop = api.po_probe_fp64_fma(w, 4, 1024, sink)
        e1.record()
        torch.cuda.synchronize()
        tf = flop / (e0.elapsed_time(e1) * 1e-3) / 1e12
        say(f"fp64 fma probe: {w} waves/SIMD, 4 chains: {tf:.1f} TFLOP/s")
        assert 10.0 < tf < 1.05 * 78.6
        v = host(sink[:n_cu * w * 256])
        assert np.all(np.isfinite(v)) and np.all((v > 3.9) & (v < 5.1))
