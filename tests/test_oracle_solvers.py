"""Pins of the oracle's field samples, kinetic-equation solver and fourth-order Magnus step.

* Field samples: E = -dA/dt and dE/dt against central differences of the samples themselves,
  A(t_f) = 0, and the midpoint samples against the synthesis tables.
* Kinetic equation (Sec. II B): fourth-order convergence of RK4 (error ratio 16 per halving),
  and the double build against the long-double build.
* Fourth-order Magnus step (the fourth-order Dirac scheme of Sec. V C): no pairs without a
  field, f in [0, 2], rotation covariance, error ratio 16 per halving of dt, the Sauter-pulse
  closed form, and the same dt -> 0 limit as the second-order scheme on a multimode pulse.
"""
import json
import math
import os

import numpy as np

from paper_1704_08919_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _pulse(seed=0, nt=1024, **kw):
    w = W.single_pulse(seed)
    return dict(w["specs"][0], nt=nt, **kw), w["coeff"][0]


def test_field_samples_derivatives(orc):
    spec, coeff = _pulse(nt=512)
    dt = spec["T"] / spec["nt"]
    h = 1e-4  # in units of dt
    c = 0.3
    E, Ed, A = orc.field_samples(spec, coeff, [c - h, c, c + h])
    E, Ed, A = E.reshape(-1, 3, 2), Ed.reshape(-1, 3, 2), A.reshape(-1, 3, 2)
    dA = (A[:, 2] - A[:, 0]) / (2 * h * dt)
    dE = (E[:, 2] - E[:, 0]) / (2 * h * dt)
    scaleE, scaleEd = np.abs(E).max(), np.abs(Ed).max()
    assert np.abs(-dA - E[:, 1]).max() <= 1e-7 * scaleE
    assert np.abs(dE - Ed[:, 1]).max() <= 1e-7 * scaleEd
    # the peak normalisation holds over the step nodes
    En, _, _ = orc.field_samples(spec, coeff, [0.0], with_end=True)
    assert abs(np.hypot(En[:, 0], En[:, 1]).max() - spec["norm_value"]) <= 1e-15


def test_field_samples_edges_and_midpoints(orc):
    spec, coeff = _pulse(nt=256)
    E, Ed, A = orc.field_samples(spec, coeff, [0.0, 0.5], with_end=True)
    assert E.shape == (2 * 256 + 1, 2)
    assert np.all(np.abs(A[-1]) <= 1e-15)            # A(t_f) = 0
    assert np.all(np.abs(E[0]) <= 1e-15) and np.all(np.abs(E[-1]) <= 1e-15)  # Hann window
    Am, Em, edge, _ = orc.synth(spec, coeff)
    np.testing.assert_allclose(A[1::2], Am, rtol=0, atol=1e-15)
    np.testing.assert_allclose(E[1::2], Em, rtol=0, atol=1e-15)
    np.testing.assert_allclose(A[0], edge[0], rtol=0, atol=1e-15)


def _circular_tables(t, T, A0, Om):
    """A(t) = A0 sin^4(pi (t + T/2)/T) (cos Om t, sin Om t) and E = -dA/dt, dE/dt, analytically."""
    k = np.pi / T
    s, c = np.sin(k * (t + T / 2)), np.cos(k * (t + T / 2))
    h, hd = s ** 4, 4 * s ** 3 * c * k
    hdd = (12 * s ** 2 * c ** 2 - 4 * s ** 4) * k * k
    cx, sx = np.cos(Om * t), np.sin(Om * t)
    A = A0 * np.stack([h * cx, h * sx], 1)
    Ad = A0 * np.stack([hd * cx - h * Om * sx, hd * sx + h * Om * cx], 1)
    Add = A0 * np.stack([hdd * cx - 2 * hd * Om * sx - h * Om ** 2 * cx,
                         hdd * sx + 2 * hd * Om * cx - h * Om ** 2 * sx], 1)
    return -Ad, -Add, A


def _qke_circular(orc, nt, p, T=120.0, A0=0.8, Om=0.35, precision="ld"):
    th = -T / 2 + np.arange(2 * nt + 1) * (T / nt) / 2
    E, Ed, A = _circular_tables(th, T, A0, Om)
    return orc.qke_tabulated(E, Ed, A, T / nt, p, precision=precision)


def test_kinetic_equation_fourth_order(orc):
    # modes with f ~ 1e-6 .. 1e-5 are in the asymptotic range from nt = 1024 on
    p = np.array([[-0.5, 0.3, 0.4], [0.7, -0.2, -0.3]])
    r = [_qke_circular(orc, nt, p) for nt in (1024, 2048, 4096)]
    ratio = (r[0] - r[1]) / (r[1] - r[2])
    assert np.all(np.abs(ratio - 16.0) < 1.0), ratio  # second order would give 4


def test_kinetic_equation_double_build(orc):
    p = np.array([[0.1, 0.2, 0.0], [-0.5, 0.3, 0.4], [1.2, -0.7, 0.1]])
    ld = _qke_circular(orc, 2048, p)
    d = _qke_circular(orc, 2048, p, precision="d")
    # f = 1 - chi_1 carries the absolute rounding of chi_1 (~ eps sqrt(nt) per component)
    assert np.all(np.abs(d - ld) <= 1e-12)


def _sauter(orc_fn, g, nt, gauss):
    E0, tau, T = g["E0"], g["tau"], g["T"]
    dt = T / nt
    n = np.arange(nt)
    if gauss:
        t = -T / 2 + (n[:, None] + np.array(gauss)[None, :]) * dt
        A = np.zeros((nt, 2, 2))
        A[:, :, 0] = -E0 * tau * np.tanh(t / tau)
    else:
        t = -T / 2 + (n + 0.5) * dt
        A = np.zeros((nt, 2))
        A[:, 0] = -E0 * tau * np.tanh(t / tau)
    edge = np.array([[-E0 * tau * math.tanh(-T / 2 / tau), 0.0], [-E0 * tau * math.tanh(T / 2 / tau), 0.0]])
    return orc_fn(A, edge, dt, np.array(g["momenta"]))


def _sauter_exact(g):
    E0, tau = g["E0"], g["tau"]
    p = np.array(g["momenta"])
    pperp2 = p[:, 1] ** 2 + p[:, 2] ** 2
    w_in = np.sqrt(1 + pperp2 + (p[:, 0] - E0 * tau) ** 2)
    w_out = np.sqrt(1 + pperp2 + (p[:, 0] + E0 * tau) ** 2)
    D = w_in - w_out
    f1 = (np.sinh(np.pi * tau * (E0 * tau + D / 2)) * np.sinh(np.pi * tau * (E0 * tau - D / 2))
          / (np.sinh(np.pi * tau * w_in) * np.sinh(np.pi * tau * w_out)))
    return 2 * f1


def test_magnus4_sauter_closed_form_and_order(orc):
    with open(os.path.join(GOLD, "sauter_pulse.json")) as fh:
        g = json.load(fh)
    exact = _sauter_exact(g)
    err = [np.abs(_sauter(orc.evolve4_points, g, nt, orc.GAUSS2) - exact) for nt in (512, 1024, 2048)]
    ratio = err[0] / err[1]
    assert np.all((ratio > 13) & (ratio < 19)), ratio
    assert np.all(err[2] <= 3e-7 * exact), err[2] / exact
    # the second-order scheme at the same step count is three orders of magnitude less accurate
    e2 = np.abs(_sauter(orc.evolve_points, g, 2048, None) - exact)
    assert np.all(err[2] < 1e-2 * e2)
    # converges to the closed form
    e8 = np.abs(_sauter(orc.evolve4_points, g, 8192, orc.GAUSS2) - exact)
    assert np.all(e8 <= 1e-9 * exact), e8 / exact


def _gauss_tables(orc, spec, coeff):
    _, _, Ag = orc.field_samples(spec, coeff, orc.GAUSS2)
    _, _, edge, _ = orc.synth(spec, coeff)
    return Ag.reshape(-1, 2, 2), edge


def test_magnus4_zero_field_unitarity_rotation(orc):
    nt = 256
    p = np.array([[0.0, 0.0, 0.0], [1.0, -0.5, 0.3], [-2.0, 1.5, -1.0]])
    A = np.zeros((nt, 2, 2))
    edge = np.zeros((2, 2))
    assert np.all(np.abs(orc.evolve4_points(A, edge, 0.1, p)) <= 1e-28)
    A[:] = [0.3, -0.2]
    edge[:] = [0.3, -0.2]
    assert np.all(np.abs(orc.evolve4_points(A, edge, 0.1, p)) <= 1e-28)
    spec, coeff = _pulse(nt=512)
    Ag, edge = _gauss_tables(orc, spec, coeff)
    dt = spec["T"] / spec["nt"]
    f0 = orc.evolve4_points(Ag, edge, dt, p)
    assert np.all((f0 >= 0) & (f0 <= 2))
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    pr = p.copy()
    pr[:, :2] = p[:, :2] @ R.T
    f1 = orc.evolve4_points(Ag @ R.T, edge @ R.T, dt, pr)
    np.testing.assert_allclose(f1, f0, rtol=1e-11)


def test_magnus4_same_limit_as_second_order(orc):
    spec, coeff = _pulse(nt=4096)
    p = np.array([[0.1, 0.2, 0.0], [-0.5, 0.3, 0.4]])
    r2 = []
    for nt in (8192, 16384):
        A, _, edge, _ = orc.synth(dict(spec, nt=nt), coeff)
        r2.append(orc.evolve_points(A, edge, spec["T"] / nt, p))
    rich = (4 * r2[1] - r2[0]) / 3
    r4 = []
    for nt in (2048, 4096, 8192):
        Ag, edge = _gauss_tables(orc, dict(spec, nt=nt), coeff)
        r4.append(orc.evolve4_points(Ag, edge, spec["T"] / nt, p))
    np.testing.assert_allclose(r4[2], rich, rtol=1e-6)
    # the fourth-order error drops ~16x per halving of dt (10x asserted)
    assert np.all(np.abs(r4[1] - rich) < 0.1 * np.abs(r4[0] - rich))


def test_kinetic_equation_quad_build(orc):
    # the quadruple-precision build agrees with the long-double one to the latter's rounding, and
    # reports the transient density max_t |1 - chi_1(t)| >= |f(t_f)|
    p = np.array([[0.1, 0.2, 0.0], [-0.5, 0.3, 0.4], [1.2, -0.7, 0.1]])
    T, nt = 120.0, 1024
    th = -T / 2 + np.arange(2 * nt + 1) * (T / nt) / 2
    E, Ed, A = _circular_tables(th, T, 0.8, 0.35)
    ld = orc.qke_tabulated(E, Ed, A, T / nt, p)
    q, fm = orc.qke_tabulated(E, Ed, A, T / nt, p, precision="q", with_fmax=True)
    assert np.all(np.abs(q - ld) <= 1e-16)
    assert np.all(fm >= np.abs(q)) and np.all(fm > 0)
