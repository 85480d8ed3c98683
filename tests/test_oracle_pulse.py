"""Pins of the oracle's pulse synthesis (Sec. III) against independent mathematics.

B-splines: partition of unity, the Bernstein closed form, scipy's BSpline, the paper's
Table I/II counts.  Field: numpy's inverse FFT of the sampled spectrum, Hann zeros.
Potential: adaptive quadrature of E, A(t_f) = 0, E = -dA/dt.  Normalisation: peak and energy,
and the sqrt(2) peak ratio of linear vs circular polarisation at fixed energy (Sec. V B).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate
from scipy.interpolate import BSpline

from paper_1704_08919_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _tables():
    with open(os.path.join(GOLD, "paper_tables.json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("order,ns", [(4, 4), (4, 8), (3, 5), (3, 10), (2, 6), (5, 9)])
def test_bspline_partition_of_unity(orc, order, ns):
    for w in np.concatenate([np.linspace(0.2, 1.3, 97), [0.2, 1.3]]):
        b = orc.bspline_basis(order, ns, 0.2, 1.3, w)
        assert np.all(b >= -1e-15)
        assert abs(b.sum() - 1.0) < 1e-14


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_bspline_bernstein_closed_form(orc, k):
    # No interior knots: the basis is the Bernstein basis of degree k-1.
    for x in np.linspace(0.0, 1.0, 41):
        w = 0.1 + 0.8 * x
        b = orc.bspline_basis(k, k, 0.1, 0.9, w)
        ref = [math.comb(k - 1, i) * x ** i * (1 - x) ** (k - 1 - i) for i in range(k)]
        np.testing.assert_allclose(b, ref, rtol=0, atol=2e-15)


@pytest.mark.parametrize("order,ns", [(4, 8), (3, 10), (4, 12)])
def test_bspline_matches_scipy(orc, order, ns):
    wmin, wmax = 0.0, 1.0
    n = ns - order + 2
    t = np.concatenate([[wmin] * order, np.linspace(wmin, wmax, n)[1:-1], [wmax] * order])
    assert t.size == 2 * order + n - 2 and ns == n + order - 2
    for w in np.linspace(wmin, wmax, 61)[:-1]:
        b = orc.bspline_basis(order, ns, wmin, wmax, w)
        for i in range(ns):
            c = np.zeros(ns)
            c[i] = 1.0
            ref = BSpline(t, c, order - 1, extrapolate=False)(w)
            assert abs(b[i] - ref) < 1e-14


def test_spectral_line_counts_of_paper_tables(orc):
    g = _tables()
    for key in ("table1", "table2"):
        tb = g[key]
        T = 1.0 / tb["dnu"]
        assert abs(T - tb["T"]) < 1e-9
        spec = W.pulse_spec(n_s=tb["n_s"][0], order=tb["order"], omega_min=2 * math.pi * tb["nu_min"],
                            omega_max=2 * math.pi * tb["nu_max"], T=T, nt=16)
        for ns in tb["n_s"]:
            spec["n_s"] = ns
            coeff = np.zeros((2, 2, ns))
            Om, E, Ph = orc.spectra(spec, coeff)
            assert Om.size == tb["n_lines"]
            dw = 2 * math.pi / T
            np.testing.assert_allclose(Om, (round(spec["omega_min"] / dw) + np.arange(Om.size)) * dw, rtol=1e-15)
            assert abs(Om[0] - spec["omega_min"]) < 1e-12 and abs(Om[-1] - spec["omega_max"]) < 1e-12


def test_spectra_are_the_bspline_expansions(orc):
    spec = W.pulse_spec(n_s=8, order=4, T=400.0, nt=16)
    coeff = W.draw_coeff(3, 1, 8)[0]
    Om, E, Ph = orc.spectra(spec, coeff)
    for j in (0, 5, 31, Om.size - 1):
        b = orc.bspline_basis(4, 8, 0.0, 1.0, Om[j])
        for l in range(2):
            assert abs(E[l, j] - coeff[l, 0] @ b) < 1e-14
            assert abs(Ph[l, j] - (math.pi * (coeff[l, 1] + 1.0)) @ b) < 1e-13


def _fft_field(Om, E, Ph, T, nmin, M):
    """E_l(t_n) / g(t_n) at t_n = -T/2 + n T/M from numpy's inverse FFT."""
    out = np.zeros((M, 2))
    for l in range(2):
        c = np.zeros(M, dtype=complex)
        for j in range(Om.size):
            k = nmin + j
            c[k] += E[l, j] * np.exp(-1j * Ph[l, j]) * (-1) ** k
        out[:, l] = np.real(M * np.fft.ifft(c))
    return out


def test_field_matches_inverse_fft(orc):
    spec = W.pulse_spec(n_s=8, order=4, T=400.0, nt=16)
    coeff = W.draw_coeff(5, 1, 8)[0]
    Om, E, Ph = orc.spectra(spec, coeff)
    M = 1024
    t = -spec["T"] / 2 + np.arange(M) * spec["T"] / M
    Ef, _ = orc.field_at(spec, coeff, t)
    ref = _fft_field(Om, E, Ph, spec["T"], 0, M) * np.cos(np.pi * t / spec["T"])[:, None] ** 2
    assert np.max(np.abs(Ef - ref)) < 1e-12 * np.max(np.abs(ref))


def test_hann_window_zeros(orc):
    spec = W.pulse_spec(n_s=8, order=4, T=400.0, nt=16)
    coeff = W.draw_coeff(6, 1, 8)[0]
    E, _ = orc.field_at(spec, coeff, [-200.0, 200.0])
    assert np.max(np.abs(E)) < 1e-28


@pytest.mark.parametrize("seed", [0, 1])
def test_potential_is_integral_of_field(orc, seed):
    spec = W.pulse_spec(n_s=8, order=4, T=400.0, nt=16)
    coeff = W.draw_coeff(seed, 1, 8)[0]
    tf = spec["T"] / 2
    ts = np.array([-200.0, -150.3, -37.7, 0.0, 12.5, 99.9, 180.0, 199.5])
    _, A = orc.field_at(spec, coeff, ts)
    Amax = np.max(np.abs(orc.field_at(spec, coeff, np.linspace(-200, 200, 401))[1]))
    for l in range(2):
        Ex = lambda s: orc.field_at(spec, coeff, [s])[0][0, l]
        for t, a in zip(ts, A[:, l]):
            val, err = integrate.quad(Ex, tf, t, limit=800, epsabs=1e-14, epsrel=1e-13)
            assert abs(a - (-val)) < 1e-10 * Amax


def test_potential_vanishes_at_tf_and_derivative_is_minus_field(orc):
    spec = W.pulse_spec(n_s=8, order=4, T=400.0, nt=16)
    coeff = W.draw_coeff(2, 1, 8)[0]
    _, A = orc.field_at(spec, coeff, [200.0])
    assert np.max(np.abs(A)) == 0.0
    h = 1e-2
    ts = np.array([-120.0, -3.3, 0.0, 77.7, 150.0])
    for t in ts:
        _, Ap = orc.field_at(spec, coeff, [t - 2 * h, t - h, t + h, t + 2 * h])
        dA = (Ap[0] - 8 * Ap[1] + 8 * Ap[2] - Ap[3]) / (12 * h)
        E, _ = orc.field_at(spec, coeff, [t])
        assert np.max(np.abs(-dA - E[0])) < 1e-9


def test_peak_normalisation(orc):
    spec = W.pulse_spec(n_s=4, order=4, T=400.0, nt=4096, norm_value=0.1)
    coeff = W.draw_coeff(0, 1, 4)[0]
    A, E, edge, s = orc.synth(spec, coeff)
    nodes = -200.0 + np.arange(spec["nt"] + 1) * spec["T"] / spec["nt"]
    En, _ = orc.field_at(spec, coeff, nodes)
    peak = np.max(np.hypot(En[:, 0], En[:, 1])) * s
    assert abs(peak - 0.1) < 1e-15
    assert np.all(edge[1] == 0.0)


def test_energy_normalisation(orc):
    spec = W.pulse_spec(n_s=8, order=4, T=400.0, nt=2048, norm=W.NORM_ENERGY, norm_value=3.0)
    coeff = W.draw_coeff(1, 1, 8)[0]
    A, E, edge, s = orc.synth(spec, coeff)
    U = np.sum(E ** 2) * spec["T"] / spec["nt"]
    assert abs(U - 3.0) < 1e-12


def test_linear_vs_circular_peak_ratio_at_fixed_energy(orc):
    # Sec. V B: at fixed integrated energy, E_lin^peak / E_circ^peak ~ sqrt(2) (exact for a single mode).
    T = 400.0
    dw = 2 * math.pi / T
    spec = W.pulse_spec(n_s=4, order=4, omega_min=40 * dw, omega_max=43 * dw, T=T, nt=8192,
                        norm=W.NORM_ENERGY, norm_value=50.0)
    amp = np.ones(4)
    lin = np.stack([np.stack([amp, -np.ones(4)]), np.stack([amp, -np.ones(4)])])        # phases 0, 0
    circ = np.stack([np.stack([amp, -np.ones(4)]), np.stack([amp, -0.5 * np.ones(4)])])  # phases 0, pi/2
    peaks = []
    for c in (lin, circ):
        _, E, _, _ = orc.synth(spec, c)
        peaks.append(np.max(np.hypot(E[:, 0], E[:, 1])))
    assert abs(peaks[0] / peaks[1] - math.sqrt(2)) < 5e-3
