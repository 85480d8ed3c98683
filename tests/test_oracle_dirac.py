"""Pins of the oracle's Dirac evolution and projection (Sec. II A) against independent results.

* Free spinors against a Hamiltonian built from Kronecker products of Pauli matrices.
* A few steps against scipy.linalg.expm of that Hamiltonian.
* Invariants: zero field gives no pairs, unitarity, f in [0, 2], rotation covariance,
  mirror symmetries, second-order convergence.
* The Sauter pulse closed form (linear polarisation) after Richardson extrapolation.
* The kinetic equation of Sec. II B (independent formulation) for linear and circular fields.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.linalg import expm

from paper_1704_08919_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")

SX = np.array([[0, 1], [1, 0]], dtype=complex)
SY = np.array([[0, -1j], [1j, 0]], dtype=complex)
SZ = np.array([[1, 0], [0, -1]], dtype=complex)
I2 = np.eye(2, dtype=complex)


def dirac_h(P):
    """alpha.P + beta m with alpha = sigma_x (x) sigma, beta = sigma_z (x) 1 (Dirac representation)."""
    sp = P[0] * SX + P[1] * SY + P[2] * SZ
    return np.kron(SX, sp) + np.kron(SZ, I2)


def test_free_spinors_are_eigenvectors(orc):
    for P in ([0.0, 0.0, 0.0], [0.3, -1.2, 0.7], [5.0, 2.0, -3.0]):
        u, v, w = orc.free_spinors(P)
        H = dirac_h(np.array(P))
        assert abs(w - math.sqrt(1 + np.dot(P, P))) < 1e-14
        for s in range(2):
            assert np.allclose(H @ u[s], w * u[s], atol=1e-13)
            assert np.allclose(H @ v[s], -w * v[s], atol=1e-13)
        B = np.concatenate([u, v])
        assert np.allclose(B.conj() @ B.T, np.eye(4), atol=1e-14)


def test_steps_match_matrix_exponential(orc):
    rng = np.random.default_rng(11)
    nt, dt = 5, 0.37
    A = rng.uniform(-1, 1, (nt, 2))
    edge = np.array([[0.2, -0.4], [-0.1, 0.3]])
    p = np.array([0.25, -0.6, 0.45])
    f, psi = orc.evolve_state(A, edge, dt, p)
    _, v, _ = orc.free_spinors(p - np.array([*edge[0], 0.0]))
    U = np.eye(4, dtype=complex)
    for n in range(nt):
        U = expm(-1j * dirac_h(p - np.array([A[n, 0], A[n, 1], 0.0])) * dt) @ U
    for s in range(2):
        assert np.allclose(psi[s], U @ v[s], atol=1e-14)
    u_out, _, _ = orc.free_spinors(p - np.array([*edge[1], 0.0]))
    fref = sum(abs(np.vdot(u_out[sp], U @ v[s])) ** 2 for s in range(2) for sp in range(2))
    assert abs(f - fref) < 1e-14


def _single_pulse_tables(orc, seed=0, nt=4096):
    w = W.single_pulse(seed)
    spec = dict(w["specs"][0], nt=nt)
    A, E, edge, s = orc.synth(spec, w["coeff"][0])
    return spec, A, edge


def test_zero_field_gives_no_pairs(orc):
    nt = 512
    A = np.zeros((nt, 2))
    edge = np.zeros((2, 2))
    p = np.array([[0.0, 0.0, 0.0], [1.0, -0.5, 0.3], [-2.0, 1.5, -1.0]])
    f = orc.evolve_points(A, edge, 0.1, p)
    assert np.all(np.abs(f) <= 1e-28)
    # a constant potential is a gauge choice: still no pairs
    A[:] = [0.3, -0.2]
    edge[:] = [0.3, -0.2]
    assert np.all(np.abs(orc.evolve_points(A, edge, 0.1, p)) <= 1e-28)


def test_unitarity_and_range(orc):
    spec, A, edge = _single_pulse_tables(orc, nt=1024)
    dt = spec["T"] / spec["nt"]
    for p in ([0.1, 0.2, 0.0], [-1.0, 0.5, 0.3]):
        f, psi = orc.evolve_state(A, edge, dt, np.array(p))
        G = psi.conj() @ psi.T
        assert np.allclose(G, np.eye(2), atol=1e-14)
        assert 0.0 <= f <= 2.0
    pts, _ = orc.grid_points(W.sheet_grid(8, 8, 1.5))
    f = orc.evolve_points(A, edge, dt, pts)
    assert np.all(f >= 0.0) and np.all(f <= 2.0)


def test_rotation_covariance(orc):
    spec, A, edge = _single_pulse_tables(orc, nt=1024)
    dt = spec["T"] / spec["nt"]
    p = np.array([[0.3, -0.4, 0.2], [1.0, 0.7, -0.5], [-0.2, 0.05, 0.0]])
    f0 = orc.evolve_points(A, edge, dt, p)
    for th in (0.3, 1.1, math.pi / 2, 2.5):
        R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        pr = p.copy()
        pr[:, :2] = p[:, :2] @ R.T
        f1 = orc.evolve_points(A @ R.T, edge @ R.T, dt, pr)
        np.testing.assert_allclose(f1, f0, rtol=1e-11)


def test_mirror_symmetries(orc):
    spec, A, edge = _single_pulse_tables(orc, nt=1024)
    dt = spec["T"] / spec["nt"]
    p = np.array([[0.3, -0.4, 0.2], [1.0, 0.7, -0.5]])
    # reflection of the out-of-plane momentum: any in-plane field
    pz = p * [1, 1, -1]
    np.testing.assert_allclose(orc.evolve_points(A, edge, dt, pz), orc.evolve_points(A, edge, dt, p), rtol=1e-12)
    # field along x only: reflection p_y -> -p_y
    Ax, ex = A.copy(), edge.copy()
    Ax[:, 1] = 0.0
    ex[:, 1] = 0.0
    py = p * [1, -1, 1]
    np.testing.assert_allclose(orc.evolve_points(Ax, ex, dt, py), orc.evolve_points(Ax, ex, dt, p), rtol=1e-12)


def test_second_order_convergence(orc):
    w = W.single_pulse(0)
    p = np.array([[0.1, 0.2, 0.0], [-0.5, 0.3, 0.4]])
    res = []
    for nt in (1024, 2048, 4096):
        spec = dict(w["specs"][0], nt=nt, norm=W.NORM_NONE)
        coeff = w["coeff"][0].copy()
        coeff[:, 0] *= 0.003
        A, E, edge, s = orc.synth(spec, coeff)
        res.append(orc.evolve_points(A, edge, spec["T"] / nt, p))
    ratio = (res[0] - res[1]) / (res[1] - res[2])
    assert np.all(np.abs(ratio - 4.0) < 0.1)  # first order would give 2, fourth order 16


def test_sauter_pulse_closed_form(orc):
    with open(os.path.join(GOLD, "sauter_pulse.json")) as fh:
        g = json.load(fh)
    E0, tau, T = g["E0"], g["tau"], g["T"]
    p = np.array(g["momenta"])
    res = []
    for nt in (8192, 16384):
        dt = T / nt
        t = -T / 2 + (np.arange(nt) + 0.5) * dt
        A = np.zeros((nt, 2))
        A[:, 0] = -E0 * tau * np.tanh(t / tau)
        edge = np.array([[-E0 * tau * math.tanh(-T / 2 / tau), 0.0], [-E0 * tau * math.tanh(T / 2 / tau), 0.0]])
        res.append(orc.evolve_points(A, edge, dt, p))
    rich = (4 * res[1] - res[0]) / 3
    pperp2 = p[:, 1] ** 2 + p[:, 2] ** 2
    w_in = np.sqrt(1 + pperp2 + (p[:, 0] - E0 * tau) ** 2)
    w_out = np.sqrt(1 + pperp2 + (p[:, 0] + E0 * tau) ** 2)
    D = w_in - w_out
    f1 = (np.sinh(np.pi * tau * (E0 * tau + D / 2)) * np.sinh(np.pi * tau * (E0 * tau - D / 2))
          / (np.sinh(np.pi * tau * w_in) * np.sinh(np.pi * tau * w_out)))
    np.testing.assert_allclose(rich, 2 * f1, rtol=1e-10)


def test_kinetic_equation_linear_field(orc):
    # Sec. II B: Dirac and kinetic formulations give the same f; linear field along x (R = 0).
    w = W.single_pulse(0)
    spec = dict(w["specs"][0], norm_value=0.3)
    coeff = w["coeff"][0].copy()
    coeff[1, 0, :] = 0.0
    _, _, _, s = orc.synth(spec, coeff)
    coeff[:, 0] *= s
    spec["norm"] = W.NORM_NONE
    p = np.array([[0.1, 0.2, 0.0], [-0.5, 0.3, 0.4]])
    res = []
    for nt in (16384, 32768):
        A, E, edge, _ = orc.synth(dict(spec, nt=nt), coeff)
        res.append(orc.evolve_points(A, edge, spec["T"] / nt, p))
    dirac = (4 * res[1] - res[0]) / 3  # second-order step: Richardson limit
    q = [orc.qke_points(spec, coeff, p, nt=nt, linear=True) for nt in (16384, 32768)]
    qke = (16 * q[1] - q[0]) / 15  # RK4: Richardson limit
    np.testing.assert_allclose(dirac, qke, rtol=1e-8)


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


def test_kinetic_equation_circular_field(orc):
    # Rotating field: the 6-component kinetic equation with R != 0 against the Dirac result.
    T, A0, Om = 120.0, 0.8, 0.35
    p = np.array([[0.1, 0.2, 0.0], [-0.5, 0.3, 0.4], [0.7, -0.2, -0.3]])
    res = []
    for nt in (8192, 16384):
        dt = T / nt
        tm = -T / 2 + (np.arange(nt) + 0.5) * dt
        _, _, Am = _circular_tables(tm, T, A0, Om)
        _, _, Ae = _circular_tables(np.array([-T / 2, T / 2]), T, A0, Om)
        res.append(orc.evolve_points(Am, Ae, dt, p))
    dirac = (4 * res[1] - res[0]) / 3
    q = []
    for nq in (16384, 32768):
        th = -T / 2 + np.arange(2 * nq + 1) * (T / nq) / 2
        E, Ed, A = _circular_tables(th, T, A0, Om)
        q.append(orc.qke_tabulated(E, Ed, A, T / nq, p))
    qke = (16 * q[1] - q[0]) / 15
    np.testing.assert_allclose(dirac, qke, rtol=1e-8)
