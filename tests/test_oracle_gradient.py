"""Pins of the oracle's finite-difference gradients (the reference for the yield-gradient kernels
that serve the local search of Sec. IV A).

* Per-entry table derivatives are linear: their contraction with a random direction equals the
  directional derivative taken directly, and predicts J(A + eps v) - J(A) to O(eps^2).
* Without a field f has its minimum 0, so the gradient vanishes there.
* Chain rule: dJ/dc equals the table gradient contracted with dA/dc of the synthesis.
* Homogeneity (Euler): without normalisation U is of degree 2 in the amplitude coefficients, so
  sum_i c_i dU/dc_i = 2 U; with the energy normalisation J and U do not change when all
  amplitudes are scaled, so sum_i c_i dJ/dc_i = 0 and dU/dc = 0.
"""
import numpy as np

from paper_1704_08919_amd import workloads as W


def _small_tables(seed=0, nt=48):
    rng = W.rng(seed)
    t = (np.arange(nt) + 0.5) / nt
    A = np.stack([0.4 * np.sin(2 * np.pi * t) * np.sin(np.pi * t), 0.3 * np.sin(4 * np.pi * t + 0.5)], 1)
    A += 0.02 * rng.normal(size=A.shape)
    edge = np.array([[0.05, -0.02], [0.0, 0.0]])
    return A, edge


def _J(orc, A, edge, dt, grid):
    p, _ = orc.grid_points(grid)
    return orc.pair_yield(grid, orc.evolve_points(A, edge, dt, p))


def test_table_gradient_is_linear_and_predicts_changes(orc):
    A, edge = _small_tables()
    nt, dt = A.shape[0], 0.7
    grid = W.grid((3, 2, 1), (-0.6, -0.4, 0.0), (0.6, 0.4, 0.0))
    g = orc.grad_table_fd(A, edge, dt, grid, np.arange(2 * nt + 4))
    rng = W.rng(3)
    v = rng.normal(size=2 * nt + 4)
    vA, ve = v[:2 * nt].reshape(nt, 2), v[2 * nt:].reshape(2, 2)
    pred = float(v @ g)
    # directional derivative by the same five-point stencil, taken directly
    h = 1e-4
    Fs = [_J(orc, A + k * h * vA, edge + k * h * ve, dt, grid) for k in (1, -1, 2, -2)]
    direct = (8 * (Fs[0] - Fs[1]) - (Fs[2] - Fs[3])) / (12 * h)
    assert abs(direct - pred) <= 1e-7 * abs(pred), (direct, pred)
    # first-order Taylor prediction of a finite change; the remainder is O(eps^2)
    J0 = _J(orc, A, edge, dt, grid)
    r = []
    for eps in (1e-3, 5e-4):
        dJ = _J(orc, A + eps * vA, edge + eps * ve, dt, grid) - J0
        r.append(abs(dJ - eps * pred))
    assert r[1] < 0.3 * r[0]  # ~1/4: second order


def test_gradient_vanishes_without_field(orc):
    nt = 32
    A = np.zeros((nt, 2))
    edge = np.zeros((2, 2))
    grid = W.grid((2, 2, 1), (-0.5, -0.5, 0.0), (0.5, 0.5, 0.0))
    g = orc.grad_table_fd(A, edge, 0.5, grid, [0, 1, 17, 40, 2 * nt, 2 * nt + 3])
    assert np.all(np.abs(g) <= 1e-15)


def test_coefficient_gradient_chain_rule(orc):
    spec = W.pulse_spec(n_s=4, order=4, T=60.0, nt=64, norm=W.NORM_NONE)
    grid = W.grid((2, 2, 1), (-0.5, -0.5, 0.0), (0.5, 0.5, 0.0))
    c = W.draw_coeff(4, 1, 4)[0]
    c[:, 0, :] *= 0.15  # field amplitude ~0.1 of the Schwinger field: J smooth on the stencil's scale
    c = c.ravel()
    J, U, gJ, gU = orc.grad_coeff_fd(spec, grid, c)
    A, _, edge, _ = orc.synth(spec, c)
    gt = orc.grad_table_fd(A, edge, spec["T"] / spec["nt"], grid, np.arange(2 * spec["nt"] + 4))
    # dA/dc by the five-point stencil on the synthesised tables
    h = 2.0 ** -14
    chain = np.zeros(c.size)
    for i in range(c.size):
        tabs = []
        for k in (1, -1, 2, -2):
            ck = c.copy()
            ck[i] += k * h
            Ak, _, ek, _ = orc.synth(spec, ck)
            tabs.append(np.concatenate([Ak.ravel(), ek.ravel()]))
        dA = (8 * (tabs[0] - tabs[1]) - (tabs[2] - tabs[3])) / (12 * h)
        chain[i] = dA @ gt
    np.testing.assert_allclose(gJ, chain, rtol=1e-6, atol=1e-9 * np.abs(gJ).max())


def test_euler_homogeneity(orc):
    grid = W.grid((2, 2, 1), (-0.5, -0.5, 0.0), (0.5, 0.5, 0.0))
    c = W.draw_coeff(5, 1, 4)[0]
    amp = np.zeros_like(c)
    amp[:, 0, :] = 1.0
    amp = amp.ravel().astype(bool)
    cf = c.ravel()
    spec = W.pulse_spec(n_s=4, order=4, T=60.0, nt=64, norm=W.NORM_NONE)
    J, U, gJ, gU = orc.grad_coeff_fd(spec, grid, cf)
    assert abs(cf[amp] @ gU[amp] - 2 * U) <= 1e-10 * U
    spec = W.pulse_spec(n_s=4, order=4, T=60.0, nt=64, norm=W.NORM_ENERGY, norm_value=1.5)
    J, U, gJ, gU = orc.grad_coeff_fd(spec, grid, cf)
    assert abs(U - 1.5) <= 1e-12
    assert np.all(np.abs(gU) <= 1e-10)
    assert abs(cf[amp] @ gJ[amp]) <= 1e-8 * np.abs(gJ).max() * np.abs(cf).max()
