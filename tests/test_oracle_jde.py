"""Pins of the oracle's self-adaptive DE (jDE) on islands and of its ring migration (Sec. IV B).

* With no self-adaptation (tau1 = tau2 = 0), one island and equal (F, CR), jDE is the plain
  DE/rand/1/bin oracle, bit for bit (that oracle is pinned by the Philox known answers and the
  DE invariants).
* Donors are distinct members of the individual's own island; the F and CR redraw rates match
  tau1 and tau2 and the redrawn values lie in [Flo, Fhi] and (0, 1).
* Selection keeps (F, CR) with the genes; migration on a hand-worked example, ties included.
"""
import math

import numpy as np

from paper_1704_08919_amd import workloads as W


def _pop(seed, N, D):
    return W.rng(seed).uniform(-1, 1, (N, D))


def test_reduces_to_plain_de(orc):
    N, D, n_s = 64, 32, 8
    pop = _pop(1, N, D)
    fcr = np.tile([0.8, 0.9], (N, 1))
    for g in (0, 5, 2 ** 33 + 7):
        t1, f1, i1 = orc.jde_propose(pop, fcr, g, 1, -1.0, 1.0, seed=77, n_s=n_s, tau1=0.0, tau2=0.0)
        t0, i0 = orc.de_propose(pop, g, 0.8, 0.9, -1.0, 1.0, seed=77, n_s=n_s)
        assert np.array_equal(t1, t0) and np.array_equal(i1, i0)
        assert np.array_equal(f1, fcr)


def test_island_donors(orc):
    N, D, K = 40, 12, 4
    S = N // K
    pop = _pop(2, N, D)
    fcr = np.tile([0.5, 0.5], (N, 1))
    seen = np.zeros((N, N), dtype=bool)
    for g in range(60):
        _, _, idx = orc.jde_propose(pop, fcr, g, K, -1.0, 1.0, seed=3)
        for i in range(N):
            a, b, c, R = idx[i]
            assert len({i, a, b, c}) == 4
            assert a // S == b // S == c // S == i // S
            assert 0 <= R < D
            seen[i, [a, b, c]] = True
    # every other member of the island is drawn at some point
    for i in range(N):
        k = i // S
        others = [j for j in range(k * S, (k + 1) * S) if j != i]
        assert seen[i, others].all()


def test_self_adaptation_rates(orc):
    N, D = 4096, 8
    pop = _pop(3, N, D)
    fcr = np.tile([0.5, 0.5], (N, 1))
    _, tf, _ = orc.jde_propose(pop, fcr, 11, 1, -1.0, 1.0, seed=9, tau1=0.1, tau2=0.25, Flo=0.1, Fhi=1.0)
    newF = tf[:, 0] != 0.5
    newC = tf[:, 1] != 0.5
    for frac, tau in ((newF.mean(), 0.1), (newC.mean(), 0.25)):
        sd = math.sqrt(tau * (1 - tau) / N)
        assert abs(frac - tau) < 5 * sd
    assert np.all((tf[newF, 0] >= 0.1) & (tf[newF, 0] <= 1.0))
    assert abs(tf[newF, 0].mean() - 0.55) < 0.05
    assert np.all((tf[newC, 1] > 0) & (tf[newC, 1] < 1))


def test_select_moves_parameters(orc):
    N, D = 6, 3
    pop = _pop(4, N, D)
    trial = _pop(5, N, D)
    fit = np.array([1.0, 2.0, 3.0, 4.0, 5.0, np.nan])
    tfit = np.array([1.0, 1.5, 3.5, np.nan, 6.0, 1.0])
    fcr = np.tile([0.5, 0.9], (N, 1))
    tfcr = np.tile([0.2, 0.1], (N, 1))
    p2, f2, c2 = orc.jde_select(pop, fit, fcr, trial, tfit, tfcr, mask=[1, 1, 1, 1, 0, 1])
    moved = np.array([True, False, True, False, False, False])  # ties move, NaN never, masked out stays
    assert np.array_equal(p2[moved], trial[moved]) and np.array_equal(p2[~moved], pop[~moved])
    assert np.array_equal(c2[moved], tfcr[moved]) and np.array_equal(c2[~moved], fcr[~moved])
    assert np.array_equal(f2[moved], tfit[moved])


def test_ring_migration_worked_example(orc):
    # islands of 2: I0 = {0, 1}, I1 = {2, 3}, I2 = {4, 5}
    pop = np.arange(12, dtype=float).reshape(6, 2)
    fit = np.array([1.0, 5.0, 2.0, 0.0, 7.0, 3.0])
    fcr = np.arange(12, dtype=float).reshape(6, 2) / 100
    p, f, c = orc.island_migrate(pop, fit, fcr, 3)
    # I0 best (1: 5) -> I1 worst (3: 0): moves; I1 best (2: 2) -> I2 worst (5: 3): stays;
    # I2 best (4: 7) -> I0 worst (0: 1): moves, from the state before the call
    assert np.array_equal(f, [7.0, 5.0, 2.0, 5.0, 7.0, 3.0])
    assert np.array_equal(p[3], pop[1]) and np.array_equal(p[0], pop[4])
    assert np.array_equal(c[3], fcr[1]) and np.array_equal(c[0], fcr[4])
    assert np.array_equal(p[[1, 2, 4, 5]], pop[[1, 2, 4, 5]])
    # ties: lowest index is best and worst; equal fits never move
    p, f, c = orc.island_migrate(pop, np.array([2.0, 2.0, 1.0, 1.0, 3.0, 3.0]), fcr, 3)
    # I0 best 0 -> I1 worst 2 (2 > 1 moves); I1 best 2 -> I2 worst 4 (1 < 3 stays); I2 best 4 -> I0 worst 0
    assert np.array_equal(f, [3.0, 2.0, 2.0, 1.0, 3.0, 3.0])
    assert np.array_equal(p[2], pop[0]) and np.array_equal(p[0], pop[4])
    # one island: the best replaces the worst of the same island
    p, f, c = orc.island_migrate(pop, np.array([1.0, 4.0, 2.0, 0.5, 3.0, 0.5]), fcr, 1)
    assert np.array_equal(f, [1.0, 4.0, 2.0, 4.0, 3.0, 0.5]) and np.array_equal(p[3], pop[1])
