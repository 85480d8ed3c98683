"""Host logic of the multistart local search (Sec. IV A): BFGS with the strong-Wolfe line search
and the augmented-Lagrangian outer loop, on functions with known optima; the lockstep driver gives
the same result as running each start alone."""
import numpy as np
import pytest

from paper_1704_08919_amd import localsearch as LS


def _run(gen, fun):
    req = next(gen)
    n = 0
    try:
        while True:
            n += 1
            req = gen.send(fun(req))
    except StopIteration as e:
        return e.value, n


def rosen(x):
    f = 100.0 * (x[1] - x[0] ** 2) ** 2 + (1 - x[0]) ** 2
    g = np.array([-400.0 * x[0] * (x[1] - x[0] ** 2) - 2 * (1 - x[0]), 200.0 * (x[1] - x[0] ** 2)])
    return f, g


def test_bfgs_rosenbrock():
    res, n = _run(LS.bfgs([-1.2, 1.0], gtol=1e-8), rosen)
    assert np.allclose(res["x"], [1.0, 1.0], atol=1e-7)
    assert res["iterations"] < 60 and n < 120


def test_strong_wolfe_conditions_hold():
    rng = np.random.default_rng(0)
    Q = rng.normal(size=(6, 6))
    Q = Q @ Q.T + np.eye(6)
    b = rng.normal(size=6)

    def fun(x):
        return 0.5 * x @ Q @ x - b @ x + 0.1 * np.sum(x ** 4), Q @ x - b + 0.4 * x ** 3

    x = rng.normal(size=6)
    f0, g0 = fun(x)
    p = -g0
    (a, fa, ga), _ = _run(LS.strong_wolfe(x, f0, g0, p, a1=1.0 / np.linalg.norm(g0)), fun)
    assert a > 0
    assert fa <= f0 + 1e-4 * a * (g0 @ p)               # sufficient decrease
    assert abs(ga @ p) <= 0.9 * abs(g0 @ p)              # curvature (strong)
    res, _ = _run(LS.bfgs(x, gtol=1e-10), fun)
    assert np.max(np.abs(fun(res["x"])[1])) <= 1e-10


def test_augmented_lagrangian_on_sphere():
    # maximise J = exp(a.x) subject to |x|^2 = U0: x* = sqrt(U0) a / |a|
    a = np.array([0.3, -1.2, 0.5, 0.8])
    U0 = 2.0

    def fun(x):
        J = np.exp(a @ x)
        return J, J * a, float(x @ x), 2 * x

    x0 = np.array([0.5, 0.5, -0.2, 0.1])
    xs = np.sqrt(U0) * a / np.linalg.norm(a)
    for log in (True, False):
        res, _ = _run(LS.augmented_lagrangian(x0, U0, J_scale=fun(x0)[0], ctol=1e-10, gtol=1e-9,
                                              log_objective=log), fun)
        assert np.allclose(res["x"], xs, atol=1e-6)
        assert abs(res["U"] - U0) <= 1e-9 * U0


def test_lockstep_driver_matches_separate_runs():
    starts = [np.array([-1.2, 1.0]), np.array([0.5, -0.7]), np.array([2.0, 2.5])]
    alone = [_run(LS.bfgs(s, gtol=1e-9), rosen)[0] for s in starts]
    calls = []

    def evaluate(idx, X):
        calls.append(list(idx))
        return [rosen(x) for x in X]

    res, evals = LS.drive([LS.bfgs(s, gtol=1e-9) for s in starts], evaluate)
    for r, a in zip(res, alone):
        assert np.array_equal(r["x"], a["x"])
    assert sum(len(c) for c in calls) == int(evals.sum())
    assert max(len(c) for c in calls) == 3


def test_run_rescales_amplitudes_onto_the_constraint():
    # a stand-in evaluator: U quadratic in the amplitudes (as without normalisation), J smooth
    n_s = 2
    amp = LS.amplitude_mask(n_s)
    w = np.linspace(0.5, 1.5, amp.sum())

    def one(x):
        xa = x[amp]
        U = float(w @ xa ** 2)
        gU = np.zeros_like(x)
        gU[amp] = 2 * w * xa
        J = float(np.exp(0.3 * np.sum(np.sin(x))))
        return J, J * 0.3 * np.cos(x), U, gU

    specs = [dict(n_s=n_s)] * 2
    x0 = np.random.default_rng(2).uniform(-1, 1, (2, 4 * n_s))
    out = LS.run(specs, None, x0, U_const=0.7, evaluate=lambda idx, X: [one(x) for x in X], ctol=1e-10, gtol=1e-10)
    for r in out["results"]:
        assert abs(r["U"] - 0.7) <= 1e-9
    assert out["evaluations"].min() > 2
    assert out["results"][out["best"]]["J"] == max(r["J"] for r in out["results"])
