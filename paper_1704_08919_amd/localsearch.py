"""Multistart local search of Sec. IV A of arXiv:1704.08919.

Maximise J subject to the energy constraint U = U_const with the augmented Lagrangian of the
paper,
    L = -J - lambda C + C^2 / (2 mu),   C = U_const - U,
minimised by BFGS with a line search that satisfies the strong Wolfe conditions; after each
minimisation lambda <- lambda - C / mu and mu <- xi mu (0 < xi < 1) until the constraint holds.
Several random starts run at once: every round evaluates J, dJ/dc, U and dU/dc for all active
starts in one batched device call (po_evaluate_gradient, the discrete adjoint of the Dirac
evaluation), and each start's BFGS state advances on the host.

Scaling (not in the paper, a numerical convenience): C is divided by U_const and the first term
is -ln J (or -J divided by its value at the start), so L is of order one; lambda and mu refer to
these scaled quantities.  ln J has the same maximisers as J.

The iteration logic is written as generators that yield a point and receive its (value,
gradient), so the host arithmetic (vectors of a few dozen entries) is independent of how points
are evaluated; `evaluate` can be any callable.
"""
from __future__ import annotations

import time

import numpy as np


# ------------------------------------------------------------------------- line search, BFGS
def _cubic_min(a, fa, da, b, fb, db):
    """Minimiser of the cubic through (a, fa, da), (b, fb, db), or None."""
    d1 = da + db - 3.0 * (fa - fb) / (a - b)
    disc = d1 * d1 - da * db
    if disc < 0:
        return None
    d2 = np.sign(b - a) * np.sqrt(disc)
    den = db - da + 2.0 * d2
    if den == 0:
        return None
    return b - (b - a) * (db + d2 - d1) / den


def _zoom(x, p, f0, d0, lo, hi, c1, c2, max_iter):
    """Zoom phase of the strong-Wolfe line search (Nocedal & Wright, Numerical Optimization,
    Alg. 3.6); lo and hi are (alpha, f, dphi, g)."""
    for _ in range(max_iter):
        a = _cubic_min(lo[0], lo[1], lo[2], hi[0], hi[1], hi[2])
        left, right = min(lo[0], hi[0]), max(lo[0], hi[0])
        width = right - left
        if a is None or not (left + 0.1 * width <= a <= right - 0.1 * width):
            a = 0.5 * (lo[0] + hi[0])
        fa, ga = yield x + a * p
        da = float(ga @ p)
        if fa > f0 + c1 * a * d0 or fa >= lo[1]:
            hi = (a, fa, da, ga)
        else:
            if abs(da) <= -c2 * d0:
                return a, fa, ga
            if da * (hi[0] - lo[0]) >= 0:
                hi = lo
            lo = (a, fa, da, ga)
        if abs(hi[0] - lo[0]) < 1e-14 * max(1.0, abs(lo[0])):
            break
    return lo[0], lo[1], lo[3]


def strong_wolfe(x, f0, g0, p, a1=1.0, c1=1e-4, c2=0.9, a_max=1e6, max_iter=25):
    """Line search for a step alpha along p satisfying the strong Wolfe conditions (Nocedal &
    Wright, Alg. 3.5).  Generator: yields trial points, receives (f, g); returns (alpha, f, g),
    alpha = 0 if no acceptable step was found."""
    d0 = float(g0 @ p)
    prev = (0.0, f0, d0, g0)
    a = a1
    for i in range(max_iter):
        fa, ga = yield x + a * p
        da = float(ga @ p)
        if fa > f0 + c1 * a * d0 or (i > 0 and fa >= prev[1]):
            return (yield from _zoom(x, p, f0, d0, prev, (a, fa, da, ga), c1, c2, max_iter))
        if abs(da) <= -c2 * d0:
            return a, fa, ga
        if da >= 0:
            return (yield from _zoom(x, p, f0, d0, (a, fa, da, ga), prev, c1, c2, max_iter))
        prev = (a, fa, da, ga)
        a = min(2.0 * a, a_max)
    return prev[0], prev[1], prev[3]


def bfgs(x0, gtol=1e-6, max_iter=200, c1=1e-4, c2=0.9, H0=None):
    """BFGS with the inverse-Hessian update and a strong-Wolfe line search (Nocedal & Wright,
    Alg. 6.1).  Without H0 the first step is scaled to unit length and H = (y.s / y.y) I after it;
    H0 (e.g. from a previous, related minimisation) is used as given.
    Generator: yields points, receives (f, g); returns dict(x, f, g, iterations, H)."""
    x = np.array(x0, dtype=float)
    f, g = yield x
    H = None if H0 is None else np.array(H0, dtype=float)
    it = 0
    while it < max_iter and np.max(np.abs(g)) > gtol:
        p = -(H @ g) if H is not None else -g
        a1 = 1.0 if H is not None else 1.0 / max(np.linalg.norm(g), 1e-300)
        a, fn, gn = yield from strong_wolfe(x, f, g, p, a1=a1, c1=c1, c2=c2)
        if a == 0.0:
            break
        s = a * p
        y = gn - g
        sy = float(s @ y)
        x, f, g = x + s, fn, gn
        it += 1
        if sy <= 1e-12 * np.linalg.norm(s) * np.linalg.norm(y):
            continue  # curvature condition failed (cannot happen under strong Wolfe): keep H
        if H is None:
            H = (sy / float(y @ y)) * np.eye(x.size)
        rho = 1.0 / sy
        V = np.eye(x.size) - rho * np.outer(s, y)
        H = V @ H @ V.T + rho * np.outer(s, s)
    return dict(x=x, f=f, g=g, iterations=it, H=H)


# ------------------------------------------------------------------- augmented Lagrangian
def augmented_lagrangian(x0, U_const, J_scale=None, mu0=1e-2, xi=1e-2, ctol=1e-6, gtol=1e-5, outer=30, inner=200,
                         log_objective=True):
    """The outer loop of Sec. IV A (steps 2-4) for one start, with the safeguards of the
    bound-constrained Lagrangian method of Nocedal & Wright (Numerical Optimization, Alg. 17.4),
    the reference the paper gives for its algorithmic details: minimise L(lambda, mu) with BFGS to
    a gradient tolerance omega; if |C| <= eta, lambda <- lambda - C/mu and the tolerances tighten
    (eta <- eta mu^0.9, omega <- omega mu); otherwise mu <- xi mu and the tolerances restart
    (eta = mu^0.1, omega = mu).  Stops once |C| <= ctol (relative to U_const) with omega <= gtol.
    The inverse Hessian is carried to the next minimisation while mu is unchanged.  With
    log_objective the first term is -ln J instead of -J / J_scale: the same maximisers, better
    scaled (J varies over orders of magnitude in parameter space).
    Generator: yields points, receives raw (J, dJ/dx, U, dU/dx); returns
    dict(x, J, U, lam, mu, outer, iterations)."""
    lam, mu = 0.0, mu0
    omega, eta = mu, mu ** 0.1
    x = np.array(x0, dtype=float)
    total_it = 0
    last = None
    H = None
    for l in range(outer):
        gen = bfgs(x, gtol=max(gtol, omega), max_iter=inner, H0=H)
        req = next(gen)
        seen = {}  # raw (J, U) of the points evaluated in this minimisation
        while True:
            J, gJ, U, gU = yield req
            last = (J, U)
            seen[req.tobytes()] = (J, U)
            c = (U_const - U) / U_const
            if log_objective:
                Lval = (-np.log(J) if J > 0 else np.inf) - lam * c + c * c / (2.0 * mu)
                gL = -gJ / J + (lam - c / mu) * gU / U_const
            else:
                Lval = -J / J_scale - lam * c + c * c / (2.0 * mu)
                gL = -gJ / J_scale + (lam - c / mu) * gU / U_const
            try:
                req = gen.send((Lval, gL))
            except StopIteration as e:
                res = e.value
                break
        x = res["x"]
        H = res["H"]
        total_it += res["iterations"]
        J, U = seen[x.tobytes()]  # the minimiser is one of the evaluated points
        last = (J, U)
        c = (U_const - U) / U_const
        if abs(c) <= max(eta, ctol):
            if abs(c) <= ctol and omega <= gtol:
                return dict(x=x, J=J, U=U, lam=lam, mu=mu, outer=l + 1, iterations=total_it)
            lam -= c / mu
            eta *= mu ** 0.9
            omega *= mu
        else:
            mu *= xi
            eta, omega = mu ** 0.1, mu
            H = None
    return dict(x=x, J=last[0], U=last[1], lam=lam, mu=mu, outer=outer, iterations=total_it)


# ------------------------------------------------------------------------------ batch driver
def drive(gens, evaluate):
    """Advances generators in lockstep: each round collects the requested points of the active
    ones, evaluates them in one call evaluate(indices, X) -> list of results, and sends each its
    result.  Returns (final values, evaluations per generator)."""
    pending = {i: next(g) for i, g in enumerate(gens)}
    done, evals = {}, np.zeros(len(gens), dtype=int)
    while pending:
        idx = sorted(pending)
        res = evaluate(idx, np.stack([pending[i] for i in idx]))
        for j, i in enumerate(idx):
            evals[i] += 1
            try:
                pending[i] = gens[i].send(res[j])
            except StopIteration as e:
                done[i] = e.value
                del pending[i]
    return [done[i] for i in range(len(gens))], evals


def device_evaluator(specs, grids):
    """evaluate(indices, X) for drive(): J, dJ/dc, U, dU/dc of the selected pulses on the device."""
    import torch
    from . import api

    def evaluate(idx, X):
        sp = [specs[i] for i in idx]
        gr = [grids[i] for i in idx]
        J, g, U, gU = api.evaluate_gradient(sp, gr, X.reshape(len(idx), -1))
        J, g, U, gU = (t.cpu().numpy() for t in (J, g, U, gU))
        n = X.shape[1]
        return [(float(J[k]), g[k * n:(k + 1) * n], float(U[k]), gU[k * n:(k + 1) * n]) for k in range(len(idx))]
    return evaluate


def amplitude_mask(n_s):
    """Entries of a flattened [2][2][n_s] coefficient vector that are amplitudes."""
    m = np.zeros((2, 2, n_s), dtype=bool)
    m[:, 0, :] = True
    return m.ravel()


def run(specs, grids, x0, U_const, mu0=1e-2, xi=1e-2, ctol=1e-6, gtol=1e-5, outer=30, inner=200, evaluate=None,
        log_objective=True):
    """Multistart local search: x0[K][D] starting coefficients (one row per start, all with the
    same spec layout).  The amplitudes of each start are first rescaled onto U = U_const (U is
    quadratic in them without normalisation).  The search runs in scaled variables y = x / d,
    d = the RMS starting amplitude for amplitude entries and 1 for phases, so both kinds of
    coefficient move on comparable scales.  Returns a dict with the per-start results (x in the
    original variables), the best start, evaluations per start and wall time."""
    evaluate = evaluate or device_evaluator(specs, grids)
    K = len(specs)
    x0 = np.array(x0, dtype=float).reshape(K, -1)
    t0 = time.perf_counter()
    first = evaluate(list(range(K)), x0)
    amp = amplitude_mask(specs[0]["n_s"])
    xs = x0.copy()
    for k in range(K):
        xs[k, amp] *= np.sqrt(U_const / first[k][2])
    d = np.ones(x0.shape[1])
    d[amp] = np.sqrt(np.mean(xs[:, amp] ** 2))

    def scaled(idx, Y):
        out = evaluate(idx, Y * d)
        return [(J, gJ * d, U, gU * d) for (J, gJ, U, gU) in out]

    again = scaled(list(range(K)), xs / d)
    Js = np.array([r[0] for r in again])
    gens = [augmented_lagrangian(xs[k] / d, U_const, Js[k], mu0, xi, ctol, gtol, outer, inner, log_objective)
            for k in range(K)]
    res, evals = drive(gens, scaled)
    for r in res:
        r["x"] = r["x"] * d
    best = int(np.argmax([r["J"] for r in res]))
    return dict(results=res, J_start=Js, best=best, evaluations=evals + 2, wall_s=time.perf_counter() - t0)
