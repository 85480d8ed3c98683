"""Surrogate-assisted differential evolution on one GPU (an addition to the paper's method).

* Evaluator: the plain FP64 objective J for a fixed-size batch of pulses sharing one spec and
  grid, through a plan (persistent launch, graph replayed every call).
* Dataset generation and training of the BF16-MFMA surrogate network (po_mlp_*), targets the
  standardised log10 J.
* surrogate_de: DE/rand/1/bin (Sec. IV B of arXiv:1704.08919) where, each generation, the network
  scores all trial vectors, only the top fraction is evaluated by the plain FP64 path, and
  selection runs on those only; the network is retrained on every plain evaluation made so far
  every `retrain_every` generations.  screen="random" picks the evaluated trials at random
  instead (the ablation without the network); plain_de evaluates every trial.

Every numerical step runs in libpairopt kernels; this module sequences calls and keeps the
history on the host.
"""
from __future__ import annotations

import math
import sys
import time

import numpy as np
import torch

from . import api
from . import workloads as W


class Evaluator:
    """J for `batch` pulses of one spec and grid; the plan's graph is replayed on every call."""

    def __init__(self, spec, grid, batch, config=None):
        self.spec, self.grid, self.batch = spec, grid, int(batch)
        self.plan = api.Plan([spec] * self.batch, [grid] * self.batch, config=config)
        self.coeff = torch.empty((self.batch, 4 * spec["n_s"]), dtype=torch.float64, device="cuda")
        self.J = torch.empty(self.batch, dtype=torch.float64, device="cuda")
        self.calls = 0

    def __call__(self, X):
        self.coeff.copy_(X)
        self.plan.evaluate(self.coeff, self.J)
        self.calls += 1
        return self.J

    def close(self):
        self.plan.close()


class Archive:
    """Every plain evaluation made so far (device tensors, preallocated)."""

    def __init__(self, capacity, dim):
        self.X = torch.empty((capacity, dim), dtype=torch.float64, device="cuda")
        self.J = torch.empty((capacity, 1), dtype=torch.float64, device="cuda")
        self.n = 0

    def add(self, X, J):
        k = X.shape[0]
        if self.n + k > self.X.shape[0]:
            raise RuntimeError("archive full")
        self.X[self.n:self.n + k].copy_(X)
        self.J[self.n:self.n + k, 0].copy_(J)
        self.n += k


def log10_stats(J_host):
    lj = np.log10(np.maximum(np.asarray(J_host, dtype=np.float64), 1e-300))
    return float(lj.mean()), float(max(lj.std(), 1e-12))


def train(net, X, J, n, epochs=1, batch=1024, lr=1e-3, seed=0, stats=None, max_steps=None):
    """Minibatch Adam on (X[:n], standardised log10 J[:n]) for `epochs` passes over a fresh
    permutation each, or at most max_steps minibatches (epochs=None: exactly max_steps, over as
    many passes as that takes); returns (mean, std, mean loss of the last pass).  The minibatch indices of all steps are uploaded once and the steps run as
    replays of the network's captured training step (po_mlp_train_indexed)."""
    mean, std = stats if stats is not None else log10_stats(J[:n, 0].cpu().numpy())
    rng = np.random.default_rng(seed)
    batch = min(batch, (n // 32) * 32)
    if batch < 32:
        raise ValueError("need at least 32 samples")
    if epochs is None and max_steps is None:
        raise ValueError("epochs=None needs max_steps")
    per_epoch = n // batch
    n_epochs = epochs if epochs is not None else -(-max_steps // per_epoch)
    idx = []
    for _ in range(n_epochs):
        idx.append(rng.permutation(n).astype(np.int32)[:per_epoch * batch])
        if max_steps is not None and len(idx) * per_epoch >= max_steps:
            break
    idx = np.concatenate(idx)
    steps = len(idx) // batch if max_steps is None else min(len(idx) // batch, max_steps)
    idx_d = torch.as_tensor(idx[:steps * batch], device="cuda")
    losses = torch.zeros(max(steps, 1), dtype=torch.float32, device="cuda")
    net.train_indexed(X, J.view(-1), idx_d, steps, batch, mean, 1.0 / std, lr=lr, losses=losses)
    tail = losses[max(0, steps - per_epoch):steps]
    last = float(tail.mean().item()) if steps else float("nan")
    return mean, std, last


def predict(net, X, n, batch=1024):
    """Network output (standardised log10 J) for X[:n] (n padded up to a multiple of 32 internally)."""
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    step = min(batch, net.max_batch, ((n + 31) // 32) * 32)
    xb = torch.zeros((step, X.shape[1]), dtype=torch.float64, device="cuda")
    for s in range(0, n, step):
        m = min(step, n - s)
        xb[:m].copy_(X[s:s + m])
        y = net.forward(xb)
        out[s:s + m].copy_(y[:m])
    return out


def generate_dataset(spec, grid, n, seed=0, batch=1024, plan_config=None):
    """n random coefficient vectors (uniform in [-1, 1]) and their plain FP64 yields."""
    D = 4 * spec["n_s"]
    X = torch.as_tensor(W.draw_coeff(seed, n, spec["n_s"]).reshape(n, D), dtype=torch.float64, device="cuda")
    J = torch.empty((n, 1), dtype=torch.float64, device="cuda")
    ev = Evaluator(spec, grid, batch, plan_config)
    for s in range(0, n, batch):
        m = min(batch, n - s)
        if m == batch:
            J[s:s + m, 0].copy_(ev(X[s:s + m]))
        else:  # last partial batch: pad with the first rows
            pad = torch.cat([X[s:s + m], X[:batch - m]])
            J[s:s + m, 0].copy_(ev(pad)[:m])
    ev.close()
    torch.cuda.synchronize()
    return X, J


def _best(fit):
    return float(fit.max().item())


def run_de(spec, grid, pop=512, generations=200, seed=0, mode="surrogate", top=0.1, retrain_every=20,
           train_steps=150, width=256, depth=3, time_limit=None,
           target=None, F=0.8, CR=0.9, plan_config=None, progress_every=0, resume=None, time_budget=None,
           record=None):
    """One DE run.  mode: "plain" (every trial evaluated), "surrogate" (network screening) or
    "random" (random screening, the ablation).  Stops after `generations`, at `time_limit`
    seconds, or once the best plain-evaluated J reaches `target`.  Returns a dict with the
    best-so-far history (seconds, plain evaluations, J).  progress_every > 0 prints the
    best-so-far to stderr every that many generations.

    The network is trained for `train_steps` minibatch steps at the start and at every retraining,
    whatever the archive's size (passes over fresh permutations of it).

    Plain runs can be split over processes: `resume` is the state a previous call returned
    (keys pop, fit, generation, evals, history, wall_s); the run continues at that generation with
    the same Philox stream, and its clock continues from wall_s (only the evaluation and DE work
    of each process is counted, not its start-up).  `time_budget` stops this process after that
    many seconds of its own work.  `record` (a list) receives (generation, trials, trial J) of
    every generation, host arrays."""
    n_s = spec["n_s"]
    D = 4 * n_s
    k = pop if mode == "plain" else int(math.ceil(top * pop))
    if resume is not None and mode != "plain":
        raise ValueError("only plain runs resume")
    torch.cuda.synchronize()
    ev_pop = Evaluator(spec, grid, pop, plan_config)
    ev_k = ev_pop if k == pop else Evaluator(spec, grid, k, plan_config)
    prm = api.de_params(pop, D, n_s, F=F, CR=CR, seed=seed + 1)
    if resume is None:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_prev = 0.0
        X0 = torch.as_tensor(W.draw_coeff(seed, pop, n_s).reshape(pop, D), dtype=torch.float64, device="cuda")
        popu = X0.clone()
        fit = ev_pop(popu).clone()
        evals = pop
        g_start = 0
        hist = None
    else:
        popu = torch.as_tensor(np.asarray(resume["pop"]), dtype=torch.float64, device="cuda").reshape(pop, D).clone()
        fit = torch.as_tensor(np.asarray(resume["fit"]), dtype=torch.float64, device="cuda").reshape(pop).clone()
        evals = int(resume["evals"])
        g_start = int(resume["generation"])
        hist = [tuple(h) for h in np.asarray(resume["history"]).tolist()]
        t_prev = float(resume["wall_s"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
    trial = torch.empty_like(popu)
    tfit = torch.empty_like(fit)
    net, archive, stats = None, None, None
    rng = torch.Generator(device="cuda")
    rng.manual_seed(seed + 3)
    if mode == "surrogate":
        archive = Archive(pop + k * generations, D)
        archive.add(popu, fit)
        net = api.MLP(D, width, depth, max_batch=max(1024, ((pop + 31) // 32) * 32), seed=seed + 2)
        stats = train(net, archive.X, archive.J, archive.n, epochs=None, seed=seed, max_steps=train_steps)[:2]
    sel = torch.empty((k, D), dtype=torch.float64, device="cuda")
    rank_corr = []

    def now():
        return t_prev + time.perf_counter() - t0

    if hist is None:
        best0 = _best(fit)  # waits for the initial evaluation before the clock is read
        hist = [(now(), evals, best0)]
    train_s = 0.0
    g = g_start - 1
    for g in range(g_start, generations):
        api.po_de_propose(prm, g, popu, trial)
        if mode == "plain":
            tfit.copy_(ev_pop(trial))
            if record is not None:
                record.append((g, trial.cpu().numpy(), tfit.cpu().numpy()))
            api.po_de_select(prm, popu, fit, trial, tfit)
        else:
            if mode == "surrogate":
                score = predict(net, trial, pop)
            else:
                score = torch.rand(pop, generator=rng, device="cuda", dtype=torch.float32)
            mask = api.po_topk_mask(score, k)
            idx = api.po_mask_indices(mask)
            api.po_gather_rows(trial, idx, k, sel)
            Jsel = ev_k(sel)
            api.po_scatter_values(Jsel, idx, k, tfit, fill=float("-inf"))
            api.po_de_select(prm, popu, fit, trial, tfit, mask)
            if mode == "surrogate":
                # rank correlation of the network's scores with the plain J of the evaluated trials
                sc = score[idx[:k].long()].cpu().numpy()
                jt = np.log10(np.maximum(Jsel.cpu().numpy(), 1e-300))
                rank_corr.append(float(np.corrcoef(np.argsort(np.argsort(sc)), np.argsort(np.argsort(jt)))[0, 1]))
                archive.add(sel, Jsel)
                if (g + 1) % retrain_every == 0:
                    ts = time.perf_counter()
                    stats = train(net, archive.X, archive.J, archive.n, epochs=None, seed=seed + g,
                                  max_steps=train_steps)[:2]
                    train_s += time.perf_counter() - ts
        evals += k
        best = _best(fit)
        hist.append((now(), evals, best))
        if progress_every and (g + 1) % progress_every == 0:
            print(f"{mode} DE generation {g + 1}: {hist[-1][0]:.1f} s, {evals} plain evaluations, best J {best:.6e}",
                  file=sys.stderr, flush=True)
        if target is not None and best >= target:
            break
        if time_limit is not None and hist[-1][0] >= time_limit:
            break
        if time_budget is not None and time.perf_counter() - t0 >= time_budget:
            break
    torch.cuda.synchronize()
    out = {"mode": mode, "pop": pop, "evaluated_per_generation": k, "generations": g + 1,
           "wall_s": now(), "plain_evaluations": evals, "best_J": _best(fit),
           "history": hist, "train_s": train_s, "final_pop": popu.cpu().numpy(), "final_fit": fit.cpu().numpy(),
           "rank_corr": rank_corr}
    for e in {id(ev_pop): ev_pop, id(ev_k): ev_k}.values():
        e.close()
    if net is not None:
        net.close()
    return out


def time_to_reach(hist, target):
    for t, _, j in hist:
        if j >= target:
            return t
    return None
