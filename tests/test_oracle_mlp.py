"""Pins of the NumPy surrogate-MLP oracle against independent implementations:
torch autograd in float64 (forward and gradients), central finite differences, torch's bfloat16
conversion (round to nearest even), torch.nn.functional.gelu (erf form) and torch.optim.Adam."""
import numpy as np
import pytest
import torch

from oracle import mlp as M

N_IN, WIDTH, DEPTH = 32, 64, 3


def random_params(seed=0, n_in=N_IN, width=WIDTH, depth=DEPTH):
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    k = n_in
    for _ in range(depth):
        Ws.append(rng.uniform(-1, 1, (k, width)) / np.sqrt(k))
        bs.append(rng.uniform(-0.1, 0.1, width))
        k = width
    Ws.append(rng.uniform(-1, 1, width) / np.sqrt(width))
    bs.append(rng.uniform(-0.1, 0.1, 1))
    return M.pack(Ws, bs)


def torch_model(params):
    Ws, bs = M.unpack(params, N_IN, WIDTH, DEPTH)
    tW = [torch.tensor(W, dtype=torch.float64, requires_grad=True) for W in Ws]
    tb = [torch.tensor(b, dtype=torch.float64, requires_grad=True) for b in bs]
    return tW, tb


def torch_forward(tW, tb, x):
    h = torch.tensor(x, dtype=torch.float64)
    for l in range(DEPTH):
        h = torch.nn.functional.gelu(h @ tW[l] + tb[l])
    return h @ tW[DEPTH] + tb[DEPTH][0]


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 3, 5000), rng.uniform(-1, 1, 5000) * 10.0 ** rng.integers(-20, 20, 5000)])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16(x), ref)


def test_gelu_matches_torch():
    z = np.linspace(-8, 8, 1001)
    ref = torch.nn.functional.gelu(torch.tensor(z, dtype=torch.float64)).numpy()
    np.testing.assert_allclose(M.gelu(z), ref, rtol=1e-14, atol=1e-15)
    zt = torch.tensor(z, dtype=torch.float64, requires_grad=True)
    torch.nn.functional.gelu(zt).sum().backward()
    np.testing.assert_allclose(M.gelu_grad(z), zt.grad.numpy(), rtol=1e-12, atol=1e-14)


def test_forward_and_gradient_match_autograd():
    p = random_params(2)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (48, N_IN))
    t = rng.normal(0, 1, 48)
    y, _ = M.forward(p, x, N_IN, WIDTH, DEPTH, bf=False)
    tW, tb = torch_model(p)
    yt = torch_forward(tW, tb, x)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-13, atol=1e-14)
    loss, g = M.loss_grad(p, x, t, N_IN, WIDTH, DEPTH, bf=False)
    lt = torch.mean((yt - torch.tensor(t)) ** 2)
    lt.backward()
    assert abs(loss - lt.item()) < 1e-13 * lt.item()
    gref = M.pack([w.grad.numpy() for w in tW], [b.grad.numpy() for b in tb])
    np.testing.assert_allclose(g, gref, rtol=1e-11, atol=1e-14)


def test_gradient_matches_finite_differences():
    p = random_params(4)
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, (16, N_IN))
    t = rng.normal(0, 1, 16)
    _, g = M.loss_grad(p, x, t, N_IN, WIDTH, DEPTH, bf=False)
    idx = rng.choice(p.size, 40, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = M.loss_grad(p + e, x, t, N_IN, WIDTH, DEPTH, bf=False)
        lm, _ = M.loss_grad(p - e, x, t, N_IN, WIDTH, DEPTH, bf=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_bf16_mode_stays_close_to_exact():
    p = random_params(6)
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, (64, N_IN))
    y0, _ = M.forward(p, x, N_IN, WIDTH, DEPTH, bf=False)
    y1, _ = M.forward(p, x, N_IN, WIDTH, DEPTH, bf=True)
    rel = np.max(np.abs(y1 - y0)) / np.max(np.abs(y0))
    assert 1e-5 < rel < 5e-2  # the bf16 path rounds (so differs) but only at the bf16 level


def test_adam_matches_torch():
    rng = np.random.default_rng(8)
    p = rng.normal(0, 1, 200)
    tp = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(1, 6):
        g = rng.normal(0, 1, 200) * (10.0 ** rng.uniform(-4, 1, 200))
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = M.adam(p, g, m, v, t)
        np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-15)
