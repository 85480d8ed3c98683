"""GPU parity of self-adaptive DE (jDE) on islands and of ring migration (Sec. IV B) against the
oracle: proposals, (F, CR) and selection bit for bit on the same Philox key; migration bit for bit;
a jDE generation equal to its separate calls."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1704_08919_amd import api  # noqa: E402
from paper_1704_08919_amd import workloads as W  # noqa: E402

from test_gpu_parity import dev, host, say  # noqa: E402


@pytest.mark.parametrize("islands", [1, 4, 16])
def test_jde_propose_bitwise(orc, islands):
    N, ns = 64, 8
    D = 4 * ns
    pop = W.rng(11).uniform(-1, 1, (N, D))
    fcr = np.stack([W.rng(12).uniform(0.1, 1.0, N), W.rng(13).uniform(0, 1, N)], 1)
    prm = api.jde_params(N, D, ns, islands=islands, tau1=0.1, tau2=0.1, seed=0xC0FFEE)
    say(f"jde propose islands={islands}")
    for gen in (0, 7, 2 ** 40 + 3):
        trial = torch.empty((N, D), dtype=torch.float64, device="cuda")
        tfcr = torch.empty((N, 2), dtype=torch.float64, device="cuda")
        idx = torch.empty((N, 4), dtype=torch.int32, device="cuda")
        api.po_jde_propose(prm, gen, dev(pop), dev(fcr), trial, tfcr, idx)
        tr, fr, ir = orc.jde_propose(pop, fcr, gen, islands, -1.0, 1.0, seed=0xC0FFEE, n_s=ns)
        assert np.array_equal(host(idx), ir)
        assert np.array_equal(host(tfcr), fr)
        assert np.array_equal(host(trial), tr)


def test_jde_without_adaptation_is_plain_de():
    N, ns = 64, 8
    D = 4 * ns
    pop = dev(W.rng(14).uniform(-1, 1, (N, D)))
    fcr = dev(np.tile([0.8, 0.9], (N, 1)))
    prm = api.jde_params(N, D, ns, islands=1, tau1=0.0, tau2=0.0, seed=99)
    t1, f1 = torch.empty_like(pop), torch.empty_like(fcr)
    api.po_jde_propose(prm, 5, pop, fcr, t1, f1)
    t0 = torch.empty_like(pop)
    api.po_de_propose(api.de_params(N, D, ns, F=0.8, CR=0.9, seed=99), 5, pop, t0)
    assert torch.equal(t1, t0) and torch.equal(f1, fcr)


def test_jde_select_and_migration_bitwise(orc):
    N, D, K = 48, 16, 4
    pop = W.rng(15).uniform(-1, 1, (N, D))
    trial = W.rng(16).uniform(-1, 1, (N, D))
    fit = W.rng(17).uniform(0, 1, N)
    tfit = W.rng(18).uniform(0, 1, N)
    tfit[5] = fit[5]
    fit[:12] = 0.5  # an island of equal fits: ties
    fcr = W.rng(19).uniform(0, 1, (N, 2))
    tfcr = W.rng(20).uniform(0, 1, (N, 2))
    mask = (W.rng(21).uniform(0, 1, N) < 0.6).astype(np.uint8)
    prm = api.jde_params(N, D, 4, islands=K, seed=1)
    for m in (None, mask):
        dp, df, dc = dev(pop), dev(fit), dev(fcr)
        api.po_jde_select(prm, dp, df, dc, dev(trial), dev(tfit), dev(tfcr), None if m is None else dev(m, torch.uint8))
        pr, fr, cr = orc.jde_select(pop, fit, fcr, trial, tfit, tfcr, m)
        assert np.array_equal(host(dp), pr) and np.array_equal(host(df), fr) and np.array_equal(host(dc), cr)
    for k in (1, 2, 4, 12):
        prm = api.jde_params(N, D, 4, islands=k, seed=1)
        dp, df, dc = dev(pop), dev(fit), dev(fcr)
        api.po_island_migrate(prm, dp, df, dc)
        pr, fr, cr = orc.island_migrate(pop, fit, fcr, k)
        assert np.array_equal(host(dp), pr) and np.array_equal(host(df), fr) and np.array_equal(host(dc), cr), k


def test_jde_generation_equals_separate_calls():
    N, ns, K = 16, 4, 4
    spec = W.pulse_spec(n_s=ns, T=400.0, nt=512, norm_value=0.1)
    grid = W.sheet_grid(16, 16, 1.5)
    prm = api.jde_params(N, 4 * ns, ns, islands=K, seed=42)
    pop = W.rng(22).uniform(-1, 1, (N, 4 * ns))
    fcr = np.tile([0.5, 0.9], (N, 1))
    fit0, _ = api.evaluate([spec] * N, [grid] * N, pop)
    dpop, dfit, dfcr = dev(pop), fit0.clone(), dev(fcr)
    trial, tfit, tfcr = torch.empty_like(dpop), torch.empty_like(dfit), torch.empty_like(dfcr)
    api.po_jde_generation(prm, 3, spec, grid, dpop, dfit, dfcr, trial, tfit, tfcr)
    trial2, tfcr2 = torch.empty_like(dpop), torch.empty_like(dfcr)
    api.po_jde_propose(prm, 3, dev(pop), dev(fcr), trial2, tfcr2)
    tfit2, _ = api.evaluate([spec] * N, [grid] * N, trial2)
    pop2, fit2, fcr2 = dev(pop), fit0.clone(), dev(fcr)
    api.po_jde_select(prm, pop2, fit2, fcr2, trial2, tfit2, tfcr2)
    assert torch.equal(trial, trial2) and torch.equal(tfit, tfit2)
    assert torch.equal(dpop, pop2) and torch.equal(dfit, fit2) and torch.equal(dfcr, fcr2)


def test_invalid_island_layouts_rejected():
    N, D = 20, 8
    pop, fit, fcr = (torch.zeros(s, dtype=torch.float64, device="cuda") for s in ((N, D), (N,), (N, 2)))
    for islands in (3, 6, 0, 65):  # 20 % 3 != 0; 20 / 6 not whole; out of range
        with pytest.raises(Exception):
            api.po_island_migrate(api.jde_params(N, D, 2, islands=islands), pop, fit, fcr)
    with pytest.raises(Exception):  # islands of 2 members cannot draw three donors
        api.po_jde_propose(api.jde_params(N, D, 2, islands=10), 0, pop, fcr, pop.clone(), fcr.clone())
