"""Series choice of the second-order evolution (the T polynomial of Sec. II A's exact midpoint step),
checked on the GPU through the per-variant mode-step counters.  The variant is chosen per block
of 512 modes and chunk of 256 steps; every (block, chunk) must use a polynomial whose error bound
covers the largest (omega dt)^2 its modes reach over the chunk's steps -- the choice may be
more conservative than needed, never less -- so, summed over blocks and chunks, the kernel's
mode-steps at variants <= k never exceed those for which variant k is admissible.  The counts
also add up to the mode-steps evolved."""
import os
import re
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on hosts without a GPU
    pytest.skip("no GPU", allow_module_level=True)

from paper_1704_08919_amd import api  # noqa: E402
from paper_1704_08919_amd import workloads as W  # noqa: E402

# Largest x = (omega dt)^2 of each tan(sqrt x)/sqrt x polynomial fit (error below 2^-57 up to there),
# read from the generated header the kernels are compiled from; beyond the last: angle halving.
_HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1704_08919_amd", "csrc",
                    "tan_fit.hpp")
XMAX = tuple(float(v) for v in re.search(r"kFitXmax\[kNumFit\] = \{([^}]*)\}", open(_HDR).read()).group(1).split(","))
BLOCK, CHUNK = 512, 256


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def momenta(grid):
    ax = []
    for k in range(3):
        n, lo, hi = grid["n"][k], grid["lo"][k], grid["hi"][k]
        ax.append(np.full(1, lo) if (n == 1 and lo == hi) else lo + (np.arange(n) + 0.5) * (hi - lo) / n)
    pz, py, px = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")   # mode index (iz ny + iy) nx + ix
    return px.ravel(), py.ravel(), pz.ravel()


def tight_histogram(A, dt, grid):
    """Mode-steps per smallest admissible variant, from the x each (block, chunk) actually reaches."""
    px, py, pz = momenta(grid)
    nt = A.shape[0]
    hist = np.zeros(len(XMAX) + 1, dtype=np.int64)
    for m0 in range(0, px.size, BLOCK):
        sl = slice(m0, m0 + BLOCK)
        nm = px[sl].size
        for c0 in range(0, nt, CHUNK):
            a = A[c0:c0 + CHUNK]
            ux = (px[sl, None] - a[None, :, 0]) ** 2
            uy = (py[sl, None] - a[None, :, 1]) ** 2
            x = dt * dt * np.max(ux + uy + 1.0 + pz[sl, None] ** 2)
            k = next((k for k, xm in enumerate(XMAX) if x <= xm), len(XMAX))
            hist[k] += nm * a.shape[0]
    return hist


def run_counts(spec, grid, coeff):
    A, edge, _, _ = api.synth([spec], coeff)
    api.po_timer_enable(True)
    api.po_timer_mode_steps()  # clear
    api.evolve([spec], [grid], A, edge, want_f=False)
    counts = api.po_timer_mode_steps()
    api.po_timer_read()
    api.po_timer_enable(False)
    return A.cpu().numpy(), np.array([counts[k] for k in api.SERIES_VARIANTS], dtype=np.int64)


CASES = {
    "weak_sheet": (W.pulse_spec(n_s=4, T=400.0, nt=4096, norm_value=0.05), W.sheet_grid(32, 16, 1.5), 3),
    "strong_sheet": (W.pulse_spec(n_s=4, T=400.0, nt=4096, norm_value=0.4), W.sheet_grid(32, 16, 1.5), 4),
    "box": (W.pulse_spec(n_s=8, T=800.0, nt=8192, norm_value=0.1), W.box_grid(8, 8, 8), 5),
    "halving": (W.pulse_spec(n_s=4, T=400.0, nt=300, norm_value=0.2), W.sheet_grid(32, 16, 2.0), 6),
    "four_blocks": (W.pulse_spec(n_s=8, T=400.0, nt=8192, norm_value=0.05), W.sheet_grid(64, 32, 2.5), 9),
    "ragged": (W.pulse_spec(n_s=8, T=400.0, nt=8000, norm_value=0.05), W.grid((40, 30, 2), (-2, -2, -0.5), (2, 2, 0.5)), 10),
}


@pytest.mark.parametrize("case", list(CASES))
def test_series_variants_are_admissible(case):
    spec, grid, seed = CASES[case]
    A, counts = run_counts(spec, grid, W.draw_coeff(seed, 1, spec["n_s"]))
    tight = tight_histogram(A, spec["T"] / spec["nt"], grid)
    say(f"{case}: counts {counts.tolist()}, tight {tight.tolist()}")
    assert counts.sum() == W.n_modes(grid) * spec["nt"]
    assert np.all(np.cumsum(counts) <= np.cumsum(tight))


def test_variants_follow_the_table_range():
    # a field that is strong in the middle of the pulse only: the chunks near the ends need lower
    # degrees than the middle ones, so more than one variant runs within one block
    spec, grid, seed = CASES["weak_sheet"]
    A, counts = run_counts(spec, grid, W.draw_coeff(seed, 1, spec["n_s"]))
    assert np.count_nonzero(counts) > 1


def test_non_finite_and_huge_tables_complete():
    # an infinite and an absurdly large table entry: the series choice stops at its cap, the call
    # returns and the affected pulses give non-finite J, the others are unaffected
    spec, grid, seed = CASES["box"]
    specs = [spec] * 3
    A, edge, _, _ = api.synth(specs, W.draw_coeff(seed, 3, spec["n_s"]))
    _, J0 = api.evolve(specs, [grid] * 3, A, edge, want_f=False)
    nt = spec["nt"]
    A[nt + 5, 0] = float("inf")
    A[2 * nt + 7, 1] = 1e200
    _, J = api.evolve(specs, [grid] * 3, A, edge, want_f=False)
    J, J0 = J.cpu().numpy(), J0.cpu().numpy()
    say(f"J with bad tables {J}, clean {J0}")
    assert J[0] == J0[0]
    assert not np.isfinite(J[1])
    assert not np.isfinite(J[2]) or abs(J[2] - J0[2]) > 1e-3 * abs(J0[2])


def test_check_finite_reports_non_finite_results():
    # with the finite check on, clean results pass through every checked entry point, and the
    # infinite table entry of the test above (which the kernels complete) or a non-finite f makes
    # the call return PO_ERR_NUMERIC; with the check off the same call returns normally
    from paper_1704_08919_amd import _lib
    spec, grid, seed = CASES["box"]
    specs, grids = [spec] * 4, [grid] * 4
    coeff = W.draw_coeff(seed, 4, spec["n_s"])
    A, edge, _, _ = api.synth(specs, coeff)
    prev = api.po_set_check_finite(True)
    try:
        A2, _, _, _ = api.synth(specs, coeff)
        f, J = api.evolve(specs, grids, A, edge)
        J2, _ = api.evaluate(specs, grids, coeff)
        assert torch.equal(A, A2) and torch.equal(J, J2)
        Jy = torch.empty_like(J)
        api.po_pair_yield(grids, f, Jy)
        prm = api.de_params(4, 4 * spec["n_s"], spec["n_s"], seed=seed)
        pop = torch.as_tensor(coeff, dtype=torch.float64).reshape(4, -1).clone().cuda()
        fit, trial, tfit = J.clone(), torch.empty_like(pop), torch.empty_like(J)
        api.po_de_generation(prm, 0, spec, grid, pop, fit, trial, tfit)
        assert torch.isfinite(tfit).all()
        A[spec["nt"] + 5, 0] = float("inf")
        with pytest.raises(_lib.POError, match=r"PO_ERR_NUMERIC.*non-finite values in d_J"):
            api.evolve(specs, grids, A, edge, want_f=False)
        with pytest.raises(_lib.POError, match=r"PO_ERR_NUMERIC.*non-finite values in d_f"):
            api.evolve(specs, grids, A, edge, want_J=False)
        f[3] = float("nan")
        with pytest.raises(_lib.POError, match=r"PO_ERR_NUMERIC: 1 non-finite values in d_J"):
            api.po_pair_yield(grids, f, Jy)
    finally:
        api.po_set_check_finite(prev)
    _, Jbad = api.evolve(specs, grids, A, edge, want_f=False)
    Jbad = Jbad.cpu().numpy()
    say(f"check off: J with an infinite table entry in pulse 1 {Jbad}")
    assert not np.isfinite(Jbad[1]) and np.all(np.isfinite(Jbad[[0, 2, 3]]))
