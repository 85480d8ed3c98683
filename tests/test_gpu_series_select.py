"""Series choice of the second-order evolution (the T series of Sec. II A's exact midpoint step),
checked on the GPU through the per-variant mode-step counters: every 512-mode block must use a
series whose remainder bound covers the largest (omega dt)^2 its modes reach over the table --
the choice may be more conservative than needed, never less -- and the counts add up to the
mode-steps evolved."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts, run on the GPU machine
    pytest.skip("no GPU", allow_module_level=True)

from paper_1704_08919_amd import api  # noqa: E402
from paper_1704_08919_amd import workloads as W  # noqa: E402

# Largest x = (omega dt)^2 at which the tan(sqrt x)/sqrt x series of degree 6, 7, ..., 13 has a
# remainder below 2^-56 (coefficient ratio bound 4/pi^2), rounded down; beyond: angle halving.
XMAX = (0.0099, 0.0197, 0.0337, 0.0518, 0.0735, 0.0985, 0.1261, 0.1558)
BLOCK = 512


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def momenta(grid):
    ax = []
    for k in range(3):
        n, lo, hi = grid["n"][k], grid["lo"][k], grid["hi"][k]
        ax.append(np.full(1, lo) if (n == 1 and lo == hi) else lo + (np.arange(n) + 0.5) * (hi - lo) / n)
    pz, py, px = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")   # mode index (iz ny + iy) nx + ix
    return px.ravel(), py.ravel(), pz.ravel()


def tight_variants(A, dt, grid):
    """Smallest admissible variant index per block from the x its modes actually reach."""
    px, py, pz = momenta(grid)
    out = []
    for m0 in range(0, px.size, BLOCK):
        sl = slice(m0, m0 + BLOCK)
        ux = (px[sl, None] - A[None, :, 0]) ** 2
        uy = (py[sl, None] - A[None, :, 1]) ** 2
        x = dt * dt * np.max(ux + uy + 1.0 + pz[sl, None] ** 2)
        out.append(next((k for k, xm in enumerate(XMAX) if x <= xm), len(XMAX)))
    return out


def run_counts(spec, grid, coeff):
    A, edge, _, _ = api.synth([spec], coeff)
    api.po_timer_enable(True)
    api.po_timer_mode_steps()  # clear
    api.evolve([spec], [grid], A, edge, want_f=False)
    counts = api.po_timer_mode_steps()
    api.po_timer_read()
    api.po_timer_enable(False)
    return A.cpu().numpy(), [counts[k] for k in api.SERIES_VARIANTS]


CASES = {
    "weak_sheet": (W.pulse_spec(n_s=4, T=400.0, nt=4096, norm_value=0.05), W.sheet_grid(32, 16, 1.5), 3),
    "strong_sheet": (W.pulse_spec(n_s=4, T=400.0, nt=4096, norm_value=0.4), W.sheet_grid(32, 16, 1.5), 4),
    "box": (W.pulse_spec(n_s=8, T=800.0, nt=8192, norm_value=0.1), W.box_grid(8, 8, 8), 5),
    "halving": (W.pulse_spec(n_s=4, T=400.0, nt=300, norm_value=0.2), W.sheet_grid(32, 16, 2.0), 6),
}


@pytest.mark.parametrize("case", list(CASES))
def test_single_block_variant_is_admissible(case):
    spec, grid, seed = CASES[case]
    assert W.n_modes(grid) == BLOCK
    coeff = W.draw_coeff(seed, 1, spec["n_s"])
    A, counts = run_counts(spec, grid, coeff)
    tight = tight_variants(A, spec["T"] / spec["nt"], grid)[0]
    used = [k for k, c in enumerate(counts) if c]
    say(f"{case}: counts {counts}, tight variant {tight}")
    assert len(used) == 1 and counts[used[0]] == BLOCK * spec["nt"]
    assert used[0] >= tight


def test_blocks_of_a_pulse_are_admissible():
    # a 64 x 32 sheet: four blocks of eight p_y rows each; aggregated over the blocks, the kernel's
    # variants dominate the tight ones (for every k, no more mode-steps at variants <= k)
    spec = W.pulse_spec(n_s=8, T=400.0, nt=8192, norm_value=0.05)
    grid = W.sheet_grid(64, 32, 2.5)
    A, counts = run_counts(spec, grid, W.draw_coeff(9, 1, 8))
    tight = tight_variants(A, spec["T"] / spec["nt"], grid)
    hist = np.zeros(len(counts), dtype=np.int64)
    for t in tight:
        hist[t] += BLOCK * spec["nt"]
    say(f"blocks: counts {counts}, tight {tight}")
    assert sum(counts) == W.n_modes(grid) * spec["nt"]
    assert np.all(np.cumsum(counts) <= np.cumsum(hist))
    assert len(set(tight)) > 1  # the case separates the blocks (|p_y| differs between them)
