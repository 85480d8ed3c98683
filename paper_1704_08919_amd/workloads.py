"""Seeded synthetic workloads: pulse specifications, momentum grids and coefficient draws.

This module holds sizes and random draws only -- none of the method's arithmetic -- so that the
HIP path and the CPU oracle can be fed identical inputs.  Every draw comes from
numpy.random.Generator(PCG64(seed)).

Conventions (units c = hbar = m = 1, Schwinger field = 1):
  * a pulse has two field components (x, y); each carries n_s amplitude coefficients and n_s
    phase coefficients, drawn uniform in [-1, 1]; coefficient layout [P][2 comp][2 kind][n_s];
  * the spectral band is angular frequency [omega_min, omega_max] in units of m;
  * t runs over [-T/2, T/2] with nt steps;
  * grids are cell-centred; n = (nx, ny, 1) with lo_z = hi_z = 0 is the p_z = 0 sheet.
"""
from __future__ import annotations

import numpy as np

NORM_NONE, NORM_PEAK, NORM_ENERGY = 0, 1, 2


def pulse_spec(n_s=8, order=4, omega_min=0.0, omega_max=1.0, T=800.0, nt=16384,
               norm=NORM_PEAK, norm_value=0.1):
    return dict(n_s=int(n_s), order=int(order), omega_min=float(omega_min), omega_max=float(omega_max),
                T=float(T), nt=int(nt), norm=int(norm), norm_value=float(norm_value))


def grid(n, lo, hi):
    return dict(n=tuple(int(x) for x in n), lo=tuple(float(x) for x in lo), hi=tuple(float(x) for x in hi))


def sheet_grid(nx, ny, half_width):
    return grid((nx, ny, 1), (-half_width, -half_width, 0.0), (half_width, half_width, 0.0))


def box_grid(nx, ny, nz, pxy=2.0, pz=1.0):
    return grid((nx, ny, nz), (-pxy, -pxy, -pz), (pxy, pxy, pz))


def n_modes(g):
    return int(g["n"][0]) * int(g["n"][1]) * int(g["n"][2])


def rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def draw_coeff(seed, n_pulses, n_s):
    """Coefficients uniform in [-1, 1], shape [P][2][2][n_s] (amplitude, phase per component)."""
    return rng(seed).uniform(-1.0, 1.0, size=(int(n_pulses), 2, 2, int(n_s)))


# ------------------------------------------------------------------------------------------
# Named workloads.
# ------------------------------------------------------------------------------------------
def single_pulse(seed=0):
    """One pulse, 2x(4 amp + 4 phase) cubic coefficients, band [0,1], T=400, nt=4096, peak |E| = 0.1,
    32x32 sheet over [-1.5, 1.5]^2 at p_z = 0."""
    spec = pulse_spec(n_s=4, order=4, T=400.0, nt=4096, norm_value=0.1)
    return dict(name="single_pulse_32x32_nt4096", specs=[spec], grids=[sheet_grid(32, 32, 1.5)],
                coeff=draw_coeff(seed, 1, 4))


def de_generation(seed=0, pop=64, nt=16384, T=800.0, n=(64, 64, 16)):
    """One plain DE generation: pop pulses, 2x(8+8) coefficients, T=800, nt=16384, peak 0.1,
    64x64x16 grid over px,py in [-2,2], pz in [-1,1]; F = 0.8, CR = 0.9."""
    spec = pulse_spec(n_s=8, order=4, T=T, nt=nt, norm_value=0.1)
    g = box_grid(*n)
    return dict(name=f"de_generation_pop{pop}_{n[0]}x{n[1]}x{n[2]}_nt{nt}", specs=[spec] * pop,
                grids=[g] * pop, coeff=draw_coeff(seed, pop, 8), F=0.8, CR=0.9)


def uneven_batch(seed=0, n_pulses=256):
    """256 pulses with nt = 2^U[12,16] rounded to a multiple of 64 at fixed dt = 800/16384
    (so T = nt dt), grid drawn from {32^2 sheet over [-1.5,1.5]^2, 64^2x8, 96^2x16 over
    [-2,2]^2 x [-1,1]}, peak |E| ~ U[0.05, 0.2], 2x(8+8) coefficients."""
    r = rng(seed + 7919)
    dt = 800.0 / 16384.0
    expo = r.uniform(12.0, 16.0, size=n_pulses)
    nts = np.clip(np.round(2.0 ** expo / 64.0) * 64, 4096, 65536).astype(int)
    kinds = r.integers(0, 3, size=n_pulses)
    epk = r.uniform(0.05, 0.2, size=n_pulses)
    grids_all = [sheet_grid(32, 32, 1.5), box_grid(64, 64, 8), box_grid(96, 96, 16)]
    specs, grids = [], []
    for i in range(n_pulses):
        specs.append(pulse_spec(n_s=8, order=4, T=float(nts[i]) * dt, nt=int(nts[i]), norm_value=float(epk[i])))
        grids.append(grids_all[int(kinds[i])])
    return dict(name=f"uneven_batch_{n_pulses}", specs=specs, grids=grids, coeff=draw_coeff(seed, n_pulses, 8))


def surrogate_data_spec():
    """Evaluator used to generate surrogate training data: T=400, nt=4096, band [0,1],
    2x(8+8) coefficients, 64x64x16 grid over px,py in [-2,2], pz in [-1,1]."""
    return pulse_spec(n_s=8, order=4, T=400.0, nt=4096, norm_value=0.1), box_grid(64, 64, 16)


def surrogate_de_spec():
    """Surrogate-assisted DE workload: pop 512, 200 generations, 2x(8+8) coefficients,
    T=800, nt=32768, 128x128x32 grid over px,py in [-2,2], pz in [-1,1]."""
    return pulse_spec(n_s=8, order=4, T=800.0, nt=32768, norm_value=0.1), box_grid(128, 128, 32)


def sample_mode_indices(seed, n_total, k):
    """k distinct mode indices (sorted) for sampled parity checks at full size."""
    k = min(int(k), int(n_total))
    return np.sort(rng(seed + 104729).choice(int(n_total), size=k, replace=False))


def mode_steps(specs, grids):
    return sum(int(s["nt"]) * n_modes(g) for s, g in zip(specs, grids))



def circular_pulse(seed=0, nt=20000, n_p=512):
    """Circularly polarised multimode pulse of the paper's 2-D study (Sec. V B, Table pulse2D,
    case (c)): band nu in [0.02, 0.03] (omega = 2 pi nu), T = 5000 (Delta nu = 0.0002, 51 lines),
    N_s = 10 quadratic B-splines (order k = 3), energy U = 50; equal amplitude coefficients on both
    components, drawn uniform in [0, 1], with phases 0 (x) and pi/2 (y), i.e. phase coefficients
    c = -1 and c = -1/2 under a^(phi) = pi (c + 1).  The optimum the paper found is not
    available: the amplitudes are a seeded draw.  Momentum sheet p_x, p_y in [-3, 3] at p_z = 0
    with n_p x n_p cells."""
    spec = pulse_spec(n_s=10, order=3, omega_min=2 * np.pi * 0.02, omega_max=2 * np.pi * 0.03, T=5000.0,
                      nt=nt, norm=NORM_ENERGY, norm_value=50.0)
    amp = rng(seed + 104729).uniform(0.0, 1.0, size=10)
    coeff = np.empty((1, 2, 2, 10))
    coeff[0, :, 0, :] = amp
    coeff[0, 0, 1, :] = -1.0
    coeff[0, 1, 1, :] = -0.5
    return dict(name=f"circular_pulse_T5000_{n_p}x{n_p}", specs=[spec], grids=[sheet_grid(n_p, n_p, 3.0)],
                coeff=coeff)


def local_search(seed=0, starts=10, nt=4096, n=(64, 64, 16)):
    """Multistart local search (Sec. IV A): `starts` random initial pulses, 2x(8+8) cubic
    coefficients, band [0,1], T = 400, nt = 4096, no normalisation -- the energy
    U = int |E|^2 dt is held at U_const = 0.1 by the augmented Lagrangian (about the energy of a
    peak-0.1 field of this kind); 64x64x16 grid over px,py in [-2,2], pz in [-1,1].  Amplitude
    coefficients are drawn uniform in [-0.005, 0.005] (peak |E| of order 0.1), phase coefficients
    uniform in [-1, 1]; the search rescales the amplitudes onto the constraint before it starts."""
    spec = pulse_spec(n_s=8, order=4, T=400.0, nt=nt, norm=NORM_NONE, norm_value=0.0)
    coeff = draw_coeff(seed + 31337, starts, 8)
    coeff[:, :, 0, :] *= 0.005
    return dict(name=f"local_search_{starts}starts_{n[0]}x{n[1]}x{n[2]}_nt{nt}", specs=[spec] * starts,
                grids=[box_grid(*n)] * starts, coeff=coeff, U_const=0.1)
