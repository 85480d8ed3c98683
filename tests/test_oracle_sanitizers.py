"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code): every entry point
of its library runs on small inputs in a child process that preloads the sanitizer runtimes and
loads the sanitized build, and the child must finish without a report."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent("""
    import numpy as np
    import oracle
    from paper_1704_08919_amd import workloads as W
    spec = dict(W.single_pulse(0)["specs"][0], nt=256)
    coeff = W.draw_coeff(1, 1, spec["n_s"])[0]
    grid = W.sheet_grid(4, 4, 1.5)
    p, dv = oracle.grid_points(grid)
    oracle.bspline_basis(4, spec["n_s"], 0.0, 1.0, 0.3)
    oracle.spectra(spec, coeff)
    oracle.field_at(spec, coeff, np.array([-10.0, 0.0, 7.5]))
    for prec in ("ld", "d"):
        A, E, edge, s = oracle.synth(spec, coeff, precision=prec)
        f = oracle.evolve_points(A, edge, spec["T"] / spec["nt"], p, precision=prec, nthreads=2)
    oracle.evolve_state(A, edge, spec["T"] / spec["nt"], p[:2])
    oracle.free_spinors(np.array([0.1, -0.2, 1.1]))
    oracle.pair_yield(grid, f)
    oracle.evaluate(spec, grid, coeff, want_f=True)
    oracle.qke_points(spec, coeff, p[:3], nt=128)
    E, Ed, Aq = oracle.field_samples(spec, coeff, (0.0, 0.5), with_end=True)
    for prec in ("ld", "q", "d"):
        oracle.qke_tabulated(E, Ed, Aq, spec["T"] / spec["nt"], p[:3], precision=prec, with_fmax=True)
    g = 0.5 - np.sqrt(3.0) / 6.0
    _, _, Ag = oracle.field_samples(spec, coeff, (g, 1.0 - g))
    oracle.evolve4_points(Ag, edge, spec["T"] / spec["nt"], p)
    oracle.evolve_split_points(A, edge, spec["T"] / spec["nt"], p, order=2)
    _, _, A4 = oracle.field_samples(spec, coeff, oracle.SPLIT4_OFFSETS)
    oracle.evolve_split_points(A4, edge, spec["T"] / spec["nt"], p, order=4)
    oracle.grad_table_fd(A, edge, spec["T"] / spec["nt"], grid, [0, 5, 2 * spec["nt"] + 1])
    oracle.grad_coeff_fd(dict(spec, norm=W.NORM_ENERGY, norm_value=1.0), grid, coeff)
    oracle.philox4x32_10([1, 2, 3, 4], [5, 6])
    pop = np.random.default_rng(0).uniform(-1, 1, (12, 4 * spec["n_s"]))
    fit = np.arange(12.0)
    trial, _ = oracle.de_propose(pop, 3, 0.8, 0.9, -1.0, 1.0, 7, n_s=spec["n_s"])
    oracle.de_select(pop, fit, trial, fit[::-1].copy(), mask=np.arange(12) % 2)
    fcr = np.tile([0.5, 0.9], (12, 1))
    trial, tfcr, _ = oracle.jde_propose(pop, fcr, 3, 3, -1.0, 1.0, 7, n_s=spec["n_s"])
    oracle.jde_select(pop, fit, fcr, trial, fit[::-1].copy(), tfcr)
    oracle.island_migrate(pop, fit, fcr, 3)
    print("sanitized oracle: done")
""")


def _runtime(name):
    r = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_clean_under_address_and_undefined_sanitizers(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("g++ sanitizer runtimes not installed")
    sys.path.insert(0, ROOT)
    from oracle import build as oracle_build
    lib = oracle_build.build_sanitized(str(tmp_path / "liboracle_san.so"))
    env = dict(os.environ, ORACLE_LIB_PATH=lib, LD_PRELOAD=f"{asan}:{ubsan}", OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", CHILD], env=env, cwd=ROOT, capture_output=True, text=True,
                       timeout=600)
    report = r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "sanitized oracle: done" in r.stdout, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
