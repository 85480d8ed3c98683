"""Host-side tests of the C ABI: the library loads, exports every declared symbol, and rejects
invalid arguments before touching the device (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1704_08919_amd import _lib
from paper_1704_08919_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            with open(os.path.join(ROOT, "include", fn)) as fh:
                text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
            names |= set(re.findall(r"\b(po_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail(f"{_lib.LIB_PATH} is not built (run python -m paper_1704_08919_amd.build)")
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert "po_pulse_synth" in names and "po_evolve_modes" in names and "po_pair_yield" in names
    assert "po_de_generation" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(_lib.SIGNATURES), "binding misses a declared entry point"


def test_abi_version(lib):
    assert lib.po_abi_version() == 1


def test_check_finite_setting_returns_previous(lib):
    # host-only switch: off by default, each call returns the setting it replaces
    prev = lib.po_set_check_finite(1)
    try:
        assert prev == 0
        assert lib.po_set_check_finite(1) == 1
        assert lib.po_set_check_finite(0) == 1
        assert lib.po_set_check_finite(0) == 0
    finally:
        lib.po_set_check_finite(0)


def _specs(**kw):
    s = W.pulse_spec(n_s=4, order=4, T=400.0, nt=64)
    s.update(kw)
    arr = (_lib.PulseSpec * 1)()
    arr[0] = _lib.PulseSpec(s["n_s"], s["order"], s["omega_min"], s["omega_max"], s["T"], s["nt"], s["norm"],
                            s["norm_value"])
    return arr


@pytest.mark.parametrize("bad", [dict(T=0.0), dict(nt=1), dict(order=5), dict(n_s=65, order=4), dict(omega_max=0.0),
                                 dict(omega_min=0.001), dict(norm=7), dict(norm_value=-1.0),
                                 dict(T=1.0, omega_max=1e6)])
def test_invalid_specs_rejected_on_host(lib, bad):
    st = lib.po_pulse_synth(1, _specs(**bad), None, None, None, None, None, None)
    assert st == _lib.PO_ERR_INVALID
    assert lib.po_last_error()


def test_invalid_counts_and_grids_rejected(lib):
    assert lib.po_pulse_synth(0, _specs(), None, None, None, None, None, None) == _lib.PO_ERR_INVALID
    g = (_lib.Grid * 1)()
    g[0].n[:] = [4, 4, 0]
    g[0].lo[:] = [-1, -1, 0]
    g[0].hi[:] = [1, 1, 0]
    assert lib.po_evolve_modes(1, _specs(), g, None, None, None, None, None, None) == _lib.PO_ERR_INVALID
    assert b"n[2]" in lib.po_last_error()
    g[0].n[:] = [4, 4, 2]
    assert lib.po_evolve_modes(1, _specs(), g, None, None, None, None, None, None) == _lib.PO_ERR_INVALID
    assert lib.po_pair_yield(0, g, None, None, None) == _lib.PO_ERR_INVALID


@pytest.mark.parametrize("bad", [dict(pop=3), dict(dim=0), dict(F=2.5), dict(CR=1.5), dict(lo=1.0, hi=-1.0)])
def test_invalid_de_params_rejected(lib, bad):
    p = dict(pop=8, dim=16, n_s=4, F=0.8, CR=0.9, lo=-1.0, hi=1.0, seed=1)
    p.update(bad)
    prm = _lib.DEParams(p["pop"], p["dim"], p["n_s"], p["F"], p["CR"], p["lo"], p["hi"], p["seed"])
    assert lib.po_de_propose(ctypes.byref(prm), 0, None, None, None, None) == _lib.PO_ERR_INVALID
    assert lib.po_de_select(ctypes.byref(prm), None, None, None, None, None, None) == _lib.PO_ERR_INVALID


def test_de_generation_requires_matching_dim(lib):
    prm = _lib.DEParams(8, 15, 4, 0.8, 0.9, -1.0, 1.0, 1)
    g = (_lib.Grid * 1)()
    g[0].n[:] = [4, 4, 1]
    g[0].lo[:] = [-1, -1, 0]
    g[0].hi[:] = [1, 1, 0]
    assert lib.po_de_generation(ctypes.byref(prm), 0, _specs(), g, None, None, None, None, None) == _lib.PO_ERR_INVALID
    assert b"4 n_s" in lib.po_last_error()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        _lib.load()


def _grid1():
    g = (_lib.Grid * 1)()
    g[0].n[:] = [4, 4, 1]
    g[0].lo[:] = [-1, -1, 0]
    g[0].hi[:] = [1, 1, 0]
    return g


def test_solver_entry_points_validate_on_host(lib):
    off = (ctypes.c_double * 2)(0.0, 0.5)
    # sample counts, offsets and outputs
    assert lib.po_field_samples(1, _specs(), None, 0, off, 1, None, None, None, None, None, None) == _lib.PO_ERR_INVALID
    assert lib.po_field_samples(1, _specs(), None, 9, off, 1, None, None, None, None, None, None) == _lib.PO_ERR_INVALID
    bad = (ctypes.c_double * 2)(0.0, 1.5)
    assert lib.po_field_samples(1, _specs(), None, 2, bad, 1, None, None, None, None, None, None) == _lib.PO_ERR_INVALID
    assert b"offsets" in lib.po_last_error()
    assert lib.po_field_samples(1, _specs(), None, 2, off, 1, None, None, None, None, None, None) == _lib.PO_ERR_INVALID
    assert b"at least one" in lib.po_last_error()
    # tables must be given
    assert lib.po_qke_modes(1, _specs(), _grid1(), None, None, None, 0, None, None, None) == _lib.PO_ERR_INVALID
    assert lib.po_evolve_modes_m4(1, _specs(), _grid1(), None, None, None, None, None) == _lib.PO_ERR_INVALID
    assert lib.po_evolve_modes_m4(0, _specs(), _grid1(), None, None, None, None, None) == _lib.PO_ERR_INVALID
    assert lib.po_probe_fp64_fma(2, 4, 16, None, None, None) == _lib.PO_ERR_INVALID
    assert lib.po_probe_fp64_fma(4, 3, 16, None, None, None) == _lib.PO_ERR_INVALID
    assert lib.po_probe_fp64_fma(4, 4, 0, None, None, None) == _lib.PO_ERR_INVALID
    for order in (2, 3, 4):
        assert lib.po_evolve_modes_split(1, _specs(), _grid1(), order, None, None, None, None,
                                         None) == _lib.PO_ERR_INVALID


@pytest.mark.parametrize("bad", [dict(islands=0), dict(islands=65), dict(pop=30, islands=4), dict(pop=12, islands=4),
                                 dict(tau1=1.5), dict(tau2=-0.1), dict(F_lo=0.5, F_hi=0.2), dict(F_hi=2.5),
                                 dict(lo=1.0, hi=-1.0)])
def test_invalid_jde_params_rejected(lib, bad):
    p = dict(pop=32, dim=16, n_s=4, islands=4, tau1=0.1, tau2=0.1, F_lo=0.1, F_hi=1.0, lo=-1.0, hi=1.0, seed=1)
    p.update(bad)
    prm = _lib.JDEParams(p["pop"], p["dim"], p["n_s"], p["islands"], p["tau1"], p["tau2"], p["F_lo"], p["F_hi"],
                         p["lo"], p["hi"], p["seed"])
    assert lib.po_jde_propose(ctypes.byref(prm), 0, None, None, None, None, None, None) == _lib.PO_ERR_INVALID
    assert lib.po_island_migrate(ctypes.byref(prm), None, None, None, None) == _lib.PO_ERR_INVALID
