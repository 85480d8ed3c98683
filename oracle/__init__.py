"""CPU oracle for the pair-yield evaluation (arXiv:1704.08919) -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg import this package.
The product path (the HIP library and its Python binding) never imports, links or calls it,
and it shares no code with that path.

The numerical work lives in oracle.cpp (plain C++, long double for parity references and double
for the timed baseline); this module only marshals numpy arrays through ctypes.  Every function
cites the passage of the paper it follows in oracle.cpp.  The MLP reference lives in
oracle/mlp.py.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_lib_fast = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_U32 = ctypes.POINTER(ctypes.c_uint32)
_I32 = ctypes.POINTER(ctypes.c_int32)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_L = ctypes.POINTER(ctypes.c_long)

NORM_NONE, NORM_PEAK, NORM_ENERGY = 0, 1, 2


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB_PATH") or _build.LIB  # the override loads a sanitizer build
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        c_int, c_long, c_double = ctypes.c_int, ctypes.c_long, ctypes.c_double
        sig = {
            "orc_bspline_ld": (None, [c_int, c_int, c_double, c_double, c_double, _D]),
            "orc_spectra_ld": (c_int, [c_int, c_int, c_double, c_double, c_double, _D, c_int, _D, _D, _D]),
            "orc_field_at_ld": (None, [c_int, c_int, c_double, c_double, c_double, _D, c_int, _D, _D, _D]),
            "orc_synth_ld": (None, [c_int, c_int, c_double, c_double, c_double, c_int, c_int, c_double,
                                    _D, _D, _D, _D, _D]),
            "orc_synth_d": (None, [c_int, c_int, c_double, c_double, c_double, c_int, c_int, c_double,
                                   _D, _D, _D, _D, _D]),
            "orc_evolve_points_ld": (None, [c_int, c_double, _D, _D, c_long, _D, _D, c_int]),
            "orc_evolve_points_d": (None, [c_int, c_double, _D, _D, c_long, _D, _D, c_int]),
            "orc_evolve_state_ld": (c_double, [c_int, c_double, _D, _D, _D, _D]),
            "orc_free_spinors_ld": (c_double, [_D, _D, _D]),
            "orc_grid_points": (c_double, [_I, _D, _D, _D]),
            "orc_yield": (c_double, [_I, _D, _D, _D]),
            "orc_evaluate_ld": (c_double, [c_int, c_int, c_double, c_double, c_double, c_int, c_int, c_double,
                                           _D, _I, _D, _D, _D, c_int]),
            "orc_evaluate_d": (c_double, [c_int, c_int, c_double, c_double, c_double, c_int, c_int, c_double,
                                          _D, _I, _D, _D, _D, c_int]),
            "orc_qke_points_ld": (None, [c_int, c_int, c_double, c_double, c_double, c_int, c_double, _D,
                                         c_int, c_int, c_long, _D, _D, c_int]),
            "orc_qke_tabulated_ld": (None, [c_int, c_double, _D, _D, _D, c_int, c_long, _D, _D, c_int]),
            "orc_qke_tabulated_d": (None, [c_int, c_double, _D, _D, _D, c_int, c_long, _D, _D, c_int]),
            "orc_qke_tabulated_q": (None, [c_int, c_double, _D, _D, _D, c_int, c_long, _D, _D, _D, c_int]),
            "orc_field_samples_ld": (None, [c_int, c_int, c_double, c_double, c_double, c_int, c_int, c_double,
                                            _D, c_int, _D, c_int, _D, _D, _D]),
            "orc_evolve4_points_ld": (None, [c_int, c_double, _D, _D, c_long, _D, _D, c_int]),
            "orc_evolve_split_points_ld": (None, [c_int, c_int, c_double, _D, _D, c_long, _D, _D, c_int]),
            "orc_grad_table_fd_ld": (None, [c_int, c_double, _D, _D, _I, _D, _D, c_double, c_int, _L, _D, c_int]),
            "orc_grad_coeff_fd_ld": (None, [c_int, c_int, c_double, c_double, c_double, c_int, c_int, c_double, _D, _I,
                                            _D, _D, c_double, _D, _D, _D, _D, c_int]),
            "orc_philox4x32_10": (None, [_U32, _U32, _U32]),
            "orc_de_propose": (None, [c_int, c_int, c_int, c_double, c_double, c_double, c_double,
                                      ctypes.c_uint64, ctypes.c_int64, _D, _D, _I32]),
            "orc_de_select": (None, [c_int, c_int, _D, _D, _D, _D, _U8]),
            "orc_jde_propose": (None, [c_int, c_int, c_int, c_int, c_double, c_double, c_double, c_double, c_double,
                                       c_double, ctypes.c_uint64, ctypes.c_int64, _D, _D, _D, _D, _I32]),
            "orc_jde_select": (None, [c_int, c_int, _D, _D, _D, _D, _D, _D, _U8]),
            "orc_island_migrate": (None, [c_int, c_int, c_int, _D, _D, _D]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def lib_fast():
    """The -O3 build with contraction allowed (timing only): double synthesis and evolution."""
    global _lib_fast
    if _lib_fast is None:
        lib()
        if not os.path.exists(_build.LIB_FAST):
            _build.build(force=False)
        L = ctypes.CDLL(_build.LIB_FAST)
        for name in ("orc_synth_d", "orc_evolve_points_d"):
            getattr(L, name).restype = getattr(_lib, name).restype
            getattr(L, name).argtypes = getattr(_lib, name).argtypes
        _lib_fast = L
    return _lib_fast


def _d(a):
    return a.ctypes.data_as(_D)


def _arr(x, dtype=np.float64):
    return np.ascontiguousarray(np.asarray(x, dtype=dtype))


# ----------------------------------------------------------------------------------- pulses
def bspline_basis(order, ns, wmin, wmax, w):
    """b_i^{(k)}(w), i = 0..ns-1 (Sec. III, Cox-de Boor recursion on clamped knots)."""
    out = np.zeros(ns)
    lib().orc_bspline_ld(order, ns, wmin, wmax, float(w), _d(out))
    return out


def spectra(spec, coeff):
    """(Omega_j, E[2][N+1], Phi[2][N+1]) sampled from the B-spline expansions (Sec. III)."""
    coeff = _arr(coeff)
    cap = 1 << 16
    Om, E, Ph = np.zeros(cap), np.zeros(2 * cap), np.zeros(2 * cap)
    n = lib().orc_spectra_ld(spec["n_s"], spec["order"], spec["omega_min"], spec["omega_max"], spec["T"],
                             _d(coeff), cap, _d(Om), _d(E), _d(Ph))
    return Om[:n].copy(), E[:2 * n].reshape(2, n).copy(), Ph[:2 * n].reshape(2, n).copy()


def field_at(spec, coeff, t):
    """Unscaled E(t)[n][2] and A(t)[n][2] (Sec. III, Eq. field and Eq. vector_potential)."""
    coeff, t = _arr(coeff), _arr(t).ravel()
    E, A = np.zeros((t.size, 2)), np.zeros((t.size, 2))
    lib().orc_field_at_ld(spec["n_s"], spec["order"], spec["omega_min"], spec["omega_max"], spec["T"],
                          _d(coeff), t.size, _d(t), _d(E), _d(A))
    return E, A


def synth(spec, coeff, precision="ld", with_E=True):
    """Scaled tables of one pulse: A_mid[nt][2], E_mid[nt][2], A_edge[2][2], scale.  precision
    "ld", "d", or "d_fast" (the double routine of the -O3 timing build)."""
    coeff = _arr(coeff)
    nt = spec["nt"]
    A, E, edge, sc = np.zeros((nt, 2)), np.zeros((nt, 2)), np.zeros((2, 2)), np.zeros(1)
    fn = {"ld": lambda: lib().orc_synth_ld, "d": lambda: lib().orc_synth_d,
          "d_fast": lambda: lib_fast().orc_synth_d}[precision]()
    fn(spec["n_s"], spec["order"], spec["omega_min"], spec["omega_max"], spec["T"], nt, spec["norm"],
       spec["norm_value"], _d(coeff), _d(A), _d(E) if with_E else None, _d(edge), _d(sc))
    return A, (E if with_E else None), edge, float(sc[0])


# --------------------------------------------------------------------------------- dynamics
def evolve_points(A_mid, A_edge, dt, p, precision="ld", nthreads=0):
    """Pair density f at momenta p[m][3] for any A table (Sec. II A); precision "ld", "d" or
    "d_fast" (the -O3 timing build)."""
    A_mid, A_edge, p = _arr(A_mid), _arr(A_edge), _arr(p).reshape(-1, 3)
    f = np.zeros(p.shape[0])
    fn = {"ld": lambda: lib().orc_evolve_points_ld, "d": lambda: lib().orc_evolve_points_d,
          "d_fast": lambda: lib_fast().orc_evolve_points_d}[precision]()
    fn(A_mid.shape[0], float(dt), _d(A_mid), _d(A_edge), p.shape[0], _d(p), _d(f), int(nthreads))
    return f


def evolve_state(A_mid, A_edge, dt, p):
    """(f, psi[2][4] complex) of one mode; psi evolved from unit-normalised v_s^in."""
    A_mid, A_edge, p = _arr(A_mid), _arr(A_edge), _arr(p).ravel()
    psi = np.zeros((2, 4, 2))
    f = lib().orc_evolve_state_ld(A_mid.shape[0], float(dt), _d(A_mid), _d(A_edge), _d(p), _d(psi))
    return f, psi[..., 0] + 1j * psi[..., 1]


def free_spinors(P):
    """Unit-normalised u_s, v_s (Sec. II A) at kinematic momentum P; returns (u[2][4], v[2][4], omega)."""
    P = _arr(P).ravel()
    u, v = np.zeros((2, 4, 2)), np.zeros((2, 4, 2))
    w = lib().orc_free_spinors_ld(_d(P), _d(u), _d(v))
    return u[..., 0] + 1j * u[..., 1], v[..., 0] + 1j * v[..., 1], w


def _grid_arrays(grid):
    n = np.ascontiguousarray(np.asarray(grid["n"], dtype=np.int32))
    lo, hi = _arr(grid["lo"]), _arr(grid["hi"])
    return n, lo, hi


def grid_points(grid):
    """Cell-centred momenta p[m][3] (x fastest) and the cell volume."""
    n, lo, hi = _grid_arrays(grid)
    p = np.zeros((int(np.prod(n.astype(np.int64))), 3))
    dv = lib().orc_grid_points(n.ctypes.data_as(_I), _d(lo), _d(hi), _d(p))
    return p, dv


def pair_yield(grid, f):
    """J = Delta V sum_p f(p) (Sec. IV A, Eq. opt_prob; midpoint rule)."""
    n, lo, hi = _grid_arrays(grid)
    f = _arr(f)
    return lib().orc_yield(n.ctypes.data_as(_I), _d(lo), _d(hi), _d(f))


def evaluate(spec, grid, coeff, precision="ld", nthreads=0, want_f=False):
    """J for one pulse (synthesis, every grid mode, yield); optionally the f array."""
    coeff = _arr(coeff)
    n, lo, hi = _grid_arrays(grid)
    m = int(np.prod(n.astype(np.int64)))
    f = np.zeros(m) if want_f else None
    fn = lib().orc_evaluate_ld if precision == "ld" else lib().orc_evaluate_d
    J = fn(spec["n_s"], spec["order"], spec["omega_min"], spec["omega_max"], spec["T"], spec["nt"],
           spec["norm"], spec["norm_value"], _d(coeff), n.ctypes.data_as(_I), _d(lo), _d(hi),
           _d(f) if want_f else None, int(nthreads))
    return (J, f) if want_f else J


def qke_points(spec, coeff, p, nt, linear=False, nthreads=0):
    """Kinetic-equation f = 1 - chi_1 (Sec. II B, Eq. qke) by RK4 with nt steps."""
    coeff, p = _arr(coeff), _arr(p).reshape(-1, 3)
    f = np.zeros(p.shape[0])
    lib().orc_qke_points_ld(spec["n_s"], spec["order"], spec["omega_min"], spec["omega_max"], spec["T"],
                            spec["norm"], spec["norm_value"], _d(coeff), int(bool(linear)), int(nt),
                            p.shape[0], _d(p), _d(f), int(nthreads))
    return f


def qke_tabulated(E, Ed, A, dt, p, linear=False, nthreads=0, precision="ld", with_fmax=False):
    """Kinetic-equation f = 1 - chi_1 for caller-supplied E, dE/dt, A at the 2 nt + 1 RK4 points.
    precision "ld" (long double), "d" (double) or "q" (__float128; with_fmax also returns the largest
    |1 - chi_1(t)| of each mode over the steps)."""
    E, Ed, A, p = _arr(E), _arr(Ed), _arr(A), _arr(p).reshape(-1, 3)
    nt = (E.shape[0] - 1) // 2
    f = np.zeros(p.shape[0])
    if precision == "q":
        fmax = np.zeros(p.shape[0])
        lib().orc_qke_tabulated_q(nt, float(dt), _d(E), _d(Ed), _d(A), int(bool(linear)), p.shape[0], _d(p), _d(f),
                                  _d(fmax), int(nthreads))
        return (f, fmax) if with_fmax else f
    fn = lib().orc_qke_tabulated_ld if precision == "ld" else lib().orc_qke_tabulated_d
    fn(nt, float(dt), _d(E), _d(Ed), _d(A), int(bool(linear)), p.shape[0], _d(p), _d(f), int(nthreads))
    return f


GAUSS2 = (0.5 - 3 ** 0.5 / 6, 0.5 + 3 ** 0.5 / 6)  # Gauss-Legendre nodes on [0, 1]


def field_samples(spec, coeff, offsets, with_end=False):
    """Scaled E, dE/dt, A at t_i + (n + c) dt for every step n and offset c (rows n len(offsets) + r),
    plus t_f as a last row when with_end; arrays [rows][2]."""
    coeff, off = _arr(coeff), _arr(offsets).ravel()
    rows = spec["nt"] * off.size + (1 if with_end else 0)
    E, Ed, A = np.zeros((rows, 2)), np.zeros((rows, 2)), np.zeros((rows, 2))
    lib().orc_field_samples_ld(spec["n_s"], spec["order"], spec["omega_min"], spec["omega_max"], spec["T"],
                               spec["nt"], spec["norm"], spec["norm_value"], _d(coeff), off.size, _d(off),
                               int(bool(with_end)), _d(E), _d(Ed), _d(A))
    return E, Ed, A


def evolve4_points(A_gauss, A_edge, dt, p, nthreads=0):
    """Pair density f by the fourth-order Magnus step; A_gauss[nt][2][2] holds A at the two
    Gauss-Legendre nodes of every step (GAUSS2), A_edge[2][2] A(t_i) and A(t_f)."""
    A_gauss, A_edge, p = _arr(A_gauss), _arr(A_edge), _arr(p).reshape(-1, 3)
    nt = A_gauss.size // 4
    f = np.zeros(p.shape[0])
    lib().orc_evolve4_points_ld(nt, float(dt), _d(A_gauss), _d(A_edge), p.shape[0], _d(p), _d(f), int(nthreads))
    return f


_W1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
SPLIT4_OFFSETS = (_W1 / 2, 0.5, 1.0 - _W1 / 2)  # substep midpoints of the fourth-order splitting


def evolve_split_points(A_tab, A_edge, dt, p, order=2, nthreads=0):
    """Pair density f by the split-operator step (Sec. II A; H_0 = alpha_z p_z + beta m against the
    field-driven transverse part): order 2 = Strang with A_tab[nt][2] at the step midpoints,
    order 4 = its triple-jump composition with A_tab[nt][3][2] at SPLIT4_OFFSETS of every step."""
    A_tab, A_edge, p = _arr(A_tab), _arr(A_edge), _arr(p).reshape(-1, 3)
    if order not in (2, 4):
        raise ValueError("order must be 2 or 4")
    nt = A_tab.size // (2 if order == 2 else 6)
    f = np.zeros(p.shape[0])
    lib().orc_evolve_split_points_ld(int(order), nt, float(dt), _d(A_tab), _d(A_edge), p.shape[0], _d(p), _d(f),
                                     int(nthreads))
    return f


# ------------------------------------------------------------------------------------- DE
def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data_as(_U32), k.ctypes.data_as(_U32), o.ctypes.data_as(_U32))
    return o


def de_propose(pop, generation, F, CR, lo, hi, seed, n_s=0):
    """DE/rand/1/bin trial vectors (Sec. IV B); returns (trial, idx[N][4] = a, b, c, R)."""
    pop = _arr(pop)
    N, D = pop.shape
    trial = np.zeros_like(pop)
    idx = np.zeros((N, 4), dtype=np.int32)
    lib().orc_de_propose(N, D, int(n_s), float(F), float(CR), float(lo), float(hi), int(seed), int(generation),
                         _d(pop), _d(trial), idx.ctypes.data_as(_I32))
    return trial, idx


def de_select(pop, fit, trial, trial_fit, mask=None):
    """Greedy selection for maximisation; returns new (pop, fit)."""
    pop, fit = _arr(pop).copy(), _arr(fit).copy()
    trial, trial_fit = _arr(trial), _arr(trial_fit)
    N, D = pop.shape
    m = None
    if mask is not None:
        mask = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        m = mask.ctypes.data_as(_U8)
    lib().orc_de_select(N, D, _d(pop), _d(fit), _d(trial), _d(trial_fit), m)
    return pop, fit


def jde_propose(pop, fcr, generation, islands, lo, hi, seed, n_s=0, tau1=0.1, tau2=0.1, Flo=0.1, Fhi=1.0):
    """Self-adaptive DE (jDE) trials on islands; returns (trial, trial_fcr, idx[N][4])."""
    pop, fcr = _arr(pop), _arr(fcr)
    N, D = pop.shape
    trial, tfcr = np.zeros_like(pop), np.zeros_like(fcr)
    idx = np.zeros((N, 4), dtype=np.int32)
    lib().orc_jde_propose(N, D, int(n_s), int(islands), float(tau1), float(tau2), float(Flo), float(Fhi), float(lo),
                          float(hi), int(seed), int(generation), _d(pop), _d(fcr), _d(trial), _d(tfcr),
                          idx.ctypes.data_as(_I32))
    return trial, tfcr, idx


def jde_select(pop, fit, fcr, trial, trial_fit, trial_fcr, mask=None):
    """jDE selection for maximisation; returns new (pop, fit, fcr)."""
    pop, fit, fcr = _arr(pop).copy(), _arr(fit).copy(), _arr(fcr).copy()
    trial, trial_fit, trial_fcr = _arr(trial), _arr(trial_fit), _arr(trial_fcr)
    N, D = pop.shape
    m = None
    if mask is not None:
        mask = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        m = mask.ctypes.data_as(_U8)
    lib().orc_jde_select(N, D, _d(pop), _d(fit), _d(fcr), _d(trial), _d(trial_fit), _d(trial_fcr), m)
    return pop, fit, fcr


def island_migrate(pop, fit, fcr, islands):
    """Ring migration (best of island k replaces the worst of island k+1); returns new (pop, fit, fcr)."""
    pop, fit, fcr = _arr(pop).copy(), _arr(fit).copy(), _arr(fcr).copy()
    N, D = pop.shape
    lib().orc_island_migrate(N, D, int(islands), _d(pop), _d(fit), _d(fcr))
    return pop, fit, fcr


def grad_table_fd(A_mid, A_edge, dt, grid, entries, h=2.0 ** -20, nthreads=0):
    """dJ/dx by a fourth-order central difference for table entries: e < 2 nt is A_mid[e//2][e%2],
    e = 2 nt + r is A_edge[r//2][r%2]; J in long double."""
    A_mid, A_edge = _arr(A_mid), _arr(A_edge)
    n, lo, hi = _grid_arrays(grid)
    idx = np.ascontiguousarray(np.asarray(entries, dtype=np.int64))
    out = np.zeros(idx.size)
    lib().orc_grad_table_fd_ld(A_mid.shape[0], float(dt), _d(A_mid), _d(A_edge), n.ctypes.data_as(_I), _d(lo),
                               _d(hi), float(h), idx.size, idx.ctypes.data_as(_L), _d(out), int(nthreads))
    return out


def grad_coeff_fd(spec, grid, coeff, h=2.0 ** -14, nthreads=0):
    """(J, U, dJ/dc, dU/dc) of one synthesised pulse by fourth-order central differences."""
    coeff = _arr(coeff).ravel()
    n, lo, hi = _grid_arrays(grid)
    gJ, gU, J, U = np.zeros(coeff.size), np.zeros(coeff.size), np.zeros(1), np.zeros(1)
    lib().orc_grad_coeff_fd_ld(spec["n_s"], spec["order"], spec["omega_min"], spec["omega_max"], spec["T"], spec["nt"],
                               spec["norm"], spec["norm_value"], _d(coeff), n.ctypes.data_as(_I), _d(lo), _d(hi),
                               float(h), _d(gJ), _d(gU), _d(J), _d(U), int(nthreads))
    return float(J[0]), float(U[0]), gJ, gU
