"""Python binding of the libpairopt C ABI (include/pairopt.h), one function per entry point.

Argument marshalling only: every step runs in the HIP kernels of libpairopt.so.  Device
arrays are torch tensors on the current HIP device (float64 unless stated, contiguous); work is
enqueued on torch's current stream.  Specs and grids are dicts as produced by
paper_1704_08919_amd.workloads.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import DEParams, Grid, JDEParams, PlanConfig, PulseSpec, check, load


def _spec_array(specs):
    arr = (PulseSpec * len(specs))()
    for i, s in enumerate(specs):
        arr[i] = PulseSpec(int(s["n_s"]), int(s["order"]), float(s["omega_min"]), float(s["omega_max"]), float(s["T"]),
                           int(s["nt"]), int(s["norm"]), float(s["norm_value"]))
    return arr


def _grid_array(grids):
    arr = (Grid * len(grids))()
    for i, g in enumerate(grids):
        arr[i].n[:] = [int(x) for x in g["n"]]
        arr[i].lo[:] = [float(x) for x in g["lo"]]
        arr[i].hi[:] = [float(x) for x in g["hi"]]
    return arr


def _ptr(t, dtype=torch.float64):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("expected a device (cuda/HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _de_params(pop, dim, n_s, F, CR, lo, hi, seed):
    return DEParams(int(pop), int(dim), int(n_s), float(F), float(CR), float(lo), float(hi), int(seed) & (2 ** 64 - 1))


def abi_version():
    return load().po_abi_version()


# ------------------------------------------------------------------------------- raw ABI
def po_pulse_synth(specs, coeff, A, A_edge, E=None, scale=None, stream=None):
    sp = _spec_array(specs)
    check(load().po_pulse_synth(len(specs), sp, _ptr(coeff), _ptr(A), _ptr(E), _ptr(A_edge), _ptr(scale),
                                _stream(stream)))


def po_evolve_modes(specs, grids, A, A_edge, f=None, J=None, plan=None, stream=None):
    sp, gr = _spec_array(specs), _grid_array(grids)
    ph = plan.handle if plan is not None else None
    check(load().po_evolve_modes(len(specs), sp, gr, _ptr(A), _ptr(A_edge), _ptr(f), _ptr(J), ph, _stream(stream)))


GAUSS2 = (0.5 - 3 ** 0.5 / 6, 0.5 + 3 ** 0.5 / 6)  # Gauss-Legendre nodes on [0, 1] (po_evolve_modes_m4)
QKE_OFFSETS = (0.0, 0.5)  # with with_end=True: the 2 nt + 1 points of po_qke_modes


def po_field_samples(specs, coeff, offsets, with_end=False, E=None, Ed=None, A=None, A_edge=None, scale=None,
                     stream=None):
    sp = _spec_array(specs)
    off = (ctypes.c_double * len(offsets))(*[float(c) for c in offsets])
    check(load().po_field_samples(len(specs), sp, _ptr(coeff), len(offsets), off, int(bool(with_end)), _ptr(E),
                                  _ptr(Ed), _ptr(A), _ptr(A_edge), _ptr(scale), _stream(stream)))


def po_qke_modes(specs, grids, E, Ed, A, linear=False, f=None, J=None, stream=None):
    sp, gr = _spec_array(specs), _grid_array(grids)
    check(load().po_qke_modes(len(specs), sp, gr, _ptr(E), _ptr(Ed), _ptr(A), int(bool(linear)), _ptr(f), _ptr(J),
                              _stream(stream)))


def po_evolve_modes_m4(specs, grids, Ag, A_edge, f=None, J=None, stream=None):
    sp, gr = _spec_array(specs), _grid_array(grids)
    check(load().po_evolve_modes_m4(len(specs), sp, gr, _ptr(Ag), _ptr(A_edge), _ptr(f), _ptr(J), _stream(stream)))


_W1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
SPLIT4_OFFSETS = (_W1 / 2, 0.5, 1.0 - _W1 / 2)  # substep midpoints of po_evolve_modes_split, order 4


def po_evolve_modes_split(specs, grids, order, At, A_edge, f=None, J=None, stream=None):
    sp, gr = _spec_array(specs), _grid_array(grids)
    check(load().po_evolve_modes_split(len(specs), sp, gr, int(order), _ptr(At), _ptr(A_edge), _ptr(f), _ptr(J),
                                       _stream(stream)))


def po_yield_gradient(specs, grids, A, A_edge, gA, J=None, gedge=None, stream=None):
    sp, gr = _spec_array(specs), _grid_array(grids)
    check(load().po_yield_gradient(len(specs), sp, gr, _ptr(A), _ptr(A_edge), _ptr(J), _ptr(gA), _ptr(gedge),
                                   _stream(stream)))


def po_synth_gradient(specs, coeff, gA, grad, gedge=None, U=None, gU=None, stream=None):
    sp = _spec_array(specs)
    check(load().po_synth_gradient(len(specs), sp, _ptr(coeff), _ptr(gA), _ptr(gedge), _ptr(grad), _ptr(U), _ptr(gU),
                                   _stream(stream)))


def po_evaluate_gradient(specs, grids, coeff, J, grad, U=None, gU=None, stream=None):
    sp, gr = _spec_array(specs), _grid_array(grids)
    check(load().po_evaluate_gradient(len(specs), sp, gr, _ptr(coeff), _ptr(J), _ptr(grad), _ptr(U), _ptr(gU),
                                      _stream(stream)))


def po_pair_yield(grids, f, J, stream=None):
    gr = _grid_array(grids)
    check(load().po_pair_yield(len(grids), gr, _ptr(f), _ptr(J), _stream(stream)))


def po_evaluate(specs, grids, coeff, A, A_edge, J, scale=None, f=None, stream=None):
    sp, gr = _spec_array(specs), _grid_array(grids)
    check(load().po_evaluate(len(specs), sp, gr, _ptr(coeff), _ptr(A), _ptr(A_edge), _ptr(scale), _ptr(f), _ptr(J),
                             None, _stream(stream)))


def po_evaluate_noalloc(specs, grids, coeff, A, A_edge, J, scale=None, f=None, stream=None):
    sp, gr = _spec_array(specs), _grid_array(grids)
    check(load().po_evaluate_noalloc(len(specs), sp, gr, _ptr(coeff), _ptr(A), _ptr(A_edge), _ptr(scale), _ptr(f),
                                     _ptr(J), _stream(stream)))


def po_de_propose(params, generation, pop, trial, idx=None, stream=None):
    check(load().po_de_propose(ctypes.byref(params), int(generation), _ptr(pop), _ptr(trial),
                               _ptr(idx, torch.int32), _stream(stream)))


def po_de_select(params, pop, fit, trial, trial_fit, mask=None, stream=None):
    check(load().po_de_select(ctypes.byref(params), _ptr(pop), _ptr(fit), _ptr(trial), _ptr(trial_fit),
                              _ptr(mask, torch.uint8), _stream(stream)))


def jde_params(pop, dim, n_s, islands=1, tau1=0.1, tau2=0.1, F_lo=0.1, F_hi=1.0, lo=-1.0, hi=1.0, seed=0):
    """Parameters of self-adaptive DE (jDE) on islands (po_jde_params)."""
    return JDEParams(int(pop), int(dim), int(n_s), int(islands), float(tau1), float(tau2), float(F_lo), float(F_hi),
                     float(lo), float(hi), int(seed) & (2 ** 64 - 1))


def po_jde_propose(params, generation, pop, fcr, trial, trial_fcr, idx=None, stream=None):
    check(load().po_jde_propose(ctypes.byref(params), int(generation), _ptr(pop), _ptr(fcr), _ptr(trial),
                                _ptr(trial_fcr), _ptr(idx, torch.int32), _stream(stream)))


def po_jde_select(params, pop, fit, fcr, trial, trial_fit, trial_fcr, mask=None, stream=None):
    check(load().po_jde_select(ctypes.byref(params), _ptr(pop), _ptr(fit), _ptr(fcr), _ptr(trial), _ptr(trial_fit),
                               _ptr(trial_fcr), _ptr(mask, torch.uint8), _stream(stream)))


def po_island_migrate(params, pop, fit, fcr, stream=None):
    check(load().po_island_migrate(ctypes.byref(params), _ptr(pop), _ptr(fit), _ptr(fcr), _stream(stream)))


def po_jde_generation(params, generation, spec, grid, pop, fit, fcr, trial, trial_fit, trial_fcr, stream=None):
    sp, gr = _spec_array([spec]), _grid_array([grid])
    check(load().po_jde_generation(ctypes.byref(params), int(generation), sp, gr, _ptr(pop), _ptr(fit), _ptr(fcr),
                                   _ptr(trial), _ptr(trial_fit), _ptr(trial_fcr), _stream(stream)))


def po_de_generation(params, generation, spec, grid, pop, fit, trial, trial_fit, stream=None):
    sp, gr = _spec_array([spec]), _grid_array([grid])
    check(load().po_de_generation(ctypes.byref(params), int(generation), sp, gr, _ptr(pop), _ptr(fit), _ptr(trial),
                                  _ptr(trial_fit), _stream(stream)))


class Plan:
    """po_plan_create / po_plan_evaluate / po_plan_destroy for a fixed batch of pulses.

    config: None (autotune) or dict(threads=, modes_per_lane=, persistent=, workgroups=), where 0
    (or -1 for persistent) leaves that choice to the autotuner."""

    def __init__(self, specs, grids, config=None, cache_path=None, stream=None):
        self.specs, self.grids = list(specs), list(grids)
        sp, gr = _spec_array(self.specs), _grid_array(self.grids)
        cfg = None
        if config is not None:
            cfg = PlanConfig(int(config.get("threads", 0)), int(config.get("modes_per_lane", 0)),
                             int(config.get("persistent", -1)), int(config.get("workgroups", 0)))
        h = ctypes.c_void_p()
        path = cache_path.encode() if cache_path else None
        check(load().po_plan_create(len(self.specs), sp, gr, ctypes.byref(cfg) if cfg is not None else None, path,
                                    _stream(stream), ctypes.byref(h)))
        self.handle = h

    @property
    def config(self):
        c = PlanConfig()
        check(load().po_plan_get_config(self.handle, ctypes.byref(c)))
        return dict(threads=c.threads, modes_per_lane=c.modes_per_lane, persistent=c.persistent,
                    workgroups=c.workgroups)

    def evaluate(self, coeff, J, f=None, stream=None):
        check(load().po_plan_evaluate(self.handle, _ptr(coeff), _ptr(J), _ptr(f), _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            load().po_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def po_set_check_finite(on=True):
    """Enables (or disables) the library's check that results are finite; returns the previous
    setting.  While enabled, the checked calls wait for their stream and raise POError
    (PO_ERR_NUMERIC) when a result holds non-finite values."""
    return bool(load().po_set_check_finite(1 if on else 0))


def po_timer_enable(on=True):
    check(load().po_timer_enable(1 if on else 0))


def po_probe_fp64_fma(waves_per_simd, chains, iters, sink, stream=None):
    """Launches the FP64 FMA issue probe; returns the FP64 operations launched."""
    flop = ctypes.c_double()
    check(load().po_probe_fp64_fma(int(waves_per_simd), int(chains), int(iters), _ptr(sink), ctypes.byref(flop),
                                   _stream(stream)))
    return flop.value


def po_timer_read():
    """(summed ms of the bracketed evolution launches, number of bracketed calls); clears them."""
    ms, n = ctypes.c_double(0.0), ctypes.c_int64(0)
    check(load().po_timer_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


class MLP:
    """po_mlp_*: the surrogate network (BF16 MFMA, FP32 accumulation and master weights, Adam)."""

    def __init__(self, n_in=32, width=256, depth=3, max_batch=1024, seed=0, stream=None):
        h = ctypes.c_void_p()
        check(load().po_mlp_create(int(n_in), int(width), int(depth), int(max_batch), int(seed) & (2 ** 64 - 1),
                                   _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.n_in, self.width, self.depth, self.max_batch = n_in, width, depth, max_batch
        self.n_params = int(load().po_mlp_param_count(h))

    def get_params(self, stream=None):
        p = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        check(load().po_mlp_get_params(self.handle, _ptr(p, torch.float32), _stream(stream)))
        return p

    def set_params(self, params, stream=None):
        check(load().po_mlp_set_params(self.handle, _ptr(params, torch.float32), _stream(stream)))

    def forward(self, x, y=None, stream=None):
        B = x.shape[0]
        y = torch.empty(B, dtype=torch.float32, device="cuda") if y is None else y
        check(load().po_mlp_forward(self.handle, _ptr(x), int(B), _ptr(y, torch.float32), _stream(stream)))
        return y

    def loss_grad(self, x, target, want_grad=True, stream=None):
        B = x.shape[0]
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda") if want_grad else None
        check(load().po_mlp_loss_grad(self.handle, _ptr(x), _ptr(target, torch.float32), int(B),
                                      _ptr(loss, torch.float32), _ptr(g, torch.float32), _stream(stream)))
        return loss, g

    def adam_step(self, grad=None, lr=1e-3, stream=None):
        check(load().po_mlp_adam_step(self.handle, _ptr(grad, torch.float32), float(lr), _stream(stream)))

    def train_step(self, x, target, lr=1e-3, loss=None, stream=None):
        check(load().po_mlp_train_step(self.handle, _ptr(x), _ptr(target, torch.float32), int(x.shape[0]), float(lr),
                                       _ptr(loss, torch.float32), _stream(stream)))

    def train_indexed(self, X, J, idx, steps, batch, mean, inv_std, lr=1e-3, losses=None, stream=None):
        """`steps` steps on minibatches X[idx[s batch:(s + 1) batch]] of a device data set, targets
        the standardised log10 J (po_mlp_train_indexed)."""
        check(load().po_mlp_train_indexed(self.handle, _ptr(X), _ptr(J), int(X.shape[0]), _ptr(idx, torch.int32),
                                          int(steps), int(batch), float(mean), float(inv_std), float(lr),
                                          _ptr(losses, torch.float32), _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            load().po_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def po_topk_mask(score, k, mask=None, stream=None):
    n = score.shape[0]
    mask = torch.empty(n, dtype=torch.uint8, device="cuda") if mask is None else mask
    check(load().po_topk_mask(_ptr(score, torch.float32), int(n), int(k), _ptr(mask, torch.uint8), _stream(stream)))
    return mask


def po_mask_indices(mask, idx=None, count=None, stream=None):
    n = mask.shape[0]
    idx = torch.empty(n, dtype=torch.int32, device="cuda") if idx is None else idx
    check(load().po_mask_indices(_ptr(mask, torch.uint8), int(n), _ptr(idx, torch.int32), _ptr(count, torch.int32),
                                 _stream(stream)))
    return idx


def po_gather_rows(src, idx, n_idx, dst=None, stream=None):
    rows, cols = src.shape
    dst = torch.empty((n_idx, cols), dtype=torch.float64, device="cuda") if dst is None else dst
    check(load().po_gather_rows(_ptr(src), int(rows), int(cols), _ptr(idx, torch.int32), int(n_idx), _ptr(dst),
                                _stream(stream)))
    return dst


def po_scatter_values(vals, idx, n_idx, dst, fill=float("-inf"), stream=None):
    check(load().po_scatter_values(_ptr(vals), _ptr(idx, torch.int32), int(n_idx), float(fill), _ptr(dst),
                                   int(dst.shape[0]), _stream(stream)))
    return dst


def po_log10_standardize(J, mean, inv_std, floor=1e-300, out=None, stream=None):
    n = J.shape[0]
    out = torch.empty(n, dtype=torch.float32, device="cuda") if out is None else out
    check(load().po_log10_standardize(_ptr(J), int(n), float(floor), float(mean), float(inv_std),
                                      _ptr(out, torch.float32), _stream(stream)))
    return out


SERIES_VARIANTS = ("tan4", "tan5", "tan6", "tan7", "tan8", "tan9", "tan10", "tan11", "cossin7_halving")


def po_timer_mode_steps():
    """Mode-steps evolved per series variant since the last read (dict); clears the counts."""
    arr = (ctypes.c_uint64 * len(SERIES_VARIANTS))()
    check(load().po_timer_mode_steps(arr, len(SERIES_VARIANTS)))
    return {k: int(v) for k, v in zip(SERIES_VARIANTS, arr)}


# ------------------------------------------------------------------------ conveniences
def table_rows(specs):
    return sum(int(s["nt"]) for s in specs)


def n_modes(grids):
    return sum(int(g["n"][0]) * int(g["n"][1]) * int(g["n"][2]) for g in grids)


def synth(specs, coeff, want_E=False, device="cuda"):
    """Allocates outputs and runs po_pulse_synth: returns (A, A_edge, scale, E or None)."""
    rows = table_rows(specs)
    coeff = torch.as_tensor(coeff, dtype=torch.float64).reshape(-1).contiguous().to(device)
    A = torch.empty((rows, 2), dtype=torch.float64, device=device)
    E = torch.empty((rows, 2), dtype=torch.float64, device=device) if want_E else None
    edge = torch.empty((len(specs), 2, 2), dtype=torch.float64, device=device)
    scale = torch.empty(len(specs), dtype=torch.float64, device=device)
    po_pulse_synth(specs, coeff, A, edge, E=E, scale=scale)
    return A, edge, scale, E


def evolve(specs, grids, A, A_edge, want_f=True, want_J=True, device="cuda"):
    """Allocates outputs and runs po_evolve_modes: returns (f or None, J or None)."""
    f = torch.empty(n_modes(grids), dtype=torch.float64, device=device) if want_f else None
    J = torch.empty(len(specs), dtype=torch.float64, device=device) if want_J else None
    po_evolve_modes(specs, grids, A, A_edge, f=f, J=J)
    return f, J


def evaluate(specs, grids, coeff, want_f=False, device="cuda"):
    """Synthesis -> evolution -> J for a batch of pulses; returns (J, f or None)."""
    rows = table_rows(specs)
    coeff = torch.as_tensor(coeff, dtype=torch.float64).reshape(-1).contiguous().to(device)
    A = torch.empty((rows, 2), dtype=torch.float64, device=device)
    edge = torch.empty((len(specs), 2, 2), dtype=torch.float64, device=device)
    J = torch.empty(len(specs), dtype=torch.float64, device=device)
    f = torch.empty(n_modes(grids), dtype=torch.float64, device=device) if want_f else None
    po_evaluate(specs, grids, coeff, A, edge, J, f=f)
    return J, f


def field_samples(specs, coeff, offsets, with_end=False, device="cuda"):
    """Allocates outputs and runs po_field_samples: returns (E, Ed, A, A_edge, scale), arrays [rows][2]."""
    rows = sum(int(s["nt"]) * len(offsets) + (1 if with_end else 0) for s in specs)
    coeff = torch.as_tensor(coeff, dtype=torch.float64).reshape(-1).contiguous().to(device)
    E, Ed, A = (torch.empty((rows, 2), dtype=torch.float64, device=device) for _ in range(3))
    edge = torch.empty((len(specs), 2, 2), dtype=torch.float64, device=device)
    scale = torch.empty(len(specs), dtype=torch.float64, device=device)
    po_field_samples(specs, coeff, offsets, with_end, E=E, Ed=Ed, A=A, A_edge=edge, scale=scale)
    return E, Ed, A, edge, scale


def qke(specs, grids, E, Ed, A, linear=False, want_f=True, want_J=True, device="cuda"):
    """Allocates outputs and runs po_qke_modes: returns (f or None, J or None)."""
    f = torch.empty(n_modes(grids), dtype=torch.float64, device=device) if want_f else None
    J = torch.empty(len(specs), dtype=torch.float64, device=device) if want_J else None
    po_qke_modes(specs, grids, E, Ed, A, linear=linear, f=f, J=J)
    return f, J


def evolve_m4(specs, grids, Ag, A_edge, want_f=True, want_J=True, device="cuda"):
    """Allocates outputs and runs po_evolve_modes_m4: returns (f or None, J or None)."""
    f = torch.empty(n_modes(grids), dtype=torch.float64, device=device) if want_f else None
    J = torch.empty(len(specs), dtype=torch.float64, device=device) if want_J else None
    po_evolve_modes_m4(specs, grids, Ag, A_edge, f=f, J=J)
    return f, J


def evolve_split(specs, grids, order, At, A_edge, want_f=True, want_J=True, device="cuda"):
    """Allocates outputs and runs po_evolve_modes_split: returns (f or None, J or None)."""
    f = torch.empty(n_modes(grids), dtype=torch.float64, device=device) if want_f else None
    J = torch.empty(len(specs), dtype=torch.float64, device=device) if want_J else None
    po_evolve_modes_split(specs, grids, order, At, A_edge, f=f, J=J)
    return f, J


def evaluate_gradient(specs, grids, coeff, device="cuda"):
    """Allocates outputs and runs po_evaluate_gradient: returns (J, dJ/dc [sum 4 n_s], U, dU/dc)."""
    coeff = torch.as_tensor(coeff, dtype=torch.float64).reshape(-1).contiguous().to(device)
    J = torch.empty(len(specs), dtype=torch.float64, device=device)
    U = torch.empty(len(specs), dtype=torch.float64, device=device)
    grad, gU = torch.empty_like(coeff), torch.empty_like(coeff)
    po_evaluate_gradient(specs, grids, coeff, J, grad, U=U, gU=gU)
    return J, grad, U, gU


def de_params(pop, dim, n_s, F=0.8, CR=0.9, lo=-1.0, hi=1.0, seed=0):
    return _de_params(pop, dim, n_s, F, CR, lo, hi, seed)
