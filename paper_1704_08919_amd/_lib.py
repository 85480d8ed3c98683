"""ctypes loader of libpairopt.so (built in-tree by paper_1704_08919_amd.build).

The product path has no fallback: if the HIP library is missing or does not load, every call
raises, naming the file that is expected.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpairopt.so")

PO_OK, PO_ERR_INVALID, PO_ERR_DEVICE, PO_ERR_NOMEM, PO_ERR_NUMERIC, PO_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
PO_NORM_NONE, PO_NORM_PEAK, PO_NORM_ENERGY = 0, 1, 2

_STATUS_NAMES = {PO_OK: "PO_OK", PO_ERR_INVALID: "PO_ERR_INVALID", PO_ERR_DEVICE: "PO_ERR_DEVICE",
                 PO_ERR_NOMEM: "PO_ERR_NOMEM", PO_ERR_NUMERIC: "PO_ERR_NUMERIC",
                 PO_ERR_UNSUPPORTED: "PO_ERR_UNSUPPORTED"}


class POError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class PulseSpec(ctypes.Structure):
    _fields_ = [("n_s", ctypes.c_int32), ("order", ctypes.c_int32), ("omega_min", ctypes.c_double),
                ("omega_max", ctypes.c_double), ("T", ctypes.c_double), ("nt", ctypes.c_int32),
                ("norm", ctypes.c_int32), ("norm_value", ctypes.c_double)]


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


class DEParams(ctypes.Structure):
    _fields_ = [("pop", ctypes.c_int32), ("dim", ctypes.c_int32), ("n_s", ctypes.c_int32), ("F", ctypes.c_double),
                ("CR", ctypes.c_double), ("lo", ctypes.c_double), ("hi", ctypes.c_double), ("seed", ctypes.c_uint64)]


class JDEParams(ctypes.Structure):
    _fields_ = [("pop", ctypes.c_int32), ("dim", ctypes.c_int32), ("n_s", ctypes.c_int32), ("islands", ctypes.c_int32),
                ("tau1", ctypes.c_double), ("tau2", ctypes.c_double), ("F_lo", ctypes.c_double),
                ("F_hi", ctypes.c_double), ("lo", ctypes.c_double), ("hi", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class PlanConfig(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("modes_per_lane", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("workgroups", ctypes.c_int32)]


_P = ctypes.c_void_p
_I32, _I64 = ctypes.c_int32, ctypes.c_int64

# name -> argtypes (restype po_status = int unless stated)
SIGNATURES = {
    "po_abi_version": ([], ctypes.c_int),
    "po_last_error": ([], ctypes.c_char_p),
    "po_pulse_synth": ([_I32, ctypes.POINTER(PulseSpec), _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "po_evolve_modes": ([_I32, ctypes.POINTER(PulseSpec), ctypes.POINTER(Grid), _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "po_pair_yield": ([_I32, ctypes.POINTER(Grid), _P, _P, _P], ctypes.c_int),
    "po_field_samples": ([_I32, ctypes.POINTER(PulseSpec), _P, _I32, ctypes.POINTER(ctypes.c_double), _I32, _P, _P, _P,
                          _P, _P, _P], ctypes.c_int),
    "po_qke_modes": ([_I32, ctypes.POINTER(PulseSpec), ctypes.POINTER(Grid), _P, _P, _P, _I32, _P, _P, _P],
                     ctypes.c_int),
    "po_yield_gradient": ([_I32, ctypes.POINTER(PulseSpec), ctypes.POINTER(Grid), _P, _P, _P, _P, _P, _P],
                          ctypes.c_int),
    "po_synth_gradient": ([_I32, ctypes.POINTER(PulseSpec), _P, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "po_evaluate_gradient": ([_I32, ctypes.POINTER(PulseSpec), ctypes.POINTER(Grid), _P, _P, _P, _P, _P, _P],
                             ctypes.c_int),
    "po_evolve_modes_m4": ([_I32, ctypes.POINTER(PulseSpec), ctypes.POINTER(Grid), _P, _P, _P, _P, _P],
                           ctypes.c_int),
    "po_evolve_modes_split": ([_I32, ctypes.POINTER(PulseSpec), ctypes.POINTER(Grid), _I32, _P, _P, _P, _P, _P],
                              ctypes.c_int),
    "po_evaluate_noalloc": ([_I32, ctypes.POINTER(PulseSpec), ctypes.POINTER(Grid), _P, _P, _P, _P, _P, _P, _P],
                            ctypes.c_int),
    "po_evaluate": ([_I32, ctypes.POINTER(PulseSpec), ctypes.POINTER(Grid), _P, _P, _P, _P, _P, _P, _P, _P],
                    ctypes.c_int),
    "po_de_propose": ([ctypes.POINTER(DEParams), _I64, _P, _P, _P, _P], ctypes.c_int),
    "po_jde_propose": ([ctypes.POINTER(JDEParams), _I64, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "po_jde_select": ([ctypes.POINTER(JDEParams), _P, _P, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "po_island_migrate": ([ctypes.POINTER(JDEParams), _P, _P, _P, _P], ctypes.c_int),
    "po_jde_generation": ([ctypes.POINTER(JDEParams), _I64, ctypes.POINTER(PulseSpec), ctypes.POINTER(Grid), _P, _P,
                           _P, _P, _P, _P, _P], ctypes.c_int),
    "po_de_select": ([ctypes.POINTER(DEParams), _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "po_de_generation": ([ctypes.POINTER(DEParams), _I64, ctypes.POINTER(PulseSpec), ctypes.POINTER(Grid), _P, _P, _P,
                          _P, _P], ctypes.c_int),
    "po_plan_create": ([_I32, ctypes.POINTER(PulseSpec), ctypes.POINTER(Grid), ctypes.POINTER(PlanConfig),
                        ctypes.c_char_p, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "po_plan_get_config": ([_P, ctypes.POINTER(PlanConfig)], ctypes.c_int),
    "po_plan_evaluate": ([_P, _P, _P, _P, _P], ctypes.c_int),
    "po_plan_destroy": ([_P], None),
    "po_mlp_create": ([_I32, _I32, _I32, _I32, ctypes.c_uint64, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "po_mlp_param_count": ([_P], ctypes.c_int64),
    "po_mlp_get_params": ([_P, _P, _P], ctypes.c_int),
    "po_mlp_set_params": ([_P, _P, _P], ctypes.c_int),
    "po_mlp_forward": ([_P, _P, _I32, _P, _P], ctypes.c_int),
    "po_mlp_loss_grad": ([_P, _P, _P, _I32, _P, _P, _P], ctypes.c_int),
    "po_mlp_adam_step": ([_P, _P, ctypes.c_float, _P], ctypes.c_int),
    "po_mlp_train_step": ([_P, _P, _P, _I32, ctypes.c_float, _P, _P], ctypes.c_int),
    "po_mlp_train_indexed": ([_P, _P, _P, _I32, _P, _I32, _I32, ctypes.c_double, ctypes.c_double, ctypes.c_float, _P,
                              _P], ctypes.c_int),
    "po_mlp_destroy": ([_P], None),
    "po_topk_mask": ([_P, _I32, _I32, _P, _P], ctypes.c_int),
    "po_log10_standardize": ([_P, _I32, ctypes.c_double, ctypes.c_double, ctypes.c_double, _P, _P], ctypes.c_int),
    "po_mask_indices": ([_P, _I32, _P, _P, _P], ctypes.c_int),
    "po_gather_rows": ([_P, _I32, _I32, _P, _I32, _P, _P], ctypes.c_int),
    "po_scatter_values": ([_P, _P, _I32, ctypes.c_double, _P, _I32, _P], ctypes.c_int),
    "po_probe_fp64_fma": ([_I32, _I32, _I64, _P, ctypes.POINTER(ctypes.c_double), _P], ctypes.c_int),
    "po_timer_enable": ([ctypes.c_int], ctypes.c_int),
    "po_set_check_finite": ([_I32], ctypes.c_int32),
    "po_timer_read": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "po_timer_mode_steps": ([ctypes.POINTER(ctypes.c_uint64), _I32], ctypes.c_int),
}

_lib = None


def load():
    """Loads libpairopt.so once; raises if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run python -m paper_1704_08919_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def check(status):
    if status != PO_OK:
        msg = load().po_last_error()
        raise POError(status, msg.decode() if msg else "")
