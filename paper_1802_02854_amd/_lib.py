"""ctypes declarations of libftkw.so (the C-ABI in include/ftkw.h).

The library must have been built (paper_1802_02854_amd.build); there is no
fallback implementation, so a missing library is an ImportError.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# FTK_LIBRARY=check loads the debug build with device bounds checks (libftkw_check.so)
LIB_PATH = os.path.join(HERE, "libftkw_check.so" if os.environ.get("FTK_LIBRARY") == "check" else "libftkw.so")

c_int, c_double, c_void_p, c_char_p = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_char_p
c_size_t, c_uint64, c_int8_p = ctypes.c_size_t, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int8)
P = ctypes.POINTER

STATUS = {0: "FTK_OK", -1: "FTK_EINVAL", -2: "FTK_ENOMEM", -3: "FTK_EDEVICE", -4: "FTK_ENUMERIC",
          -5: "FTK_EBUSY", -6: "FTK_ENOTREADY", -7: "FTK_ECANCELED"}


class FTKError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class ClusterC(ctypes.Structure):
    _fields_ = [("n_sites", c_int), ("n_bonds", c_int), ("bond_i", c_void_p), ("bond_j", c_void_p),
                ("bond_gamma", c_void_p), ("site_xy", c_void_p)]


class TsParamsC(ctypes.Structure):
    _fields_ = [("seed", c_uint64), ("first_vector", c_int), ("n_vectors", c_int),
                ("anchor_beta", c_void_p), ("n_anchors", c_int), ("E_b", c_void_p), ("eps", c_void_p),
                ("L", c_int), ("M", c_int), ("n_steps", c_int), ("taylor_lambda", c_double),
                ("gaussian_dev", c_void_p), ("block_steps", c_int), ("window_margin", c_double),
                ("resid_tol", c_double), ("shell_moments", c_int)]


class SpecParamsC(ctypes.Structure):
    _fields_ = [("q_xy", c_void_p), ("n_q", c_int), ("alpha_mask", c_int), ("omega", c_void_p),
                ("n_omega", c_int), ("eta", c_double), ("n_steps", c_int), ("rhs_block", c_int),
                ("resid_tol", c_double), ("first_shell", c_int), ("n_shells", c_int), ("solver", c_int),
                ("seed_tol", c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_size_t, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)


class PairParamsC(ctypes.Structure):
    _fields_ = [("op_a", c_void_p), ("op_b", c_void_p), ("n_pairs", c_int), ("omega", c_void_p),
                ("n_omega", c_int), ("eta", c_double), ("n_steps", c_int), ("rhs_block", c_int),
                ("resid_tol", c_double), ("solver", c_int), ("seed_tol", c_double)]


class ServingStatsC(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("failed", ctypes.c_int64), ("waiting", ctypes.c_int64),
                ("running", c_int), ("p50_latency_s", c_double), ("p99_latency_s", c_double),
                ("requests_per_s", c_double), ("hbm_budget", c_size_t), ("hbm_reserved", c_size_t),
                ("hbm_reserved_peak", c_size_t), ("max_peak_over_footprint", c_double),
                ("cancelled", ctypes.c_int64)]


# name -> argtypes (restype is ftk_status = int unless noted)
SIGNATURES = {
    "ftk_ctx_create": [c_int, c_void_p, P(c_void_p)],
    "ftk_ctx_destroy": [c_void_p],
    "ftk_sync": [c_void_p],
    "ftk_ctx_memory": [c_void_p, P(c_size_t)],
    "ftk_ctx_peak_memory": [c_void_p, P(c_size_t), c_int],
    "ftk_ctx_set_timing": [c_void_p, c_int],
    "ftk_set_tuning": [c_char_p, c_int],
    "ftk_ctx_kernel_time": [c_void_p, c_char_p, P(c_int), P(c_double)],
    "ftk_honeycomb_cluster": [c_int, c_int, c_int, c_int, P(c_int), P(c_int), c_void_p, c_void_p, c_void_p,
                              c_void_p],
    "ftk_honeycomb_momenta": [c_int, c_int, c_int, c_int, P(c_int), c_void_p],
    "ftk_named_momentum": [c_char_p, c_void_p],
    "ftk_build_hamiltonian": [c_void_p, P(ClusterC), c_double, c_double, P(c_void_p)],
    "ftk_hamiltonian_destroy": [c_void_p],
    "ftk_hv_plan": [P(ClusterC), P(c_int), P(c_int), c_void_p],
    "ftk_plan_layout": [P(ClusterC), c_void_p, c_void_p, P(c_int)],
    "ftk_hamiltonian_info": [c_void_p, P(c_int), P(c_double)],
    "ftk_apply_h": [c_void_p, c_void_p, c_void_p, c_int],
    "ftk_apply_h_strided": [c_void_p, c_void_p, c_void_p, c_int, ctypes.c_int64],
    "ftk_apply_h_noalloc": [c_void_p, c_void_p, c_void_p, c_int],
    "ftk_random_vector": [c_void_p, c_uint64, c_uint64, c_int, c_void_p],
    "ftk_filter_coefficients": [c_void_p, c_void_p, c_int, c_double, c_double, c_double, c_int, c_int, c_void_p],
    "ftk_taylor_plan": [c_int, c_double, c_double, c_double, P(c_int), P(c_int), P(c_double), P(c_double)],
    "ftk_typical_states": [c_void_p, P(TsParamsC), P(c_void_p)],
    "ftk_states_scalars": [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
    "ftk_states_window": [c_void_p, c_void_p, c_void_p],
    "ftk_states_moments": [c_void_p, c_void_p, c_void_p],
    "ftk_spectrum_norms": [c_void_p, c_void_p],
    "ftk_reweight_observable": [c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p, c_int, c_int, c_void_p, c_void_p],
    "ftk_thermodynamics": [c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                           c_void_p, c_int, c_int, c_void_p, c_void_p],
    "ftk_thermo_diagnostics": [c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                               c_int, c_void_p, c_int, c_int, c_void_p, c_void_p],
    "ftk_choose_anchors": [c_int, c_void_p, c_void_p, c_void_p, c_double, c_int, c_void_p, P(c_int)],
    "ftk_states_lanczos": [c_void_p, c_int, c_int, c_void_p, c_void_p, P(c_int)],
    "ftk_states_copy_shell": [c_void_p, c_int, c_int, c_int, c_void_p],
    "ftk_states_destroy": [c_void_p],
    "ftk_shifted_krylov_spectrum": [c_void_p, c_void_p, P(SpecParamsC), P(c_void_p)],
    "ftk_spectrum_raw": [c_void_p, c_void_p, c_void_p],
    "ftk_autotune": [c_void_p, c_int, P(c_int), P(c_double)],
    "ftk_autotune_layout": [c_void_p, c_int, P(c_int)],
    "ftk_autotune_candidates": [c_void_p, c_int, c_int, P(c_int), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
    "ftk_truncation_steps": [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_int, c_double, P(c_int)],
    "ftk_residual_history": [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_int, c_void_p],
    "ftk_fit_asymmetric_lorentzian": [c_void_p, c_void_p, c_int, c_double, c_double, c_void_p, c_int, c_void_p,
                                      c_void_p, c_void_p, c_void_p],
    "ftk_shell_window": [c_void_p, c_void_p, c_int, c_int, c_double, P(c_double), P(c_double)],
    "ftk_spectrum_lanczos": [c_void_p, c_int, c_int, c_int, c_int, c_int, c_void_p, c_void_p, P(c_int)],
    "ftk_spectrum_destroy": [c_void_p],
    "ftk_device_checks": [c_void_p, P(c_int), P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32), c_int],
    "ftk_device_checks_selftest": [c_void_p, P(ctypes.c_uint32)],
    "ftk_green_seq_create": [c_void_p, c_void_p, c_void_p, c_int, c_double, c_double, c_int, P(c_void_p)],
    "ftk_green_seq_advance": [c_void_p, c_int, P(c_int)],
    "ftk_green_seq_read": [c_void_p, c_void_p, c_void_p, c_void_p, P(c_int), P(c_double), P(c_int)],
    "ftk_green_seq_save": [c_void_p, c_void_p, c_size_t, P(c_size_t)],
    "ftk_green_seq_restore": [c_void_p, c_void_p, c_size_t, P(c_void_p)],
    "ftk_green_seq_info": [c_void_p, P(c_int), P(c_int), P(c_size_t)],
    "ftk_green_seq_destroy": [c_void_p],
    "ftk_spectrum_work": [c_void_p, P(ctypes.c_int64), P(c_int)],
    "ftk_spectrum_cocg": [c_void_p, c_int, c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, P(c_int),
                          P(c_int)],
    "ftk_reweight_spectrum": [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p],
    "ftk_ctx_create_with_allocator": [c_int, c_void_p, ALLOC_FN, FREE_FN, c_void_p, P(c_void_p)],
    "ftk_pair_green": [c_void_p, c_void_p, P(PairParamsC), P(c_void_p)],
    "ftk_pair_raw": [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
    "ftk_pair_lanczos": [c_void_p, c_int, c_int, c_int, c_int, c_int, c_void_p, c_void_p, P(c_int)],
    "ftk_pair_destroy": [c_void_p],
    "ftk_pair_cocg": [c_void_p, c_int, c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, P(c_int), P(c_int)],
    "ftk_momentum_operator": [c_int, c_void_p, c_int, c_double, c_double, c_void_p],
    "ftk_reweight_pair": [c_int, c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                          c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p],
    "ftk_reweight": [c_int, c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                     c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p],
    "ftk_request_footprint": [c_int, P(TsParamsC), P(SpecParamsC), c_int, P(c_size_t)],
    "ftk_server_create": [c_int, c_size_t, c_int, P(c_void_p)],
    "ftk_server_cancel": [c_void_p, c_uint64],
    "ftk_server_submit": [c_void_p, P(ClusterC), c_double, c_double, P(TsParamsC), P(SpecParamsC), c_void_p,
                          c_int, P(c_uint64)],
    "ftk_server_poll": [c_void_p, c_uint64, c_void_p, c_void_p, P(c_double)],
    "ftk_server_wait": [c_void_p, c_uint64, c_double],
    "ftk_server_stats": [c_void_p, P(ServingStatsC)],
    "ftk_server_occupancy": [c_void_p, c_void_p, c_void_p, c_int, P(c_int)],
    "ftk_server_destroy": [c_void_p],
}

_lib = None


def lib():
    """The loaded library (raises ImportError if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1802_02854_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = c_int
        L.ftk_last_error.argtypes = []
        L.ftk_last_error.restype = c_char_p
        _lib = L
    return _lib


def check(status):
    if status != 0:
        raise FTKError(status, lib().ftk_last_error().decode())
    return status


def call(name, *args):
    return check(getattr(lib(), name)(*args))
