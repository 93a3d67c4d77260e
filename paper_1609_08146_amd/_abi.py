"""ctypes declarations of the C ABI in include/sc.h (argument marshalling only).

The shared library is the product: if it is missing or cannot be loaded this
module raises immediately -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SC_LIBRARY", os.path.join(HERE, "lib", "libsc.so"))

SC_OK, SC_E_INVAL, SC_E_NOMEM, SC_E_DEVICE, SC_E_STATE, SC_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
SC_E_TIMEOUT, SC_E_CANCELLED, SC_E_REJECTED = -6, -7, -8
SC_FP64, SC_FP32_SPLIT, SC_FP32 = 0, 1, 2
SC_BEAM_LINEAR, SC_BEAM_RADIAL, SC_BEAM_AZIMUTHAL = 0, 1, 2
SC_NOALLOC_SCRATCH_BYTES = 64 << 20

STATUS_NAMES = {0: "SC_OK", -1: "SC_E_INVAL", -2: "SC_E_NOMEM", -3: "SC_E_DEVICE", -4: "SC_E_STATE",
                -5: "SC_E_UNSUPPORTED", -6: "SC_E_TIMEOUT", -7: "SC_E_CANCELLED", -8: "SC_E_REJECTED"}


class ScError(RuntimeError):
    def __init__(self, status: int, func: str, message: str):
        super().__init__(f"{func}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class sc_timing(ctypes.Structure):
    _fields_ = [("prep_ms", ctypes.c_double), ("quad_ms", ctypes.c_double), ("reduce_ms", ctypes.c_double),
                ("time_ms", ctypes.c_double), ("evals", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("chunk", ctypes.c_int32)]


class sc_launch(ctypes.Structure):
    _fields_ = [("obs_per_lane", ctypes.c_int), ("waves_per_block", ctypes.c_int), ("chunk", ctypes.c_int),
                ("blocks_per_cu", ctypes.c_int), ("freq_per_lane", ctypes.c_int)]


class sc_lg_mode(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("l", ctypes.c_int), ("ex", ctypes.c_double * 2), ("ey", ctypes.c_double * 2)]


class sc_request(ctypes.Structure):
    _fields_ = [("f", ctypes.c_double), ("r_max", ctypes.c_double), ("n_r", ctypes.c_int), ("n_phi", ctypes.c_int),
                ("n_k", ctypes.c_int), ("k", ctypes.c_void_p), ("spectrum", ctypes.c_void_p),
                ("w0", ctypes.c_double), ("pol_angle", ctypes.c_double), ("consistent", ctypes.c_int),
                ("n_obs", ctypes.c_int), ("obs", ctypes.c_void_p), ("prec", ctypes.c_int), ("n_t", ctypes.c_int),
                ("t", ctypes.c_void_p), ("dk", ctypes.c_double), ("beam", ctypes.c_int)]


class sc_request_stats(ctypes.Structure):
    _fields_ = [("queue_ms", ctypes.c_double), ("run_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("evals", ctypes.c_int64), ("device_bytes", ctypes.c_size_t)]


class sc_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("cancelled", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("running", ctypes.c_int64), ("hbm_in_use", ctypes.c_size_t), ("hbm_budget", ctypes.c_size_t),
                ("launches", ctypes.c_int64), ("evals_done", ctypes.c_int64), ("evals_launched", ctypes.c_int64),
                ("quad_ms", ctypes.c_double), ("prep_ms", ctypes.c_double), ("prep_host_ms", ctypes.c_double),
                ("host_in_use", ctypes.c_size_t), ("host_budget", ctypes.c_size_t)]


V, I, D, P = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
PP = ctypes.POINTER(ctypes.c_void_p)

# name -> argtypes (every function returns int status unless listed in _RESTYPE)
SIGNATURES = {
    "sc_last_error": [],
    "sc_version": [],
    "sc_ctx_create": [I, V, PP],
    "sc_ctx_destroy": [V],
    "sc_ctx_synchronize": [V],
    "sc_ctx_set_profiling": [V, I],
    "sc_get_timing": [V, ctypes.POINTER(sc_timing)],
    "sc_set_launch": [V, ctypes.POINTER(sc_launch)],
    "sc_get_launch": [V, I, ctypes.POINTER(sc_launch)],
    "sc_autotune": [V, I, D, ctypes.POINTER(sc_launch)],
    "sc_set_batch_launch": [V, I, ctypes.POINTER(sc_launch)],
    "sc_autotune_batch": [V, PP, I, I, D, ctypes.POINTER(sc_launch)],
    "sc_autotune_load": [V, ctypes.c_char_p],
    "sc_autotune_save": [V, ctypes.c_char_p],
    "sc_prob_create": [V, PP],
    "sc_prob_destroy": [V],
    "sc_set_mirror": [V, D, D, I, I],
    "sc_set_surface": [V, I, P, P, I, P, P, P],
    "sc_get_num_nodes": [V, ctypes.POINTER(I), ctypes.POINTER(I)],
    "sc_get_nodes": [V, P, P, P],
    "sc_set_frequencies": [V, P, I],
    "sc_set_incident": [V, P, P, I],
    "sc_set_incident_gaussian": [V, D, D, P, I],
    "sc_set_incident_beam": [V, I, D, D, P, I],
    "sc_set_incident_lg": [V, ctypes.POINTER(sc_lg_mode), I, D, P],
    "sc_get_incident_power": [V, P],
    "sc_scale_spectrum": [V, P],
    "sc_normalize_energy": [V, P, D, D],
    "sc_set_table_storage": [V, I],
    "sc_set_factoring": [V, I],
    "sc_get_factoring": [V, ctypes.POINTER(I)],
    "sc_get_factoring_for": [V, I, ctypes.POINTER(I)],
    "sc_set_observation": [V, P, I, I],
    "sc_evaluate": [V, I, P, P, I],
    "sc_evaluate_noalloc": [V, I, P, P],
    "sc_get_result": [V, P, P, I],
    "sc_to_time": [V, D, D, I, P, P, I],
    "sc_to_time_at": [V, D, P, I, P, P, I],
    "sc_stencil_points": [P, I, D, P],
    "sc_maxwell_residual_freq": [V, I, D, P],
    "sc_maxwell_residual_time": [V, I, D, P, I, D, D, P],
    "sc_field_energy": [V, P, I, D, D, P],
    "sc_evaluate_batch": [V, PP, I, I],
    "sc_prob_device_bytes": [V, ctypes.POINTER(ctypes.c_size_t)],
    "sc_server_create": [V, ctypes.c_size_t, I, D, PP],
    "sc_server_submit": [V, ctypes.POINTER(sc_request), ctypes.POINTER(ctypes.c_uint64)],
    "sc_server_wait": [V, ctypes.c_uint64, D, P, P, P, P, ctypes.POINTER(sc_request_stats)],
    "sc_server_cancel": [V, ctypes.c_uint64],
    "sc_server_get_stats": [V, ctypes.POINTER(sc_server_stats)],
    "sc_server_destroy": [V],
}
_RESTYPE = {"sc_last_error": ctypes.c_char_p, "sc_version": ctypes.c_char_p}

_lib = None


def load(path: str = LIB_PATH):
    """Load libsc.so (raises if it is not built: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libsc.so not found at {path}: build it with `python -m paper_1609_08146_amd.build` "
                          "(the gfx950 library is required; there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = _RESTYPE.get(name, ctypes.c_int)
    _lib = lib
    return lib


def call(name: str, *args) -> int:
    """Call an entry point; raise ScError on a non-OK status."""
    lib = load()
    st = getattr(lib, name)(*args)
    if st != SC_OK:
        raise ScError(st, name, lib.sc_last_error().decode(errors="replace"))
    return st


def call_status(name: str, *args) -> int:
    """Call an entry point and return its status (no exception)."""
    return getattr(load(), name)(*args)


def last_error() -> str:
    return load().sc_last_error().decode(errors="replace")
