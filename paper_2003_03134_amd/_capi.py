"""ctypes declarations of the C ABI in include/gbp.h (argument marshalling
only; every step of the GBP sweep runs in the HIP library)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgbp_hip.so")

GBP_OK, GBP_EINVAL, GBP_ENOMEM, GBP_EDEVICE, GBP_ENUMERIC, GBP_ESTATE = 0, -1, -2, -3, -4, -5
GBP_FP64, GBP_FP32 = 0, 1
GBP_DAMP_ETA, GBP_DAMP_ETA_LAMBDA = 0, 1
GBP_PAIR_KEYFRAMES, GBP_PAIR_LANDMARKS, GBP_PAIR_ODOMETRY = 0, 1, 2

STATUS_NAMES = {0: "GBP_OK", -1: "GBP_EINVAL", -2: "GBP_ENOMEM", -3: "GBP_EDEVICE",
                -4: "GBP_ENUMERIC", -5: "GBP_ESTATE"}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_u8p = C.POINTER(C.c_uint8)
_u16p = C.POINTER(C.c_uint16)


class gbp_graph(C.Structure):
    _fields_ = [("n_keyframes", C.c_int32), ("n_landmarks", C.c_int32),
                ("n_factors", C.c_int32), ("factor_kf", _ip), ("factor_lm", _ip),
                ("kf_init", _dp), ("lm_init", _dp), ("kf_anchor_info", _dp)]


class gbp_camera(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double),
                ("cy", C.c_double), ("sigma_px", C.c_double)]


class gbp_measurements(C.Structure):
    _fields_ = [("z", _dp)]


class gbp_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("damp_mode", C.c_int32),
                ("beta", C.c_double), ("relin_min_interval", C.c_int32),
                ("undamped_after_relin", C.c_int32), ("anneal", C.c_int32),
                ("prior_anneal_iters", C.c_int32), ("prior_weaken", C.c_double),
                ("huber_k", C.c_double), ("zmin", C.c_double),
                ("max_keyframes", C.c_int32), ("max_landmarks", C.c_int32),
                ("max_factors", C.c_int32), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t), ("stream", C.c_void_p)]


class gbp_reproj(C.Structure):
    _fields_ = [("are_all", C.c_double), ("are_quadratic", C.c_double),
                ("are_ref", C.c_double), ("n_valid", C.c_int64),
                ("n_quadratic", C.c_int64), ("n_linear", C.c_int64),
                ("n_invalid", C.c_int64), ("n_ref", C.c_int64),
                ("n_linear_ref", C.c_int64)]


EXPORTS = ["gbp_default_options", "gbp_workspace_bytes", "gbp_create",
           "gbp_create_batch", "gbp_relinearise", "gbp_iterate", "gbp_beliefs",
           "gbp_reproj_error", "gbp_reproj_stats", "gbp_set_reference", "gbp_add_pair_factors",
           "gbp_iterate_logged", "gbp_add_keyframe", "gbp_set_damping_model",
           "gbp_reset", "gbp_apply_depth_model", "gbp_set_damping_judges", "gbp_fallback_flags", "gbp_factor_features", "gbp_factor_messages", "gbp_mlp_infer", "gbp_mlp_infer_bf16",
           "gbp_mlp_train_workspace_bytes", "gbp_mlp_train_step", "gbp_mlp_train_step_static",
           "gbp_phase_times", "gbp_counters", "gbp_autotune", "gbp_sizes", "gbp_last_error", "gbp_destroy"]

MLP_PARAMS = 5378
GBP_MLP_STATIC_MAX_BATCH = 8192   # batch limit of gbp_mlp_train_step_static
GBP_MAX_BATCH_ITEMS = 1 << 30     # keyframes, landmarks, factors per batch, at most
LOG_COLS = 5           # GBP_LOG_COLS: columns of a gbp_iterate_logged row
MLP_FEATURES = 16

_LIB = None


class HipLibraryMissing(RuntimeError):
    pass


def load():
    """Load libgbp_hip.so; raises HipLibraryMissing when it is not built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise HipLibraryMissing(
            f"{LIB_PATH} is not built; run `python -m paper_2003_03134_amd.build` from the repository root")
    # torch first: its HIP runtime (soname libamdhip64.so.7) then satisfies the
    # library's dependency, so the process holds a single HIP runtime
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.gbp_default_options.argtypes = [C.POINTER(gbp_options)]
    lib.gbp_default_options.restype = None
    lib.gbp_workspace_bytes.argtypes = [C.c_int32, C.POINTER(gbp_graph), C.POINTER(gbp_options),
                                        C.POINTER(C.c_size_t)]
    lib.gbp_create.argtypes = [C.POINTER(gbp_graph), C.POINTER(gbp_camera),
                               C.POINTER(gbp_measurements), C.POINTER(gbp_options), C.POINTER(P)]
    lib.gbp_create_batch.argtypes = [C.c_int32, C.POINTER(gbp_graph), C.POINTER(gbp_camera),
                                     C.POINTER(gbp_measurements), C.POINTER(gbp_options),
                                     C.POINTER(P)]
    lib.gbp_relinearise.argtypes = [P, C.c_double, _ip]
    lib.gbp_iterate.argtypes = [P, C.c_int32, C.c_double, C.c_double]
    lib.gbp_iterate_logged.argtypes = [P, C.c_int32, C.c_double, C.c_double, C.c_int32, _dp]
    lib.gbp_beliefs.argtypes = [P, _dp, _dp, _dp, _dp]
    lib.gbp_reproj_error.argtypes = [P, _dp, _dp, _ip]
    lib.gbp_reproj_stats.argtypes = [P, C.c_int32, C.POINTER(gbp_reproj)]
    lib.gbp_set_reference.argtypes = [P, _dp, _u8p]
    lib.gbp_add_pair_factors.argtypes = [P, C.c_int32, C.c_int32, _ip, _ip, _dp, _dp]
    lib.gbp_add_keyframe.argtypes = [P, _dp, C.c_int32, _dp, C.c_int32, _ip, _ip, _dp]
    lib.gbp_set_damping_model.argtypes = [P, _u16p, C.c_int32, C.c_double]
    lib.gbp_reset.argtypes = [P]
    lib.gbp_set_damping_judges.argtypes = [P, _ip]
    lib.gbp_apply_depth_model.argtypes = [P, _ip, C.c_int32]
    lib.gbp_fallback_flags.argtypes = [P, _ip]
    lib.gbp_factor_features.argtypes = [P, P, C.c_int32, P]
    lib.gbp_factor_messages.argtypes = [P, P, C.c_int32, P]
    lib.gbp_mlp_infer.argtypes = [P, P, C.c_int32, P, P, P]
    lib.gbp_mlp_infer_bf16.argtypes = [P, P, C.c_int32, P, P, P]
    lib.gbp_mlp_train_workspace_bytes.argtypes = [C.c_int32, C.POINTER(C.c_size_t)]
    lib.gbp_mlp_train_step.argtypes = [P, P, P, C.c_int32, P, C.c_int32, P, P, P, P, C.c_float, C.c_int32,
                                       P, P, P, C.c_size_t, P]
    lib.gbp_mlp_train_step_static.argtypes = [P, P, P, C.c_int32, P, C.c_int32, P, P, P, P, C.c_float,
                                              C.c_int32, P, P, P]
    lib.gbp_phase_times.argtypes = [P, C.c_int32, C.c_double, C.c_double, _dp]
    lib.gbp_counters.argtypes = [P, C.POINTER(C.c_int64)]
    lib.gbp_autotune.argtypes = [P, C.c_int32, C.c_char_p, _ip]
    lib.gbp_sizes.argtypes = [P, _ip, _ip, _ip, _ip, _ip]
    lib.gbp_last_error.argtypes = [P]
    lib.gbp_last_error.restype = C.c_char_p
    lib.gbp_destroy.argtypes = [P]
    lib.gbp_destroy.restype = None
    for name in EXPORTS:
        fn = getattr(lib, name)
        if fn.restype is C.c_int:  # default
            fn.restype = C.c_int32
    _LIB = lib
    return lib
