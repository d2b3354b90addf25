"""ctypes declarations of the C-ABI in include/rpot.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# RPOT_LIB names another build of the same library (the host sanitizer build)
LIB_PATH = os.environ.get("RPOT_LIB") or os.path.join(HERE, "librpot.so")

RP_OK = 0
STATUS = {0: "RP_OK", 1: "RP_ERR_ARG", 2: "RP_ERR_GEOMETRY", 3: "RP_ERR_NOMEM",
          4: "RP_ERR_STATE", 5: "RP_ERR_DEVICE", 6: "RP_ERR_UNSUPPORTED"}
PRECISION = {"fp64": 0, "fp32": 1, "fp32_ring_fp16": 2, "fp32_ring_bf16": 3, "fp32_ring_i16": 4}

EXPORTS = ["rp_plan_domains", "rp_plan_targets", "rp_workspace_bytes", "rp_bind_workspace", "rp_bind_workspace_static",
           "rp_set_green_kernels",
           "rp_push_sources", "rp_retarded_step", "rp_plan_info", "rp_plan_stats",
           "rp_profile_lagsum", "rp_lagsum_time", "rp_set_tuning", "rp_get_tuning",
           "rp_autotune", "rp_capture_step", "rp_launch_step", "rp_mlp_create", "rp_mlp_workspace_bytes",
           "rp_mlp_bind", "rp_mlp_n_params", "rp_mlp_set_params", "rp_mlp_get_params", "rp_mlp_forward",
           "rp_mlp_loss_grad", "rp_mlp_train_step", "rp_mlp_destroy", "rp_plan_destroy", "rp_last_error",
           "rp_mlp_last_error", "rp_surrogate_configure", "rp_surrogate_info", "rp_surrogate_pairs",
           "rp_surrogate_attach", "rp_surrogate_multipole", "rp_surrogate_multipole_response", "rp_surrogate_features", "rp_surrogate_pair_response", "rp_surrogate_judge", "rp_surrogate_readmit",
           "rp_osc_create", "rp_osc_workspace_bytes", "rp_osc_bind", "rp_osc_set_state", "rp_osc_sources",
           "rp_osc_step", "rp_osc_state", "rp_osc_destroy", "rp_osc_last_error", "rp_history_split",
           "rp_history_host", "rp_history_host_bytes", "rp_bind_history_host",
           "rp_class_info", "rp_set_class_tuning", "rp_get_class_tuning", "rp_read_stream",
           "rp_surrogate_teacher", "rp_surrogate_data_scales", "rp_surrogate_scale_data", "rp_mlp_relative_rms",
           "rp_surrogate_sample", "rp_surrogate_sample_fields", "rp_surrogate_judge_stats"]
TUNE = {"lagsum_unroll": 1, "lagsum_persistent": 2, "fft_lds": 4, "lagsum_steps": 8, "lagsum_cached": 16,
        "lagsum_tile_major": 32, "fft_reg": 64, "fft_plane": 128}


class RpotError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class RpStats(ctypes.Structure):
    _fields_ = [("n_triples", ctypes.c_int64), ("n_spectra", ctypes.c_int64),
                ("n_entries", ctypes.c_int64), ("points", ctypes.c_int64),
                ("lagsum_bytes", ctypes.c_double), ("ring_bytes", ctypes.c_double),
                ("spectra_bytes", ctypes.c_double), ("fft_bytes_fwd", ctypes.c_double),
                ("fft_bytes_inv", ctypes.c_double), ("history_bytes", ctypes.c_double),
                ("split_rings", ctypes.c_int64), ("n_classes", ctypes.c_int64),
                ("fused_additions", ctypes.c_int64)]


_LIB = None


def load():
    """Load librpot.so; raise if it has not been built (there is no fallback)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2311_15429_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    P = ctypes.POINTER
    lib.rp_plan_domains.argtypes = [P(vp), i32, P(i32), P(ctypes.c_double), P(i32), ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_int, vp]
    lib.rp_workspace_bytes.argtypes = [vp, P(sz)]
    lib.rp_plan_targets.argtypes = [vp, P(i32), i32]
    lib.rp_read_stream.argtypes = [vp, sz, vp, i32, i32, vp]
    lib.rp_bind_workspace.argtypes = [vp, vp, sz]
    lib.rp_bind_workspace_static.argtypes = [vp]
    lib.rp_surrogate_teacher.argtypes = [vp, vp, vp, i32]
    lib.rp_surrogate_data_scales.argtypes = [vp, vp, i64, i32, vp, vp, vp]
    lib.rp_surrogate_scale_data.argtypes = [vp, vp, i64, i32, vp, vp, vp]
    lib.rp_mlp_relative_rms.argtypes = [vp, vp, vp, i64, vp, P(ctypes.c_double)]
    lib.rp_set_green_kernels.argtypes = [vp]
    lib.rp_push_sources.argtypes = [vp, i64, P(vp)]
    lib.rp_retarded_step.argtypes = [vp, i64, P(vp)]
    lib.rp_plan_info.argtypes = [vp, i32, i32, P(i32), P(i32), P(i32), P(i32)]
    lib.rp_plan_stats.argtypes = [vp, P(RpStats)]
    lib.rp_profile_lagsum.argtypes = [vp, i32]
    lib.rp_lagsum_time.argtypes = [vp, P(ctypes.c_double), P(i64)]
    lib.rp_set_tuning.argtypes = [vp, i32, i32]
    lib.rp_get_tuning.argtypes = [vp, i32, P(i32)]
    lib.rp_autotune.argtypes = [vp, i32, P(i32), P(i32), P(ctypes.c_double)]
    lib.rp_capture_step.argtypes = [vp, P(vp), P(vp)]
    lib.rp_launch_step.argtypes = [vp, i64]
    lib.rp_plan_destroy.argtypes = [vp]
    lib.rp_last_error.argtypes = [vp]
    lib.rp_last_error.restype = ctypes.c_char_p
    lib.rp_mlp_create.argtypes = [P(vp), i32, i32, i32, i32, vp]
    lib.rp_mlp_workspace_bytes.argtypes = [vp, P(sz)]
    lib.rp_mlp_bind.argtypes = [vp, vp, sz]
    lib.rp_mlp_n_params.argtypes = [vp, P(i64)]
    lib.rp_mlp_set_params.argtypes = [vp, vp]
    lib.rp_mlp_get_params.argtypes = [vp, vp]
    lib.rp_mlp_forward.argtypes = [vp, vp, i32, vp]
    lib.rp_mlp_loss_grad.argtypes = [vp, vp, vp, i32, vp, vp]
    lib.rp_mlp_train_step.argtypes = [vp, vp, vp, i32, ctypes.c_float, vp]
    lib.rp_mlp_destroy.argtypes = [vp]
    lib.rp_mlp_last_error.argtypes = [vp]
    lib.rp_mlp_last_error.restype = ctypes.c_char_p
    dp = P(ctypes.c_double)
    lib.rp_surrogate_configure.argtypes = [vp, ctypes.c_double, i32, P(i32), i32]
    lib.rp_surrogate_info.argtypes = [vp, P(i32), P(i32), P(i32), P(i32)]
    lib.rp_surrogate_pairs.argtypes = [vp, P(i32), P(i32), dp, P(i32), P(i32)]
    lib.rp_surrogate_attach.argtypes = [vp, vp, P(ctypes.c_float), P(ctypes.c_float)]
    lib.rp_surrogate_features.argtypes = [vp, vp]
    lib.rp_surrogate_multipole.argtypes = [vp, i32]
    lib.rp_surrogate_multipole_response.argtypes = [vp, vp]
    lib.rp_surrogate_pair_response.argtypes = [vp, vp, vp]
    lib.rp_surrogate_judge.argtypes = [vp, P(vp), ctypes.c_double, P(i32), dp, P(i32)]
    lib.rp_surrogate_readmit.argtypes = [vp, ctypes.c_double]
    lib.rp_surrogate_sample.argtypes = [vp, i32, i32]
    lib.rp_surrogate_sample_fields.argtypes = [vp, P(i32), i32, vp]
    lib.rp_surrogate_judge_stats.argtypes = [vp, P(i32), P(i32), P(i32), P(i32)]
    lib.rp_history_split.argtypes = [vp, i32]
    lib.rp_history_host.argtypes = [vp, i32]
    lib.rp_history_host_bytes.argtypes = [vp, P(ctypes.c_size_t)]
    lib.rp_bind_history_host.argtypes = [vp, vp, ctypes.c_size_t]
    lib.rp_class_info.argtypes = [vp, i32, P(i32), P(i32), P(i32)]
    lib.rp_set_class_tuning.argtypes = [vp, i32, i32, i32]
    lib.rp_get_class_tuning.argtypes = [vp, i32, i32, P(i32)]
    lib.rp_osc_create.argtypes = [P(vp), vp, P(i32), dp]
    lib.rp_osc_workspace_bytes.argtypes = [vp, P(sz)]
    lib.rp_osc_bind.argtypes = [vp, vp, sz, P(vp)]
    lib.rp_osc_set_state.argtypes = [vp, dp, dp]
    lib.rp_osc_sources.argtypes = [vp, P(vp)]
    lib.rp_osc_step.argtypes = [vp, P(vp), ctypes.c_double, P(vp)]
    lib.rp_osc_state.argtypes = [vp, dp, dp, dp, dp]
    lib.rp_osc_destroy.argtypes = [vp]
    lib.rp_osc_last_error.argtypes = [vp]
    lib.rp_osc_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("rp_last_error", "rp_mlp_last_error", "rp_osc_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _LIB = lib
    return lib


def check(lib, plan, code):
    if code != RP_OK:
        msg = lib.rp_last_error(plan)
        raise RpotError(code, msg.decode() if msg else "")


def check_mlp(lib, mlp, code):
    if code != RP_OK:
        msg = lib.rp_mlp_last_error(mlp)
        raise RpotError(code, msg.decode() if msg else "")


def check_osc(lib, osc, code):
    if code != RP_OK:
        msg = lib.rp_osc_last_error(osc)
        raise RpotError(code, msg.decode() if msg else "")
