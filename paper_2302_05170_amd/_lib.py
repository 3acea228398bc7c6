"""ctypes declarations of the C ABI in include/sl7.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsl7.so")

SL7_OK, SL7_EINVAL, SL7_EUNSUPPORTED, SL7_EHIP, SL7_ENOMEM, SL7_ENUMERIC, SL7_EIO = 0, -1, -2, -3, -4, -5, -6
GBM, OU, CIR = 0, 1, 2
F64, F32, BF16, F16, BF16X3, F16X3, PWL32, PWL64 = 0, 1, 2, 3, 4, 5, 6, 7
RELU, SOFTPLUS = 0, 1
MAX_DIN = 8

c_i32, c_i64, c_u32, c_u64, c_dbl, c_p = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                         ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p)


class Problem(ctypes.Structure):
    _fields_ = [("model", c_i32), ("m", c_i32), ("M", c_i32), ("reserved0", c_i32),
                ("N", c_i64), ("theta", c_dbl * 4), ("Y0", c_dbl), ("T", c_dbl), ("K", c_dbl),
                ("path_offset", c_i64), ("instance", c_u32), ("reserved1", c_u32)]


class Stats(ctypes.Structure):
    _fields_ = [("mean", c_dbl * 2), ("var", c_dbl * 2), ("se", c_dbl * 2), ("n", c_i64),
                ("n_clamped", c_i64), ("n_out_of_domain", c_i64), ("reserved", c_i64)]


class MlpDesc(ctypes.Structure):
    _fields_ = [("d_in", c_i32), ("width", c_i32), ("depth", c_i32), ("m", c_i32),
                ("act", c_i32), ("model", c_i32), ("in_scale", c_dbl * MAX_DIN),
                ("in_shift", c_dbl * MAX_DIN), ("dom_lo", c_dbl * MAX_DIN),
                ("dom_hi", c_dbl * MAX_DIN)]


class Plan(ctypes.Structure):
    _fields_ = [("waves_per_block", c_i32), ("blocks_per_cu", c_i32), ("grab", c_i32),
                ("reserved", c_i32)]


# name -> (restype, argtypes)
SIGNATURES = {
    "sl7_last_error": (ctypes.c_char_p, []),
    "sl7_version": (ctypes.c_char_p, []),
    "sl7_gh_nodes": (ctypes.c_int, [ctypes.c_int, c_p, c_p]),
    "sl7_mlp_n_params": (c_i64, [c_p]),
    "sl7_mlp_create": (ctypes.c_int, [c_p, c_p, c_p]),
    "sl7_mlp_load": (ctypes.c_int, [ctypes.c_char_p, c_p]),
    "sl7_mlp_save": (ctypes.c_int, [c_p, ctypes.c_char_p]),
    "sl7_mlp_get_desc": (ctypes.c_int, [c_p, c_p]),
    "sl7_mlp_get_params": (ctypes.c_int, [c_p, c_p]),
    "sl7_mlp_set_params": (ctypes.c_int, [c_p, c_p]),
    "sl7_mlp_free": (None, [c_p]),
    "sl7_eval_H": (ctypes.c_int, [c_p, ctypes.c_int, c_p, c_i64, c_p, c_p]),
    "sl7_simulate": (ctypes.c_int, [c_p, c_p, ctypes.c_int, c_u64, c_p, c_p, c_p, c_p]),
    "sl7_simulate_noalloc": (ctypes.c_int, [c_p, c_p, ctypes.c_int, c_u64, c_p, c_p, c_p, c_p]),
    "sl7_simulate_cdc": (ctypes.c_int, [c_p, c_p, ctypes.c_int, c_u64, c_p, c_p, c_p]),
    "sl7_pwl_compile": (ctypes.c_int, [c_p, c_p, ctypes.c_int, c_p, c_p, c_p, c_p, c_p]),
    "sl7_simulate_batched": (ctypes.c_int, [c_p, ctypes.c_int, c_p, ctypes.c_int, c_u64, c_p, c_p,
                                            ctypes.c_int, c_p]),
    "sl7_default_plan": (ctypes.c_int, [ctypes.c_int, c_i64, ctypes.c_int, c_p]),
    "sl7_autotune": (ctypes.c_int, [c_p, c_p, ctypes.c_int, ctypes.c_char_p, c_p, c_p]),
    "sl7_autotune_batched": (ctypes.c_int, [c_p, ctypes.c_int, c_p, ctypes.c_int, ctypes.c_char_p,
                                            c_p, c_p]),
    "sl7_labels": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, c_p, c_i64, ctypes.c_int, ctypes.c_int,
                                  c_u64, c_i64, c_p, c_p]),
    "sl7_train": (ctypes.c_int, [c_p, c_p, c_p, c_p, c_i64, c_p, c_p, c_p]),
    "sl7_train_grad": (ctypes.c_int, [c_p, c_p, c_p, c_i64, c_p, c_p, c_p]),
    "sl7_adjoint_ws_bytes": (ctypes.c_size_t, [c_p, ctypes.c_int, ctypes.c_int]),
    "sl7_adjoint": (ctypes.c_int, [c_p, c_p, ctypes.c_int, c_u64, ctypes.c_int, ctypes.c_int, c_p,
                                   c_p, c_p, ctypes.c_size_t, c_p]),
}


class Greeks(ctypes.Structure):
    _fields_ = [("value", c_dbl), ("value_se", c_dbl), ("grad", c_dbl * 5), ("grad_se", c_dbl * 5),
                ("n_grad", c_i32), ("reserved", c_i32)]


class TrainSpec(ctypes.Structure):
    _fields_ = [("epochs", c_i32), ("batch", c_i32), ("lr", c_dbl), ("beta1", c_dbl),
                ("beta2", c_dbl), ("eps", c_dbl)]

_lib = None


class Sl7Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sl7 error {code}: {msg}")
        self.code = code


def lib():
    """The loaded libsl7.so.  Raises if it has not been built: there is no
    fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                               "`python -m paper_2302_05170_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != SL7_OK:
        msg = lib().sl7_last_error()
        raise Sl7Error(rc, msg.decode() if msg else "")
