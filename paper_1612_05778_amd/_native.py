"""ctypes binding of ``libzpm.so`` (the C-ABI declared in ``include/zpm.h``).

Argument marshalling only: every step of a product runs in the library's HIP
kernels.  Importing this module fails loudly when the library is not built;
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libzpm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1612_05778_amd.build` "
        "(hipcc, gfx950). There is no CPU fallback.")

# One HIP runtime per process: torch ships its own libamdhip64, and the library must
# bind to that same copy (same SONAME).  Loading libzpm.so first would pull in the
# system runtime and leave torch without a usable device.
import torch  # noqa: E402,F401

lib = ctypes.CDLL(LIB_PATH)

c_i32, c_i64, c_u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
c_vp = ctypes.c_void_p

ZPM_OK = 0
ZPM_EINVAL = -1
ZPM_ENOMEM = -2
ZPM_EDEVICE = -3
ZPM_ERANGE = -4
ZPM_EUNSUPPORTED = -5
ZPM_ENOTIMPL = -6
ZPM_EBUSY = -7
ZPM_ENOTFOUND = -8
ZPM_ETOOBIG = -9


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("da", c_i64), ("db", c_i64), ("Na", c_i32), ("Nb", c_i32),
        ("K", c_i32), ("M", c_i32), ("np", c_i32),
        ("log2_L", c_i32), ("log2_L1", c_i32), ("ncol", c_i32), ("col_log2n", c_i32 * 4),
        ("col_tile", c_i32 * 4), ("W", c_i32), ("log2P", c_i32), ("nout_bits", c_i32),
        ("workspace_bytes", c_i64),
    ]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["col_log2n"] = list(self.col_log2n)[: self.ncol]
        d["col_tile"] = list(self.col_tile)[: self.ncol]
        return d


def _sig(name, res, args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = args
    return f


zpm_version = _sig("zpm_version", ctypes.c_int, [])
zpm_strerror = _sig("zpm_strerror", ctypes.c_char_p, [ctypes.c_int])
zpm_out_bits = _sig("zpm_out_bits", c_i32, [c_i64, c_i32, c_i64, c_i32])
zpm_plan = _sig("zpm_plan", ctypes.c_int,
                [c_i64, c_i32, c_i64, c_i32, c_i32, c_i32, ctypes.POINTER(PlanInfo)])
zpm_prime = _sig("zpm_prime", ctypes.c_int,
                 [c_i32, ctypes.POINTER(c_u32), ctypes.POINTER(c_u32)])
zpm_crt_matrix = _sig("zpm_crt_matrix", ctypes.c_int,
                      [c_i32, ctypes.POINTER(ctypes.c_int8), c_i64, ctypes.POINTER(c_i32)])
zpm_create = _sig("zpm_create", ctypes.c_int, [ctypes.POINTER(c_vp), ctypes.c_int])
zpm_destroy = _sig("zpm_destroy", None, [c_vp])
zpm_mul = _sig("zpm_mul", ctypes.c_int,
               [c_vp, c_vp, c_i64, c_i32, c_vp, c_i64, c_i32, c_vp, c_i32, c_vp])
zpm_mul_ex = _sig("zpm_mul_ex", ctypes.c_int,
                  [c_vp, c_vp, c_i64, c_i32, c_vp, c_i64, c_i32, c_vp, c_i32,
                   c_i32, c_i32, c_i32, c_vp, c_vp])
zpm_sync = _sig("zpm_sync", ctypes.c_int, [c_vp, c_vp])
zpm_reserve = _sig("zpm_reserve", ctypes.c_int, [c_vp, ctypes.c_size_t, c_i64, c_i32, c_i32])
ZPM_OPT_CHECK_INPUTS = 1
zpm_set_option = _sig("zpm_set_option", ctypes.c_int, [c_vp, c_i32, c_i64])


class Job(ctypes.Structure):
    _fields_ = [("a", c_vp), ("da", c_i64), ("Na", c_i32), ("b", c_vp), ("db", c_i64),
                ("Nb", c_i32), ("c", c_vp), ("wc", c_i32)]


ZPM_BATCH_GRAPH = 1
zpm_mul_batch = _sig("zpm_mul_batch", ctypes.c_int, [c_vp, ctypes.POINTER(Job), c_i64, c_i32, c_vp])
zpm_mul_batch_ex = _sig("zpm_mul_batch_ex", ctypes.c_int,
                        [c_vp, ctypes.POINTER(Job), c_i64, c_i32, c_i32, c_vp])
ZPM_BATCH_PERSISTENT = 2
zpm_batch_schedule = _sig("zpm_batch_schedule", ctypes.c_int,
                          [ctypes.POINTER(Job), c_i64, c_i32, ctypes.POINTER(c_i64),
                           ctypes.POINTER(c_i64), c_i64])
zpm_tune = _sig("zpm_tune", ctypes.c_int, [c_vp, ctypes.POINTER(Job), c_i64, ctypes.c_char_p, c_vp])
zpm_tune_load = _sig("zpm_tune_load", ctypes.c_int, [c_vp, ctypes.c_char_p])
zpm_tune_get = _sig("zpm_tune_get", ctypes.c_int,
                    [c_vp, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32), ctypes.POINTER(c_i32), c_i32,
                     ctypes.POINTER(c_i32)])
zpm_device_limits = _sig("zpm_device_limits", ctypes.c_int,
                         [ctypes.c_int, ctypes.POINTER(c_i32), ctypes.POINTER(c_i64),
                          ctypes.POINTER(c_i64)])


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", c_i64), ("total_ms", ctypes.c_double)]


zpm_profile_begin = _sig("zpm_profile_begin", ctypes.c_int, [c_vp])
zpm_profile_begin_kinds = _sig("zpm_profile_begin_kinds", ctypes.c_int, [c_vp, ctypes.c_uint32])
zpm_profile_end = _sig("zpm_profile_end", ctypes.c_int,
                       [c_vp, ctypes.POINTER(KernelTime), c_i32, ctypes.POINTER(c_i32)])


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("n_streams", c_i32), ("max_batch", c_i32),
                ("large_bits", ctypes.c_double), ("single_product", c_i32), ("large_streams", c_i32),
                ("min_batch", c_i32), ("linger_s", ctypes.c_double)]


class ServerReport(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("admission_waits", ctypes.c_uint64),
                ("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double),
                ("max_s", ctypes.c_double), ("mean_s", ctypes.c_double),
                ("out_bits", ctypes.c_double), ("bits_per_s", ctypes.c_double),
                ("mean_batch", ctypes.c_double),
                ("hbm_budget", c_i64), ("hbm_peak", c_i64), ("hbm_in_use", c_i64),
                ("inflight", c_i64), ("inflight_peak", c_i64), ("queued", c_i64)]

    def as_dict(self) -> dict:
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


c_u64 = ctypes.c_uint64
zpm_server_create = _sig("zpm_server_create", ctypes.c_int,
                         [c_vp, ctypes.c_size_t, c_i32, ctypes.POINTER(c_vp)])
zpm_server_create_ex = _sig("zpm_server_create_ex", ctypes.c_int,
                            [c_vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(c_vp)])
zpm_server_create_simulated = _sig("zpm_server_create_simulated", ctypes.c_int,
                                   [ctypes.POINTER(ServerConfig), ctypes.c_double, ctypes.c_double,
                                    c_i32, ctypes.POINTER(c_vp)])
zpm_server_submit = _sig("zpm_server_submit", ctypes.c_int,
                         [c_vp, ctypes.POINTER(Job), ctypes.POINTER(c_u64)])
zpm_server_poll = _sig("zpm_server_poll", ctypes.c_int,
                       [c_vp, c_u64, ctypes.POINTER(c_i32), ctypes.POINTER(ctypes.c_double)])
zpm_server_wait = _sig("zpm_server_wait", ctypes.c_int,
                       [c_vp, c_u64, ctypes.c_double, ctypes.POINTER(c_i32),
                        ctypes.POINTER(ctypes.c_double)])
zpm_server_completions = _sig("zpm_server_completions", ctypes.c_int,
                              [c_vp, ctypes.POINTER(c_u64), ctypes.POINTER(c_i32),
                               ctypes.POINTER(ctypes.c_double), c_i64, ctypes.POINTER(c_i64)])
zpm_server_stats = _sig("zpm_server_stats", ctypes.c_int, [c_vp, ctypes.POINTER(ServerReport)])
zpm_server_reset_stats = _sig("zpm_server_reset_stats", ctypes.c_int, [c_vp])
zpm_server_destroy = _sig("zpm_server_destroy", None, [c_vp])

zpm_operand_create = _sig("zpm_operand_create", ctypes.c_int,
                          [c_vp, c_vp, c_i64, c_i32, c_i64, c_i32, c_i32, ctypes.POINTER(c_vp), c_vp])
zpm_mul_operand = _sig("zpm_mul_operand", ctypes.c_int,
                       [c_vp, c_vp, c_i64, c_i32, c_vp, c_vp, c_i32, c_vp])
zpm_operand_info = _sig("zpm_operand_info", ctypes.c_int, [c_vp, ctypes.POINTER(PlanInfo)])
zpm_operand_destroy = _sig("zpm_operand_destroy", None, [c_vp])


class OperandJob(ctypes.Structure):
    _fields_ = [("a", c_vp), ("da", c_i64), ("Na", c_i32), ("op", c_vp), ("c", c_vp),
                ("wc", c_i32)]


zpm_mul_operand_batch = _sig("zpm_mul_operand_batch", ctypes.c_int,
                             [c_vp, ctypes.POINTER(OperandJob), c_i64, c_i32, c_vp])
zpm_server_submit_operand = _sig("zpm_server_submit_operand", ctypes.c_int,
                                 [c_vp, ctypes.POINTER(OperandJob), ctypes.POINTER(c_u64)])

class KronInfo(ctypes.Structure):
    _fields_ = [("chunk_bits", c_i32), ("s_a", c_i32), ("s_b", c_i32), ("S", c_i32),
                ("da2", c_i64), ("db2", c_i64), ("N2", c_i32), ("wc2", c_i32),
                ("inner", PlanInfo)]

    def as_dict(self) -> dict:
        d = {f[0]: getattr(self, f[0]) for f in self._fields_ if f[0] != "inner"}
        d["inner"] = self.inner.as_dict()
        return d


zpm_mul_kronecker = _sig("zpm_mul_kronecker", ctypes.c_int,
                         [c_vp, c_vp, c_i64, c_i32, c_vp, c_i64, c_i32, c_vp, c_i32, c_i32, c_vp])
zpm_kronecker_plan = _sig("zpm_kronecker_plan", ctypes.c_int,
                          [c_i64, c_i32, c_i64, c_i32, c_i32, ctypes.POINTER(KronInfo)])



class P64Info(ctypes.Structure):
    _fields_ = [("da", c_i64), ("db", c_i64), ("Na", c_i32), ("Nb", c_i32), ("K", c_i32),
                ("M", c_i32), ("np", c_i32), ("log2_L", c_i32), ("npass", c_i32),
                ("pass_log2n", c_i32 * 3), ("log2_tx", c_i32), ("log2_ti", c_i32),
                ("log2P", c_i32), ("nout_bits", c_i32), ("workspace_bytes", c_i64)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["pass_log2n"] = list(self.pass_log2n)[: self.npass]
        return d


zpm_plan_p64 = _sig("zpm_plan_p64", ctypes.c_int,
                    [c_i64, c_i32, c_i64, c_i32, c_i32, c_i32, ctypes.POINTER(P64Info)])
zpm_prime64 = _sig("zpm_prime64", ctypes.c_int,
                   [c_i32, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)])
zpm_mul_p64 = _sig("zpm_mul_p64", ctypes.c_int,
                   [c_vp, c_vp, c_i64, c_i32, c_vp, c_i64, c_i32, c_vp, c_i32, c_i32, c_i32, c_vp])

class GfpInfo(ctypes.Structure):
    _fields_ = [("da", c_i64), ("db", c_i64), ("Na", c_i32), ("Nb", c_i32), ("k", c_i32),
                ("r", c_i32), ("K", c_i32), ("M", c_i32), ("log2_L", c_i32), ("npass", c_i32),
                ("pass_log2n", c_i32 * 6), ("log2p", c_i32), ("nout_bits", c_i32),
                ("workspace_bytes", c_i64)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["pass_log2n"] = list(self.pass_log2n)[: self.npass]
        return d


zpm_gfp_prime = _sig("zpm_gfp_prime", ctypes.c_int,
                     [c_i32, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32)])
zpm_gfp_root = _sig("zpm_gfp_root", ctypes.c_int, [c_i32, c_i32, ctypes.POINTER(c_i32)])
zpm_plan_gfp = _sig("zpm_plan_gfp", ctypes.c_int,
                    [c_i64, c_i32, c_i64, c_i32, c_i32, c_i32, ctypes.POINTER(GfpInfo)])
zpm_mul_gfp = _sig("zpm_mul_gfp", ctypes.c_int,
                   [c_vp, c_vp, c_i64, c_i32, c_vp, c_i64, c_i32, c_vp, c_i32, c_i32, c_i32, c_vp])

zpm_butterfly_ceiling = _sig("zpm_butterfly_ceiling", ctypes.c_int,
                              [ctypes.c_int, c_i32, ctypes.POINTER(ctypes.c_double)])

zpm_noalloc_max_bytes = _sig("zpm_noalloc_max_bytes", c_i64, [])
zpm_mul_noalloc = _sig("zpm_mul_noalloc", ctypes.c_int,
                       [c_vp, c_vp, c_i64, c_i32, c_vp, c_i64, c_i32, c_vp, c_i32, c_vp])

EXPORTS = ["zpm_version", "zpm_strerror", "zpm_out_bits", "zpm_plan", "zpm_prime",
           "zpm_create", "zpm_destroy", "zpm_mul", "zpm_mul_ex", "zpm_sync", "zpm_reserve",
           "zpm_set_option",
           "zpm_profile_begin", "zpm_profile_begin_kinds", "zpm_profile_end", "zpm_mul_batch", "zpm_mul_batch_ex",
           "zpm_device_limits", "zpm_batch_schedule", "zpm_tune", "zpm_tune_load",
           "zpm_tune_get", "zpm_server_create", "zpm_server_create_ex",
           "zpm_server_create_simulated", "zpm_server_submit", "zpm_server_poll",
           "zpm_server_wait", "zpm_server_completions", "zpm_server_stats",
           "zpm_server_reset_stats", "zpm_server_destroy", "zpm_operand_create",
           "zpm_mul_operand", "zpm_operand_info", "zpm_operand_destroy",
           "zpm_mul_operand_batch", "zpm_server_submit_operand", "zpm_mul_kronecker",
           "zpm_kronecker_plan", "zpm_plan_p64", "zpm_prime64", "zpm_mul_p64",
           "zpm_noalloc_max_bytes", "zpm_mul_noalloc", "zpm_gfp_prime", "zpm_gfp_root",
           "zpm_plan_gfp", "zpm_mul_gfp", "zpm_butterfly_ceiling", "zpm_crt_matrix"]


class ZpmError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {zpm_strerror(code).decode()} ({code})")


def check(code: int, what: str = "zpm") -> None:
    if code != ZPM_OK:
        raise ZpmError(code, what)
