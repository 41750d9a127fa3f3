"""ctypes declarations of libspme.so (the C ABI in include/spme.h).

Argument marshalling only: every step of the SPME path runs in the HIP
library.  Loading fails loudly when the library has not been built.
"""
import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspme.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "spme.h")

PME_FP64 = 0
PME_FP32_FIXED = 1
PME_FP32_FIXED_HALF = 2
PME_FP32_FIXED_BF16 = 3
PME_FLAG_NONFINITE = 1
PME_FLAG_OVERFLOW = 2
PME_FLAG_BUCKETS = 4

PME_EBUSY = 8
PME_SCRATCH_BYTES = 32 << 20  # static scratch of pme_step_noalloc (include/spme.h)
PME_CONV_FUSED, PME_CONV_SPLIT, PME_CONV_REG = 0, 1, 2
PME_INTERP_FUSED, PME_INTERP_SPLIT = 0, 1
PME_VAR_CONV_FUSED, PME_VAR_CONV_SPLIT, PME_VAR_INTERP_FUSED, PME_VAR_INTERP_SPLIT = 1, 2, 4, 8
PME_VAR_CONV_REG = 16

STATUS = {0: "PME_OK", 1: "PME_EINVAL", 2: "PME_EUNSUPPORTED", 3: "PME_EWORKSPACE",
          4: "PME_EOVERFLOW", 5: "PME_EDEVICE", 6: "PME_ENONFINITE", 7: "PME_ESTATE",
          8: "PME_EBUSY"}


class Tuning(ctypes.Structure):
    """pme_tuning: the kernel variants of a plan."""
    _fields_ = [("conv", ctypes.c_int), ("interp", ctypes.c_int), ("bin_chunk", ctypes.c_int)]

    def as_dict(self):
        return {"conv": int(self.conv), "interp": int(self.interp), "bin_chunk": int(self.bin_chunk)}


class SystemDesc(ctypes.Structure):
    """pme_system_desc: one system of a batch."""
    _fields_ = [("K1", ctypes.c_int), ("K2", ctypes.c_int), ("K3", ctypes.c_int),
                ("order", ctypes.c_int), ("beta", ctypes.c_double), ("precision", ctypes.c_int),
                ("max_atoms", ctypes.c_int), ("pos", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("N", ctypes.c_int), ("box", ctypes.c_double * 9), ("forces", ctypes.c_void_p),
                ("ev", ctypes.c_void_p)]

_lib = None


class SpmeError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        msg = _lib.pme_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {STATUS.get(code, code)} ({msg})")


def declared_functions():
    """Names of the functions include/spme.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pme_[a-z_]+)\s*\(", text)))


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_2009_12617_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    dp = ctypes.POINTER(ctypes.c_double)
    lib.pme_version.restype = i
    lib.pme_version.argtypes = []
    lib.pme_strerror.restype = ctypes.c_char_p
    lib.pme_strerror.argtypes = [i]
    lib.pme_workspace_bytes.restype = sz
    lib.pme_workspace_bytes.argtypes = [i, i, i, i, i, i]
    lib.pme_create.restype = i
    lib.pme_create.argtypes = [ctypes.POINTER(vp), i, i, i, i, d, i, i, i, d, vp, sz, vp]
    lib.pme_destroy.restype = i
    lib.pme_destroy.argtypes = [vp]
    lib.pme_set_stream.restype = i
    lib.pme_set_stream.argtypes = [vp, vp]
    lib.pme_spread.restype = i
    lib.pme_spread.argtypes = [vp, vp, vp, i, dp]
    lib.pme_solve.restype = i
    lib.pme_solve.argtypes = [vp, vp]
    lib.pme_gather.restype = i
    lib.pme_gather.argtypes = [vp, vp, i]
    lib.pme_step.restype = i
    lib.pme_step.argtypes = [vp, vp, vp, i, dp, vp, i, vp]
    lib.pme_bind.restype = i
    lib.pme_bind.argtypes = [vp, vp, vp, i, dp, vp, i, vp]
    lib.pme_batch_run.restype = i
    lib.pme_batch_run.argtypes = [ctypes.POINTER(vp), i, vp]
    lib.pme_set_debug.restype = i
    lib.pme_set_debug.argtypes = [vp, i]
    lib.pme_debug_grid.restype = i
    lib.pme_debug_grid.argtypes = [vp, i, vp]
    lib.pme_debug_grid_bytes.restype = sz
    lib.pme_debug_grid_bytes.argtypes = [vp, i]
    lib.pme_check.restype = i
    lib.pme_check.argtypes = [vp, ctypes.POINTER(ctypes.c_uint)]
    lib.pme_kernel_timing.restype = i
    lib.pme_kernel_timing.argtypes = [vp, i]
    lib.pme_kernel_times.restype = i
    lib.pme_kernel_times.argtypes = [vp, dp, i, ctypes.POINTER(ctypes.c_int)]
    lib.pme_real_workspace_bytes.restype = sz
    lib.pme_real_workspace_bytes.argtypes = [i, i]
    lib.pme_real.restype = i
    lib.pme_real.argtypes = [vp, vp, i, dp, d, d, d, vp, vp, vp, i, vp, vp, sz, i, i, vp]
    tp = ctypes.POINTER(Tuning)
    sdp = ctypes.POINTER(SystemDesc)
    lib.pme_tuning_variants.restype = ctypes.c_uint
    lib.pme_tuning_variants.argtypes = [i, i, i, i, i]
    lib.pme_default_tuning.restype = i
    lib.pme_default_tuning.argtypes = [i, i, i, i, i, tp]
    lib.pme_get_tuning.restype = i
    lib.pme_get_tuning.argtypes = [vp, tp]
    lib.pme_set_tuning.restype = i
    lib.pme_set_tuning.argtypes = [vp, tp]
    lib.pme_autotune.restype = i
    lib.pme_autotune.argtypes = [vp, vp, vp, i, dp, vp, vp, i, tp, dp, dp, i]
    lib.pme_batch_footprint.restype = sz
    lib.pme_batch_footprint.argtypes = [sdp]
    lib.pme_batch_create.restype = i
    lib.pme_batch_create.argtypes = [ctypes.POINTER(vp), i, vp, sz, vp]
    lib.pme_batch_destroy.restype = i
    lib.pme_batch_destroy.argtypes = [vp]
    lib.pme_batch_admit.restype = i
    lib.pme_batch_admit.argtypes = [vp, sdp, ctypes.POINTER(i)]
    lib.pme_batch_update.restype = i
    lib.pme_batch_update.argtypes = [vp, i, vp, vp, i, dp, vp, vp]
    lib.pme_batch_retire.restype = i
    lib.pme_batch_retire.argtypes = [vp, i]
    lib.pme_batch_launch.restype = i
    lib.pme_batch_launch.argtypes = [vp, ctypes.POINTER(i), i]
    lib.pme_batch_io.restype = i
    lib.pme_batch_io.argtypes = [vp, i] + [ctypes.POINTER(ctypes.c_void_p)] * 4
    lib.pme_batch_stats.restype = i
    lib.pme_batch_stats.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(sz), ctypes.POINTER(sz)]
    lib.pme_batch_plan.restype = vp
    lib.pme_batch_plan.argtypes = [vp, i]
    lib.pme_step_probe.restype = i
    lib.pme_step_probe.argtypes = [vp, vp, vp, i, dp, vp, vp, i]
    lib.pme_step_noalloc.restype = i
    lib.pme_step_noalloc.argtypes = [i, i, i, i, d, i, i, d, vp, vp, i, dp, vp, i, vp, vp]
    _lib = lib
    return lib


def check(code, what):
    if code != 0:
        raise SpmeError(code, what)
