"""ctypes declarations of the C ABI in include/mtgp.h (argument marshalling only).

The shared library is built in-tree by ``build.py``; there is no fallback:
if it is missing or fails to load, every entry point raises.
"""
import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmtgp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mtgp.h")

c_i32, c_i64, c_u32, c_sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
vp = ctypes.c_void_p


class Design(ctypes.Structure):
    _fields_ = [("T", c_i32), ("d", c_i32), ("family", c_i32),
                ("m", ctypes.POINTER(c_i32)), ("gen", ctypes.POINTER(c_u32)),
                ("shift", ctypes.POINTER(c_u32)), ("kernel_order", c_i32),
                ("adaptive", c_i32), ("rank_s", c_i32), ("profile_tau", c_i32)]


SIGNATURES = {
    "mtgp_plan_create": (ctypes.c_int, [ctypes.POINTER(Design), c_i32, ctypes.POINTER(vp)]),
    "mtgp_plan_destroy": (ctypes.c_int, [vp]),
    "mtgp_plan_set_schedule": (ctypes.c_int, [vp, c_i32, c_i32, c_i64]),
    "mtgp_plan_set_overlap": (ctypes.c_int, [vp, c_i32]),
    "mtgp_plan_set_elimination": (ctypes.c_int, [vp, c_i32]),
    "mtgp_plan_set_fused_occupancy": (ctypes.c_int, [vp, c_i32]),
    "mtgp_plan_enable_timing": (ctypes.c_int, [vp, c_i32]),
    "mtgp_phase_times": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double), c_i32,
                                        ctypes.POINTER(c_i32)]),
    "mtgp_phase_name": (ctypes.c_char_p, [c_i32]),
    "mtgp_theta_size": (c_i64, [vp]),
    "mtgp_workspace_bytes": (c_sz, [vp]),
    "mtgp_num_points": (c_i64, [vp]),
    "mtgp_num_columns": (c_i32, [vp]),
    "mtgp_column_info": (ctypes.c_int, [vp, c_i32, ctypes.POINTER(c_i32), ctypes.POINTER(c_i64),
                                        ctypes.POINTER(c_i32), ctypes.POINTER(c_i32)]),
    "mtgp_gen_points": (ctypes.c_int, [vp, c_i32, c_i64, c_i64, vp, vp]),
    "mtgp_kernel_cols": (ctypes.c_int, [vp, vp, vp, vp, vp]),
    "mtgp_fwht": (ctypes.c_int, [vp, c_i64, c_i32, c_i32, vp]),
    "mtgp_fft": (ctypes.c_int, [vp, vp, vp, c_i64, c_i32, c_i32, c_i32, vp]),
    "mtgp_fft_noalloc": (ctypes.c_int, [vp, vp, c_i64, c_i32, c_i32, c_i32, vp]),
    "mtgp_set_data": (ctypes.c_int, [vp, vp, vp, vp]),
    "mtgp_nll": (ctypes.c_int, [vp, vp, vp, vp, vp, vp]),
    "mtgp_nll_grad": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
    "mtgp_predict": (ctypes.c_int, [vp, vp, vp, c_i64, vp, vp, vp]),
    "mtgp_predict_net_scratch_bytes": (c_sz, [vp, c_i32]),
    "mtgp_predict_net": (ctypes.c_int, [vp, vp, ctypes.POINTER(c_u32), c_i32, vp, vp, vp, vp]),
    "mtgp_predict_var_scratch_bytes": (c_sz, [vp, c_i32]),
    "mtgp_predict_var": (ctypes.c_int, [vp, vp, vp, c_i64, c_i32, vp, vp, vp, vp]),
    "mtgp_status": (ctypes.c_int, [vp, vp, ctypes.POINTER(c_i64)]),
    "mtgp_gcv": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
    "mtgp_cubature": (ctypes.c_int, [vp, vp, vp, vp, vp, vp]),
    "mtgp_nll_grad_batched": (ctypes.c_int, [c_i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                             ctypes.POINTER(vp), ctypes.POINTER(vp),
                                             ctypes.POINTER(vp), vp]),
    "mtgp_batch_workspace_bytes": (c_sz, [c_i32, ctypes.POINTER(vp)]),
    "mtgp_batch_create": (ctypes.c_int, [c_i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.POINTER(vp), vp, ctypes.POINTER(vp)]),
    "mtgp_batch_destroy": (ctypes.c_int, [vp]),
    "mtgp_batch_nll_grad": (ctypes.c_int, [vp, vp]),
    "mtgp_batch_adam_step": (ctypes.c_int, [vp, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, vp]),
    "mtgp_adam_step": (ctypes.c_int, [vp, vp, vp, vp, c_i64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, vp, vp, vp]),
    "mtgp_strerror": (ctypes.c_char_p, [ctypes.c_int]),
}

_LIB = None


def header_functions():
    """Names of the functions declared in include/mtgp.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mtgp_[a-z0-9_]+)\s*\(", text)))


def load():
    """Loads libmtgp.so and declares every entry point; raises if it is absent."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


class MTGPError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        msg = load().mtgp_strerror(code).decode()
        super().__init__(f"{what} failed: {msg} (code {code})")


def check(code, what):
    if code != 0:
        raise MTGPError(code, what)
    return code
