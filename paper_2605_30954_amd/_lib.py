"""ctypes binding of libgpgomea_eval.so (argument marshalling only).

The shared library is the product: every step of the evaluation runs in its
HIP kernels.  If it has not been built, importing this module raises; there is
no CPU fallback.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpgomea_eval.so")

OK = 0
E_ARG, E_SHAPE, E_PROGRAM, E_HIP, E_WORKSPACE, E_UNSUPPORTED = -1, -2, -3, -4, -5, -6
LINEAR_SCALING, FP64_NODES, PLAIN, NO_GRAPH = 0x1, 0x2, 0x4, 0x8
MAX_LEN, MAX_CONSTS, MAX_FEATURES = 511, 256, 64

# C declarations of include/gpgomea_eval.h: name -> (restype, argtypes)
_c = ctypes
_p = _c.c_void_p
_i32, _i64, _u32, _sz = _c.c_int32, _c.c_int64, _c.c_uint32, _c.c_size_t
SIGNATURES = {
    "gpgomea_version": (_c.c_int, []),
    "gpgomea_last_error": (_c.c_char_p, []),
    "gpgomea_workspace_bytes": (_sz, [_i32, _i32, _i32, _i32, _i64, _u32]),
    "gpgomea_eval_batch": (_c.c_int, [_p, _i32, _i32, _p, _i32, _p, _i32, _i64, _i64, _p, _u32,
                                      _p, _p, _p, _p, _sz, _p]),
    "gpgomea_grad_consts": (_c.c_int, [_p, _i32, _i32, _p, _i32, _p, _i32, _i64, _i64, _p, _u32,
                                       _p, _p, _p, _p, _p, _sz, _p]),
    "gpgomea_eval_design1": (_c.c_int, [_p, _i32, _i32, _p, _i32, _p, _i32, _i64, _i64, _p, _i32,
                                        _p, _p, _p]),
    "gpgomea_eval_design2": (_c.c_int, [_p, _i32, _i32, _p, _i32, _p, _i32, _i64, _i64, _p, _i32,
                                        _i32, _p, _p, _p, _p]),
    "gpgomea_adam_consts": (_c.c_int, [_p, _i32, _i32, _p, _p, _p, _p, _p, _i32, _c.c_double,
                                       _c.c_double, _c.c_double, _c.c_double, _p]),
    "gpgomea_noalloc_scratch_bytes": (_sz, []),
    "gpgomea_eval_batch_noalloc": (_c.c_int, [_p, _i32, _i32, _p, _i32, _p, _i32, _i64, _i64, _p, _u32,
                                              _p, _p, _p, _p]),
    "gpgomea_encode": (_c.c_int, [_p, _p, _i32, _i32, _i32, _p, _p, _i32, _p, _i32, _p, _p, _p]),
    "gpgomea_decode": (_c.c_int, [_p, _p, _i32, _i32, _i32, _i32, _p, _p, _p]),
    "gpgomea_validate": (_c.c_int, [_p, _i32, _i32, _i32, _i32, _i32, _p, _p]),
    "gpgomea_autotune": (_c.c_int, [_p, _i32, _i32, _p, _i32, _p, _i32, _i64, _i64, _p, _u32,
                                    _i32, _p, _sz, _c.c_char_p, _i32, _c.c_char_p, _i32, _p]),
    "gpgomea_load_tuning": (_c.c_int, [_c.c_char_p]),
    "gpgomea_clear_graphs": (_c.c_int, []),
    "gpgomea_graph_count": (_c.c_int, []),
    "gpgomea_profile": (_c.c_int, [_i32]),
    "gpgomea_profile_report": (_c.c_int, [_c.c_char_p, _i32]),
    "gpgomea_op_costs": (_c.c_int, [_p, _i32, _i32, _p, _p]),
}


class LibraryError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gpgomea error {code}: {msg}")
        self.code = code


def hip_runtimes():
    """Distinct HIP runtime files mapped into this process."""
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                p = line.split()[-1]
                if "libamdhip64" in p:
                    paths.add(os.path.realpath(p))
    except OSError:
        pass
    return sorted(paths)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_2605_30954_amd/build.py` (hipcc, gfx950)")
    # torch brings its own HIP runtime (same soname).  Load it first so the
    # library binds to that one: torch's streams and memory then belong to the
    # same runtime instance, and only one runtime opens the device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    rts = hip_runtimes()
    if len(rts) > 1:
        raise ImportError(f"two HIP runtimes are loaded in this process: {rts}")
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def last_error() -> str:
    return lib.gpgomea_last_error().decode()


def check(code: int) -> int:
    if code < 0:
        raise LibraryError(code, last_error())
    return code
