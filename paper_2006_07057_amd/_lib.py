"""ctypes view of the C ABI in include/sinkhorn.h (argument marshalling only).

Loading fails loudly when the HIP library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsinkhorn.so")

SK_OK, SK_EINVAL, SK_ENOMEM, SK_ERANGE, SK_ENOTCONV, SK_EHIP, SK_ETIMEOUT, \
    SK_ENOTSUP = range(8)
SK_MAX_R = 4096
SK_NOALLOC_SCRATCH_BYTES = 64 << 20
SK_RANGE_EXTENDED, SK_RANGE_LINEAR = 0, 1

c_i32, c_i64, c_f32p, c_dbl = ctypes.c_int32, ctypes.c_int64, \
    ctypes.c_void_p, ctypes.c_double
c_size, c_void = ctypes.c_size_t, ctypes.c_void_p


class sk_solve_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", c_i32),
                ("fixed_iter", c_i32), ("warm_start", c_i32),
                ("range", c_i32)]


class sk_solve_info(ctypes.Structure):
    _fields_ = [("iters", c_i32), ("status", c_i32), ("err", ctypes.c_double),
                ("w_hat", ctypes.c_double)]


class sk_problem(ctypes.Structure):
    _fields_ = [("X", c_void), ("Y", c_void), ("a", c_void), ("b", c_void),
                ("U", c_void), ("n", c_i64), ("m", c_i64), ("d", c_i64),
                ("r", c_i64), ("eps", ctypes.c_double), ("q", ctypes.c_double)]


class sk_solve_spec(ctypes.Structure):
    _fields_ = [("Prow", c_void), ("Pcol", c_void), ("a", c_void), ("b", c_void),
                ("srow", c_void), ("scol", c_void), ("u", c_void), ("v", c_void),
                ("w", c_void), ("z", c_void), ("info", c_void), ("n", c_i64),
                ("m", c_i64), ("r", c_i64), ("eps", ctypes.c_double)]


class sk_state_layout(ctypes.Structure):
    _fields_ = [("phix", c_size), ("phiy", c_size), ("sx", c_size),
                ("sy", c_size), ("u", c_size * 3), ("v", c_size * 3),
                ("w", c_size * 3), ("z", c_size * 3), ("info", c_size),
                ("out", c_size), ("meta", c_size), ("total", c_size)]


# name -> (restype, argtypes)
SIGNATURES = {
    "sinkhorn_gaussian_q": (c_i32, [c_dbl, c_dbl, c_i64,
                                    ctypes.POINTER(ctypes.c_double)]),
    "sinkhorn_gaussian_anchors": (c_i32, [c_void, c_i64, c_i64, c_dbl, c_dbl, c_dbl,
                                          c_void, ctypes.POINTER(ctypes.c_double)]),
    "sinkhorn_features": (c_i32, [c_void, c_i64, c_i64, c_void, c_i64, c_dbl,
                                  c_dbl, c_i32, c_void, c_void, c_void]),
    "sinkhorn_features_arccos": (c_i32, [c_void, c_i64, c_i64, c_void, c_i64, c_i32,
                                         c_dbl, c_dbl, c_void, c_void, c_void]),
    "sinkhorn_solve_workspace_size": (c_size, [c_i64, c_i64, c_i64]),
    "sinkhorn_solve": (c_i32, [c_void, c_i64, c_void, c_i64, c_i64, c_void,
                               c_void, ctypes.POINTER(sk_solve_opts), c_void,
                               c_void, c_void, c_void, c_void, c_void, c_size,
                               c_void]),
    "sinkhorn_solve_noalloc": (c_i32, [c_void, c_i64, c_void, c_i64, c_i64, c_void,
                                       c_void, ctypes.POINTER(sk_solve_opts), c_void,
                                       c_void, c_void, c_void, c_void, c_void]),
    "sinkhorn_state_layout": (c_i32, [c_i64, c_i64, c_i64,
                                      ctypes.POINTER(sk_state_layout)]),
    "sinkhorn_divergence_workspace_size": (c_size, [ctypes.POINTER(sk_problem)]),
    "sinkhorn_divergence": (c_i32, [ctypes.POINTER(sk_problem),
                                    ctypes.POINTER(sk_solve_opts), c_void,
                                    c_void, c_size, c_void, c_size, c_void]),
    "sinkhorn_divergence_arccos_workspace_size": (c_size, [ctypes.POINTER(sk_problem)]),
    "sinkhorn_divergence_arccos": (c_i32, [ctypes.POINTER(sk_problem), c_i32, c_dbl, c_dbl,
                                           ctypes.POINTER(sk_solve_opts), c_void, c_void,
                                           c_size, c_void, c_size, c_void]),
    "sinkhorn_divergence_assemble": (c_i32, [c_void, c_i32, c_void, c_void]),
    "sinkhorn_batched_workspace_size": (c_size, [ctypes.POINTER(sk_problem),
                                                 c_i32]),
    "sinkhorn_divergence_batched": (c_i32, [ctypes.POINTER(sk_problem), c_i32,
                                            ctypes.POINTER(sk_solve_opts),
                                            c_void, ctypes.POINTER(c_void),
                                            c_void, c_size, c_void]),
    "sinkhorn_solve_batched_workspace_size": (c_size, [ctypes.POINTER(sk_solve_spec),
                                                       c_i32]),
    "sinkhorn_solve_batched": (c_i32, [ctypes.POINTER(sk_solve_spec), c_i32,
                                       ctypes.POINTER(sk_solve_opts), c_void,
                                       c_size, c_void]),
    "sinkhorn_solve_accelerated_workspace_size": (c_size, [ctypes.POINTER(sk_solve_spec)]),
    "sinkhorn_solve_accelerated": (c_i32, [ctypes.POINTER(sk_solve_spec),
                                           ctypes.POINTER(sk_solve_opts), ctypes.c_double,
                                           c_void, c_void, c_size, c_void]),
    "sinkhorn_divergence_accelerated_workspace_size": (c_size, [ctypes.POINTER(sk_problem)]),
    "sinkhorn_divergence_accelerated": (c_i32, [ctypes.POINTER(sk_problem),
                                                ctypes.POINTER(sk_solve_opts),
                                                ctypes.c_double, c_void, c_void, c_size,
                                                c_void, c_size, c_void]),
    "sinkhorn_features_backward": (c_i32, [c_void, c_i64, c_i64, c_void, c_i64,
                                           c_void, c_void, c_void,
                                           ctypes.c_float, c_i32, c_i32, c_void,
                                           c_void]),
    "sinkhorn_divergence_backward": (c_i32, [ctypes.POINTER(sk_problem),
                                             c_void, c_void, c_void, c_void,
                                             c_void, c_void, c_void, c_size,
                                             c_void]),
    "sinkhorn_divergence_backward_anchors_workspace_size": (
        c_size, [ctypes.POINTER(sk_problem)]),
    "sinkhorn_divergence_backward_anchors": (c_i32, [ctypes.POINTER(sk_problem), c_void,
                                                     c_void, c_void, c_void, c_size,
                                                     c_void]),
    "sinkhorn_tune_set": (c_i32, [c_i64, c_i64]),
    "sinkhorn_tune_get": (c_i64, [c_i64]),
    "sinkhorn_solver_layouts": (c_i32, [c_i64, c_void, c_i32]),
    "sinkhorn_tune_set_layout": (c_i32, [c_i64, c_i32]),
    "sinkhorn_tune_get_layout": (c_i32, [c_i64]),
    "sinkhorn_profile": (c_i32, [c_i32]),
    "sinkhorn_profile_read": (c_i32, [c_i32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(c_i64),
                                      ctypes.POINTER(ctypes.c_double)]),
    "sinkhorn_strerror": (ctypes.c_char_p, [c_i32]),
    "sinkhorn_version": (ctypes.c_char_p, []),
}

_lib = None


class SinkhornError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        msg = _strerror(status)
        super().__init__(f"{where}: {msg}" if where else msg)


def _strerror(status):
    try:
        return lib().sinkhorn_strerror(int(status)).decode()
    except Exception:  # pragma: no cover - library missing
        return f"status {status}"


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2006_07057_amd.build` (there is no CPU "
                "fallback)")
        # torch carries its own HIP runtime.  Load it first, so that this
        # library's dependency on the runtime resolves to the one torch
        # uses: the streams and device memory passed in come from torch,
        # and a second runtime loaded before torch does not know them
        # (launches then fail with a HIP error).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status, where=""):
    if status != SK_OK:
        raise SinkhornError(status, where)
