"""ctypes binding of libg3pcf.so: argument marshalling only.

The structure below mirrors ``g3pcf_problem`` in include/g3pcf.h field by
field.  Nothing here computes any part of the estimator.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libg3pcf.so")

OK, EINVAL, EWORKSPACE, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4
LOS_Z, LOS_OBSERVER = 0, 1
PREC_FP64, PREC_FP32, PREC_BF16X3 = 0, 1, 2
F32, F64 = 0, 1
BASIS_CARTESIAN, BASIS_SPIN, BASIS_SPIN_T = 0, 1, 2  # SPIN_T: diagnostic table only

EXPORTED = ["g3pcf_zeta_len", "g3pcf_num_terms", "g3pcf_workspace_bytes", "g3pcf_forward",
            "g3pcf_backward", "g3pcf_last_error", "g3pcf_conj_ylm_via_monomials",
            "g3pcf_trace_create", "g3pcf_trace_reset", "g3pcf_trace_read",
            "g3pcf_trace_destroy", "g3pcf_isotropic", "g3pcf_degenerate_term",
            "g3pcf_forward_regions", "g3pcf_alm_bytes", "g3pcf_forward_batch",
            "g3pcf_forward_noalloc"]
STAGES = {0: "cells", 1: "pairs", 2: "zeta", 3: "adj_coef", 4: "pair_adjoint", 5: "distinct"}


class Problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("pos", ctypes.c_void_p),
        ("pos_dtype", ctypes.c_int),
        ("w", ctypes.c_void_p),
        ("box", ctypes.c_double * 3),
        ("box_lo", ctypes.c_double * 3),
        ("periodic", ctypes.c_int),
        ("observer", ctypes.c_double * 3),
        ("rmax", ctypes.c_double),
        ("nbins", ctypes.c_int),
        ("lmax", ctypes.c_int),
        ("los", ctypes.c_int),
        ("pair_prec", ctypes.c_int),
        ("zeta_prec", ctypes.c_int),
        ("basis", ctypes.c_int),
        ("primary_mask", ctypes.c_void_p),
        ("accumulate", ctypes.c_int),
        ("pairs_out", ctypes.POINTER(ctypes.c_int64)),
        ("trace", ctypes.c_void_p),
        ("distinct", ctypes.c_int),
        ("alm", ctypes.c_void_p),
        ("alm_bytes", ctypes.c_size_t),
    ]


class G3pcfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"g3pcf error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load the in-tree library; fail loudly if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(Problem)
    lib.g3pcf_zeta_len.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.g3pcf_zeta_len.restype = ctypes.c_size_t
    lib.g3pcf_num_terms.argtypes = [ctypes.c_int]
    lib.g3pcf_num_terms.restype = ctypes.c_int
    lib.g3pcf_workspace_bytes.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    lib.g3pcf_workspace_bytes.restype = ctypes.c_int
    lib.g3pcf_alm_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.g3pcf_alm_bytes.restype = ctypes.c_int
    lib.g3pcf_forward_batch.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p]
    lib.g3pcf_forward_batch.restype = ctypes.c_int
    lib.g3pcf_forward.argtypes = [P, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p]
    lib.g3pcf_forward.restype = ctypes.c_int
    lib.g3pcf_forward_noalloc.argtypes = [P, ctypes.c_void_p, ctypes.c_void_p]
    lib.g3pcf_forward_noalloc.restype = ctypes.c_int
    lib.g3pcf_backward.argtypes = [P, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_size_t, ctypes.c_void_p]
    lib.g3pcf_backward.restype = ctypes.c_int
    lib.g3pcf_last_error.argtypes = []
    lib.g3pcf_last_error.restype = ctypes.c_char_p
    lib.g3pcf_conj_ylm_via_monomials.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                 ctypes.c_double, ctypes.c_double,
                                                 ctypes.POINTER(ctypes.c_double)]
    lib.g3pcf_conj_ylm_via_monomials.restype = ctypes.c_int
    lib.g3pcf_trace_create.argtypes = [ctypes.c_int]
    lib.g3pcf_trace_create.restype = ctypes.c_void_p
    lib.g3pcf_trace_reset.argtypes = [ctypes.c_void_p]
    lib.g3pcf_trace_reset.restype = None
    lib.g3pcf_trace_read.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_float), ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int)]
    lib.g3pcf_trace_read.restype = ctypes.c_int
    lib.g3pcf_trace_destroy.argtypes = [ctypes.c_void_p]
    lib.g3pcf_trace_destroy.restype = None
    lib.g3pcf_forward_regions.argtypes = [P, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.g3pcf_forward_regions.restype = ctypes.c_int
    lib.g3pcf_isotropic.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p]
    lib.g3pcf_isotropic.restype = ctypes.c_int
    lib.g3pcf_degenerate_term.argtypes = [ctypes.c_int, ctypes.c_double,
                                          ctypes.POINTER(ctypes.c_double)]
    lib.g3pcf_degenerate_term.restype = ctypes.c_int
    _lib = lib
    return lib


def check(rc: int):
    if rc != OK:
        msg = load().g3pcf_last_error().decode(errors="replace")
        raise G3pcfError(rc, msg)


def zeta_len(lmax: int, nbins: int) -> int:
    return int(load().g3pcf_zeta_len(lmax, nbins))


def num_terms(basis: int) -> int:
    return int(load().g3pcf_num_terms(basis))


def workspace_bytes(prob: Problem, backward: int) -> int:
    out = ctypes.c_size_t(0)
    check(load().g3pcf_workspace_bytes(ctypes.byref(prob), int(backward), ctypes.byref(out)))
    return int(out.value)


def alm_bytes(prob: Problem) -> int:
    out = ctypes.c_size_t(0)
    check(load().g3pcf_alm_bytes(ctypes.byref(prob), ctypes.byref(out)))
    return int(out.value)


def forward(prob: Problem, zeta_ptr: int, ws_ptr: int, ws_bytes: int, stream: int):
    check(load().g3pcf_forward(ctypes.byref(prob), ctypes.c_void_p(zeta_ptr),
                               ctypes.c_void_p(ws_ptr), ctypes.c_size_t(ws_bytes),
                               ctypes.c_void_p(stream)))


def forward_noalloc(prob: Problem, zeta_ptr: int, stream: int):
    """g3pcf_forward_noalloc: the forward pass in the library's static scratch."""
    check(load().g3pcf_forward_noalloc(ctypes.byref(prob), ctypes.c_void_p(zeta_ptr),
                                       ctypes.c_void_p(stream)))


def backward(prob: Problem, gz_ptr: int, gw_ptr: int, ws_ptr: int, ws_bytes: int, stream: int):
    check(load().g3pcf_backward(ctypes.byref(prob), ctypes.c_void_p(gz_ptr),
                                ctypes.c_void_p(gw_ptr), ctypes.c_void_p(ws_ptr),
                                ctypes.c_size_t(ws_bytes), ctypes.c_void_p(stream)))


def conj_ylm_via_monomials(basis: int, lmax: int, u) -> list:
    n = (lmax + 1) * (lmax + 2)
    out = (ctypes.c_double * n)()
    check(load().g3pcf_conj_ylm_via_monomials(int(basis), int(lmax), float(u[0]), float(u[1]),
                                              float(u[2]), out))
    return [complex(out[2 * k], out[2 * k + 1]) for k in range(n // 2)]


def degenerate_term(lmax: int, uz: float) -> list:
    """conj(Y_lm(u)) Y_l'm(u) as [m][l][l'] nested lists (host diagnostic)."""
    L1 = lmax + 1
    out = (ctypes.c_double * (L1 * L1 * L1))()
    check(load().g3pcf_degenerate_term(int(lmax), float(uz), out))
    return [[[out[(m * L1 + l) * L1 + lp] for lp in range(L1)] for l in range(L1)]
            for m in range(L1)]


class Trace:
    """Per-stage HIP-event timing recorded by the library on its stream."""

    def __init__(self, capacity: int = 8192):
        self.capacity = capacity
        self.handle = load().g3pcf_trace_create(int(capacity))
        if not self.handle:
            raise G3pcfError(EHIP, load().g3pcf_last_error().decode(errors="replace"))

    def reset(self):
        load().g3pcf_trace_reset(self.handle)

    def read(self):
        """[(stage_name, ms), ...] -- call after synchronising the stream."""
        st = (ctypes.c_int * self.capacity)()
        ms = (ctypes.c_float * self.capacity)()
        dropped = ctypes.c_int(0)
        n = load().g3pcf_trace_read(self.handle, st, ms, self.capacity, ctypes.byref(dropped))
        if n < 0:
            check(n)
        if dropped.value:
            raise RuntimeError(f"trace dropped {dropped.value} records; raise its capacity")
        return [(STAGES.get(st[k], str(st[k])), float(ms[k])) for k in range(n)]

    def __del__(self):
        try:
            if self.handle:
                load().g3pcf_trace_destroy(self.handle)
                self.handle = None
        except Exception:
            pass
