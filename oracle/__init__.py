"""FP64 CPU oracle for the anisotropic 3PCF (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it.

``liboracle.so`` is built from ``oracle.cpp`` with g++ (``build()``); the
functions below marshal NumPy arrays into it through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile the oracle with g++ (FP64, no FMA contraction, OpenMP)."""
    out = LIB if not sanitize else os.path.join(HERE, "liboracle_san.so")
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-shared", "-fPIC", SRC, "-o", out + ".tmp"]
        if sanitize:
            cmd[1:1] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g"]
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)
    return out


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        d = ctypes.c_double
        pd = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        vp = ctypes.c_void_p
        lib.oracle_ylm.argtypes = [d, d, d, ctypes.c_int, pd]
        lib.oracle_ylm.restype = None
        common = [i64, vp, vp, vp, vp, ctypes.c_int, vp, d, ctypes.c_int, ctypes.c_int,
                  ctypes.c_int, vp]
        lib.oracle_zeta.argtypes = common + [vp, vp, ctypes.c_int]
        lib.oracle_zeta.restype = ctypes.c_int
        lib.oracle_grad.argtypes = common + [vp, vp, ctypes.c_int]
        lib.oracle_grad.restype = ctypes.c_int
        _lib = lib
    return _lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def ylm(u, lmax: int) -> np.ndarray:
    """Y_lm(u), 0 <= m <= l <= lmax, complex, triangular (l, m) order."""
    lib = _load()
    u = np.asarray(u, dtype=np.float64)
    nlm = (lmax + 1) * (lmax + 2) // 2
    out = np.zeros(2 * nlm)
    lib.oracle_ylm(float(u[0]), float(u[1]), float(u[2]), int(lmax),
                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out[0::2] + 1j * out[1::2]


def _args(cat, primary_mask):
    pos = np.ascontiguousarray(cat.pos, dtype=np.float64)  # float32 -> float64 is exact
    w = np.ascontiguousarray(cat.w, dtype=np.float64)
    L = np.ascontiguousarray(cat.box, dtype=np.float64)
    lo = np.ascontiguousarray(cat.box_lo, dtype=np.float64)
    obs = np.ascontiguousarray(cat.observer, dtype=np.float64)
    mask = None
    if primary_mask is not None:
        mask = np.ascontiguousarray(primary_mask, dtype=np.uint8)
    los = 0 if cat.los == "z" else 1
    keep = (pos, w, L, lo, obs, mask)
    return keep, [pos.shape[0], _p(pos), _p(w), _p(L), _p(lo), int(bool(cat.periodic)),
                  _p(obs), float(cat.rmax), int(cat.nbins), int(cat.lmax), los, _p(mask)]


def zeta(cat, primary_mask=None, nthreads: int | None = None, return_pairs: bool = False):
    """zeta^m_{l l'}(b1, b2) as float64 [m][l][l'][b1][b2][re, im]."""
    lib = _load()
    keep, args = _args(cat, primary_mask)
    shape = (cat.lmax + 1, cat.lmax + 1, cat.lmax + 1, cat.nbins, cat.nbins, 2)
    out = np.zeros(shape, dtype=np.float64)
    pairs = np.zeros(1, dtype=np.int64)
    rc = lib.oracle_zeta(*args, _p(out), _p(pairs), int(nthreads or default_threads()))
    del keep
    if rc != 0:
        raise ValueError(f"oracle_zeta failed with code {rc}")
    return (out, int(pairs[0])) if return_pairs else out


def grad(cat, c, primary_mask=None, nthreads: int | None = None) -> np.ndarray:
    """d(sum c * zeta)/dw for every weight (c laid out like zeta)."""
    lib = _load()
    keep, args = _args(cat, primary_mask)
    c = np.ascontiguousarray(c, dtype=np.float64)
    out = np.zeros(cat.n, dtype=np.float64)
    rc = lib.oracle_grad(*args, _p(c), _p(out), int(nthreads or default_threads()))
    del keep
    if rc != 0:
        raise ValueError(f"oracle_grad failed with code {rc}")
    return out
