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
            cmd[1:1] = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer", "-g"]
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)
    return out


def _load():
    global _lib
    if _lib is None:
        # G3PCF_ORACLE_SANITIZED=1 loads the AddressSanitizer / UBSan build
        # (the process must run with the ASan runtime preloaded)
        san = os.environ.get("G3PCF_ORACLE_SANITIZED") == "1"
        lib = ctypes.CDLL(build(sanitize=san))
        d = ctypes.c_double
        pd = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        vp = ctypes.c_void_p
        lib.oracle_ylm.argtypes = [d, d, d, ctypes.c_int, pd]
        lib.oracle_ylm.restype = None
        common = [i64, vp, vp, vp, vp, ctypes.c_int, vp, d, ctypes.c_int, ctypes.c_int,
                  ctypes.c_int, vp]
        lib.oracle_zeta.argtypes = common + [vp, vp, ctypes.c_int, ctypes.c_int]
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


def zeta(cat, primary_mask=None, nthreads: int | None = None, return_pairs: bool = False,
         distinct: bool = False):
    """zeta^m_{l l'}(b1, b2) as float64 [m][l][l'][b1][b2][re, im].

    ``distinct`` leaves out the degenerate triangles j = k (the same secondary
    on both sides), which the product of the a_lm (Sec. 3.1) contains."""
    lib = _load()
    keep, args = _args(cat, primary_mask)
    shape = (cat.lmax + 1, cat.lmax + 1, cat.lmax + 1, cat.nbins, cat.nbins, 2)
    out = np.zeros(shape, dtype=np.float64)
    pairs = np.zeros(1, dtype=np.int64)
    rc = lib.oracle_zeta(*args, _p(out), _p(pairs), int(nthreads or default_threads()),
                         int(bool(distinct)))
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


def isotropic(z) -> np.ndarray:
    """Isotropic multipoles zeta_l(b1, b2) = sum_i w_i sum_{j in b1, k in b2}
    w_j w_k P_l(u_ij . u_ik), shape [l][b1][b2], from the anisotropic ones by the
    addition theorem (Sec. 2: the Legendre polynomial of the opening angle is
    4 pi / (2l + 1) times the sum over m of Y_lm Y*_lm):
    zeta_l = 4 pi / (2l + 1) [zeta^0_ll + 2 sum_{m >= 1} Re zeta^m_ll]
    (zeta^{-m} is the conjugate of zeta^m for real weights)."""
    z = np.asarray(z, dtype=np.float64)
    lmax, nb = z.shape[0] - 1, z.shape[3]
    out = np.zeros((lmax + 1, nb, nb))
    for l in range(lmax + 1):
        s = z[0, l, l, :, :, 0].copy()
        for m in range(1, l + 1):
            s = s + 2.0 * z[m, l, l, :, :, 0]
        out[l] = 4.0 * np.pi / (2 * l + 1) * s
    return out
