"""PyTorch front end of libg3pcf.

PyTorch provides device memory and the stream; every step of the estimator
runs in the library's HIP kernels.  There is no CPU fallback: on a machine
without the built library or without a GPU these functions raise.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import torch

from . import _lib

_PREC = {"fp64": (_lib.PREC_FP64, _lib.PREC_FP64),
         "fp32": (_lib.PREC_FP32, _lib.PREC_FP32),
         "bf16x3": (_lib.PREC_FP32, _lib.PREC_BF16X3)}
_ZPREC = {"fp64": _lib.PREC_FP64, "fp32": _lib.PREC_FP32, "bf16x3": _lib.PREC_BF16X3}
_BASIS = {"cartesian": _lib.BASIS_CARTESIAN, "spin": _lib.BASIS_SPIN}


@dataclasses.dataclass(frozen=True)
class Config:
    """Estimator settings (everything except the arrays)."""

    box: Sequence[float]
    rmax: float
    nbins: int = 10
    lmax: int = 10
    los: str = "z"                     # "z" or "observer"
    observer: Sequence[float] = (0.0, 0.0, 0.0)
    periodic: bool = True
    box_lo: Sequence[float] = (0.0, 0.0, 0.0)
    precision: str = "fp32"            # "fp64", "fp32" or "bf16x3"
    zeta_precision: Optional[str] = None  # override the zeta-stage precision
    basis: str = "cartesian"           # "cartesian" (eq. 1 monomials) or "spin"
    distinct: bool = False             # leave out the degenerate triangles j = k (forward only)

    def pair_prec(self) -> int:
        return _PREC[self.precision][0]

    def zeta_prec(self) -> int:
        if self.zeta_precision is not None:
            return _ZPREC[self.zeta_precision]
        return _PREC[self.precision][1]


def zeta_shape(lmax: int, nbins: int):
    return (lmax + 1, lmax + 1, lmax + 1, nbins, nbins, 2)


def _require_cuda(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor (HIP); got {t.device}")


def make_problem(pos: torch.Tensor, w: torch.Tensor, cfg: Config,
                 primary_mask: Optional[torch.Tensor] = None, accumulate: bool = False,
                 pairs_out=None, trace: Optional["_lib.Trace"] = None,
                 alm: Optional[torch.Tensor] = None) -> _lib.Problem:
    _require_cuda(pos, "pos")
    _require_cuda(w, "w")
    if pos.dim() != 2 or pos.shape[1] != 3:
        raise ValueError("pos must have shape (n, 3)")
    if pos.dtype not in (torch.float32, torch.float64):
        raise ValueError("pos must be float32 or float64")
    if w.dtype != torch.float64 or w.shape != (pos.shape[0],):
        raise ValueError("w must be float64 with shape (n,)")
    if not (pos.is_contiguous() and w.is_contiguous()):
        raise ValueError("pos and w must be contiguous")
    p = _lib.Problem()
    p.n = pos.shape[0]
    p.pos = pos.data_ptr() if p.n else None
    p.pos_dtype = _lib.F32 if pos.dtype == torch.float32 else _lib.F64
    p.w = w.data_ptr() if p.n else None
    for k in range(3):
        p.box[k] = float(cfg.box[k])
        p.box_lo[k] = float(cfg.box_lo[k])
        p.observer[k] = float(cfg.observer[k])
    p.periodic = 1 if cfg.periodic else 0
    p.rmax = float(cfg.rmax)
    p.nbins = int(cfg.nbins)
    p.lmax = int(cfg.lmax)
    p.los = _lib.LOS_Z if cfg.los == "z" else _lib.LOS_OBSERVER
    p.pair_prec = cfg.pair_prec()
    p.zeta_prec = cfg.zeta_prec()
    p.basis = _BASIS[cfg.basis]
    if primary_mask is not None:
        _require_cuda(primary_mask, "primary_mask")
        if primary_mask.dtype != torch.uint8 or primary_mask.shape != (p.n,):
            raise ValueError("primary_mask must be uint8 with shape (n,)")
        p.primary_mask = primary_mask.data_ptr()
    else:
        p.primary_mask = None
    p.accumulate = 1 if accumulate else 0
    p.pairs_out = pairs_out
    p.trace = trace.handle if trace is not None else None
    p.distinct = 1 if cfg.distinct else 0
    if alm is not None:
        _require_cuda(alm, "alm")
        if alm.dtype != torch.uint8 or alm.dim() != 1 or not alm.is_contiguous():
            raise ValueError("alm must be a contiguous 1-d uint8 tensor (see alm_store)")
        p.alm = alm.data_ptr()
        p.alm_bytes = alm.numel()
    else:
        p.alm = None
        p.alm_bytes = 0
    return p


def alm_store(pos: torch.Tensor, w: torch.Tensor, cfg: Config) -> torch.Tensor:
    """An uninitialised a_lm store for (pos, w, cfg): a device uint8 tensor of
    g3pcf_alm_bytes bytes (n * nbins * (lmax+1)^2 doubles and a header).

    Pass it as ``alm=`` to :func:`zeta`, which fills it, and then to
    :func:`zeta_backward` with the same inputs, which reads the a_lm from it
    instead of recomputing them (a mismatch gives a NaN gradient)."""
    nbytes = _lib.alm_bytes(make_problem(pos, w, cfg))
    return torch.empty(nbytes, dtype=torch.uint8, device=pos.device)


class Workspace:
    """A reusable device workspace (grows on demand)."""

    def __init__(self):
        self.buf: Optional[torch.Tensor] = None

    def get(self, nbytes: int, device) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = None
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        return self.buf


_default_ws = Workspace()


def zeta(pos: torch.Tensor, w: torch.Tensor, cfg: Config,
         primary_mask: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
         accumulate: bool = False, workspace: Optional[Workspace] = None,
         return_pairs: bool = False, trace: Optional["_lib.Trace"] = None,
         alm: Optional[torch.Tensor] = None):
    """zeta^m_{l l'}(b1, b2) as a float64 device tensor [m][l][l'][b1][b2][re, im].

    alm: an a_lm store (:func:`alm_store`) to keep the a_lm in for the backward pass."""
    import ctypes
    pairs = ctypes.c_int64(0)
    p = make_problem(pos, w, cfg, primary_mask, accumulate,
                     ctypes.pointer(pairs) if return_pairs else None, trace, alm)
    shape = zeta_shape(cfg.lmax, cfg.nbins)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=pos.device)
    elif out.shape != shape or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of shape " + str(shape))
    ws = (workspace or _default_ws).get(_lib.workspace_bytes(p, 0), pos.device)
    stream = torch.cuda.current_stream(pos.device).cuda_stream
    _lib.forward(p, out.data_ptr(), ws.data_ptr(), ws.numel(), stream)
    if return_pairs:
        return out, int(pairs.value)
    return out


def zeta_regions(pos: torch.Tensor, w: torch.Tensor, cfg: Config, region: torch.Tensor,
                 nregions: int, primary_mask: Optional[torch.Tensor] = None,
                 accumulate: bool = False, out: Optional[torch.Tensor] = None,
                 workspace: Optional[Workspace] = None, return_pairs: bool = False,
                 trace: Optional["_lib.Trace"] = None):
    """Partial zeta of each region of primaries, float64 [nregions][m][l][l'][b1][b2][2].

    ``region`` (int32, device, shape (n,)): galaxy i is a primary of region
    region[i] when 0 <= region[i] < nregions; every galaxy is a secondary."""
    import ctypes
    _require_cuda(region, "region")
    if region.dtype != torch.int32 or region.shape != (pos.shape[0],) or not region.is_contiguous():
        raise ValueError("region must be a contiguous int32 tensor of shape (n,)")
    pairs = ctypes.c_int64(0)
    p = make_problem(pos, w, cfg, primary_mask, accumulate,
                     ctypes.pointer(pairs) if return_pairs else None, trace)
    shape = (nregions,) + zeta_shape(cfg.lmax, cfg.nbins)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=pos.device)
    elif out.shape != shape or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of shape " + str(shape))
    ws = (workspace or _default_ws).get(_lib.workspace_bytes(p, 0), pos.device)
    stream = torch.cuda.current_stream(pos.device).cuda_stream
    _lib.check(_lib.load().g3pcf_forward_regions(
        ctypes.byref(p), ctypes.c_void_p(region.data_ptr() if p.n else 0), int(nregions),
        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
        ctypes.c_size_t(ws.numel()), ctypes.c_void_p(stream)))
    if return_pairs:
        return out, int(pairs.value)
    return out


def zeta_batch(pos: torch.Tensor, w: torch.Tensor, cfg: Config, offsets: Sequence[int],
               primary_mask: Optional[torch.Tensor] = None, accumulate: bool = False,
               out: Optional[torch.Tensor] = None, workspace: Optional[Workspace] = None,
               return_pairs: bool = False, trace: Optional["_lib.Trace"] = None):
    """zeta of each catalogue of a batch, float64 [ncat][m][l][l'][b1][b2][2].

    Catalogue c is rows offsets[c]:offsets[c+1] of ``pos`` / ``w`` (concatenated
    catalogues of one geometry, e.g. randoms or mocks); pairs never cross
    catalogues."""
    import ctypes
    offs = [int(o) for o in offsets]
    ncat = len(offs) - 1
    pairs = ctypes.c_int64(0)
    p = make_problem(pos, w, cfg, primary_mask, accumulate,
                     ctypes.pointer(pairs) if return_pairs else None, trace)
    shape = (ncat,) + zeta_shape(cfg.lmax, cfg.nbins)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=pos.device)
    elif out.shape != shape or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of shape " + str(shape))
    ws = (workspace or _default_ws).get(_lib.workspace_bytes(p, 0), pos.device)
    stream = torch.cuda.current_stream(pos.device).cuda_stream
    arr = (ctypes.c_int64 * len(offs))(*offs)
    _lib.check(_lib.load().g3pcf_forward_batch(
        ctypes.byref(p), int(ncat), arr, ctypes.c_void_p(out.data_ptr()),
        ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()), ctypes.c_void_p(stream)))
    if return_pairs:
        return out, int(pairs.value)
    return out


def zeta_backward(pos: torch.Tensor, w: torch.Tensor, cfg: Config, grad_zeta: torch.Tensor,
                  primary_mask: Optional[torch.Tensor] = None,
                  workspace: Optional[Workspace] = None,
                  trace: Optional["_lib.Trace"] = None,
                  alm: Optional[torch.Tensor] = None) -> torch.Tensor:
    """d(sum grad_zeta * zeta)/dw as a float64 device tensor (n,).

    alm: the a_lm store a :func:`zeta` call over the same inputs filled; the
    a_lm are then read from it instead of recomputed on the pair kernel."""
    p = make_problem(pos, w, cfg, primary_mask, trace=trace, alm=alm)
    shape = zeta_shape(cfg.lmax, cfg.nbins)
    gz = grad_zeta.to(torch.float64).contiguous()
    if gz.shape != shape:
        raise ValueError("grad_zeta must have shape " + str(shape))
    gw = torch.empty(pos.shape[0], dtype=torch.float64, device=pos.device)
    ws = (workspace or _default_ws).get(_lib.workspace_bytes(p, 1), pos.device)
    stream = torch.cuda.current_stream(pos.device).cuda_stream
    _lib.backward(p, gz.data_ptr(), gw.data_ptr(), ws.data_ptr(), ws.numel(), stream)
    return gw


def isotropic(zeta_t: torch.Tensor, lmax: int, nbins: int) -> torch.Tensor:
    """Isotropic multipoles [l][b1][b2] from zeta by the addition theorem, on the
    library's kernel: 4 pi / (2l + 1) (zeta^0_ll + 2 sum_{m >= 1} Re zeta^m_ll)."""
    import ctypes
    _require_cuda(zeta_t, "zeta")
    if (zeta_t.shape != zeta_shape(lmax, nbins) or zeta_t.dtype != torch.float64
            or not zeta_t.is_contiguous()):
        raise ValueError("zeta must be a contiguous float64 tensor of shape "
                         + str(zeta_shape(lmax, nbins)))
    out = torch.empty((lmax + 1, nbins, nbins), dtype=torch.float64, device=zeta_t.device)
    stream = torch.cuda.current_stream(zeta_t.device).cuda_stream
    _lib.check(_lib.load().g3pcf_isotropic(int(lmax), int(nbins),
                                           ctypes.c_void_p(zeta_t.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()),
                                           ctypes.c_void_p(stream)))
    return out


def _keep_alm(pos: torch.Tensor, w: torch.Tensor, cfg: Config, keep) -> Optional[torch.Tensor]:
    """The a_lm store for an autograd forward: always (keep=True), never
    (False, the default: the backward recomputes the a_lm), or (None) when it
    takes at most a quarter of the free device memory."""
    if keep is False or cfg.distinct:
        return None
    nbytes = _lib.alm_bytes(make_problem(pos, w, cfg))
    if keep is None:
        free, _ = torch.cuda.mem_get_info(pos.device)
        if nbytes > free // 4:
            return None
    return torch.empty(nbytes, dtype=torch.uint8, device=pos.device)


class G3PCF(torch.autograd.Function):
    """zeta as a differentiable function of the weights.

    forward(w, pos, cfg, primary_mask, keep_alm) -> zeta.  Saves ``pos``, ``w``
    and the mask; the backward pass recomputes the a_lm on the pair kernel
    (about n * nbins * (lmax+1)^2 * 8 bytes are never held).  keep_alm=True
    (or None: when it fits in a quarter of the free device memory) also keeps
    the a_lm store, and the backward reads the a_lm from it instead.
    Position gradients are not provided (None).
    """

    @staticmethod
    def forward(ctx, w, pos, cfg: Config, primary_mask=None, keep_alm=False):
        ctx.cfg = cfg
        ctx.save_for_backward(w, pos, primary_mask if primary_mask is not None else
                              torch.empty(0, dtype=torch.uint8, device=pos.device))
        ctx.has_mask = primary_mask is not None
        wd = w.detach()
        ctx.alm = _keep_alm(pos, wd, cfg, keep_alm)
        return zeta(pos, wd, cfg, primary_mask, alm=ctx.alm)

    @staticmethod
    def backward(ctx, grad_out):
        w, pos, mask = ctx.saved_tensors
        gw = zeta_backward(pos, w.detach(), ctx.cfg, grad_out,
                           mask if ctx.has_mask else None, alm=ctx.alm)
        ctx.alm = None
        return gw, None, None, None, None


def zeta_autograd(w, pos, cfg: Config, primary_mask=None, keep_alm=False):
    """zeta through torch.autograd; keep_alm as in :class:`G3PCF`."""
    return G3PCF.apply(w, pos, cfg, primary_mask, keep_alm)
