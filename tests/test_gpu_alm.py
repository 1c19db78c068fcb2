"""The a_lm store: the forward pass keeps every primary's a_lm for the backward.

With the store the backward reads the a_lm the forward wrote instead of
recomputing them on the pair kernel.  The pair kernel is deterministic (one
wave per primary, a fixed order of candidates), so zeta is bitwise the same
with or without the store and the gradient differs only by the order of the
atomic additions of the secondary terms.  A store written for other inputs
makes the gradient NaN.
"""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1709_00086_amd import _lib, api, catalogues as C

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def cfg_of(cat, precision, basis):
    return api.Config(box=cat.box, rmax=cat.rmax, nbins=cat.nbins, lmax=cat.lmax, los=cat.los,
                      observer=cat.observer, periodic=cat.periodic, box_lo=cat.box_lo,
                      precision=precision, basis=basis)


def tensors(cat, dev, mask=None):
    pos = torch.from_numpy(np.ascontiguousarray(cat.pos)).to(dev)
    w = torch.from_numpy(np.ascontiguousarray(cat.w)).to(dev)
    m = torch.from_numpy(mask).to(dev) if mask is not None else None
    return pos, w, m


SMALL = dict(n=1500, L=200.0, seed=15, rmax=45.0, nbins=7, lmax=10, periodic=True, los="z")
OPEN = dict(n=900, L=150.0, seed=19, rmax=40.0, nbins=5, lmax=9, periodic=False,
            los="observer", observer=(-300.0, 40.0, -90.0))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("basis", ["spin", "cartesian"])
@pytest.mark.parametrize("key", ["small", "open"])
def test_store_matches_recompute_and_oracle(dev, key, basis, precision):
    say(f"case alm {key} {basis} {precision}")
    cat = C.tiny(**(SMALL if key == "small" else OPEN))
    mask = None
    if key == "open":
        mask = (np.random.default_rng(73).uniform(size=cat.n) < 0.6).astype(np.uint8)
    pos, w, m = tensors(cat, dev, mask)
    cfg = cfg_of(cat, precision, basis)
    c = torch.from_numpy(np.random.default_rng(74).standard_normal(
        C.zeta_shape(cat.lmax, cat.nbins))).to(dev)
    z0 = api.zeta(pos, w, cfg, primary_mask=m)
    g0 = api.zeta_backward(pos, w, cfg, c, primary_mask=m)
    store = api.alm_store(pos, w, cfg)
    z1 = api.zeta(pos, w, cfg, primary_mask=m, alm=store)
    g1 = api.zeta_backward(pos, w, cfg, c, primary_mask=m, alm=store)
    # the same kernels write the same a_lm rows elsewhere: zeta is bitwise equal
    assert torch.equal(z0, z1)
    g0, g1 = g0.cpu().numpy(), g1.cpu().numpy()
    scale = np.abs(g0).max()
    d = np.abs(g1 - g0).max() / scale
    ref = oracle.grad(cat, c.cpu().numpy(), primary_mask=mask)
    e = np.abs(g1 - ref).max() / np.abs(ref).max()
    say(f"  store vs recompute {d:.2e}; store vs oracle {e:.2e}")
    # only the order of the secondary terms' atomic additions differs
    assert d <= (1e-13 if precision == "fp64" else 1e-6)
    assert e <= (1e-10 if precision == "fp64" else 1e-4)


def test_autograd_keeps_the_store(dev):
    """zeta_autograd with keep_alm False (the default: recompute) / True /
    None (keep when it fits): the same gradient."""
    say("case alm autograd")
    cat = C.config1_weighted()
    pos, w0, _ = tensors(cat, dev)
    cfg = cfg_of(cat, "fp64", "spin")
    c = torch.from_numpy(C.loss_weights(cat.lmax, cat.nbins, seed=55)).to(dev)
    grads = []
    for keep in (False, True, None):
        w = w0.clone().requires_grad_(True)
        z = api.zeta_autograd(w, pos, cfg, keep_alm=keep)
        (z * c).sum().backward()
        grads.append(w.grad.cpu().numpy())
    ref = oracle.grad(cat, c.cpu().numpy())
    for g in grads:
        assert np.abs(g - grads[0]).max() <= 1e-13 * np.abs(grads[0]).max()
        assert np.abs(g - ref).max() <= 1e-10 * np.abs(ref).max()


def test_store_from_other_inputs_gives_nan(dev):
    """Changed weight, changed mask, changed settings: NaN gradient; the right
    inputs afterwards: a finite gradient again (the check is per call)."""
    say("case alm mismatch")
    cat = C.tiny(**SMALL)
    pos, w, _ = tensors(cat, dev)
    cfg = cfg_of(cat, "fp32", "spin")
    c = torch.from_numpy(np.random.default_rng(75).standard_normal(
        C.zeta_shape(cat.lmax, cat.nbins))).to(dev)
    store = api.alm_store(pos, w, cfg)
    api.zeta(pos, w, cfg, alm=store)
    w2 = w.clone()
    w2[17] += 1e-3
    assert torch.isnan(api.zeta_backward(pos, w2, cfg, c, alm=store)).all()
    pos2 = pos.clone()
    pos2[3, 1] += 1e-2
    assert torch.isnan(api.zeta_backward(pos2, w, cfg, c, alm=store)).all()
    mask = torch.ones(cat.n, dtype=torch.uint8, device=dev)
    mask[100] = 0
    assert torch.isnan(api.zeta_backward(pos, w, cfg, c, primary_mask=mask, alm=store)).all()
    cfg_cart = cfg_of(cat, "fp32", "cartesian")
    assert torch.isnan(api.zeta_backward(pos, w, cfg_cart, c, alm=store)).all()
    g = api.zeta_backward(pos, w, cfg, c, alm=store)
    assert torch.isfinite(g).all()
    # accumulate = 1 adds NaN into the caller's array as well
    gw = torch.zeros(cat.n, dtype=torch.float64, device=dev)
    p = api.make_problem(pos, w2, cfg, accumulate=True, alm=store)
    ws = api.Workspace().get(_lib.workspace_bytes(p, 1), dev)
    _lib.backward(p, c.contiguous().data_ptr(), gw.data_ptr(), ws.data_ptr(), ws.numel(),
                  torch.cuda.current_stream(dev).cuda_stream)
    assert torch.isnan(gw).all()


def test_store_pairs_and_empty_catalogue(dev):
    """pairs_out of the backward with the store (the adjoint pass's count) is
    the forward's; n = 0 with a store is a no-op."""
    say("case alm pairs / empty")
    cat = C.tiny(**SMALL)
    pos, w, _ = tensors(cat, dev)
    cfg = cfg_of(cat, "fp32", "spin")
    store = api.alm_store(pos, w, cfg)
    _, pairs = api.zeta(pos, w, cfg, alm=store, return_pairs=True)
    c = torch.ones(api.zeta_shape(cat.lmax, cat.nbins), dtype=torch.float64, device=dev)
    cnt = ctypes.c_int64(-1)
    p = api.make_problem(pos, w, cfg, pairs_out=ctypes.pointer(cnt), alm=store)
    ws = api.Workspace().get(_lib.workspace_bytes(p, 1), dev)
    gw = torch.empty(cat.n, dtype=torch.float64, device=dev)
    _lib.backward(p, c.data_ptr(), gw.data_ptr(), ws.data_ptr(), ws.numel(),
                  torch.cuda.current_stream(dev).cuda_stream)
    assert cnt.value == pairs > 0
    e_pos = torch.empty((0, 3), dtype=torch.float64, device=dev)
    e_w = torch.empty(0, dtype=torch.float64, device=dev)
    e_store = api.alm_store(e_pos, e_w, cfg)
    assert e_store.numel() == 256
    z = api.zeta(e_pos, e_w, cfg, alm=e_store)
    assert torch.count_nonzero(z) == 0
    g = api.zeta_backward(e_pos, e_w, cfg, c, alm=e_store)
    assert g.numel() == 0


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_store_full_size_matches_recompute(dev, precision):
    """N = 2^20 (the uniform 1000 Mpc/h box, R_max = 200, 10 shells), spin basis,
    in the benchmark's launch configuration: zeta bitwise equal, gradient with
    the store against the recomputed one.  Each galaxy's secondary terms, about
    3.5e4 of them, are summed by atomics in no fixed order: in FP32 two runs
    of the same path differ by a few 1e-6 of max|g| (bound 1e-5, ten times
    under the FP32 parity bound against the oracle), in FP64 by ~1e-15."""
    say(f"case alm config2 full size {precision}")
    cat = C.config2()
    pos, w, _ = tensors(cat, dev)
    cfg = cfg_of(cat, precision, "spin")
    c = torch.from_numpy(C.loss_weights(cat.lmax, cat.nbins, seed=55)).to(dev)
    ws = api.Workspace()
    z0 = api.zeta(pos, w, cfg, workspace=ws)
    g0 = api.zeta_backward(pos, w, cfg, c, workspace=ws).cpu().numpy()
    store = api.alm_store(pos, w, cfg)
    z1 = api.zeta(pos, w, cfg, workspace=ws, alm=store)
    g1 = api.zeta_backward(pos, w, cfg, c, workspace=ws, alm=store).cpu().numpy()
    del store
    assert torch.equal(z0, z1)
    d = np.abs(g1 - g0).max() / np.abs(g0).max()
    say(f"  full size: store vs recompute max|dg|/max|g| = {d:.2e}")
    assert d <= (1e-5 if precision == "fp32" else 1e-12)
