"""g3pcf_forward_noalloc (the forward pass in the library's static scratch,
for callers that cannot allocate) against g3pcf_forward, through the C ABI.

Two calls in a row on one GPU, the second with a smaller catalogue (the
scratch keeps the first call's contents, so everything the second needs
cleared must be cleared by the call itself); each is compared with
g3pcf_forward on the same input: equal pair counts, and zeta within 1e-12 of
max|zeta| (only the FP64 sums across blocks of primaries are ordered
differently; the pair stage and every block's Gram product are the same).
A problem too large for the scratch is refused before anything is enqueued.
"""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

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


def noalloc(cat, dev, cfg):
    pos = torch.from_numpy(np.ascontiguousarray(cat.pos)).to(dev)
    w = torch.from_numpy(np.ascontiguousarray(cat.w)).to(dev)
    pairs = ctypes.c_int64(-1)
    p = api.make_problem(pos, w, cfg, pairs_out=ctypes.pointer(pairs))
    z = torch.full(api.zeta_shape(cat.lmax, cat.nbins), float("nan"), dtype=torch.float64,
                   device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    _lib.forward_noalloc(p, z.data_ptr(), stream)
    torch.cuda.synchronize()
    return z.cpu().numpy(), int(pairs.value)


def with_workspace(cat, dev, cfg):
    pos = torch.from_numpy(np.ascontiguousarray(cat.pos)).to(dev)
    w = torch.from_numpy(np.ascontiguousarray(cat.w)).to(dev)
    z, pairs = api.zeta(pos, w, cfg, return_pairs=True)
    return z.cpu().numpy(), pairs


CATS = [
    # 20,000 galaxies (five pair-blocks of the scratch layout), then 3,000
    lambda: C.uniform(20000, 400.0, seed=61, dtype=np.float32, weights="uniform", rmax=60.0),
    lambda: C.tiny(n=3000, L=150.0, seed=62, rmax=40.0, nbins=6, lmax=8, periodic=False,
                   los="observer", observer=(-100.0, 20.0, -50.0), dtype=np.float32),
]


@pytest.mark.parametrize("precision,basis", [("fp32", "spin"), ("fp64", "cartesian"),
                                             ("fp32", "cartesian"), ("bf16x3", "spin")])
def test_noalloc_matches_workspace_forward(dev, precision, basis):
    for k, make in enumerate(CATS):
        cat = make()
        say(f"case noalloc call {k + 1} n={cat.n} {precision} {basis}")
        cfg = cfg_of(cat, precision, basis)
        z, pairs = noalloc(cat, dev, cfg)
        ref, pref = with_workspace(cat, dev, cfg)
        e = np.abs(z - ref).max() / np.abs(ref).max()
        say(f"  pairs {pairs} (workspace {pref}), max|dz|/max|z| = {e:.3e}")
        assert pairs == pref
        assert np.isfinite(z).all()
        assert e <= 1e-12


def test_noalloc_refuses_a_problem_beyond_the_scratch(dev):
    say("case noalloc size limit")
    cat = C.uniform(1 << 21, 1000.0, seed=63, dtype=np.float32, weights="uniform", rmax=200.0)
    cfg = cfg_of(cat, "fp32", "spin")
    with pytest.raises(_lib.G3pcfError) as ei:
        noalloc(cat, dev, cfg)
    assert ei.value.code == _lib.EINVAL and "scratch" in str(ei.value)
