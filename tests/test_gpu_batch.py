"""A batch of catalogues of one geometry in one call (randoms / mocks).

Each catalogue's zeta from g3pcf_forward_batch is bitwise the zeta of a
separate g3pcf_forward on that catalogue alone (the same kernels on the same
inputs), pairs never cross catalogues, and the oracle agrees per catalogue.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1709_00086_amd import api, catalogues as C

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def batch_of(sizes, L, seed, dtype=np.float64):
    return C.mock_batch(sizes, L, seed, dtype)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("basis", ["spin", "cartesian"])
def test_batch_equals_separate_calls_and_oracle(dev, basis, precision):
    say(f"case batch {basis} {precision}")
    L, rmax, nbins, lmax = 300.0, 60.0, 6, 10
    sizes = [900, 0, 1, 2, 1500, 700]
    pos, w, offs = batch_of(sizes, L, seed=91)
    cfg = api.Config(box=(L, L, L), rmax=rmax, nbins=nbins, lmax=lmax, precision=precision,
                     basis=basis)
    pt = torch.from_numpy(pos).to(dev)
    wt = torch.from_numpy(w).to(dev)
    zb, pairs = api.zeta_batch(pt, wt, cfg, offs, return_pairs=True)
    total = 0
    for c in range(len(sizes)):
        a, b = int(offs[c]), int(offs[c + 1])
        zc, pc = api.zeta(pt[a:b].contiguous(), wt[a:b].contiguous(), cfg, return_pairs=True)
        assert torch.equal(zb[c], zc), c
        total += pc
    assert pairs == total
    # the oracle on two of the catalogues
    for c in (0, 4):
        a, b = int(offs[c]), int(offs[c + 1])
        cat = C.Catalogue(name=f"batch{c}", pos=pos[a:b], w=w[a:b], box=(L, L, L), rmax=rmax,
                          nbins=nbins, lmax=lmax, los="z", observer=(0.0, 0.0, 0.0),
                          periodic=True, box_lo=(0.0, 0.0, 0.0))
        ref = oracle.zeta(cat)
        err = np.abs(zb[c].cpu().numpy() - ref).max() / np.abs(ref).max()
        say(f"  catalogue {c}: max|dzeta|/max|zeta| = {err:.2e}")
        assert err <= (1e-10 if precision == "fp64" else 1e-5)
    # a catalogue with fewer than two galaxies has no pairs
    for c in (1, 2):
        assert torch.count_nonzero(zb[c]) == 0


def test_batch_masked_observer_and_accumulate(dev):
    """Non-periodic catalogues with an observer line of sight and a primary
    mask; accumulate = 1 adds into the output."""
    say("case batch masked observer")
    L, rmax = 200.0, 50.0
    sizes = [600, 800, 500]
    pos, w, offs = batch_of(sizes, L, seed=92)
    mask = (np.random.default_rng(93).uniform(size=len(w)) < 0.5).astype(np.uint8)
    cfg = api.Config(box=(L, L, L), rmax=rmax, nbins=5, lmax=8, los="observer",
                     observer=(-400.0, 100.0, 50.0), periodic=False, precision="fp64",
                     basis="spin")
    pt, wt = torch.from_numpy(pos).to(dev), torch.from_numpy(w).to(dev)
    mt = torch.from_numpy(mask).to(dev)
    zb = api.zeta_batch(pt, wt, cfg, offs, primary_mask=mt)
    for c in range(len(sizes)):
        a, b = int(offs[c]), int(offs[c + 1])
        zc = api.zeta(pt[a:b].contiguous(), wt[a:b].contiguous(), cfg,
                      primary_mask=mt[a:b].contiguous())
        assert torch.equal(zb[c], zc), c
    out = zb.clone()
    api.zeta_batch(pt, wt, cfg, offs, primary_mask=mt, accumulate=True, out=out)
    assert torch.allclose(out, 2 * zb, rtol=1e-14, atol=0)


def test_batch_full_size_mocks(dev):
    """Eight 2^17-galaxy catalogues in the 1000 Mpc/h box (R_max = 200, 10
    shells, FP32 spin, float32 positions): each zeta bitwise equal to its
    separate forward, one sampled catalogue against the oracle on 256
    primaries."""
    say("case batch 8 x 2^17")
    sizes = [1 << 17] * 8
    pos, w, offs = batch_of(sizes, 1000.0, seed=94, dtype=np.float32)
    cfg = api.Config(box=(1000.0,) * 3, rmax=200.0, nbins=10, lmax=10, precision="fp32",
                     basis="spin")
    pt, wt = torch.from_numpy(pos).to(dev), torch.from_numpy(w).to(dev)
    zb = api.zeta_batch(pt, wt, cfg, offs)
    for c in (0, 5):
        a, b = int(offs[c]), int(offs[c + 1])
        zc = api.zeta(pt[a:b].contiguous(), wt[a:b].contiguous(), cfg)
        assert torch.equal(zb[c], zc), c
    c = 3
    a, b = int(offs[c]), int(offs[c + 1])
    mask = C.primary_mask(b - a, 256, seed=95)
    cat = C.Catalogue(name="mock3", pos=pos[a:b], w=w[a:b], box=(1000.0,) * 3, rmax=200.0,
                      nbins=10, lmax=10, los="z", observer=(0.0, 0.0, 0.0), periodic=True,
                      box_lo=(0.0, 0.0, 0.0))
    ref = oracle.zeta(cat, primary_mask=mask)
    zs = api.zeta(pt[a:b].contiguous(), wt[a:b].contiguous(), cfg,
                  primary_mask=torch.from_numpy(mask).to(dev))
    err = np.abs(zs.cpu().numpy() - ref).max() / np.abs(ref).max()
    say(f"  mock 3 sample: max|dzeta|/max|zeta| = {err:.2e}")
    assert err <= 1e-5
