"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: FP64 mode max|dz| <= 1e-10 max|z_oracle|; FP32 pair stage (FP32
or BF16x3 zeta stage) max|dz| <= 1e-5 max|z_oracle|.  Pair counts are integers
and must match exactly in FP64 mode; in FP32 mode a pair whose separation lies
within FP32 rounding of a shell edge or of R_max may fall on the other side, so
the count may differ by a few pairs.
"""
import dataclasses
import functools
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


def cfg_of(cat, precision, basis="cartesian", zeta_precision=None):
    return api.Config(box=cat.box, rmax=cat.rmax, nbins=cat.nbins, lmax=cat.lmax, los=cat.los,
                      observer=cat.observer, periodic=cat.periodic, box_lo=cat.box_lo,
                      precision=precision, basis=basis, zeta_precision=zeta_precision)


def run_gpu(cat, dev, precision, basis="cartesian", mask=None, zeta_precision=None):
    pos = torch.from_numpy(np.ascontiguousarray(cat.pos)).to(dev)
    w = torch.from_numpy(np.ascontiguousarray(cat.w)).to(dev)
    m = torch.from_numpy(mask).to(dev) if mask is not None else None
    z, pairs = api.zeta(pos, w, cfg_of(cat, precision, basis, zeta_precision), primary_mask=m,
                        return_pairs=True)
    return z.cpu().numpy(), pairs


def compare(z, ref, tol, label):
    scale = np.abs(ref).max()
    err = np.abs(z - ref).max() / scale
    big = np.abs(ref) >= 1e-8 * scale
    per_entry = (np.abs(z - ref)[big] / np.abs(ref)[big]).max() if big.any() else 0.0
    say(f"  {label}: max|dz|/max|z| = {err:.3e}, max per-entry rel (|z| >= 1e-8 max) = "
        f"{per_entry:.3e}")
    assert np.isfinite(z).all()
    assert err <= tol, (label, err)
    return err


@functools.lru_cache(maxsize=None)
def oracle_of(key):
    cat, mask = _CATS[key]()
    z, pairs = oracle.zeta(cat, primary_mask=mask, return_pairs=True)
    return z, pairs


def _tiny(**kw):
    return lambda: (C.tiny(**kw), None)


_CATS = {
    "tiny_periodic_tight": _tiny(n=48, L=100.0, seed=11, rmax=50.0, nbins=4, lmax=10,
                                 periodic=True, los="z"),
    "tiny_open": _tiny(n=64, L=100.0, seed=12, rmax=45.0, nbins=5, lmax=6, periodic=False,
                       los="z"),
    "tiny_observer_open": _tiny(n=64, L=100.0, seed=13, rmax=50.0, nbins=3, lmax=8,
                                periodic=False, los="observer", observer=(-250.0, -120.0, -60.0)),
    "tiny_observer_periodic": _tiny(n=64, L=80.0, seed=14, rmax=40.0, nbins=4, lmax=5,
                                    periodic=True, los="observer", observer=(300.0, 200.0, 500.0)),
    "small_periodic": _tiny(n=2000, L=200.0, seed=15, rmax=45.0, nbins=7, lmax=10,
                            periodic=True, los="z"),
    "small_open_f32": _tiny(n=2000, L=200.0, seed=16, rmax=60.0, nbins=10, lmax=10,
                            periodic=False, los="z", dtype=np.float32, box_lo=(-50.0, 10.0, 3.0)),
    # the maximum number of shells (list entries carry shells >= 16 in their
    # top bits); float32 positions whose separations all keep >= 9e-5 from a
    # shell edge and from R_max, so FP32 binning agrees with FP64 binning
    "small_32_shells": _tiny(n=600, L=200.0, seed=19, rmax=60.0, nbins=32, lmax=10,
                             periodic=True, los="z", dtype=np.float32),
    "config1": lambda: (C.config1(), None),
    "config1_weighted": lambda: (C.config1_weighted(), None),
}

SMALL = ["tiny_periodic_tight", "tiny_open", "tiny_observer_open", "tiny_observer_periodic",
         "small_periodic", "small_open_f32", "small_32_shells"]


@pytest.mark.parametrize("basis", ["cartesian", "spin"])
@pytest.mark.parametrize("key", SMALL)
def test_small_cases_fp64(dev, key, basis):
    say(f"case {key} fp64 {basis}")
    cat, _ = _CATS[key]()
    ref, pairs_ref = oracle_of(key)
    z, pairs = run_gpu(cat, dev, "fp64", basis)
    compare(z, ref, 1e-10, f"{key} fp64 {basis}")
    assert pairs == pairs_ref


@pytest.mark.parametrize("basis", ["cartesian", "spin"])
@pytest.mark.parametrize("key", SMALL)
def test_small_cases_fp32(dev, key, basis):
    say(f"case {key} fp32 {basis}")
    cat, _ = _CATS[key]()
    ref, pairs_ref = oracle_of(key)
    z, pairs = run_gpu(cat, dev, "fp32", basis)
    compare(z, ref, 1e-5, f"{key} fp32 {basis}")
    assert abs(pairs - pairs_ref) <= 2 + 1e-6 * pairs_ref


@pytest.mark.parametrize("basis", ["cartesian", "spin"])
def test_config1_fp64_full(dev, basis):
    say(f"case config1 fp64 {basis}")
    cat, _ = _CATS["config1"]()
    ref, pairs_ref = oracle_of("config1")
    z, pairs = run_gpu(cat, dev, "fp64", basis)
    compare(z, ref, 1e-10, f"config1 fp64 {basis}")
    assert pairs == pairs_ref
    say(f"  pairs {pairs}")


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("basis", ["cartesian", "spin"])
def test_config1_split_precisions(dev, basis, precision):
    say(f"case config1 {precision} {basis}")
    cat, _ = _CATS["config1"]()
    ref, _ = oracle_of("config1")
    z, _ = run_gpu(cat, dev, precision, basis)
    compare(z, ref, 1e-5, f"config1 {precision} {basis}")


def test_zeta_stage_precision_sweep_same_pairs(dev):
    """Same FP64 pair stage, three zeta-stage precisions (isolates that stage)."""
    say("case config1 zeta-stage sweep")
    cat, _ = _CATS["config1"]()
    ref, _ = oracle_of("config1")
    for zp in ["fp64", "fp32", "bf16x3"]:
        z, _ = run_gpu(cat, dev, "fp64", "spin", zeta_precision=zp)
        compare(z, ref, 1e-10 if zp == "fp64" else 1e-5, f"zeta stage {zp}")


def test_mask_additivity_and_accumulate(dev):
    say("case mask additivity")
    cat, _ = _CATS["small_periodic"]()
    rng = np.random.default_rng(8)
    a = (rng.uniform(size=cat.n) < 0.3).astype(np.uint8)
    b = (1 - a).astype(np.uint8)
    za, _ = run_gpu(cat, dev, "fp64", "spin", mask=a)
    zb, _ = run_gpu(cat, dev, "fp64", "spin", mask=b)
    zall, _ = run_gpu(cat, dev, "fp64", "spin")
    assert np.abs(za + zb - zall).max() <= 1e-13 * np.abs(zall).max()
    # accumulate = 1 adds into the output
    pos = torch.from_numpy(cat.pos).to(dev)
    w = torch.from_numpy(cat.w).to(dev)
    cfg = cfg_of(cat, "fp64", "spin")
    out = api.zeta(pos, w, cfg, primary_mask=torch.from_numpy(a).to(dev))
    api.zeta(pos, w, cfg, primary_mask=torch.from_numpy(b).to(dev), out=out, accumulate=True)
    assert np.abs(out.cpu().numpy() - zall).max() <= 1e-13 * np.abs(zall).max()


def test_degenerate_inputs(dev):
    say("case degenerate inputs")
    cat, _ = _CATS["tiny_open"]()
    z, pairs = run_gpu(cat, dev, "fp32", mask=np.zeros(cat.n, np.uint8))
    assert pairs == 0 and np.abs(z).max() == 0.0
    empty = dataclasses.replace(cat, pos=np.zeros((0, 3)), w=np.zeros(0))
    z, pairs = run_gpu(empty, dev, "fp64")
    assert pairs == 0 and np.abs(z).max() == 0.0
    one = dataclasses.replace(cat, pos=cat.pos[:1].copy(), w=cat.w[:1].copy())
    z, pairs = run_gpu(one, dev, "fp64")
    assert pairs == 0 and np.abs(z).max() == 0.0
    # coincident galaxies are excluded (r = 0), duplicates elsewhere are counted
    dup = dataclasses.replace(cat, pos=np.concatenate([cat.pos, cat.pos[:5]]),
                              w=np.concatenate([cat.w, cat.w[:5]]))
    ref, pref = oracle.zeta(dup, return_pairs=True)
    z, pairs = run_gpu(dup, dev, "fp64")
    compare(z, ref, 1e-10, "duplicates fp64")
    assert pairs == pref


def test_repeatable(dev):
    say("case repeatability")
    cat, _ = _CATS["small_periodic"]()
    for prec in ["fp64", "fp32"]:
        z1, _ = run_gpu(cat, dev, prec, "cartesian")
        z2, _ = run_gpu(cat, dev, prec, "cartesian")
        assert np.array_equal(z1, z2), prec


@functools.lru_cache(maxsize=None)
def _dense_case():
    # ~23k pairs per primary in two shells: the outer shell holds more
    # secondaries than a wave's spill list (16,384), the inner one fewer, so the
    # multi-chunk bases take both the replay path and the repeated-search path
    cat = C.tiny(n=60000, L=100.0, seed=21, rmax=45.0, nbins=2, lmax=10, periodic=True,
                 los="z", dtype=np.float32)
    mask = C.primary_mask(cat.pos.shape[0], 256, seed=22)
    ref, pairs = oracle.zeta(cat, primary_mask=mask, return_pairs=True)
    return cat, mask, ref, pairs


@pytest.mark.parametrize("precision,basis", [("fp64", "cartesian"), ("fp64", "spin"),
                                             ("fp32", "cartesian"), ("fp32", "spin")])
def test_dense_shells_beyond_spill_capacity(dev, precision, basis):
    say(f"case dense two-shell catalogue {precision} {basis}")
    cat, mask, ref, pairs_ref = _dense_case()
    assert pairs_ref > 256 * 16384  # the outer shell overflows a spill list
    z, pairs = run_gpu(cat, dev, precision, basis, mask=mask)
    compare(z, ref, 1e-10 if precision == "fp64" else 1e-5, f"dense {precision} {basis}")
    if precision == "fp64":
        assert pairs == pairs_ref
    else:
        assert abs(pairs - pairs_ref) <= 2 + 1e-6 * pairs_ref
