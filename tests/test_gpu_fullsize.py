"""Parity at the full workload sizes, in the configuration bench.py runs.

The oracle cannot compute zeta for 2^20 primaries in test time, so
  * the full catalogues run on the GPU with a seeded sample of primaries (every
    galaxy is still a secondary) and the sample's zeta is compared with the
    oracle's, through exactly the same pair-blocks and zeta blocks;
  * the full zeta (all primaries) is checked for properties that hold at any
    size: Hermitian symmetry, Im zeta^0 = 0, a positive semi-definite Gram per
    m, finiteness, and additivity over a partition of the primaries.
"""
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


@functools.lru_cache(maxsize=None)
def catalogue(name):
    return getattr(C, name)()


@functools.lru_cache(maxsize=None)
def oracle_sample(name, count, seed):
    cat = catalogue(name)
    mask = C.primary_mask(cat.n, count, seed=seed)
    z, pairs = oracle.zeta(cat, primary_mask=mask, return_pairs=True)
    return mask, z, pairs


def cfg_of(cat, precision, basis, zeta_precision=None):
    return api.Config(box=cat.box, rmax=cat.rmax, nbins=cat.nbins, lmax=cat.lmax, los=cat.los,
                      observer=cat.observer, periodic=cat.periodic, box_lo=cat.box_lo,
                      precision=precision, basis=basis, zeta_precision=zeta_precision)


_ws = api.Workspace()


def run(cat, dev, precision, basis, mask=None, zeta_precision=None):
    pos = torch.from_numpy(cat.pos).to(dev)
    w = torch.from_numpy(cat.w).to(dev)
    m = torch.from_numpy(mask).to(dev) if mask is not None else None
    z, pairs = api.zeta(pos, w, cfg_of(cat, precision, basis, zeta_precision), primary_mask=m,
                        workspace=_ws, return_pairs=True)
    return z.cpu().numpy(), pairs


def rel(z, ref):
    return float(np.abs(z - ref).max() / np.abs(ref).max())


@pytest.mark.parametrize("name", ["config2", "config3", "config5"])
def test_sampled_primaries_vs_oracle(dev, name):
    say(f"case full-size sample {name}")
    cat = catalogue(name)
    mask, ref, pairs_ref = oracle_sample(name, 1024, 7)
    for precision, basis, tol in [("fp64", "cartesian", 1e-10), ("fp64", "spin", 1e-10),
                                  ("fp32", "cartesian", 1e-5), ("fp32", "spin", 1e-5),
                                  ("bf16x3", "spin", 1e-5)]:
        z, pairs = run(cat, dev, precision, basis, mask)
        e = rel(z, ref)
        say(f"  {name} {precision} {basis}: max|dz|/max|z| = {e:.3e}, pairs {pairs} "
            f"(oracle {pairs_ref})")
        assert e <= tol
        if precision == "fp64":
            assert pairs == pairs_ref
        else:
            assert abs(pairs - pairs_ref) <= 1e-5 * pairs_ref


def check_properties(z, lmax, nbins, label):
    assert np.isfinite(z).all()
    zc = z[..., 0] + 1j * z[..., 1]
    herm = np.abs(zc - np.conj(np.transpose(zc, (0, 2, 1, 4, 3)))).max() / np.abs(zc).max()
    im0 = np.abs(z[0, ..., 1]).max() / np.abs(zc).max()
    worst_neg = 0.0
    for m in range(lmax + 1):
        d = (lmax + 1 - m) * nbins
        Hm = zc[m, m:, m:].transpose(0, 2, 1, 3).reshape(d, d)
        ev = np.linalg.eigvalsh(0.5 * (Hm + Hm.conj().T))
        worst_neg = max(worst_neg, -ev.min() / max(ev.max(), 1e-300))
    zero_ok = all(np.abs(z[m, :m]).max() == 0 and np.abs(z[m, :, :m]).max() == 0
                  for m in range(1, lmax + 1))
    say(f"  {label}: hermitian {herm:.2e}, Im zeta^0 {im0:.2e}, most negative eigenvalue "
        f"{worst_neg:.2e}")
    return herm, im0, worst_neg, zero_ok


@pytest.mark.parametrize("name", ["config2", "config3"])
def test_full_zeta_properties(dev, name):
    say(f"case full-size properties {name}")
    cat = catalogue(name)
    z, pairs = run(cat, dev, "fp32", "spin")
    herm, im0, neg, zero_ok = check_properties(z, cat.lmax, cat.nbins, f"{name} fp32 spin")
    assert herm <= 1e-6 and im0 <= 1e-6 and neg <= 1e-6 and zero_ok
    say(f"  accepted pairs {pairs}")
    if name == "config2":
        # uniform expectation: N n V(R) = N (N / L^3) (4/3) pi R^3 ~ 35,138 per primary
        expect = cat.n * (cat.n / 1000.0 ** 3) * 4.0 / 3.0 * np.pi * 200.0 ** 3
        assert abs(pairs / expect - 1.0) < 1e-3
    # additivity over a partition of the primaries, full launch configuration
    rng = np.random.default_rng(17)
    a = (rng.uniform(size=cat.n) < 0.5).astype(np.uint8)
    za, pa = run(cat, dev, "fp64", "spin", a)
    zb, pb = run(cat, dev, "fp64", "spin", (1 - a).astype(np.uint8))
    z64, p64 = run(cat, dev, "fp64", "spin")
    assert pa + pb == p64
    e = rel(za + zb, z64)
    say(f"  partition additivity (fp64): {e:.3e}")
    assert e <= 1e-12
    # the FP32 and FP64 full results agree within the FP32 tolerance
    e32 = rel(z, z64)
    say(f"  full fp32 vs fp64: {e32:.3e}")
    assert e32 <= 1e-5
    # the benchmark's default form: FP32 pairs, BF16x3 zeta stage over every
    # block of primaries
    zb, pbf = run(cat, dev, "bf16x3", "spin")
    herm, im0, neg, zero_ok = check_properties(zb, cat.lmax, cat.nbins, f"{name} bf16x3 spin")
    assert herm <= 1e-6 and im0 <= 1e-6 and neg <= 1e-6 and zero_ok
    assert pbf == pairs
    eb = rel(zb, z64)
    say(f"  full bf16x3 vs fp64: {eb:.3e}")
    assert eb <= 1e-5


def test_zeta_stage_sweep_across_blocks(dev):
    """Config-2 catalogue, 65,536 seeded primaries (16 zeta blocks of 4096):
    the same FP64 pair stage with FP64, FP32 and BF16x3 zeta stages, each
    compared with the FP64 one, exercises the FP64 cross-block sum."""
    say("case zeta-stage sweep over 16 blocks")
    cat = catalogue("config2")
    mask = C.primary_mask(cat.n, 65536, seed=9)
    z64, _ = run(cat, dev, "fp64", "spin", mask, zeta_precision="fp64")
    scale = np.abs(z64).max()
    big = np.abs(z64) >= 1e-8 * scale
    for zp in ["fp32", "bf16x3"]:
        z, _ = run(cat, dev, "fp64", "spin", mask, zeta_precision=zp)
        e = np.abs(z - z64).max() / scale
        pe = (np.abs(z - z64)[big] / np.abs(z64)[big]).max()
        say(f"  zeta stage {zp}: max|dz|/max|z| = {e:.3e}, max per-entry rel = {pe:.3e}")
        assert e <= 1e-5


def test_ragged_pair_blocks_add_up(dev):
    """Config-2 catalogue, primaries split into 2^19 + 777 and the rest: one
    side runs a full pair-block of 524,288 primaries plus a ragged one of 777,
    the other a single ragged block; the two zetas add up to the zeta of all
    primaries (two full blocks) in FP64, and their pair counts to its count."""
    say("case ragged pair-blocks")
    cat = catalogue("config2")
    perm = np.random.default_rng(19).permutation(cat.n)
    a = np.zeros(cat.n, dtype=np.uint8)
    a[perm[: (1 << 19) + 777]] = 1
    za, pa = run(cat, dev, "fp64", "spin", a)
    zb, pb = run(cat, dev, "fp64", "spin", (1 - a).astype(np.uint8))
    z64, p64 = run(cat, dev, "fp64", "spin")
    assert pa + pb == p64
    e = rel(za + zb, z64)
    say(f"  ragged blocks additivity (fp64): {e:.3e}")
    assert e <= 1e-12


def test_large_catalogue_2e23(dev):
    """N = 2^23 uniform in a periodic 2000 Mpc/h box (R_max = 200, 10 shells,
    float32 positions, w ~ U(0.5, 1.5), spin basis): 16 pair-blocks of 2^19
    primaries over a grid of 4.1 million cells, 2.8e11 pairs.  The full FP32
    zeta is finite, Hermitian and PSD per m, with the uniform pair count; 128
    seeded primaries agree with the oracle in FP32 and FP64."""
    say("case large catalogue 2^23")
    cat = C.uniform(1 << 23, 2000.0, seed=23, dtype=np.float32, weights="uniform",
                    rmax=200.0, name="uniform_n8388608_L2000_r200_f32")
    z, pairs = run(cat, dev, "fp32", "spin")
    herm, im0, neg, zero_ok = check_properties(z, cat.lmax, cat.nbins, "2^23 fp32 spin")
    assert herm <= 1e-6 and im0 <= 1e-6 and neg <= 1e-6 and zero_ok
    expect = cat.n * (cat.n / 2000.0 ** 3) * 4.0 / 3.0 * np.pi * 200.0 ** 3
    say(f"  accepted pairs {pairs} (uniform expectation {expect:.4e})")
    assert abs(pairs / expect - 1.0) < 1e-3
    mask = C.primary_mask(cat.n, 128, seed=24)
    ref, pref = oracle.zeta(cat, primary_mask=mask, return_pairs=True)
    for precision, tol in (("fp32", 1e-5), ("fp64", 1e-10)):
        zs, ps = run(cat, dev, precision, "spin", mask)
        e = rel(zs, ref)
        say(f"  sample {precision}: max|dz|/max|z| = {e:.3e}, pairs {ps} (oracle {pref})")
        assert e <= tol
        if precision == "fp64":
            assert ps == pref
