"""Pins of the oracle's degenerate-triangle option and isotropic multipoles.

With distinct secondaries the triangles j = k (the same secondary on both
sides of the primary) are left out of zeta.  Pins: O(N^3) triplet sums that
skip j = k, the Legendre brute force of the isotropic 3PCF without j = k, the
two-galaxy case (nothing but j = k triangles, so zero), and the structure of
the removed part (b1 = b2 only, real, a sum of w_i w_j^2 |Y|^2-type terms).
Every test here runs on the CPU.
"""
import math

import numpy as np
import pytest

import oracle
import oracle.brute as brute
from paper_1709_00086_amd import catalogues as C

CASES = [
    dict(n=48, L=100.0, seed=111, rmax=50.0, nbins=4, lmax=10, periodic=True, los="z"),
    dict(n=44, L=100.0, seed=112, rmax=45.0, nbins=3, lmax=6, periodic=False, los="observer",
         observer=(-250.0, -120.0, -60.0)),
]


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("case", CASES)
def test_distinct_zeta_matches_triplets_without_j_equal_k(case):
    cat = C.tiny(**case)
    z = oracle.zeta(cat, distinct=True)
    zb = brute.zeta_triplets(cat, distinct=True)
    assert rel(z, zb) <= 1e-12
    # and it differs from the full zeta (the j = k part is not negligible)
    assert rel(z, oracle.zeta(cat)) > 1e-3


@pytest.mark.parametrize("distinct", [False, True])
@pytest.mark.parametrize("los", ["z", "observer"])
def test_isotropic_matches_legendre_brute_force(los, distinct):
    cat = C.tiny(60, 100.0, seed=131, rmax=50.0, nbins=4, lmax=7, periodic=False, los=los,
                 observer=(-200.0, 50.0, -300.0))
    iso = oracle.isotropic(oracle.zeta(cat, distinct=distinct))
    ref = brute.isotropic_triplets(cat, distinct=distinct)
    assert rel(iso, ref) <= 1e-12


def test_isotropic_monopole_is_weighted_pair_count_product():
    # P_0 = 1: zeta_0(b1, b2) = sum_i w_i W_i(b1) W_i(b2), W_i(b) = sum_{j in b} w_j
    cat = C.tiny(300, 200.0, seed=121, rmax=60.0, nbins=6, lmax=2, periodic=True)
    W = brute.bin_counts_kdtree(cat)
    ref = np.einsum("i,ib,ic->bc", cat.w, W, W)
    iso = oracle.isotropic(oracle.zeta(cat))
    assert np.abs(iso[0] - ref).max() <= 1e-12 * ref.max()


def test_two_galaxies_have_no_distinct_triangles():
    rng = np.random.default_rng(141)
    for _ in range(3):
        d = rng.standard_normal(3)
        d *= rng.uniform(5, 45) / np.linalg.norm(d)
        p1 = np.array([50.0, 50.0, 50.0])
        cat = C.Catalogue("two", np.stack([p1, p1 + d]), rng.uniform(0.5, 1.5, 2),
                          (100.0,) * 3, (0.0,) * 3, False, 50.0, 5, 10, "z")
        assert np.abs(oracle.zeta(cat)).max() > 1e-3
        assert np.abs(oracle.zeta(cat, distinct=True)).max() <= 1e-15


def test_removed_part_is_diagonal_real_and_matches_direct_sum():
    cat = C.tiny(50, 100.0, seed=151, rmax=50.0, nbins=4, lmax=5, periodic=True, los="z")
    d = oracle.zeta(cat) - oracle.zeta(cat, distinct=True)
    nb = cat.nbins
    off = ~np.eye(nb, dtype=bool)
    assert np.abs(d[..., off, :]).max() == 0.0
    assert np.abs(d[..., 1]).max() <= 1e-15 * np.abs(d).max()
    # direct sum of w_i w_j^2 conj(Y_lm) Y_l'm over pairs with SciPy's Y_lm
    ref = np.zeros(d.shape[:3] + (nb,))
    w = np.asarray(cat.w)
    for i, (j, b, u) in enumerate(brute.neighbour_table(cat)):
        if j.size == 0:
            continue
        Y = brute.ylm_matrix(u, cat.lmax)
        for t in range(j.size):
            v = w[i] * w[j[t]] ** 2 * np.conj(Y[t])[:, None, :] * Y[t][None, :, :]
            ref[:, :, :, b[t]] += np.moveaxis(v.real, 2, 0)
    for m in range(cat.lmax + 1):
        ref[m, :m] = 0.0
        ref[m, :, :m] = 0.0
    got = np.stack([d[..., k, k, 0] for k in range(nb)], axis=-1)
    assert rel(got, ref) <= 1e-12
