"""Seeded synthetic galaxy catalogues for the anisotropic 3PCF hot path.

This module only draws random numbers and arranges them into arrays. It holds
none of the estimator's arithmetic, so both the FP64 CPU oracle (test
infrastructure) and the HIP path can take their inputs from it.

The paper measures on the Outer Rim halo catalogue (Sec. "Problem
Configuration"), which is not available here; the uniform and Neyman-Scott
catalogues below stand in for it with the same kind of geometry: 3-D positions
in a cube, R_max of 100-200 Mpc/h, 10 radial bins and l_max = 10 (Sec. 3.1 and
the vectorisation section, eq. 1).

Draw order for every catalogue: positions as an (N, 3) float64 array, cast to
the stated dtype (a float32 value that rounds up to the box edge is wrapped
back to the low edge), then weights.  All generators use NumPy's PCG64
``default_rng(seed)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Catalogue:
    """A catalogue plus the estimator settings it is measured with."""

    name: str
    pos: np.ndarray          # (N, 3) float32 or float64, row-major
    w: np.ndarray            # (N,) float64 weights
    box: tuple               # box side lengths (Lx, Ly, Lz)
    box_lo: tuple            # low corner of the box
    periodic: bool
    rmax: float
    nbins: int
    lmax: int
    los: str                 # "z" or "observer"
    observer: tuple = (0.0, 0.0, 0.0)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def subset(self, idx) -> "Catalogue":
        """A catalogue holding only the galaxies ``idx`` (same settings)."""
        idx = np.asarray(idx)
        return dataclasses.replace(self, pos=np.ascontiguousarray(self.pos[idx]),
                                   w=np.ascontiguousarray(self.w[idx]))


def _cast_positions(pos64: np.ndarray, dtype, lo, L) -> np.ndarray:
    pos = pos64.astype(dtype)
    if dtype == np.float32:
        lo32 = np.asarray(lo, dtype=np.float32)
        hi = (np.asarray(lo, np.float64) + np.asarray(L, np.float64)).astype(np.float32)
        for a in range(3):
            col = pos[:, a]
            col[col >= hi[a]] = lo32[a]
    return np.ascontiguousarray(pos)


def uniform(n: int, L: float, seed: int, dtype=np.float64, weights: str = "unit",
            rmax: float = 100.0, nbins: int = 10, lmax: int = 10,
            name: str = "uniform") -> Catalogue:
    """N galaxies uniform in the periodic cube [0, L)^3.

    ``weights`` is "unit" (w = 1) or "uniform" (w ~ U(0.5, 1.5)).
    """
    rng = np.random.default_rng(seed)
    pos64 = rng.uniform(0.0, L, size=(n, 3))
    pos = _cast_positions(pos64, dtype, (0.0, 0.0, 0.0), (L, L, L))
    if weights == "unit":
        w = np.ones(n, dtype=np.float64)
    elif weights == "uniform":
        w = rng.uniform(0.5, 1.5, size=n)
    else:
        raise ValueError(weights)
    return Catalogue(name, pos, w, (L, L, L), (0.0, 0.0, 0.0), True, rmax, nbins,
                     lmax, "z")


def neyman_scott(n: int, L: float, centre, n_parents: int, sigma: float, seed: int,
                 dtype=np.float32, rmax: float = 200.0, nbins: int = 10,
                 lmax: int = 10, name: str = "neyman_scott") -> Catalogue:
    """Clustered catalogue: Gaussian blobs around uniform parents.

    Parents are uniform in the cube of side ``L`` centred on ``centre``; each
    gets Poisson(n / n_parents) members displaced by N(0, sigma^2) per axis.
    Members outside the cube are rejected.  If fewer than ``n`` survive,
    another batch of ``n_parents`` parents is drawn.  The first ``n`` members in
    generation order are kept.  Unit weights, no periodicity, observer at the
    origin.
    """
    rng = np.random.default_rng(seed)
    lo = np.asarray(centre, np.float64) - L / 2.0
    hi = lo + L
    lam = n / float(n_parents)
    kept = []
    total = 0
    while total < n:
        parents = lo + rng.uniform(0.0, L, size=(n_parents, 3))
        counts = rng.poisson(lam, size=n_parents)
        members = np.repeat(parents, counts, axis=0)
        members = members + rng.normal(0.0, sigma, size=members.shape)
        members = members.astype(dtype).astype(np.float64)
        inside = np.all((members >= lo) & (members < hi), axis=1)
        members = members[inside]
        kept.append(members)
        total += members.shape[0]
    pos64 = np.concatenate(kept, axis=0)[:n]
    pos = np.ascontiguousarray(pos64.astype(dtype))
    w = np.ones(n, dtype=np.float64)
    return Catalogue(name, pos, w, (L, L, L), tuple(lo.tolist()), False, rmax, nbins,
                     lmax, "observer", (0.0, 0.0, 0.0))


# ----------------------------------------------------------------------------
# The five workloads.  Sizes follow the estimator settings the paper uses
# (R_max = 200 Mpc/h, l_max = 10) scaled to one GPU.
# ----------------------------------------------------------------------------

def config1() -> Catalogue:
    """N = 4096 uniform, periodic L = 500, float64, unit weights, R_max = 100."""
    return uniform(4096, 500.0, seed=1, dtype=np.float64, weights="unit", rmax=100.0,
                   name="uniform_n4096_L500_r100_f64")


def config2() -> Catalogue:
    """N = 2^20 uniform, periodic L = 1000, float32, w ~ U(0.5,1.5), R_max = 200."""
    return uniform(1 << 20, 1000.0, seed=2, dtype=np.float32, weights="uniform",
                   rmax=200.0, name="uniform_n1048576_L1000_r200_f32")


def config3() -> Catalogue:
    """N = 2^21 Neyman-Scott blobs in a non-periodic cube 2000 Mpc/h away."""
    c = 2000.0 / math.sqrt(3.0)
    return neyman_scott(1 << 21, 1500.0, (c, c, c), 20000, 5.0, seed=3,
                        dtype=np.float32, rmax=200.0,
                        name="neyman_scott_n2097152_L1500_r200_f32_observer")


def config5() -> Catalogue:
    """N = 2^18 uniform, periodic L = 650, float64, w ~ U(0.5,1.5), R_max = 150."""
    return uniform(1 << 18, 650.0, seed=5, dtype=np.float64, weights="uniform",
                   rmax=150.0, name="uniform_n262144_L650_r150_f64")


def config1_weighted() -> Catalogue:
    """Config-1 positions with w ~ U(0.5, 1.5) drawn from seed 51."""
    cat = config1()
    rng = np.random.default_rng(51)
    cat.w = rng.uniform(0.5, 1.5, size=cat.n)
    cat.name = "uniform_n4096_L500_r100_f64_weighted"
    return cat


def primary_mask(n: int, count: int, seed: int = 7) -> np.ndarray:
    """uint8 mask with ``count`` primaries chosen without replacement."""
    rng = np.random.default_rng(seed)
    m = np.zeros(n, dtype=np.uint8)
    m[rng.choice(n, size=count, replace=False)] = 1
    return m


def mock_batch(sizes, L: float, seed: int, dtype=np.float64):
    """Seeded uniform catalogues of one periodic box L^3 (stand-ins for randoms
    or mocks of one geometry), concatenated: positions (sum(sizes), 3) of
    ``dtype``, weights ~ U(0.5, 1.5) float64, and offsets [len(sizes) + 1]
    int64 (catalogue c is rows offsets[c]:offsets[c+1]).  Draw order per
    catalogue: positions, then weights."""
    rng = np.random.default_rng(seed)
    pos, w = [], []
    for n in sizes:
        pos.append(_cast_positions(rng.uniform(0.0, L, size=(n, 3)), dtype, (0.0, 0.0, 0.0),
                                   (L, L, L)))
        w.append(rng.uniform(0.5, 1.5, size=n))
    offs = np.concatenate([[0], np.cumsum(sizes, dtype=np.int64)]).astype(np.int64)
    return np.concatenate(pos), np.concatenate(w), offs


def loss_weights(lmax: int, nbins: int, seed: int = 55) -> np.ndarray:
    """c ~ N(0, 1) float64 shaped like zeta: [m][l][l'][b1][b2][re,im]."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((lmax + 1, lmax + 1, lmax + 1, nbins, nbins, 2))


def fd_indices(n: int, count: int = 64, seed: int = 56) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.choice(n, size=count, replace=False)


def tiny(n: int, L: float, seed: int, rmax: float, nbins: int = 4, lmax: int = 4,
         periodic: bool = True, los: str = "z", weights: str = "uniform",
         dtype=np.float64, observer=(0.0, 0.0, 0.0), box_lo=(0.0, 0.0, 0.0)) -> Catalogue:
    """Small catalogue for brute-force checks (N <= 64 typically)."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(box_lo, np.float64)
    pos64 = lo + rng.uniform(0.0, L, size=(n, 3))
    pos = _cast_positions(pos64, dtype, lo, (L, L, L))
    if weights == "unit":
        w = np.ones(n)
    else:
        w = rng.uniform(0.5, 1.5, size=n)
    return Catalogue("tiny", pos, w, (L, L, L), tuple(lo.tolist()), periodic, rmax,
                     nbins, lmax, los, tuple(observer))


def zeta_shape(lmax: int, nbins: int):
    return (lmax + 1, lmax + 1, lmax + 1, nbins, nbins, 2)
