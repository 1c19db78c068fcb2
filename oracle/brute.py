"""Brute-force references that pin the oracle (test infrastructure).

Nothing here is used by the product.  These routines use SciPy's spherical
harmonics and Legendre polynomials, a different line-of-sight rotation
construction from the oracle's, and O(N^3) triplet sums with no factorisation
through a_lm, so that a mistake in the oracle's recurrence, rotation, binning or
reduction shows up as a disagreement.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import eval_legendre, sph_harm_y


def _wrapped(cat):
    pos = np.asarray(cat.pos, dtype=np.float64).copy()
    if cat.periodic:
        for c in range(3):
            lo, L = cat.box_lo[c], cat.box[c]
            t = np.fmod(pos[:, c] - lo, L)
            t = np.where(t < 0, t + L, t)
            t = np.where(t >= L, 0.0, t)
            pos[:, c] = lo + t
    return pos


def _rodrigues_to_z(n):
    """A rotation R with R n = z, built with Rodrigues' formula about n x z
    (the identity for n = 0: a primary on the observer keeps the box frame)."""
    n = np.asarray(n, dtype=np.float64)
    if not np.any(n):
        return np.eye(3)
    n = n / np.linalg.norm(n)
    z = np.array([0.0, 0.0, 1.0])
    v = np.cross(n, z)
    c = float(np.dot(n, z))
    if c < -1.0 + 1e-12:
        return np.diag([1.0, -1.0, -1.0])
    vx = np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])
    return np.eye(3) + vx + vx @ vx / (1.0 + c)


def neighbour_table(cat, azimuth_seed=None):
    """For each galaxy i: (j indices, bins, unit vectors in i's frame).

    ``azimuth_seed`` adds an independent random rotation about the line of
    sight for every primary (the result must not depend on it)."""
    pos = _wrapped(cat)
    n = pos.shape[0]
    L = np.asarray(cat.box, dtype=np.float64)
    rng = np.random.default_rng(azimuth_seed) if azimuth_seed is not None else None
    out = []
    for i in range(n):
        d = pos - pos[i]
        if cat.periodic:
            d = d - L * np.round(d / L)
        r2 = np.einsum("ij,ij->i", d, d)
        ok = (r2 > 0) & (r2 < cat.rmax ** 2)
        ok[i] = False
        j = np.nonzero(ok)[0]
        r = np.sqrt(r2[j])
        b = np.minimum(cat.nbins - 1, np.floor(r * cat.nbins / cat.rmax).astype(int))
        u = d[j] / r[:, None]
        if cat.los == "observer":
            R = _rodrigues_to_z(pos[i] - np.asarray(cat.observer, dtype=np.float64))
            if rng is not None:
                a = rng.uniform(0, 2 * math.pi)
                Rz = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0],
                               [0, 0, 1.0]])
                R = Rz @ R
            u = u @ R.T
        out.append((j, b, u))
    return out


def ylm_matrix(u, lmax):
    """Y[n, l, m] (m >= 0) via scipy.special.sph_harm_y (orthonormal, CS phase)."""
    u = np.atleast_2d(u)
    rho = np.hypot(u[:, 0], u[:, 1])
    theta = np.arctan2(rho, u[:, 2])   # accurate near the poles, unlike arccos(u_z)
    phi = np.arctan2(u[:, 1], u[:, 0])
    Y = np.zeros((u.shape[0], lmax + 1, lmax + 1), dtype=np.complex128)
    for l in range(lmax + 1):
        for m in range(l + 1):
            Y[:, l, m] = sph_harm_y(l, m, theta, phi)
    return Y


def zeta_triplets(cat, primary_mask=None, azimuth_seed=None, distinct=False):
    """zeta from an explicit sum over ordered triplets (i, j, k), j, k != i,
    j = k included (left out with ``distinct``), with no factorisation through a_lm:
      zeta^m_{ll'}(b_ij, b_ik) += w_i w_j w_k conj(Y_lm(u_ij)) Y_l'm(u_ik)."""
    lmax, nb = cat.lmax, cat.nbins
    z = np.zeros((lmax + 1, lmax + 1, lmax + 1, nb, nb), dtype=np.complex128)
    tab = neighbour_table(cat, azimuth_seed)
    w = np.asarray(cat.w, dtype=np.float64)
    for i, (j, b, u) in enumerate(tab):
        if primary_mask is not None and not primary_mask[i]:
            continue
        if j.size == 0:
            continue
        Y = ylm_matrix(u, lmax)
        wj = w[j]
        # every ordered triplet (i, j, k): T[j, k, m, l, l'] = conj(Y_lm(u_ij)) Y_l'm(u_ik)
        T = np.einsum("jam,kbm->jkmab", np.conj(Y), Y)
        f = w[i] * np.outer(wj, wj)
        if distinct:
            np.fill_diagonal(f, 0.0)
        T = T * f[:, :, None, None, None]
        bj = np.repeat(b, j.size)
        bk = np.tile(b, j.size)
        T = T.reshape(j.size * j.size, lmax + 1, lmax + 1, lmax + 1)
        for t in range(T.shape[0]):
            z[:, :, :, bj[t], bk[t]] += T[t]
    # zero the l < m and l' < m entries (Y_lm with m > l are zero already)
    out = np.zeros(z.shape + (2,))
    out[..., 0] = z.real
    out[..., 1] = z.imag
    return out


def isotropic_triplets(cat, primary_mask=None, distinct=False):
    """sum_i w_i sum_{j in b1, k in b2} w_j w_k P_l(u_ij . u_ik), shape [l][b1][b2]
    (j = k left out with ``distinct``)."""
    lmax, nb = cat.lmax, cat.nbins
    out = np.zeros((lmax + 1, nb, nb))
    w = np.asarray(cat.w, dtype=np.float64)
    for i, (j, b, u) in enumerate(neighbour_table(cat)):
        if primary_mask is not None and not primary_mask[i]:
            continue
        if j.size == 0:
            continue
        mu = np.clip(u @ u.T, -1.0, 1.0)
        ww = w[i] * np.outer(w[j], w[j])
        if distinct:
            np.fill_diagonal(ww, 0.0)
        for l in range(lmax + 1):
            P = eval_legendre(l, mu) * ww
            np.add.at(out[l], (b[:, None].repeat(j.size, 1), b[None, :].repeat(j.size, 0)), P)
    return out


def isotropic_from_zeta(z):
    """(4 pi / (2l+1)) [zeta^0_ll + 2 sum_{m>=1} Re zeta^m_ll]  (addition theorem)."""
    lmax = z.shape[0] - 1
    nb = z.shape[3]
    out = np.zeros((lmax + 1, nb, nb))
    for l in range(lmax + 1):
        s = z[0, l, l, :, :, 0].copy()
        for m in range(1, l + 1):
            s += 2.0 * z[m, l, l, :, :, 0]
        out[l] = 4.0 * math.pi / (2 * l + 1) * s
    return out


def bin_counts_kdtree(cat):
    """Per-primary weighted neighbour sums W_i(b) using scipy's cKDTree."""
    from scipy.spatial import cKDTree
    pos = _wrapped(cat)
    if cat.periodic:
        lo = np.asarray(cat.box_lo)
        tree = cKDTree(pos - lo, boxsize=np.asarray(cat.box))
        q = pos - lo
    else:
        tree = cKDTree(pos)
        q = pos
    n = pos.shape[0]
    W = np.zeros((n, cat.nbins))
    w = np.asarray(cat.w, dtype=np.float64)
    L = np.asarray(cat.box, dtype=np.float64)
    lists = tree.query_ball_point(q, cat.rmax)
    for i in range(n):
        j = np.asarray(lists[i], dtype=np.int64)
        j = j[j != i]
        d = pos[j] - pos[i]
        if cat.periodic:
            d = d - L * np.round(d / L)
        r = np.sqrt(np.einsum("ij,ij->i", d, d))
        ok = (r > 0) & (r < cat.rmax)
        b = np.minimum(cat.nbins - 1, np.floor(r[ok] * cat.nbins / cat.rmax).astype(int))
        np.add.at(W[i], b, w[j[ok]])
    return W
