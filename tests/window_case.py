"""A catalogue whose pair-kernel windows hold 64 runs of one candidate each.

The pair kernel reads a shell's candidates as runs of cell-order slots: per
(cy, cz) row of cells, the cells of the row that can hold a separation in the
shell's annulus (the outer sphere's x-interval minus the inner sphere's, so up
to two ranges per row), 64 rows at a time, and maps 64 candidates at a time to
their runs.  A window of 64 candidates that spans 64 runs has a run start at
every position (all 64 of its run-start marks set), the extreme case of that
mapping.  This module builds a catalogue
in which one primary's annulus runs are all one galaxy long and more than 64
of them fall into one block of rows, and it replays the grid and run
construction on the host (same formulas as the library's cell grid and run
build) to show that the windows really are made of single-galaxy runs.

Geometry (non-periodic box [0, 260)^3, R_max = 100, 10 shells): the primary P
sits at the box centre; for every row whose annulus of shell 8 ([80, 90)) has
two separate x-ranges, one galaxy at distance 85 from P in each range, at the
row's (y, z) centre; rows with a single x-range get one galaxy; rows near the
boundary between the two cases get none.  Filler galaxies farther than 130
from P bring the count to N = 20,000, so that the grid keeps its cells of
R_max/64 along x and R_max/8 across (the grid has at most 4 N cells).
"""
from __future__ import annotations

import math

import numpy as np

from paper_1709_00086_amd import catalogues as C

RMAX = 100.0
NBINS = 10
SHELL = 8
L = 260.0
N = 20000


def grid(n, box, box_lo, rmax, periodic):
    """Host replay of the library's cell grid (cell sides, counts, margin)."""
    ext = max(abs(box_lo[a]) + abs(box[a]) for a in range(3))
    rsearch = rmax * (1.0 + 1e-5) + 1e-6 * ext + 1e-9
    target = [rmax / 64.0, rmax / 8.0, rmax / 8.0]
    cap = min(max(64, 4 * n), 1 << 24)
    nc = [int(max(1.0, min(math.floor(box[a] / target[a]), 4096.0))) for a in range(3)]
    while nc[0] * nc[1] * nc[2] > cap:
        nc = [max(1, (c * 4) // 5) for c in nc]
    s = [box[a] / nc[a] for a in range(3)]
    return dict(nc=nc, s=s, inv_s=[nc[a] / box[a] for a in range(3)], lo=list(box_lo),
                rsearch=rsearch, periodic=periodic)


def _axis_range(prel, cu, nc, s):
    lo, hi = cu - prel, cu - prel + 1.0
    if cu == 0:
        lo = -math.inf
    if cu == nc - 1:
        hi = math.inf
    return max(0.0, max(lo, -hi)) * s, max(abs(lo), abs(hi)) * s


def shell_rows(g, p, shell, nbins, rmax):
    """Per row of the shell's search window (in the kernel's row order): the
    cell ranges of x that the pair kernel reads for primary p (open box)."""
    margin = g["rsearch"] - rmax
    r0 = max(0.0, shell * rmax / nbins - margin)
    r1 = g["rsearch"] if shell + 1 == nbins else (shell + 1) * rmax / nbins + margin
    nc, lo, inv_s, s = g["nc"], g["lo"], g["inv_s"], g["s"]

    def cl(v, a):
        c = int(math.floor((v - lo[a]) * inv_s[a]))
        return min(max(c, 0), nc[a] - 1)
    c0 = [0, cl(p[1] - r1, 1), cl(p[2] - r1, 2)]
    c1 = [0, cl(p[1] + r1, 1), cl(p[2] + r1, 2)]
    nyr, nzr = c1[1] - c0[1] + 1, c1[2] - c0[2] + 1
    prel = [(p[a] - lo[a]) * inv_s[a] for a in range(3)]
    rows = []
    for r in range(nyr * nzr):
        cz, cy = c0[2] + r // nyr, c0[1] + r % nyr
        dzmin, dzmax = _axis_range(prel[2], cz, nc[2], s[2])
        dymin, dymax = _axis_range(prel[1], cy, nc[1], s[1])
        d2min, d2max = dymin ** 2 + dzmin ** 2, dymax ** 2 + dzmax ** 2
        ranges = []
        if d2min < r1 * r1:
            hx1 = math.sqrt(r1 * r1 - d2min)
            cut = r0 > 0 and r0 * r0 > d2max
            hx0 = math.sqrt(r0 * r0 - d2max) if cut else 0.0

            def cx(v):
                return min(max(int(math.floor(prel[0] + v * inv_s[0])), 0), nc[0] - 1)
            a1, b1, a2, b2 = cx(-hx1), cx(-hx0), cx(hx0), cx(hx1)
            ranges = [(a1, b2)] if a2 <= b1 + 1 else [(a1, b1), (a2, b2)]
        rows.append(((cy, cz), ranges, (hx0 if d2min < r1 * r1 else 0.0,
                                          hx1 if d2min < r1 * r1 else 0.0)))
    return rows


def cells_of(g, pos):
    pos = np.asarray(pos, np.float64)
    idx = []
    for a in range(3):
        f = np.floor((pos[:, a] - g["lo"][a]) * g["inv_s"][a])
        idx.append(np.clip(f, 0, g["nc"][a] - 1).astype(np.int64))
    return idx


def build(dtype=np.float64, seed=41):
    """(catalogue, primary mask selecting P = galaxy 0)."""
    g = grid(N, (L, L, L), (0.0, 0.0, 0.0), RMAX, False)
    P = np.array([L / 2, L / 2, L / 2])
    rmid = (SHELL + 0.5) * RMAX / NBINS
    s = g["s"]
    pts = [P]
    for (cy, cz), ranges, (hx0, hx1) in shell_rows(g, P, SHELL, NBINS, RMAX):
        yc, zc = (cy + 0.5) * s[1], (cz + 0.5) * s[2]
        d = math.hypot(yc - P[1], zc - P[2])
        if not ranges or d >= rmid:
            continue
        h = math.sqrt(rmid * rmid - d * d)
        # keep every galaxy at least two x-cells inside its range, and the two
        # ranges of a row at least three cells apart, so that rounding in the
        # kernel's FP32 chords cannot move a galaxy or merge the ranges
        if (len(ranges) == 2 and hx0 > 3 * s[0] and h - hx0 > 2 * s[0]
                and hx1 - h > 2 * s[0]):
            pts += [[P[0] - h, yc, zc], [P[0] + h, yc, zc]]
        elif len(ranges) == 1 and hx1 - h > 2 * s[0] and hx0 == 0.0:
            pts.append([P[0] + h, yc, zc])
    rng = np.random.default_rng(seed)
    fill = []
    while len(pts) + len(fill) < N:
        q = rng.uniform(0.0, L, size=(4 * N, 3))
        q = q[np.linalg.norm(q - P, axis=1) > 1.3 * RMAX]
        fill.extend(q[: N - len(pts) - len(fill)].tolist())
    pos64 = np.array(pts + fill, dtype=np.float64)
    pos = pos64.astype(dtype)
    w = rng.uniform(0.5, 1.5, size=N)
    cat = C.Catalogue("window_runs", np.ascontiguousarray(pos), w, (L, L, L), (0.0, 0.0, 0.0),
                      False, RMAX, NBINS, 10, "z")
    mask = np.zeros(N, np.uint8)
    mask[0] = 1
    return cat, mask


def window_runs(cat):
    """Run lengths of P's shell-8 search, per block of 64 rows (host replay)."""
    g = grid(cat.n, cat.box, cat.box_lo, cat.rmax, cat.periodic)
    cx, cy, cz = cells_of(g, cat.pos)
    P = np.asarray(cat.pos[0], np.float64)
    rows = shell_rows(g, P, SHELL, cat.nbins, cat.rmax)
    by_row = {}
    for k in range(cat.n):
        by_row.setdefault((int(cy[k]), int(cz[k])), []).append(int(cx[k]))
    blocks = []
    for b0 in range(0, len(rows), 64):
        runs = []
        for (ry, rz), ranges, _ in rows[b0:b0 + 64]:
            xs = by_row.get((ry, rz), [])
            for a, b in ranges:
                cnt = sum(1 for x in xs if a <= x <= b)
                if cnt:
                    runs.append(cnt)
        blocks.append(runs)
    return blocks


# ---- a dense open box: blocks of 64 rows with several spans of run-start marks
# (the kernel marks run starts for 4096 candidates of a block at a time)

DENSE_N = 250000
MARK_SPAN = 4096


def build_dense(dtype=np.float64, seed=47, nprim=4):
    """Uniform galaxies in the open box [0, 260)^3 (R_max = 100, 10 shells);
    primaries: the nprim galaxies nearest the box centre.  (catalogue, mask)"""
    rng = np.random.default_rng(seed)
    pos64 = rng.uniform(0.0, L, size=(DENSE_N, 3))
    w = rng.uniform(0.5, 1.5, size=DENSE_N)
    cat = C.Catalogue("dense_open_box", np.ascontiguousarray(pos64.astype(dtype)), w,
                      (L, L, L), (0.0, 0.0, 0.0), False, RMAX, NBINS, 10, "z")
    d = np.linalg.norm(pos64 - L / 2, axis=1)
    mask = np.zeros(DENSE_N, np.uint8)
    mask[np.argsort(d)[:nprim]] = 1
    return cat, mask


def block_totals(cat, k, shell):
    """Candidates per block of 64 rows of galaxy k's search of `shell`
    (host replay of the run construction, open box)."""
    g = grid(cat.n, cat.box, cat.box_lo, cat.rmax, cat.periodic)
    cx, cy, cz = cells_of(g, cat.pos)
    rows = shell_rows(g, np.asarray(cat.pos[k], np.float64), shell, cat.nbins, cat.rmax)
    key = cy.astype(np.int64) * (g["nc"][2] + 1) + cz
    order = np.argsort(key, kind="stable")
    ks, xs = key[order], cx[order]
    totals = []
    for b0 in range(0, len(rows), 64):
        t = 0
        for (ry, rz), ranges, _ in rows[b0:b0 + 64]:
            kk = ry * (g["nc"][2] + 1) + rz
            lo, hi = np.searchsorted(ks, kk), np.searchsorted(ks, kk, side="right")
            row_x = xs[lo:hi]
            for a, b in ranges:
                t += int(np.count_nonzero((row_x >= a) & (row_x <= b)))
        totals.append(t)
    return totals
