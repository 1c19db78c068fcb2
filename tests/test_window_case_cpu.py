"""Host check of the single-galaxy-run catalogue used by the GPU parity test
of the pair kernel's window mapping (no GPU, no oracle)."""
import numpy as np

import window_case as WC


def test_some_window_holds_64_single_galaxy_runs():
    for dtype in (np.float64, np.float32):
        cat, mask = WC.build(dtype)
        blocks = WC.window_runs(cat)
        # every run of the shell's search is a single galaxy ...
        assert all(all(r == 1 for r in runs) for runs in blocks)
        # ... and some block of 64 rows has more than 64 of them, so a window
        # of 64 candidates spans 64 runs (a run start at every position)
        assert max(len(runs) for runs in blocks) > 64
        # each galaxy of the construction is at distance 85 from the primary,
        # in the middle of shell 8 ([80, 90)), far from both edges
        p = cat.pos.astype(np.float64)
        d = np.linalg.norm(p[1:] - p[0], axis=1)
        near = d[d < 100.0]
        assert near.size == sum(len(r) for r in blocks)
        assert np.abs(near - 85.0).max() < 1e-3


def test_dense_box_blocks_span_several_mark_spans():
    cat, mask = WC.build_dense(np.float64)
    assert int(mask.sum()) == 4
    best = 0
    for k in np.flatnonzero(mask):
        for shell in (8, 9):
            best = max(best, max(WC.block_totals(cat, int(k), shell)))
    # a block of 64 rows with candidates in three spans of run-start marks
    assert best > 2 * WC.MARK_SPAN
