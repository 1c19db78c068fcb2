"""Host-side checks of the parity cases themselves (no GPU, no oracle)."""
import numpy as np

from paper_1709_00086_amd import catalogues as C


def _edge_margin(cat):
    """Smallest distance of any pair separation from a shell edge or R_max."""
    pos = cat.pos.astype(np.float64)
    L = np.asarray(cat.box, dtype=np.float64)
    d = pos[:, None, :] - pos[None, :, :]
    if cat.periodic:
        d -= L * np.rint(d / L)
    r = np.sqrt((d * d).sum(-1))
    r = r[(r > 0) & (r < cat.rmax + 1.0)]
    x = r * cat.nbins / cat.rmax
    return float(np.abs(x - np.rint(x)).min() * cat.rmax / cat.nbins)


def test_32_shell_case_is_clear_of_shell_edges():
    # FP32 separations of float32 positions in [0, 200) carry absolute errors
    # of a few 1e-6; a margin far above that means FP32 and FP64 binning agree
    # for every pair of the 32-shell parity case, so it can be held to 1e-5.
    cat = C.tiny(n=600, L=200.0, seed=19, rmax=60.0, nbins=32, lmax=10, periodic=True, los="z",
                 dtype=np.float32)
    assert _edge_margin(cat) > 9e-5


def test_non_finite_case_is_clear_of_shell_edges():
    # the GPU test of non-finite positions holds the FP32 gradient to 1e-4 of
    # the oracle's: no finite pair of its catalogue may sit near a shell edge
    for periodic in (True, False):
        cat = C.tiny(n=400, L=100.0, seed=48, rmax=40.0, nbins=4, lmax=10, periodic=periodic,
                     los="z")
        assert _edge_margin(cat) > 1e-4


def test_observer_case_is_clear_of_shell_edges():
    cat = C.tiny(n=64, L=100.0, seed=13, rmax=50.0, nbins=3, lmax=8, periodic=False,
                 los="observer")
    assert _edge_margin(cat) > 1e-3
