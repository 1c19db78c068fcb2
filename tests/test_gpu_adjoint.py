"""The adjoint d(sum c * zeta)/dw on the GPU, through torch.autograd.

Checked against the FP64 oracle's analytic gradient (itself pinned by exact
finite differences on the CPU) and against central finite differences of the
FP64 GPU forward.  zeta is quadratic in any single weight, so the central
difference is exact up to the forward's rounding divided by h.
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


def cfg_of(cat, precision, basis):
    return api.Config(box=cat.box, rmax=cat.rmax, nbins=cat.nbins, lmax=cat.lmax, los=cat.los,
                      observer=cat.observer, periodic=cat.periodic, box_lo=cat.box_lo,
                      precision=precision, basis=basis)


def gpu_grad(cat, c, dev, precision, basis, mask=None):
    pos = torch.from_numpy(np.ascontiguousarray(cat.pos)).to(dev)
    w = torch.from_numpy(np.ascontiguousarray(cat.w)).to(dev).requires_grad_(True)
    m = torch.from_numpy(mask).to(dev) if mask is not None else None
    z = api.zeta_autograd(w, pos, cfg_of(cat, precision, basis), m)
    loss = (z * torch.from_numpy(c).to(dev)).sum()
    loss.backward()
    return w.grad.cpu().numpy(), float(loss)


CASES = {
    "tiny_periodic_tight": dict(n=48, L=100.0, seed=11, rmax=50.0, nbins=4, lmax=10,
                                periodic=True, los="z"),
    "tiny_observer_open": dict(n=64, L=100.0, seed=13, rmax=50.0, nbins=3, lmax=8,
                               periodic=False, los="observer", observer=(-250.0, -120.0, -60.0)),
    "small_periodic": dict(n=1500, L=200.0, seed=15, rmax=45.0, nbins=7, lmax=10,
                           periodic=True, los="z"),
}


@pytest.mark.parametrize("basis", ["cartesian", "spin"])
@pytest.mark.parametrize("key", sorted(CASES))
def test_gradient_matches_oracle(dev, key, basis):
    say(f"case adjoint {key} {basis}")
    cat = C.tiny(**CASES[key])
    c = np.random.default_rng(71).standard_normal(C.zeta_shape(cat.lmax, cat.nbins))
    mask = None
    if key == "small_periodic":
        mask = (np.random.default_rng(72).uniform(size=cat.n) < 0.7).astype(np.uint8)
    ref = oracle.grad(cat, c, primary_mask=mask)
    scale = np.abs(ref).max()
    g64, _ = gpu_grad(cat, c, dev, "fp64", basis, mask)
    e64 = np.abs(g64 - ref).max() / scale
    g32, _ = gpu_grad(cat, c, dev, "fp32", basis, mask)
    e32 = np.abs(g32 - ref).max() / scale
    say(f"  fp64 max|dg|/max|g| = {e64:.3e}; fp32 = {e32:.3e}")
    assert e64 <= 1e-10
    assert e32 <= 1e-4


def test_gradient_config1_weighted_vs_oracle(dev):
    """N = 4096 (config-1 positions, w ~ U(0.5, 1.5)): the oracle gradient."""
    say("case adjoint config1_weighted")
    cat = C.config1_weighted()
    c = C.loss_weights(cat.lmax, cat.nbins, seed=55)
    ref = oracle.grad(cat, c)
    scale = np.abs(ref).max()
    for basis in ["cartesian", "spin"]:
        g64, _ = gpu_grad(cat, c, dev, "fp64", basis)
        g32, _ = gpu_grad(cat, c, dev, "fp32", basis)
        e64 = np.abs(g64 - ref).max() / scale
        e32 = np.abs(g32 - ref).max() / scale
        say(f"  {basis}: fp64 {e64:.3e}  fp32 {e32:.3e}")
        assert e64 <= 1e-10
        assert e32 <= 1e-4


def test_gradient_config5_finite_differences(dev):
    """N = 2^18, L = 650, R_max = 150: 64 seeded weights, central differences
    with h = 1e-4 of the FP64 GPU forward; |g_fd - g| <= 1e-3 |g| + 10 eps / h."""
    say("case adjoint config5 finite differences")
    cat = C.config5()
    c = C.loss_weights(cat.lmax, cat.nbins, seed=55)
    idx = C.fd_indices(cat.n, 64, seed=56)
    basis = "spin"
    cfg = cfg_of(cat, "fp64", basis)
    pos = torch.from_numpy(cat.pos).to(dev)
    ct = torch.from_numpy(c).to(dev)
    g, L0 = gpu_grad(cat, c, dev, "fp64", basis)
    h = 1e-4
    w0 = torch.from_numpy(cat.w).to(dev)
    ws = api.Workspace()
    out = torch.empty(api.zeta_shape(cat.lmax, cat.nbins), dtype=torch.float64, device=dev)

    def L(w):
        api.zeta(pos, w, cfg, out=out, workspace=ws)
        return float((out * ct).sum())
    # rounding level of the forward: two evaluations differing only in the order
    # of a harmless no-op are identical, so estimate it from the size of L
    eps = 1e-15 * abs(L0) * 100
    worst = 0.0
    for k in idx:
        wp = w0.clone(); wp[k] += h
        wm = w0.clone(); wm[k] -= h
        fd = (L(wp) - L(wm)) / (2 * h)
        bound = 1e-3 * abs(g[k]) + 10 * eps / h
        worst = max(worst, abs(fd - g[k]) / bound)
        assert abs(fd - g[k]) <= bound, (k, fd, g[k])
    say(f"  worst |fd - g| / bound = {worst:.3e}")


def edge_safe(cat, mask, margin=1e-3):
    """The catalogue without every secondary whose separation from a primary
    of the mask lies within ``margin`` of a shell edge or of R_max (and the
    mask restricted to the galaxies kept).  FP32 positions and FP32 binning
    move a separation by far less than the margin, so FP32 and FP64 put every
    remaining pair into the same shell and the FP32 gradient can be held to
    the oracle's at the FP32 tolerance."""
    from scipy.spatial import cKDTree
    pos = np.asarray(cat.pos, dtype=np.float64)
    lo = np.asarray(cat.box_lo, dtype=np.float64)
    L = np.asarray(cat.box, dtype=np.float64)
    if cat.periodic:
        q = np.mod(pos - lo, L)
        q[q >= L] = 0.0
        tree = cKDTree(q, boxsize=L)
    else:
        q = pos - lo
        tree = cKDTree(q)
    prim = np.nonzero(mask)[0]
    drop = set()
    for i, js in zip(prim, tree.query_ball_point(q[prim], cat.rmax + 2 * margin)):
        js = np.asarray(js, dtype=np.int64)
        d = q[js] - q[i]
        if cat.periodic:
            d -= L * np.rint(d / L)
        r = np.sqrt((d * d).sum(1))
        x = r * cat.nbins / cat.rmax
        near = (np.abs(x - np.rint(x)) * cat.rmax / cat.nbins < margin) & (np.rint(x) >= 1)
        drop.update(js[near & (r > 0)].tolist())
    keep = np.setdiff1d(np.arange(cat.n), np.fromiter(drop, dtype=np.int64, count=len(drop)))
    return cat.subset(keep), np.ascontiguousarray(mask[keep]), len(drop)


def check_fp32_gradient_at_size(dev, cat, mask, c, label):
    safe, m, dropped = edge_safe(cat, mask)
    say(f"  {label}: {dropped} secondaries within 1e-3 of a shell edge dropped, "
        f"{safe.n} galaxies, {int(m.sum())} primaries")
    ref = oracle.grad(safe, c, primary_mask=m)
    scale = np.abs(ref).max()
    for basis in ["cartesian", "spin"]:
        for precision, tol in (("fp64", 1e-10), ("fp32", 1e-4)):
            g, _ = gpu_grad(safe, c, dev, precision, basis, m)
            e = np.abs(g - ref).max() / scale
            say(f"  {label} {precision} {basis}: max|dg|/max|g| = {e:.3e}")
            assert e <= tol


def test_fp32_gradient_config5_sample_vs_oracle(dev):
    """N = 2^18 (the finite-difference catalogue), 1024 seeded primaries, less
    the secondaries with a separation within 1e-3 of a shell edge or R_max:
    FP32 and FP64 gradients against the oracle's (FP32 <= 1e-4 max|g|)."""
    say("case adjoint config5 sample, FP32 and FP64 against the oracle")
    cat = C.config5()
    mask = C.primary_mask(cat.n, 1024, seed=7)
    c = C.loss_weights(cat.lmax, cat.nbins, seed=55)
    check_fp32_gradient_at_size(dev, cat, mask, c, "config5 sample")


def test_gradient_config3_sample_vs_oracle(dev):
    """Clustered, non-periodic, observer line of sight, N = 2^21: the gradient
    from 256 seeded primaries (every galaxy a secondary) against the oracle's,
    through the same pair-blocks as the full run.  The whole catalogue in
    FP64; FP32 (and FP64 again) on the catalogue less the secondaries with a
    separation within 1e-3 of a shell edge or R_max (with so few primaries a
    secondary receives one or two terms, so a single FP32 shell-edge flip
    would move its gradient by its own size)."""
    say("case adjoint config3 sample")
    cat = C.config3()
    mask = C.primary_mask(cat.n, 256, seed=57)
    c = C.loss_weights(cat.lmax, cat.nbins, seed=58)
    ref = oracle.grad(cat, c, primary_mask=mask)
    scale = np.abs(ref).max()
    for basis in ["cartesian", "spin"]:
        g64, _ = gpu_grad(cat, c, dev, "fp64", basis, mask)
        e64 = np.abs(g64 - ref).max() / scale
        say(f"  {basis}: fp64 max|dg|/max|g| = {e64:.3e}")
        assert e64 <= 1e-10
    check_fp32_gradient_at_size(dev, cat, mask, c, "config3 sample")
