"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle is rebuilt with -fsanitize=address,undefined and run in a child
process with the ASan runtime preloaded on small cases of every code path
(both lines of sight, periodic and open boxes, a mask, distinct secondaries,
the gradient, non-finite positions).  Any memory error or undefined behaviour
aborts the child; its results must also equal those of the ordinary build.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
import numpy as np
sys.path.insert(0, ROOT)
import oracle
from paper_1709_00086_amd import catalogues as C
out = {}
for k, case in enumerate(CASES):
    cat = C.tiny(**case)
    if k == 1:
        cat.pos[2, 0] = np.nan
    mask = (np.arange(cat.n) % 3 != 0).astype(np.uint8)
    z, pairs = oracle.zeta(cat, nthreads=2, return_pairs=True)
    zd = oracle.zeta(cat, primary_mask=mask, nthreads=3, distinct=True)
    c = np.random.default_rng(k).standard_normal(zd.shape)
    g = oracle.grad(cat, c, primary_mask=mask, nthreads=2)
    out[str(k)] = [float(np.abs(z).sum()), int(pairs), float(np.abs(zd).sum()),
                   float(np.abs(g).sum())]
print("RESULT " + json.dumps(out))
"""

CASES = [
    dict(n=40, L=100.0, seed=11, rmax=50.0, nbins=4, lmax=10, periodic=True, los="z"),
    dict(n=40, L=100.0, seed=12, rmax=45.0, nbins=5, lmax=6, periodic=False, los="z"),
    dict(n=40, L=100.0, seed=13, rmax=50.0, nbins=3, lmax=8, periodic=False, los="observer",
         observer=(-250.0, -120.0, -60.0)),
    dict(n=30, L=80.0, seed=14, rmax=40.0, nbins=4, lmax=5, periodic=True, los="observer",
         observer=(300.0, 200.0, 500.0)),
]


def _run(env_extra):
    code = f"ROOT = {ROOT!r}\nCASES = {CASES!r}\n" + CHILD
    env = dict(os.environ, **env_extra)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("RESULT ")][-1]
    return json.loads(line[len("RESULT "):])


def test_oracle_clean_under_asan_and_ubsan():
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no AddressSanitizer runtime")
    oracle.build(force=True, sanitize=True)
    san = _run({"G3PCF_ORACLE_SANITIZED": "1", "LD_PRELOAD": asan,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    plain = _run({"G3PCF_ORACLE_SANITIZED": "0"})
    assert san.keys() == plain.keys()
    for k in san:
        assert np.allclose(san[k], plain[k], rtol=1e-12, atol=0.0), (k, san[k], plain[k])
