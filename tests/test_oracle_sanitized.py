"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

A child interpreter preloads libasan and loads the instrumented build of the oracle
(oracle.build(sanitize=True), selected by QLA_ORACLE_SANITIZE=1). It runs the fast
oracle pins and a battery of every C entry point on ragged lattices (widths and
heights down to one site, every operator, every potential mode); any sanitizer report
ends the child with a non-zero status. The slow convergence pins are left out here
(about five minutes instrumented); the same child environment runs them too:
    python -c "import oracle; oracle.build(sanitize=True)"
    env $(python -c "import oracle; print(' '.join(f'{k}={v}' for k, v in
        oracle.sanitizer_env({}).items()))") PATH=$PATH python -m pytest tests/test_oracle_pins.py
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

BATTERY = r"""
import numpy as np
import oracle
assert oracle._load()._name.endswith("liboracle_san.so"), oracle._load()._name
rng = np.random.default_rng(1)
for ny, nx in ((1, 1), (1, 9), (3, 5), (8, 9), (17, 4), (5, 33)):
    n = 1.0 + rng.random((ny, nx))
    oracle.coefficients(n, 0.25)
    for vmode in (oracle.V_SKEW_HALF, oracle.V_PAPER, oracle.V_NONE, oracle.V_BSTREAM):
        q = rng.normal(size=(6, ny, nx))
        for op in range(oracle.OP_STEP + 1):
            oracle.apply(op, q, n, 0.25, vmode)
        oracle.advance(q, n, 0.25, 3, vmode)
        assert np.isfinite(oracle.energy(q))
    for planar in (True, False):
        q = oracle.packet(n, nx / 3, ny / 2, 2.0, 4.0, phi=0.3, planar=planar)
        assert np.isfinite(q).all()
print("battery ok")
"""


def _have_asan():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                           text=True, check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return False
    return os.path.isabs(p) and os.path.exists(p)


@pytest.mark.skipif(not _have_asan(), reason="gcc has no AddressSanitizer runtime here")
def test_oracle_is_clean_under_address_and_undefined_behaviour_sanitizers():
    oracle.build(sanitize=True)
    env = oracle.sanitizer_env()
    env["PYTHONPATH"] = ROOT
    r = subprocess.run([sys.executable, "-c", BATTERY], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "battery ok" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]
    for bad in ("ERROR: AddressSanitizer", "runtime error:"):
        assert bad not in r.stderr, r.stderr[-4000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-k", "not converge and not translation and not fresnel"],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    for bad in ("ERROR: AddressSanitizer", "runtime error:"):
        assert bad not in r.stdout + r.stderr
