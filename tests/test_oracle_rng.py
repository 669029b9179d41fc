"""Pins of the oracle's counter-based random numbers (Philox4x32-10)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answer_vectors():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert oracle.philox(v[0:4], v[4:6]) == v[6:10]


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand(tmp_path):
    exe = tmp_path / "philox_rocrand"
    subprocess.run(["hipcc", "-O1", "-o", str(exe), os.path.join(HERE, "golden", "philox_rocrand.cpp")],
                   check=True, capture_output=True)
    rng = np.random.default_rng(11)
    cases = [(int(rng.integers(0, 2 ** 63)), int(rng.integers(0, 2 ** 40)), int(rng.integers(0, 1000)), int(k))
             for k in (0, 1) for _ in range(8)]
    args = [str(v) for c in cases for v in c]
    out = subprocess.run([str(exe)] + args, check=True, capture_output=True, text=True).stdout.split("\n")
    for (seed, pid, e, k), line in zip(cases, out):
        ref = [int(x) for x in line.split()]
        mine = oracle.philox([pid & 0xFFFFFFFF, pid >> 32, e, k], [seed & 0xFFFFFFFF, seed >> 32])
        assert mine == ref


def test_u24_map_endpoints_and_exactness():
    assert oracle.u24(0) == 2.0 ** -24
    assert oracle.u24(0xFFFFFFFF) == 1.0
    assert oracle.u24(0x000000FF) == 2.0 ** -24          # low 8 bits dropped
    assert oracle.u24(0x80000000) == 0.5 + 2.0 ** -24
    for w in (1, 12345678, 0xDEADBEEF):
        u = oracle.u24(w)
        assert np.float32(u) == u                          # exact in FP32


def test_uniform_chi2():
    words = []
    for p in range(4000):
        words += oracle.philox([p, 0, 0, 0], [7, 0])
    u = np.array([oracle.u24(w) for w in words])
    h, _ = np.histogram(u, bins=32, range=(0, 1))
    e = u.size / 32
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 < 70      # 31 dof; p ~ 1e-4
    assert 0.0 < u.min() and u.max() <= 1.0
