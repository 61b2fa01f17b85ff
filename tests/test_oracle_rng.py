"""Pins of the oracle's counter-based Gaussian noise (Philox4x32-10 + Box-Muller)."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    """Published Philox4x32-10 known-answer vectors (Salmon et al., SC'11)."""
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert oracle.philox4x32_10(ctr, key) == want


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_on_host(tmp_path):
    """rocRAND's independent philox4x32_10 engine, run on the host, evaluates
    the block at counter (0, 0, subsequence lo, hi) with key (seed lo, hi)."""
    exe = tmp_path / "rr"
    src = os.path.join(HERE, "golden", "rocrand_philox_host.cpp")
    subprocess.run(["hipcc", "-O1", "-x", "hip", "--offload-arch=gfx950", src, "-o", str(exe)],
                   check=True, capture_output=True, timeout=600)
    rng = np.random.default_rng(7)
    cases = [(0, 0), (0xFFFFFFFFFFFFFFFF, 0xFFFFFFFFFFFFFFFF)]
    cases += [(int(rng.integers(0, 2**63)), int(rng.integers(0, 2**63))) for _ in range(30)]
    inp = "".join(f"{s:x} {q:x}\n" for s, q in cases)
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True,
                         timeout=60).stdout.split("\n")
    for (seed, sub), line in zip(cases, out):
        want = [int(t, 16) for t in line.split()]
        got = oracle.philox4x32_10([0, 0, sub & 0xFFFFFFFF, sub >> 32],
                                   [seed & 0xFFFFFFFF, seed >> 32])
        assert got == want


def _normals(count, key=(0, 0)):
    out = np.empty(2 * count)
    for i in range(count):
        out[2 * i], out[2 * i + 1] = oracle.normal_pair([i, 5, 9, 0], key)
    return out


def test_box_muller_distribution():
    """Box-Muller normals: mean 0, variance 1, Kolmogorov-Smirnov against N(0,1),
    and the cos/sin outputs of one block uncorrelated."""
    z = _normals(200_000)
    n = z.size
    assert abs(z.mean()) < 5.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    a, b = z[0::2], z[1::2]
    assert abs(np.corrcoef(a, b)[0, 1]) < 5.0 / np.sqrt(a.size)
    # fourth moment of N(0,1) is 3
    assert abs((z ** 4).mean() - 3.0) < 5.0 * np.sqrt(96.0 / n)


def test_normals_depend_on_every_counter_word():
    base = oracle.normal_pair([1, 2, 3, 4], [5, 6])
    for w in range(4):
        ctr = [1, 2, 3, 4]
        ctr[w] += 1
        assert oracle.normal_pair(ctr, [5, 6]) != base
    assert oracle.normal_pair([1, 2, 3, 4], [5, 7]) != base
    assert oracle.normal_pair([1, 2, 3, 4], [6, 6]) != base
