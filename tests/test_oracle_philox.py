"""Pins for the oracle's uniform integers J (Section 3 notation; reading R1).

* External reference: rocRAND's header-only Philox4x32-10 engine compiled for the
  host here and run on a grid of counters and keys.  rocRAND's engine with
  (seed, subsequence, offset = 4 b) yields the block for counter
  (b mod 2^32, b div 2^32, subsequence mod 2^32, subsequence div 2^32) and key
  (seed mod 2^32, seed div 2^32).
* Statistical: chi-square of top-q-bit histograms and per-bit balance.
* Layout: the cached per-step words equal direct stream lookups; packed field 0
  is the top q bits of the unpacked word.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

from oracle import philox

SRC = r'''
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>
int main(){
  unsigned long long seed, sub, off;
  while (scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    uint4 r = e.next4();
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
}
'''


@pytest.fixture(scope="module")
def rocrand_exe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("rocRAND headers / hipcc absent: Philox parity unpinned against an external reference")
    d = tempfile.mkdtemp(prefix="rr_philox_")
    src, exe = os.path.join(d, "x.cpp"), os.path.join(d, "x")
    with open(src, "w") as f:
        f.write(SRC)
    subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-O1", src, "-o", exe],
                   check=True, capture_output=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(rocrand_exe):
    rng = np.random.default_rng(7)
    cases = [(0, 0, 0, 0, 0, 0), (2**32 - 1,) * 6, (1, 2, 3, 4, 5, 6)]
    for _ in range(300):
        cases.append(tuple(int(v) for v in rng.integers(0, 2**32, size=6, dtype=np.uint64)))
    lines = []
    for c0, c1, c2, c3, k0, k1 in cases:
        seed = k0 | (k1 << 32)
        sub = c2 | (c3 << 32)
        off = 4 * (c0 | (c1 << 32))
        lines.append(f"{seed} {sub} {off % 2**64}")
    # offsets of 4 b overflow 64 bits when c1 >= 2^30: keep b < 2^62
    out = subprocess.run([rocrand_exe], input="\n".join(lines), capture_output=True,
                         text=True, check=True).stdout.split("\n")
    for (c0, c1, c2, c3, k0, k1), line in zip(cases, out):
        if c1 >= 2**30:
            continue
        ref = tuple(int(v) for v in line.split())
        got = tuple(int(v) for v in philox.philox4x32_10(c0, c1, c2, c3, k0, k1))
        assert got == ref, (c0, c1, c2, c3, k0, k1)


def test_philox_vectorised_equals_scalar():
    rng = np.random.default_rng(3)
    c = rng.integers(0, 2**32, size=(4, 64), dtype=np.uint64)
    out = philox.philox4x32_10(c[0], c[1], c[2], c[3], 11, 22)
    for i in range(64):
        s = philox.philox4x32_10(int(c[0, i]), int(c[1, i]), int(c[2, i]), int(c[3, i]), 11, 22)
        assert tuple(int(o[i]) for o in out) == tuple(int(v) for v in s)


@pytest.mark.parametrize("q", [4, 6, 8])
def test_top_bits_uniform_chi2(q):
    w = philox.stream_words(1234, 0, 3, 1, np.arange(200_000, dtype=np.uint64))
    k = (w.astype(np.int64) >> (32 - q))
    hist = np.bincount(k, minlength=1 << q)
    p = stats.chisquare(hist).pvalue
    assert 1e-4 < p, p


def test_bit_balance():
    w = philox.stream_words(99, 5, 0, 0, np.arange(100_000, dtype=np.uint64)).astype(np.int64)
    for bit in range(32):
        frac = ((w >> bit) & 1).mean()
        assert abs(frac - 0.5) < 5 * 0.5 / np.sqrt(w.size), bit


@pytest.mark.parametrize("level", [0, 1, 2, 5])
def test_step_words_follow_layout(level):
    paths = np.array([0, 1, 2, 7, 1000, 2**31 + 5], dtype=np.uint64)
    sw = philox.StepWords(1234, 3, level, 2, paths)
    for n in range(1 << level):
        g = paths * np.uint64(1 << level) + np.uint64(n)
        direct = philox.stream_words(1234, 3, level, 2, g)
        assert np.array_equal(sw.word(n), direct)


def test_stream_ids_distinct():
    g = np.arange(4096, dtype=np.uint64)
    a = philox.stream_words(1, 0, 3, 1, g)
    b = philox.stream_words(1, 0, 3, 2, g)
    c = philox.stream_words(1, 0, 4, 1, g)
    d = philox.stream_words(1, 1, 3, 1, g)
    e = philox.stream_words(2, 0, 3, 1, g)
    for x in (b, c, d, e):
        assert (a == x).mean() < 0.01


@pytest.mark.parametrize("q", [4, 6, 8])
def test_packed_field0_is_top_bits(q):
    F = 32 // q
    level = 3
    paths = np.arange(64, dtype=np.uint64)
    sw = philox.StepWords(77, 0, level, 1, paths)
    for n in range(1 << level):
        idx = sw.packed_index(n, q)
        g = paths * np.uint64(1 << level) + np.uint64(n)
        field0 = (g % np.uint64(F)) == 0
        J = philox.stream_words(77, 0, level, 1, g // np.uint64(F)).astype(np.int64)
        assert np.array_equal(idx[field0], (J >> (32 - q))[field0])
        assert idx.min() >= 0 and idx.max() < (1 << q)
