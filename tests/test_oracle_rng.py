"""Pins of the oracle's Philox4x32-10 generator and the uniforms built on it.

* known-answer vectors published with the Random123 library (Salmon et al.,
  SC'11), golden file tests/golden/philox4x32_10_kat.txt;
* bitwise agreement with an independent implementation called at test time:
  PyTorch's header-only engine ATen/core/PhiloxRNGEngine.h, compiled here
  into a small driver (key = seed, counter = (offset lo, offset hi,
  subsequence lo, subsequence hi));
* range and uniformity of the derived uniforms.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers(orc):
    rows = _kat()
    assert len(rows) >= 3
    for ctr, key, want in rows:
        got = orc.philox(ctr, key)
        assert [int(x) for x in got] == want


_DRIVER = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cinttypes>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
    uint64_t sub = (uint64_t)c2 | ((uint64_t)c3 << 32);
    uint64_t off = (uint64_t)c0 | ((uint64_t)c1 << 32);
    at::Philox4_32 e(seed, sub, off);
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%08x %08x %08x %08x\n", a, b, c, d);
  }
  return 0;
}
"""


def _torch_include():
    try:
        import torch
    except Exception:
        return None
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    return inc if os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")) else None


def test_philox_matches_torch_engine(orc):
    inc = _torch_include()
    if inc is None or shutil.which("g++") is None:
        pytest.skip("torch headers or g++ not available")
    rng = np.random.default_rng(1234)
    cases = rng.integers(0, 2 ** 32, size=(200, 6), dtype=np.uint64)
    cases[0] = 0
    cases[1] = 2 ** 32 - 1
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "drv.cpp")
        exe = os.path.join(d, "drv")
        open(src, "w").write(_DRIVER)
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", inc, "-o", exe, src])
        inp = "\n".join(" ".join("%x" % int(v) for v in row) for row in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for row, line in zip(cases, out):
        want = [int(x, 16) for x in line.split()]
        got = [int(x) for x in orc.philox(row[:4], row[4:6])]
        assert got == want


def test_uniforms_range_and_uniformity(orc):
    from scipy import stats
    us = np.array([orc.unit_uniform(7, q, 3, 5, orc.ST_HID) for q in range(20000)])
    assert us.min() > 0.0 and us.max() < 1.0
    counts = np.histogram(us, bins=20, range=(0, 1))[0]
    assert stats.chisquare(counts).pvalue > 1e-4
    ms = np.array([orc.mh_uniform(7, t, 11) for t in range(20000)])
    assert ms.min() > 0.0 and ms.max() < 1.0
    counts = np.histogram(ms, bins=20, range=(0, 1))[0]
    assert stats.chisquare(counts).pvalue > 1e-4


def test_unit_uniform_uses_documented_word(orc):
    # unit q of a stream uses word q & 3 of the block with counter (q>>2, t, g, tag)
    seed, t, g, tag = 0x0123456789ABCDEF, 17, 42, orc.ST_VIS | (2 << 8)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for q in (0, 1, 2, 3, 4, 9, 1023):
        w = orc.philox([q >> 2, t, g, tag], key)[q & 3]
        assert orc.unit_uniform(seed, q, t, g, tag) == (float(w) + 0.5) / 2 ** 32


def test_init_state_is_balanced(orc):
    s = orc.init_state(3, 64, 1, 16)
    assert set(np.unique(s)) <= {-1, 1}
    m = s.mean()
    assert abs(m) < 0.03
    # chain offset g0 shifts the chain index only
    s2 = orc.init_state(3, 4, 1, 16, g0=10)
    assert np.array_equal(s2, orc.init_state(3, 14, 1, 16)[10:])
