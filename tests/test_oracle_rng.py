"""Pins of the oracle's Philox4x32-10 stream and the draws taken from it.

Known-answer vectors published with Random123 (Salmon et al., SC'11), a
cross-check against the open-source rocRAND Philox engine header compiled for
the host, and uniformity of the partner index and of u.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def kat_rows():
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            yield v[0:4], v[4:6], v[6:10]


def test_known_answer_vectors(oracle):
    n = 0
    for ctr, key, out in kat_rows():
        assert list(oracle.philox(ctr, key)) == out
        n += 1
    assert n == 3


ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
    unsigned int c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned int a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_matches_rocrand_engine(oracle, tmp_path):
    src = tmp_path / "probe.cpp"
    exe = tmp_path / "probe"
    src.write_text(ROCRAND_PROBE)
    subprocess.run(["hipcc", "-O1", "-o", str(exe), str(src)], check=True, capture_output=True)
    g = np.random.default_rng(5)
    rows = g.integers(0, 2**32, size=(200, 6), dtype=np.uint64)
    rows[:, 1] %= 2**30  # keep 4*(c0 | c1 << 32) inside 64 bits
    inp = "\n".join(" ".join(str(int(x)) for x in r) for r in rows) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
    got = np.array([[int(x) for x in line.split()] for line in out.strip().splitlines()])
    for r, ref in zip(rows, got):
        mine = oracle.philox(r[:4], r[4:6])
        assert list(mine) == list(ref)


def test_partner_and_u_are_uniform(oracle):
    """k = floor(w0 * Z1 / 2^32) uniform over the Z1 directions and u uniform
    in [0, 1), over the counters a sweep actually uses."""
    Z1 = 8
    n = 20000
    ks = np.empty(n, np.int64)
    us = np.empty(n)
    for a in range(n):
        w = oracle.philox([a, 0, 7, 0], [0, 0])
        ks[a] = (int(w[0]) * Z1) >> 32
        us[a] = ((int(w[1]) << 21) | (int(w[2]) >> 11)) * 2.0**-53
    counts = np.bincount(ks, minlength=Z1)
    assert stats.chisquare(counts).pvalue > 1e-4
    assert stats.kstest(us, "uniform").pvalue > 1e-4
    assert us.min() >= 0.0 and us.max() < 1.0
