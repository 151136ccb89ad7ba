"""Pins of the oracle's primitives against values fixed outside the oracle:
published known-answer vectors, an independent library generator (rocRAND),
exact integer arithmetic, and 200-bit mpmath logarithms."""
import os
import shutil
import subprocess

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NATIVE = os.path.join(os.path.dirname(__file__), "native")


def _kat():
    rows = []
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append([int(x, 16) for x in line.split()])
    return rows


def test_philox_known_answers():
    for row in _kat():
        ctr, key, want = row[0:4], row[4:6], row[6:10]
        assert list(O.philox(ctr, key)) == want


@pytest.fixture(scope="module")
def rocrand_exe(tmp_path_factory):
    inc = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not os.path.exists(inc) or shutil.which("g++") is None:
        pytest.skip("rocRAND headers or g++ not available")
    exe = str(tmp_path_factory.mktemp("rocrand") / "rp")
    subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(NATIVE, "rocrand_philox.cpp"), "-o", exe], check=True)
    return exe


def test_philox_matches_rocrand(rocrand_exe):
    rng = np.random.default_rng(7)
    ctrs = rng.integers(0, 2**32, (300, 4), dtype=np.uint64)
    keys = rng.integers(0, 2**32, (300, 2), dtype=np.uint64)
    # the counters the simulation actually uses: small draw index, node, day, stream
    ctrs[:100, 0] = rng.integers(0, 50, 100)
    ctrs[:100, 2] = rng.integers(0, 1461, 100)
    ctrs[:100, 3] = rng.integers(0, 2, 100)
    inp = "\n".join(" ".join(f"{int(x):x}" for x in (*c, *k)) for c, k in zip(ctrs, keys)) + "\n"
    res = subprocess.run([rocrand_exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for c, k, line in zip(ctrs, keys, res):
        assert list(O.philox(c, k)) == [int(x, 16) for x in line.split()]


def test_u53_exact_and_open_interval():
    assert O.u53(0, 0) == 2.0 ** -53
    assert O.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    rng = np.random.default_rng(1)
    for lo, hi in rng.integers(0, 2**32, (2000, 2), dtype=np.uint64):
        x = (int(hi) << 32) | int(lo)
        u = O.u53(int(lo), int(hi))
        assert u == (2 * (x >> 12) + 1) / 2.0 ** 53            # exact in binary64
        assert 0.0 < u < 1.0
        # symmetric lattice: complementing every bit reflects u about 1/2
        assert u + O.u53(0xFFFFFFFF - int(lo), 0xFFFFFFFF - int(hi)) == 1.0


def test_mulhi64_exact():
    rng = np.random.default_rng(2)
    vals = [0, 1, 2**32 - 1, 2**32, 2**63, 2**64 - 1]
    vals += [int(x) for x in rng.integers(0, 2**63, 50, dtype=np.uint64)] + \
            [int(x) | (1 << 63) for x in rng.integers(0, 2**63, 50, dtype=np.uint64)]
    for a in vals:
        for b in vals[::7]:
            assert O.mulhi64(a, b) == (a * b) >> 64


def _ulp(x):
    return np.spacing(abs(x))


def test_neglog_within_two_ulp_of_mpmath():
    mp.mp.prec = 200
    rng = np.random.default_rng(3)
    us = [O.u53(int(a), int(b)) for a, b in rng.integers(0, 2**32, (20000, 2), dtype=np.uint64)]
    # powers of two, the fold point sqrt(2)/2, both ends of the U53 lattice, near 1
    us += [2.0 ** -k for k in range(1, 54)]
    us += [np.nextafter(1 / np.sqrt(2), 0), 1 / np.sqrt(2), np.nextafter(1 / np.sqrt(2), 1)]
    us += [2.0 ** -53, 1 - 2.0 ** -53, 1 - 2.0 ** -40, 0.5 + 2.0 ** -53, 0.75, 0.999]
    worst = 0.0
    for u in us:
        got = O.neglog(u)
        exact = -mp.log(mp.mpf(u))
        err = abs(float((mp.mpf(got) - exact) / mp.mpf(_ulp(float(exact)))))
        worst = max(worst, err)
    assert worst <= 2.0, worst


def test_neglog_exact_cases():
    # m = 1 exactly: the series vanishes and -log(2^-k) = k ln 2 from the split constant
    assert O.neglog(0.5) == float(mp.log(2))
    for k in (1, 2, 10, 53):
        assert abs(O.neglog(2.0 ** -k) - k * float(mp.log(2))) <= 2 * _ulp(k * float(mp.log(2)))


def test_quarter_matches_paper_table():
    for line in open(os.path.join(GOLDEN, "beta_season.txt")):
        if line.strip() and not line.startswith("#"):
            t, q = map(int, line.split())
            assert O.quarter(t) == q, t
