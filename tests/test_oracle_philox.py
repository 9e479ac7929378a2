"""Pins for the oracle's counter-based generator (Philox4x32-10).

* known-answer vectors published with the generator's reference
  implementation (tests/golden/philox4x32_10_kat.txt);
* rocRAND's own Philox4x32-10 engine, run on the host, for the counter
  layout the method uses: (step, instance, 0, 0);
* the toy oracle's separate Python implementation;
* uniformity of the 53-bit uniforms (Kolmogorov-Smirnov).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import tiny

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                w = [int(v, 16) for v in line.split()]
                rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,want", _kat())
def test_c_oracle_known_answers(oracle_lib, ctr, key, want):
    assert list(oracle.philox4x32_10(ctr, key)) == want


@pytest.mark.parametrize("ctr,key,want", _kat())
def test_python_philox_known_answers(ctr, key, want):
    assert list(tiny.philox4x32_10(ctr, key)) == want


def _cases():
    rng = np.random.default_rng(12345)
    cases = [(0, 0, 0), (0, 1, 0), (0, 4095, 0), (0, 7, 511), (1, 0, 0), (2**64 - 1, 3, 17)]
    for _ in range(40):
        cases.append((int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2)),
                      int(rng.integers(0, 1 << 20)), int(rng.integers(0, 1 << 16))))
    return cases


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available to build the rocRAND driver")
def test_against_rocrand_engine(oracle_lib, tmp_path):
    exe = tmp_path / "rocrand_philox_ref"
    subprocess.run(["hipcc", "-O1", "-o", str(exe), os.path.join(HERE, "helpers", "rocrand_philox_ref.cpp")],
                   check=True, capture_output=True)
    cases = _cases()
    inp = "".join(f"{s} {m} {i}\n" for s, m, i in cases)
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for (s, m, i), line in zip(cases, out):
        want = [int(v, 16) for v in line.split()]
        got = oracle.philox4x32_10((m, i, 0, 0), (s & 0xFFFFFFFF, s >> 32))
        assert list(got) == want, (s, m, i)


def test_c_and_python_agree_and_u53():
    for s, m, i in _cases():
        a = oracle.philox4x32_10((m, i, 0, 0), (s & 0xFFFFFFFF, s >> 32))
        b = tiny.philox4x32_10((m, i, 0, 0), (s & 0xFFFFFFFF, s >> 32))
        assert list(a) == list(b)
        u = oracle.uniform(s, m, i)
        assert u == tiny.uniform(s, m, i)
        assert 0.0 <= u < 1.0
        # 53 significant bits: u * 2^53 is an integer built from r0>>5 and r1>>6
        assert float(u * 2**53).is_integer()
        assert int(u * 2**53) >> 26 == int(a[0]) >> 5
        assert int(u * 2**53) & ((1 << 26) - 1) == int(a[1]) >> 6


def test_uniformity_ks():
    us = np.array([oracle.uniform(0, m, 0) for m in range(20000)])
    assert stats.kstest(us, "uniform").pvalue > 1e-4
    us2 = np.array([oracle.uniform(7, 3, i) for i in range(20000)])
    assert stats.kstest(us2, "uniform").pvalue > 1e-4
