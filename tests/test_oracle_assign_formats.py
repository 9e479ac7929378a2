"""Pins for the oracle's assignment (output O of the paper's Algorithm 1) and
for its storage formats used by the precision forms.

* assignment: FP64 argmin against torch.cdist (a library routine), with
  exact ties on an integer lattice resolved to the smallest centre index;
* BF16: round-to-nearest-even encoding against torch's CPU conversion, on
  random values and on constructed ties, overflow, subnormals and NaN;
* FP8 E4M3FN (OCP): decoding of all 256 codes and encoding against torch's
  float8_e4m3fn conversion; per-row power-of-two exponent rule.
"""
import numpy as np
import torch

import oracle
import kmpp_synth


def test_assign_matches_cdist(oracle_lib):
    X = kmpp_synth.gaussian(3000, 7, seed=1).numpy()
    C = kmpp_synth.gaussian(37, 7, seed=2).numpy()
    lab, mind, sec = oracle.assign(X, C)
    dist = torch.cdist(torch.from_numpy(X).double(), torch.from_numpy(C).double()).square()
    ref = dist.argmin(dim=1).numpy()
    np.testing.assert_array_equal(lab, ref)
    np.testing.assert_allclose(mind, dist.min(dim=1).values.numpy(), rtol=1e-10)
    srt = dist.sort(dim=1).values.numpy()
    np.testing.assert_allclose(sec, srt[:, 1], rtol=1e-10)
    l2, m2, _ = oracle.assign_rows(X, np.arange(0, 3000, 7), C)
    np.testing.assert_array_equal(l2, lab[::7])
    np.testing.assert_array_equal(m2, mind[::7])
    pd = oracle.pair_dist(X, np.arange(0, 3000, 7), C, lab[::7])
    np.testing.assert_array_equal(pd, mind[::7])


def test_assign_ties_go_to_smallest_index(oracle_lib):
    X = np.array([[0, 0], [2, 0], [1, 1]], dtype=np.float32)
    C = np.array([[5, 5], [1, 0], [-1, 0], [1, 0]], dtype=np.float32)
    lab, mind, _ = oracle.assign(X, C)
    # x0 is at distance 1 from centres 1 and 2 (and 3): smallest is 1
    assert list(lab) == [1, 1, 1]
    assert list(mind) == [1.0, 1.0, 1.0]


def _bf16_torch(x):
    return torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)


def test_bf16_encoding_matches_torch(oracle_lib):
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(20000).astype(np.float32) * 10 ** rng.uniform(-30, 30, 20000).astype(np.float32),
        np.array([0.0, -0.0, 1.0, -1.0, 3.4e38, -3.4e38, 1e-40, -1e-42, np.inf, -np.inf], dtype=np.float32),
    ]).astype(np.float32)
    # exact ties: mantissa low half 0x8000 with even and odd kept bit
    ties = (np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x00018000, 0x7F7F8000], dtype=np.uint32)).view(np.float32)
    x = np.concatenate([x, ties])
    got = oracle.bf16_encode(x)
    np.testing.assert_array_equal(got, _bf16_torch(x))
    back = oracle.bf16_decode(got)
    np.testing.assert_array_equal(back, torch.from_numpy(x).to(torch.bfloat16).float().numpy())
    assert np.isnan(oracle.bf16_decode(oracle.bf16_encode(np.array([np.nan], np.float32))))[0]


def test_fp8_decode_all_codes(oracle_lib):
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).double().numpy()
    got = np.array([oracle.fp8_decode(int(c)) for c in codes])
    nan = np.isnan(ref)
    assert np.array_equal(nan, np.isnan(got))
    assert nan.sum() == 2                         # S.1111.111 only
    np.testing.assert_array_equal(got[~nan], ref[~nan])
    assert np.nanmax(got) == 448.0
    assert oracle.fp8_decode(1) == 2.0 ** -9      # smallest subnormal


def test_fp8_encoding_matches_torch(oracle_lib):
    rng = np.random.default_rng(1)
    v = np.concatenate([rng.uniform(-448, 448, 5000), rng.standard_normal(5000) * 0.01,
                        rng.standard_normal(2000) * 1e-3])
    # every midpoint between neighbouring codes is an exact tie
    pos = np.array([oracle.fp8_decode(c) for c in range(127)])
    mids = 0.5 * (pos[:-1] + pos[1:])
    v = np.concatenate([v, mids, -mids, pos, -pos]).astype(np.float32)
    got = np.array([oracle.fp8_encode(float(a)) for a in v], dtype=np.uint8)
    ref = torch.from_numpy(v).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(got, ref)
    # saturation (torch's conversion is not saturating, so pinned by value)
    assert oracle.fp8_encode(1000.0) == 0x7E and oracle.fp8_encode(-500.0) == 0xFE


def test_fp8_row_exponent_rule(oracle_lib):
    rng = np.random.default_rng(2)
    for _ in range(500):
        row = (rng.standard_normal(16) * 10 ** rng.uniform(-8, 8)).astype(np.float32)
        e = oracle.fp8_row_exponent(row)
        amax = float(np.abs(row.astype(np.float64)).max())
        assert amax <= 448.0 * 2.0 ** e
        assert amax > 448.0 * 2.0 ** (e - 1)
    assert oracle.fp8_row_exponent(np.zeros(8, np.float32)) == 0
    assert oracle.fp8_row_exponent(np.array([448.0], np.float32)) == 0
    assert oracle.fp8_row_exponent(np.array([448.5], np.float32)) == 1
    assert oracle.fp8_row_exponent(np.array([224.0], np.float32)) == -1


def test_fp8_row_quantisation_roundtrip(oracle_lib):
    X = kmpp_synth.gaussian(64, 16, seed=3, scale=50.0).numpy()
    q, e = oracle.fp8_quantize_rows(X)
    Xh = oracle.fp8_dequantize_rows(q, e)
    for i in range(64):
        s = 2.0 ** int(e[i])
        ref = torch.from_numpy((X[i].astype(np.float64) / s).astype(np.float32)).to(torch.float8_e4m3fn)
        np.testing.assert_array_equal(q[i], ref.view(torch.uint8).numpy())
        np.testing.assert_array_equal(Xh[i], (ref.double().numpy() * s).astype(np.float32))
    rel = np.abs(Xh - X) / np.abs(X).max(axis=1, keepdims=True)
    assert rel.max() <= 2.0 ** -4 + 1e-12           # half an ulp of a 3-bit mantissa, relative to amax


def test_fp8_bisection_encoder_equals_definition(oracle_lib):
    pos = np.array([oracle.fp8_decode(c) for c in range(127)])
    mids = 0.5 * (pos[:-1] + pos[1:])
    rng = np.random.default_rng(9)
    v = np.concatenate([pos, mids, np.nextafter(mids, 0), np.nextafter(mids, 1000), rng.uniform(0, 500, 20000),
                        rng.standard_normal(5000) * 1e-3, [448.0, 449.0, 1e9, 0.0]])
    v = np.concatenate([v, -v])
    for a in v:
        assert oracle.fp8_encode_bisect(a) == oracle.fp8_encode(a), a
    X = kmpp_synth.gaussian(300, 33, seed=4, scale=30.0).numpy()
    q1, e1 = oracle.fp8_quantize_rows(X)
    q2, e2 = oracle.fp8_quantize_rows_fast(X)
    np.testing.assert_array_equal(q1, q2)
    np.testing.assert_array_equal(e1, e2)
