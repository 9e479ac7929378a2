"""GPU parity of the seed pass in every memory-space combination: the point
rows through cached, non-temporal or buffer-descriptor loads, the current
centre through LDS, scalar loads or per-lane global loads (the memory spaces
the paper compares in Section II and Figs. 2c and 3c).

A row's arithmetic does not depend on where its values come from, so at one
launch schedule every combination must give bit-identical seeds, centres and
D; one of them is checked against the oracle's parity rules as well.
"""
import numpy as np
import pytest
import torch

import kmpp_synth
import oracle
from gpu_util import check_D, check_seed_run, run_seed

pytestmark = pytest.mark.gpu

ROWS = {"cached": 0, "nontemporal": 1, "buffer": 2}
CENTRES = {"lds": 1, "scalar": 2, "global": 3}
# rows per tile: several tiles and a ragged last one at these sizes
CASES = {2: (100_003, 2048), 32: (40_009, 1024), 64: (20_011, 512), 128: (12_007, 256)}


@pytest.fixture(scope="module")
def kl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_02136_amd as k
    k.lib()
    return k


def _say(*a):
    print(*a, flush=True)


def _all_combinations(kl, X, K, seed, rpt):
    out = {}
    for rn, rl in ROWS.items():
        for cn, cs in CENTRES.items():
            _say(f"  rows={rn} centre={cn}")
            idx, C, D, st = run_seed(kl, X, K, seed, threads=256, loads_per_lane=8, rows_per_tile=rpt,
                                     row_loads=rl, centre_source=cs)
            assert st == 0, (rn, cn, st)
            out[(rn, cn)] = (idx, C, D)
    return out


@pytest.mark.parametrize("d", sorted(CASES))
def test_memory_spaces_bit_identical_and_parity(kl, d):
    N, rpt = CASES[d]
    K = 24
    Xh = kmpp_synth.gaussian(N, d, seed=500 + d)
    _say(f"memory spaces N={N} d={d} K={K} rows/tile={rpt}")
    runs = _all_combinations(kl, Xh.cuda(), K, 7, rpt)
    idx0, C0, D0 = runs[("cached", "lds")]
    check_seed_run(Xh.numpy(), K, 7, idx0, C0, D0)
    for key, (idx, C, D) in runs.items():
        np.testing.assert_array_equal(idx, idx0, err_msg=str(key))
        np.testing.assert_array_equal(C, C0, err_msg=str(key))
        np.testing.assert_array_equal(D, D0, err_msg=str(key))


def test_memory_spaces_integer_lattice_exact(kl):
    # integer points: distances and sums exact, so every combination must
    # equal the oracle bit for bit
    N, d, K = 65_537, 2, 30
    Xh = kmpp_synth.lattice(N, d, seed=11)
    _say(f"memory spaces lattice N={N} d={d} K={K}")
    runs = _all_combinations(kl, Xh.cuda(), K, 5, 2048)
    for key, (idx, C, D) in runs.items():
        check_seed_run(Xh.numpy(), K, 5, idx, C, D, exact=True)


def test_memory_spaces_paper_shape(kl):
    # the two-dimensional points of the paper's cluster sweep: N = 4M, K = 100
    w = kmpp_synth.paper_shape("paper_k")
    Xh, N, d, K = w.X, w.N, w.d, w.K
    _say(f"memory spaces paper shape N={N} d={d} K={K}")
    runs = _all_combinations(kl, Xh.cuda(), K, 0, 0)
    idx0, C0, D0 = runs[("cached", "lds")]
    for key, (idx, C, D) in runs.items():
        np.testing.assert_array_equal(idx, idx0, err_msg=str(key))
        np.testing.assert_array_equal(D, D0, err_msg=str(key))
    X = Xh.numpy()
    r = oracle.seed(X, 4, seed=0, replay=idx0[:4])
    assert int(r.idx[0]) == int(idx0[0])
    for m in range(1, 4):
        assert oracle.seed_index_ok(int(idx0[m]), r.rec[m], int(r.idx[m])), m
    rows = np.random.default_rng(3).choice(N, 3000, replace=False)
    _, om, _ = oracle.assign_rows(X, rows, C0)
    check_D(D0[rows], om)


def test_memory_spaces_unsupported(kl):
    X = torch.randn((1000, 33), device="cuda")
    for cs in (2, 3):
        with pytest.raises(kl.KmppError) as e:
            kl.kmpp_seed(X, 4, 0, threads=256, loads_per_lane=8, centre_source=cs)
        assert e.value.code == -5
    with pytest.raises(kl.KmppError) as e:
        kl.kmpp_seed(X, 4, 0, threads=256, loads_per_lane=8, row_loads=2)
    assert e.value.code == -5
    Xb = torch.randn((1000, 32), device="cuda")
    Xq, _ = kl.kmpp_quantize(Xb, kl.KMPP_BF16)
    with pytest.raises(kl.KmppError) as e:
        kl.kmpp_seed(Xb, 4, 0, Xq=Xq, dtype=kl.KMPP_BF16, centre_source=2)
    assert e.value.code == -5
    with pytest.raises(kl.KmppError) as e:
        kl.kmpp_seed(Xb, 4, 0, row_loads=3)
    assert e.value.code == -1
