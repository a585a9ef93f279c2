"""OSD with G in registers, two rows of G per lane (the default for codes with
<= 1024 checks) against one row per lane and against the oracle.

LBP_OSD_ROWS_PER_LANE=1 at decoder creation selects one row per lane.  The cases
cover every register width (8, 16, 28 and 32 words per row), codes whose second
rows fill only part of the block or none of it, OSD-0 and OSD-CS, and the float
formats.  Bars: bit for bit equal to the one-row decode (corrections, flags,
iterations, lambda); Int3.4 also bit-exact against the oracle.
"""
import sys

import pytest

import oracle
from tests.gpu_util import batch, gpu_decode, oracle_params

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _params(**kw):
    from paper_2605_00038_amd import DecoderParams
    return DecoderParams(**kw)


CASES = [
    # name (m x n), p, shots, data seed, params
    ("surface5_phen", 0.03, 2000, 1601, dict(msg=2, max_iter=30, lottery=True, osd=2, osd_order=10, seed=3)),  # 60
    ("surface7_phenpf", 0.008, 1500, 1602, dict(msg=2, max_iter=60, lottery=True, osd=2, osd_order=10, seed=4)),  # 192
    ("usurface7_phenpf", 0.008, 1500, 1603, dict(msg=2, max_iter=60, lottery=True, osd=1, seed=5)),  # 336
    ("surface9_phen", 0.008, 800, 1604, dict(msg=1, max_iter=60, lottery=True, osd=2, osd_order=10, seed=6)),  # 360
    ("bb144_phen", 0.006, 600, 1605, dict(msg=2, max_iter=60, lottery=True, osd=2, osd_order=10, seed=7)),  # 864
    ("surface11_phen", 0.01, 400, 1606, dict(msg=0, max_iter=60, lottery=True, osd=2, osd_order=10, seed=8)),  # 660
    ("bb144_phenpf", 0.02, 300, 1607, dict(msg=2, max_iter=60, lottery=True, osd=1, seed=9)),  # 936
    ("bb144_phenpf", 0.02, 300, 1608, dict(msg=2, max_iter=60, lottery=True, osd=2, osd_order=10, seed=10)),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{i}" for i, c in enumerate(CASES)])
def test_two_rows_match_one_row_and_oracle(case, monkeypatch):
    name, p, shots, seed, kw = case
    _say("osd rows", name, p, shots, kw)
    h, e, syn = batch(name, p, shots, seed)
    prm = _params(**kw)
    monkeypatch.delenv("LBP_OSD_ROWS_PER_LANE", raising=False)
    two = gpu_decode(h, p, prm, syn, first_shot_id=5, want_llr=True)
    monkeypatch.setenv("LBP_OSD_ROWS_PER_LANE", "1")
    one = gpu_decode(h, p, prm, syn, first_shot_id=5, want_llr=True)
    monkeypatch.delenv("LBP_OSD_ROWS_PER_LANE")
    _say("  OSD shots", int(((two["flags"] & 2) != 0).sum()), "of", shots)
    assert ((two["flags"] & 2) != 0).sum() >= 4
    for k in ("corr", "flags", "iters", "llr"):
        assert (two[k] == one[k]).all(), k
    if prm.msg == 2:
        o = oracle.decode(h, p, oracle_params(prm), syn, first_shot_id=5, want_llr=True, n_threads=8)
        for k in ("corr", "flags", "iters", "llr"):
            assert (two[k] == o[k]).all(), k


def _random_code(m, n, cdeg, seed):
    """Random code with column degree <= cdeg and row degree <= n * cdeg / m
    (configuration model, repeated edges dropped; n * cdeg divisible by m)."""
    import numpy as np
    import scipy.sparse as sps
    rng = np.random.default_rng(seed)
    cols = np.repeat(np.arange(n), cdeg)
    assert len(cols) % m == 0
    rows = rng.permutation(np.repeat(np.arange(m), len(cols) // m))
    h = sps.csr_matrix((np.ones(len(cols), dtype=np.uint8), (rows, cols)), shape=(m, n))
    h.data[:] = 1  # repeated (row, column) pairs were summed: keep one edge
    h.eliminate_zeros()
    return h


@pytest.mark.parametrize("m", [1023, 1024], ids=["m1023-registers", "m1024-lds"])
@pytest.mark.parametrize("osd", [1, 2], ids=["osd0", "osdcs"])
def test_register_kernel_boundary(m, osd):
    """The last size with G in registers (m = 1023: rows 512..1022 in the second
    slot of 511 lanes) and the first with G in LDS, on random codes whose rows
    reach the 8-slot limit; Int3.4 bit-exact against the oracle."""
    from workloads import sample
    h = _random_code(m, 2 * m, 4, 1700 + m)
    assert h.shape == (m, 2 * m) and h.getnnz(axis=1).max() <= 8 and h.getnnz(axis=0).max() <= 4
    p = 0.07
    e, syn = sample.make_batch(h, p, 60, 1710 + m)
    prm = _params(msg=2, max_iter=8, lottery=False, osd=osd, osd_order=10)
    from paper_2605_00038_amd import Code, Decoder
    variant = Decoder(Code.from_scipy(h, p), prm, 60).shape()["osd_variant"]
    _say("osd boundary", m, osd, "variant", variant)
    # the two sides of the boundary run the two kernels: G in registers (two 32-word
    # rows per lane), then G in LDS
    assert variant == (232 if m == 1023 else 0)
    g = gpu_decode(h, p, prm, syn, want_llr=True)
    o = oracle.decode(h, p, oracle_params(prm), syn, want_llr=True, n_threads=8)
    assert ((g["flags"] & 2) != 0).sum() >= 20
    for k in ("corr", "flags", "iters", "llr"):
        assert (g[k] == o[k]).all(), k
