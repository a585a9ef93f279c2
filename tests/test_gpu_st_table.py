"""The Int3.4 kernel with the compact space-time offset table (the Eq. 1
structure H = [I_r (x) H0 | D (x) I_m0] turned into per-check arithmetic on a
table of the base code) against the oracle and the per-check table: bit for bit,
with the table in LDS (LBP_INT8_TABLE=1) and in global memory (=2)."""
import os
import sys

import numpy as np
import pytest

import oracle
from tests.gpu_util import batch, gpu_decode, oracle_params

pytestmark = pytest.mark.gpu

CASES = [
    ("bb144_phen", 0.004, 3000, 1401, dict(max_iter=200, msg=2, lottery=True, osd=2, osd_order=10, seed=41)),
    ("surface11_phen", 0.01, 1500, 1402, dict(max_iter=100, msg=2, lottery=True, osd=1, seed=42, flip=1)),
    ("surface9_phen", 0.006, 2000, 1403, dict(max_iter=100, msg=2, lottery=True, osd=1, seed=43)),
]


@pytest.mark.parametrize("table", [1, 2])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_compact_table_bit_exact(case, table, monkeypatch):
    from paper_2605_00038_amd import DecoderParams
    name, p, shots, seed, kw = case
    h, e, syn = batch(name, p, shots, seed)
    prm = DecoderParams(**kw)
    ref = gpu_decode(h, p, prm, syn, first_shot_id=3, want_llr=True)
    monkeypatch.setenv("LBP_INT8_TABLE", str(table))
    g = gpu_decode(h, p, prm, syn, first_shot_id=3, want_llr=True)
    for k in ("corr", "flags", "iters", "llr"):
        assert np.array_equal(g[k], ref[k]), k
    o = oracle.decode(h, p, oracle_params(prm), syn, first_shot_id=3, n_threads=8)
    assert np.array_equal(g["corr"], o["corr"]) and np.array_equal(g["flags"], o["flags"])
    assert np.array_equal(g["iters"], o["iters"])
    print(f"{name} table {table}: {shots} shots bit-exact", file=sys.stderr, flush=True)
