"""The wide column table (u32 slot positions), which codes with more than 8191
checks need, against the oracle and against the narrow table.

Setting LBP_WIDE_COLUMN_TABLE=1 at code creation gives small codes the same
layout, so every kernel that reads it (general BP kernel in all formats, the
lottery's worst-check and neighbour rules, OSD with G in LDS and in global
memory, the global-memory comparison path) is checked at sizes the oracle
finishes in seconds; the surface d=27 case is the size that needs it.
Bars: Int3.4 bit-exact against the oracle; every format bit-exact against the
same decode with the narrow table (the layout must not change any result).
"""
import sys

import numpy as np
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
    # name, p, shots, data seed, params (m > 1024 keeps Int3.4 on the general kernel)
    ("surface13_phen", 0.006, 300, 1401, dict(msg=2, max_iter=100, lottery=True, osd=2, osd_order=10, seed=3)),
    ("surface13_phen", 0.008, 300, 1402, dict(msg=2, max_iter=60, lottery=True, lottery_rule=0x31, osd=1, seed=4)),
    ("surface13_phen", 0.008, 200, 1403, dict(msg=2, max_iter=60, lottery=True, lottery_rule=0x21, osd=0, seed=5,
                                             flip=1)),
    ("surface17_phen", 0.01, 24, 1010, dict(msg=2, max_iter=3, lottery=False, osd=2, osd_order=6)),
    ("surface11_phen", 0.01, 400, 1404, dict(msg=0, max_iter=100, lottery=True, osd=1, seed=6)),
    ("surface11_phen", 0.01, 400, 1405, dict(msg=1, max_iter=100, lottery=True, lottery_rule=0x11, osd=2, seed=7)),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{i}" for i, c in enumerate(CASES)])
def test_wide_table_matches_narrow_and_oracle(case, monkeypatch):
    name, p, shots, seed, kw = case
    _say("wide table", name, p, shots, kw)
    h, e, syn = batch(name, p, shots, seed)
    prm = _params(**kw)
    monkeypatch.delenv("LBP_WIDE_COLUMN_TABLE", raising=False)
    narrow = gpu_decode(h, p, prm, syn, first_shot_id=9, want_llr=True)
    monkeypatch.setenv("LBP_WIDE_COLUMN_TABLE", "1")
    wide = gpu_decode(h, p, prm, syn, first_shot_id=9, want_llr=True)
    monkeypatch.delenv("LBP_WIDE_COLUMN_TABLE")
    for k in ("corr", "flags", "iters", "llr"):
        assert (wide[k] == narrow[k]).all(), k
    if prm.osd:
        assert (wide["flags"] & 2).any()
    if prm.msg == 2:
        o = oracle.decode(h, p, oracle_params(prm), syn, first_shot_id=9, want_llr=True, n_threads=8)
        for k in ("corr", "flags", "iters", "llr"):
            assert (wide[k] == o[k]).all(), k


@pytest.mark.parametrize("msg", [0, 1], ids=["fp32", "fp16"])
def test_wide_table_comparison_path(msg, monkeypatch):
    import torch
    from paper_2605_00038_amd import Code, Decoder
    h, e, syn = batch("surface11_phen", 0.01, 300, 1406)
    prm = _params(msg=msg, max_iter=100, lottery=True, lottery_rule=0x21, osd=1, seed=8)
    s = torch.from_numpy(np.ascontiguousarray(syn).view(np.int32)).cuda()
    out = []
    for wide in (False, True):
        if wide:
            monkeypatch.setenv("LBP_WIDE_COLUMN_TABLE", "1")
        dec = Decoder(Code.from_scipy(h, 0.01), prm, syn.shape[0])
        monkeypatch.delenv("LBP_WIDE_COLUMN_TABLE", raising=False)
        out.append([t.cpu().numpy() for t in dec.decode_baseline(s, first_shot_id=2)])
        torch.cuda.synchronize()
    for a, b in zip(*out):
        assert (a == b).all()


def test_surface27_final_readout():
    """Surface d=27 over 27 rounds with the final read-out (10192 x 29511): the size
    whose slot positions exceed 16 bits. Int3.4 on the general kernel, OSD-0 with G
    and the per-column arrays in global memory; bit-exact against the oracle."""
    h, e, syn = batch("surface27_phenpf", 0.0015, 40, 1407)
    assert h.shape == (10192, 29511)
    prm = _params(msg=2, max_iter=100, lottery=True, osd=1, seed=10)
    g = gpu_decode(h, 0.0015, prm, syn, want_llr=True)
    o = oracle.decode(h, 0.0015, oracle_params(prm), syn, want_llr=True, n_threads=8)
    _say("  d=27: OSD shots", int(((g["flags"] & 2) != 0).sum()), "of", syn.shape[0])
    assert ((g["flags"] & 2) != 0).sum() >= 8
    for k in ("flags", "iters", "llr", "corr"):
        assert (g[k] == o[k]).all(), k
