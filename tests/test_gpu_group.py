"""Workgroup-per-shot BP (the GRP variant of bp_kernel) against the wave-per-shot
kernel and the oracle.

Large codes choose it by themselves (surface d >= 21, covered by the
large-code parity tests); LBP_BP_GROUP=g at decoder creation forces groups of
g waves on small codes, so the variant is checked here in every format,
lottery rule and flip mode, in batch decoding and in the serving loop.
Bars: bit for bit equal to the wave-per-shot decode (corrections, flags,
iterations, lambda); Int3.4 also bit-exact against the oracle.
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
    # name, p, shots, data seed, group, params (m > 1024 keeps Int3.4 on the general kernel)
    ("surface13_phen", 0.006, 300, 1501, 4, dict(msg=2, max_iter=100, lottery=True, osd=2, osd_order=10, seed=3)),
    ("surface13_phen", 0.008, 300, 1502, 16, dict(msg=2, max_iter=60, lottery=True, lottery_rule=0x31, osd=1,
                                                  seed=4, flip=1)),
    ("surface13_phen", 0.008, 200, 1503, 2, dict(msg=2, max_iter=60, lottery=True, lottery_rule=0x21, osd=0, seed=5)),
    ("surface11_phen", 0.01, 400, 1504, 8, dict(msg=0, max_iter=100, lottery=True, osd=1, seed=6)),
    ("bb144_phen", 0.004, 400, 1505, 4, dict(msg=1, max_iter=100, lottery=True, lottery_rule=0x11, osd=2, seed=7)),
    ("surface5_cc", 0.05, 500, 1506, 2, dict(msg=0, max_iter=50, scale_mode=1, scale=0.625, lottery=True, osd=1,
                                             seed=8)),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-g{c[4]}-{i}" for i, c in enumerate(CASES)])
def test_group_matches_wave_and_oracle(case, monkeypatch):
    name, p, shots, seed, group, kw = case
    _say("group", group, name, p, shots, kw)
    h, e, syn = batch(name, p, shots, seed)
    prm = _params(**kw)
    monkeypatch.delenv("LBP_BP_GROUP", raising=False)
    wave = gpu_decode(h, p, prm, syn, first_shot_id=11, want_llr=True)
    monkeypatch.setenv("LBP_BP_GROUP", str(group))
    grp = gpu_decode(h, p, prm, syn, first_shot_id=11, want_llr=True)
    monkeypatch.delenv("LBP_BP_GROUP")
    for k in ("corr", "flags", "iters", "llr"):
        assert (grp[k] == wave[k]).all(), k
    if prm.msg == 2:
        o = oracle.decode(h, p, oracle_params(prm), syn, first_shot_id=11, want_llr=True, n_threads=8)
        for k in ("corr", "flags", "iters", "llr"):
            assert (grp[k] == o[k]).all(), k


def test_group_ragged_batches(monkeypatch):
    """Batches smaller than, equal to and larger than the grid's shot slots."""
    import torch
    from paper_2605_00038_amd import Code, Decoder
    h, e, syn = batch("surface13_phen", 0.006, 1500, 1507)
    prm = _params(msg=2, max_iter=100, lottery=True, osd=1, seed=9)
    monkeypatch.setenv("LBP_BP_GROUP", "16")
    dec = Decoder(Code.from_scipy(h, 0.006), prm, 1500)
    monkeypatch.delenv("LBP_BP_GROUP")
    s = torch.from_numpy(syn.view(np.int32)).cuda()
    full = [t.cpu().numpy() for t in dec.decode(s, first_shot_id=0)[:3]]
    for lo, hi in ((0, 1), (5, 6), (100, 357), (0, 1500)):
        part = [t.cpu().numpy() for t in dec.decode(s[lo:hi].contiguous(), first_shot_id=lo)[:3]]
        for a, b in zip(full, part):
            assert (a[lo:hi] == b).all()
    o = oracle.decode(h, 0.006, oracle_params(prm), syn[:200], n_threads=8)
    assert (full[0].view(np.uint32)[:200] == o["corr"]).all()


def test_group_serving_equals_lone_decodes(monkeypatch):
    from paper_2605_00038_amd import Code, Server
    rng = np.random.default_rng(8)
    h, e, syn = batch("surface13_phen", 0.006, 2000, 1508)
    kw = dict(msg=2, max_iter=100, lottery=True, osd=1)
    srv = Server(max_slots=2)
    monkeypatch.setenv("LBP_BP_GROUP", "4")
    slot = srv.add_code(Code.from_scipy(h, 0.006), _params(**kw))
    monkeypatch.delenv("LBP_BP_GROUP")
    reqs = []
    for _ in range(120):
        size = int(rng.integers(1, 30))
        lo = int(rng.integers(0, syn.shape[0] - size + 1))
        seed = int(rng.integers(0, 1 << 62))
        first = int(rng.integers(0, 1 << 40))
        reqs.append((srv.submit(slot, syn[lo:lo + size], seed, first), lo, size, seed, first))
    for t, lo, size, seed, first in reqs:
        r = srv.wait(t, slot, size, timeout_us=60_000_000)
        assert r is not None, "request did not complete"
        corr, flags, iters = r
        ref = gpu_decode(h, 0.006, _params(**kw, seed=seed), syn[lo:lo + size], first_shot_id=first)
        assert np.array_equal(corr, ref["corr"]) and np.array_equal(flags, ref["flags"])
        assert np.array_equal(iters, ref["iters"])
    srv.close()
