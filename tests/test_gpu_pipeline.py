"""Pipelined decode of large batches (BP of one chunk on the caller's stream while
OSD of the previous chunk runs on a side stream): every output is identical to
the one-pass decode, for consecutive and keyed shot ids, and for chunk counts
that leave a short last chunk.  Large OSD-heavy batches of BB[[144,12,12]]
phenomenological noise at p = 0.006 put a few thousand shots through OSD-CS."""
import os
import sys

import numpy as np
import pytest

from tests.gpu_util import batch

pytestmark = pytest.mark.gpu

SHOTS = 150_001  # above the 2^17-shot threshold; 3 and 7 chunks leave a short last one


def _decode(dec, torch, s, chunks, keys=None):
    old = os.environ.get("LBP_PIPELINE_CHUNKS")
    os.environ["LBP_PIPELINE_CHUNKS"] = str(chunks)
    try:
        if keys is None:
            corr, flags, iters, _ = dec.decode(s, first_shot_id=77)
        else:
            corr, flags, iters = dec.decode_keyed(s, keys)
        torch.cuda.synchronize()
    finally:
        if old is None:
            del os.environ["LBP_PIPELINE_CHUNKS"]
        else:
            os.environ["LBP_PIPELINE_CHUNKS"] = old
    return corr.cpu().numpy(), flags.cpu().numpy(), iters.cpu().numpy()


@pytest.mark.parametrize("msg", [2, 1], ids=["int8", "fp16"])
def test_pipelined_decode_equals_one_pass(msg):
    import torch
    from paper_2605_00038_amd import Code, Decoder, DecoderParams
    h, _, syn = batch("bb144_phen", 0.006, SHOTS, 1501)
    prm = DecoderParams(max_iter=200, msg=msg, lottery=True, lottery_skip=6, osd=2, osd_order=10, seed=2501)
    dec = Decoder(Code.from_scipy(h, 0.006), prm, SHOTS)
    s = torch.from_numpy(np.ascontiguousarray(syn).view(np.int32)).cuda()
    ref = _decode(dec, torch, s, 1)
    n_osd = int(((ref[1] & 2) != 0).sum())
    assert n_osd > 1000
    for k in (2, 3, 7):
        got = _decode(dec, torch, s, k)
        print(f"msg={msg} chunks={k}: {n_osd} OSD shots", file=sys.stderr, flush=True)
        for a, b in zip(ref, got):
            np.testing.assert_array_equal(a, b)
    # keyed shot ids: (seed, id) pairs, chunk offsets must follow the pairs
    rng = np.random.default_rng(9)
    keys = np.stack([np.full(SHOTS, 2501, np.uint64), rng.integers(0, 1 << 40, SHOTS, dtype=np.uint64)], axis=1)
    kt = torch.from_numpy(keys.view(np.int64)).cuda()
    ref_k = _decode(dec, torch, s, 1, kt)
    got_k = _decode(dec, torch, s, 3, kt)
    for a, b in zip(ref_k, got_k):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("cap", [None, 300], ids=["staging", "overflow"])
def test_osd_alongside_bp_equals_osd_after_bp(cap):
    """An OSD grid takes failures while BP runs (the Int3.4 kernel; the default,
    LBP_EARLY_OSD=0 turns it off) and the launch after BP takes the rest; every
    output equals the decoder that runs OSD after BP only, also when more shots
    fail than the staging holds (the overflow passes run the same way)."""
    import torch
    from paper_2605_00038_amd import Code, Decoder, DecoderParams
    h, _, syn = batch("bb144_phen", 0.006, SHOTS, 1502)
    prm = DecoderParams(max_iter=200, msg=2, lottery=True, lottery_skip=6, osd=2, osd_order=10, seed=2502)
    s = torch.from_numpy(np.ascontiguousarray(syn).view(np.int32)).cuda()
    outs = []
    for early in (0, 1):
        old = os.environ.get("LBP_EARLY_OSD")
        os.environ["LBP_EARLY_OSD"] = str(early)
        try:
            dec = Decoder(Code.from_scipy(h, 0.006), prm, SHOTS)
        finally:
            if old is None:
                del os.environ["LBP_EARLY_OSD"]
            else:
                os.environ["LBP_EARLY_OSD"] = old
        if cap is not None:
            dec.set_osd_capacity(cap)
        runs = []
        for rep in range(2):
            corr, flags, iters, _ = dec.decode(s, first_shot_id=5)
            torch.cuda.synchronize()
            runs.append((corr.cpu().numpy(), flags.cpu().numpy(), iters.cpu().numpy()))
        outs.append(runs)
        del dec
    n_osd = int(((outs[0][0][1] & 2) != 0).sum())
    print(f"cap={cap}: {n_osd} OSD shots", file=sys.stderr, flush=True)
    assert n_osd > 1000
    for r in range(2):
        for a, b in zip(outs[0][0], outs[1][r]):
            np.testing.assert_array_equal(a, b)
