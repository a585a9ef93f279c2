"""Global-memory comparison path (lbp_decode_baseline) against the oracle.

The comparison path computes in fp32 only: column sums are exact TwoSum pairs
in the oracle's order, each stored message is rounded once to the storage
format, so its corrections, flags and iteration counts should agree with the
oracle on (essentially) every shot; the bar is the float bar of the fused
kernels, identical corrections on >= 99.9% of shots.  It must also agree with
the fused LDS kernel of the same format at that bar.
"""
import sys

import numpy as np
import pytest

import oracle
from tests.gpu_util import batch, gpu_decode, oracle_params

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _baseline(h, p, prm, syn, first_shot_id=0):
    import torch
    from paper_2605_00038_amd import Code, Decoder
    dec = Decoder(Code.from_scipy(h, p), prm, syn.shape[0])
    s = torch.from_numpy(np.ascontiguousarray(syn).view(np.int32)).cuda()
    corr, flags, iters = dec.decode_baseline(s, first_shot_id=first_shot_id)
    torch.cuda.synchronize()
    return dict(corr=corr.cpu().numpy().view(np.uint32), flags=flags.cpu().numpy(), iters=iters.cpu().numpy())


CASES = [
    # name, p, shots, seed, params
    ("surface5_cc", 0.05, 2000, 1001, dict(max_iter=50, scale_mode=1, scale=0.625, lottery=True, osd=1, seed=3)),
    ("surface11_phen", 0.01, 600, 1002, dict(max_iter=100, lottery=True, osd=1, seed=2002)),
    ("bb144_phen", 0.003, 1500, 1004, dict(max_iter=200, lottery=True, osd=2, osd_order=10, seed=2004)),
    ("bb144_phen", 0.01, 300, 1005, dict(max_iter=60, lottery=True, osd=2, osd_order=10, seed=7, flip=1)),
]


@pytest.mark.parametrize("msg", [0, 1], ids=["fp32", "fp16"])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{i}" for i, c in enumerate(CASES)])
def test_baseline_matches_oracle_and_fused(case, msg):
    from paper_2605_00038_amd import DecoderParams
    name, p, shots, seed, kw = case
    _say("baseline parity", msg, name, p, shots, kw)
    h, e, syn = batch(name, p, shots, seed)
    prm = DecoderParams(msg=msg, **kw)
    b = _baseline(h, p, prm, syn, first_shot_id=5)
    o = oracle.decode(h, p, oracle_params(prm), syn, first_shot_id=5, n_threads=8)
    same = (b["corr"] == o["corr"]).all(axis=1)
    _say("  vs oracle: identical", same.mean(), "flags", (b["flags"] == o["flags"]).mean(),
         "iters", (b["iters"] == o["iters"]).mean())
    assert same.mean() >= 0.999
    assert (b["flags"] == o["flags"]).mean() >= 0.999
    f = gpu_decode(h, p, prm, syn, first_shot_id=5)
    same_f = (b["corr"] == f["corr"]).all(axis=1)
    _say("  vs fused: identical", same_f.mean())
    assert same_f.mean() >= 0.999


def test_baseline_rejects_int8_and_handles_empty():
    import torch
    from paper_2605_00038_amd import Code, Decoder, DecoderParams
    from paper_2605_00038_amd._lib import LbpError, LBP_EUNSUPPORTED
    h, e, syn = batch("surface5_cc", 0.05, 10, 1)
    dec = Decoder(Code.from_scipy(h, 0.05), DecoderParams(msg=2), 10)
    with pytest.raises(LbpError) as ei:
        dec.decode_baseline(torch.from_numpy(syn.view(np.int32)).cuda())
    assert ei.value.status == LBP_EUNSUPPORTED
    dec = Decoder(Code.from_scipy(h, 0.05), DecoderParams(msg=0), 10)
    corr, flags, iters = dec.decode_baseline(torch.zeros((0, syn.shape[1]), dtype=torch.int32, device="cuda"))
    assert corr.shape[0] == 0
