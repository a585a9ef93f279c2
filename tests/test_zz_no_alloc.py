"""lbp_decode_noalloc (the entry point that allocates nothing) against lbp_decode.

The no-allocation variant runs the same kernels on the library's static scratch
array, so every output must be bit for bit the one of lbp_decode on the same
inputs: two calls in a row per case, the second with fewer shots (the scratch
keeps the first call's contents, which must not leak into the second), through
the C ABI.
"""
import sys

import numpy as np
import pytest

from tests.gpu_util import batch

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


CASES = [
    # name, p, params, shots of the first and the second call
    ("bb144_phen", 0.003, dict(max_iter=200, msg=2, lottery=True, osd=2, osd_order=10, seed=2004), 6000, 1500),
    ("bb144_phen", 0.004, dict(max_iter=100, msg=1, lottery=True, osd=2, osd_order=10, seed=5), 1200, 300),
    ("surface11_phen", 0.01, dict(max_iter=100, msg=0, lottery=True, osd=1, seed=2002), 2500, 700),
    ("surface13_phen", 0.003, dict(max_iter=100, msg=2, lottery=True, osd=1, seed=20), 400, 90),
]


def _run(dec, s, first, noalloc):
    import torch
    shots = s.shape[0]
    out = (torch.empty((shots, dec.nw), dtype=torch.int32, device="cuda"),
           torch.empty(shots, dtype=torch.uint8, device="cuda"),
           torch.empty(shots, dtype=torch.int32, device="cuda"),
           torch.empty((shots, dec.code.n), dtype=torch.float32, device="cuda"))
    if noalloc:
        dec.decode_noalloc(s, out, first_shot_id=first)
    else:
        dec.decode(s, first_shot_id=first, out=out)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-msg{c[2]['msg']}" for c in CASES])
def test_noalloc_matches_decode(case):
    import torch
    from paper_2605_00038_amd import Code, Decoder, DecoderParams
    name, p, kw, n1, n2 = case
    _say("noalloc", name, kw, n1, n2)
    h, e, syn = batch(name, p, n1 + n2, 4100)
    dec = Decoder(Code.from_scipy(h, p), DecoderParams(**kw), n1)
    for shots, lo, first in ((n1, 0, 11), (n2, n1, 7000)):
        s = torch.from_numpy(np.ascontiguousarray(syn[lo:lo + shots]).view(np.int32)).cuda()
        got = _run(dec, s, first, True)
        ref = _run(dec, s, first, False)
        osd = int(((ref[1] & 2) != 0).sum())
        _say(f"  {shots} shots: {osd} via OSD")
        for a, b, what in zip(got, ref, ("corrections", "flags", "iterations", "lambda")):
            assert np.array_equal(a, b), (what, shots)


def test_noalloc_rejects_batches_beyond_the_scratch():
    import torch
    from paper_2605_00038_amd import Code, Decoder, DecoderParams
    from paper_2605_00038_amd._lib import LbpError, LBP_EINVAL
    h, e, syn = batch("bb144_phen", 0.003, 8, 4101)
    dec = Decoder(Code.from_scipy(h, 0.003), DecoderParams(max_iter=200, msg=2, osd=2, osd_order=10), 8)
    big = 200_000   # 2n bytes of lambda staging per shot alone exceed 128 MiB at this size
    s = torch.zeros((big, dec.mw), dtype=torch.int32, device="cuda")
    out = (torch.empty((big, dec.nw), dtype=torch.int32, device="cuda"),
           torch.empty(big, dtype=torch.uint8, device="cuda"), None, None)
    with pytest.raises(LbpError) as ei:
        dec.decode_noalloc(s, out)
    assert ei.value.status == LBP_EINVAL and "at most" in str(ei.value)
    _say(str(ei.value))
    # the rejected call launched nothing: a valid call right after still matches lbp_decode
    s8 = torch.from_numpy(np.ascontiguousarray(syn).view(np.int32)).cuda()
    assert all(np.array_equal(a, b) for a, b in zip(_run(dec, s8, 3, True), _run(dec, s8, 3, False)))
