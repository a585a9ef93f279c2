"""Fixed-point message formats Int x.y (LBP_MSG_FIXED) on the GPU against the oracle.

The 7-bit formats saturate at 63, the 8-bit ones at 127; every format is
bit-exact (corrections, flags, iteration counts, lambda) in the fused kernel
(m <= 1024) and in the general kernel (m > 1024).
"""
import sys

import pytest

import oracle
from tests.gpu_util import batch, gpu_decode, oracle_params

pytestmark = pytest.mark.gpu

FORMATS = [(2, 4), (3, 3), (4, 2), (2, 5), (4, 3), (3, 4)]
CASES = [
    # name, p, shots, data seed, params
    ("surface9_phenpf", 0.004, 1500, 1201, dict(max_iter=80, lottery=True, osd=2, osd_order=10, seed=51)),
    ("bb144_phen", 0.006, 800, 1202, dict(max_iter=60, lottery=True, osd=1, seed=52, flip=1)),
    ("surface13_phenpf", 0.003, 300, 1203, dict(max_iter=60, lottery=True, osd=0, seed=53)),  # m > 1024
]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("fx", FORMATS, ids=[f"int{x}.{y}" for x, y in FORMATS])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fixed_point_bit_exact(case, fx):
    from paper_2605_00038_amd import DecoderParams, msg_fixed
    name, p, shots, seed, kw = case
    _say("fixed point", fx, name, p, shots)
    h, e, syn = batch(name, p, shots, seed)
    prm = DecoderParams(msg=msg_fixed(*fx), **kw)
    g = gpu_decode(h, p, prm, syn, first_shot_id=9, want_llr=True)
    o = oracle.decode(h, p, oracle_params(prm), syn, first_shot_id=9, want_llr=True, n_threads=8)
    assert (g["flags"] == o["flags"]).all()
    assert (g["iters"] == o["iters"]).all()
    assert (g["llr"] == o["llr"]).all()
    assert (g["corr"] == o["corr"]).all()


def test_fixed_point_formats_validated():
    from paper_2605_00038_amd import Code, Decoder, DecoderParams, msg_fixed
    from paper_2605_00038_amd._lib import LbpError, LBP_EINVAL
    h, e, syn = batch("surface5_cc", 0.05, 4, 1)
    code = Code.from_scipy(h, 0.05)
    for bad in (msg_fixed(4, 4), msg_fixed(0, 0), msg_fixed(15, 15), 0x300, 3):
        with pytest.raises(LbpError) as ei:
            Decoder(code, DecoderParams(msg=bad), 4)
        assert ei.value.status == LBP_EINVAL
    Decoder(code, DecoderParams(msg=msg_fixed(1, 0)), 4)       # 2-bit messages: accepted
