"""Lottery design-space rules (Sec. III-B, Table I) on the GPU against the oracle.

Every rule (random / worst check x proposed, Q-first, unreliable, random
neighbour) goes through the fused Int3.4 kernel (bit-exact: corrections, flags,
iteration counts, lambda), the fused float kernels and the global-memory
comparison path (identical corrections on >= 99.9% of shots).
"""
import sys

import numpy as np
import pytest

import oracle
from tests.gpu_util import batch, gpu_decode, oracle_params

pytestmark = pytest.mark.gpu

RULES = [0x01, 0x10, 0x11, 0x20, 0x21, 0x30, 0x31]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _params(**kw):
    from paper_2605_00038_amd import DecoderParams
    return DecoderParams(**kw)


INT8_CASES = [
    # name, p, shots, data seed, params
    ("bb144_phen", 0.01, 600, 1101, dict(max_iter=60, lottery=True, osd=1, seed=41)),
    ("surface11_phen", 0.012, 600, 1102, dict(max_iter=60, lottery=True, lottery_skip=2, osd=0, seed=42)),
    ("bb144_cc", 0.06, 1000, 1103, dict(max_iter=60, lottery=True, osd=0, seed=43, flip=1)),
]


@pytest.mark.parametrize("rule", RULES, ids=[f"r{r:02x}" for r in RULES])
@pytest.mark.parametrize("case", INT8_CASES, ids=[c[0] for c in INT8_CASES])
def test_int8_rules_bit_exact(case, rule):
    name, p, shots, seed, kw = case
    _say("int8 rule", hex(rule), name, p, shots, kw)
    h, e, syn = batch(name, p, shots, seed)
    prm = _params(msg=2, lottery_rule=rule, **kw)
    g = gpu_decode(h, p, prm, syn, first_shot_id=3, want_llr=True)
    o = oracle.decode(h, p, oracle_params(prm), syn, first_shot_id=3, want_llr=True, n_threads=8)
    assert (g["flags"] == o["flags"]).all()
    assert (g["iters"] == o["iters"]).all()
    assert (g["llr"] == o["llr"]).all()
    assert (g["corr"] == o["corr"]).all()
    # the rule reached the kernel: the outcome differs from the proposed rule somewhere
    base = oracle.decode(h, p, oracle_params(prm, policy=0), syn, first_shot_id=3, n_threads=8)
    assert not (base["iters"] == o["iters"]).all()


@pytest.mark.parametrize("msg", [0, 1], ids=["fp32", "fp16"])
@pytest.mark.parametrize("rule", [0x01, 0x20, 0x31], ids=["worst", "unreliable", "worst-random"])
def test_float_rules_fused_and_comparison_path(rule, msg):
    import torch
    from paper_2605_00038_amd import Code, Decoder
    name, p, shots, seed = "bb144_phen", 0.01, 800, 1104
    _say("float rule", hex(rule), msg, name, p, shots)
    h, e, syn = batch(name, p, shots, seed)
    prm = _params(msg=msg, max_iter=60, lottery=True, osd=1, seed=44, lottery_rule=rule)
    o = oracle.decode(h, p, oracle_params(prm), syn, n_threads=8)
    g = gpu_decode(h, p, prm, syn)
    same = (g["corr"] == o["corr"]).all(axis=1)
    _say("  fused identical", same.mean())
    assert same.mean() >= 0.999
    dec = Decoder(Code.from_scipy(h, p), prm, shots)
    corr, flags, iters = dec.decode_baseline(torch.from_numpy(np.ascontiguousarray(syn).view(np.int32)).cuda())
    torch.cuda.synchronize()
    same_b = (corr.cpu().numpy().view(np.uint32) == o["corr"]).all(axis=1)
    _say("  comparison path identical", same_b.mean())
    assert same_b.mean() >= 0.999


def test_unknown_rule_rejected():
    from paper_2605_00038_amd import Code, Decoder
    from paper_2605_00038_amd._lib import LbpError, LBP_EINVAL
    h, e, syn = batch("surface5_cc", 0.05, 4, 1)
    code = Code.from_scipy(h, 0.05)
    for bad in (0x02, 0x03, 0x40, 0x04, 0x100, -1):
        with pytest.raises(LbpError) as ei:
            Decoder(code, _params(lottery_rule=bad), 4)
        assert ei.value.status == LBP_EINVAL
