"""Multi-group plans (lbp_plan_*): uneven codes, formats and parameters in one
persistent launch, replayed from a captured HIP graph.

Every group's outputs must equal lbp_decode of that group alone (bit for bit:
the same arithmetic runs, only the launch is shared), and the Int3.4 groups
must equal the oracle.  Graph replays are checked one by one against eager
decodes of the syndromes written into the bound buffers before each replay,
with the program's own eager work and synchronisations in between."""
import sys

import numpy as np
import pytest

import oracle
from tests.gpu_util import batch, gpu_decode, oracle_params

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


# the code-capacity and space-time workloads of the batching configuration, plus a
# large-code group and an OSD-CS group: name, p, shots, params
GROUPS = [
    ("surface5_cc", 0.05, 3000, dict(max_iter=50, msg=0, scale_mode=1, scale=0.625, lottery=False, osd=1)),
    ("bb144_cc", 0.04, 2000, dict(max_iter=100, msg=2, lottery=True, osd=1, seed=11)),
    ("bb144_cc", 0.02, 1500, dict(max_iter=100, msg=1, lottery=True, osd=1, seed=12)),
    ("surface11_phen", 0.01, 300, dict(max_iter=100, msg=2, lottery=True, osd=2, osd_order=10, seed=13)),
    ("bb144_phen", 0.004, 400, dict(max_iter=200, msg=2, lottery=True, osd=2, osd_order=10, seed=14)),
]


def _make(groups, seed0, autotune=True):
    import torch
    from paper_2605_00038_amd import Code, Decoder, DecoderParams, Plan
    decs, data, gl = [], [], []
    for j, (name, p, shots, kw) in enumerate(groups):
        h, e, syn = batch(name, p, shots, seed0 + j)
        dec = Decoder(Code.from_scipy(h, p), DecoderParams(**kw), max(1, shots))
        s = torch.from_numpy(np.ascontiguousarray(syn).view(np.int32)).cuda()
        gl.append((dec, s, 1000 * j + 5))
        decs.append(dec)
        data.append((name, h, p, kw, syn))
    return Plan(gl, autotune=autotune), decs, data, gl


def _check_group(plan, g, h, p, kw, syn, first, with_oracle):
    from paper_2605_00038_amd import DecoderParams
    corr, flags, iters = (t.cpu().numpy() for t in plan.outputs[g])
    ref = gpu_decode(h, p, DecoderParams(**kw), syn, first_shot_id=first)
    assert np.array_equal(corr.view(np.uint32), ref["corr"]), g
    assert np.array_equal(flags, ref["flags"]), g
    assert np.array_equal(iters, ref["iters"]), g
    if with_oracle and kw.get("msg") == 2 and syn.shape[0] > 0:
        k = min(400, syn.shape[0])
        o = oracle.decode(h, p, oracle_params(DecoderParams(**kw)), syn[:k], first_shot_id=first, n_threads=8)
        assert np.array_equal(corr[:k].view(np.uint32), o["corr"]), g
        assert np.array_equal(flags[:k], o["flags"]), g
        assert np.array_equal(iters[:k], o["iters"]), g
    return int(((flags & 2) != 0).sum())


def test_plan_groups_equal_lone_decodes_and_oracle():
    plan, decs, data, gl = _make(GROUPS, 5100)
    wpb, blocks, ms = plan.info()
    _say(f"plan shape: {wpb} waves per block x {blocks} blocks; candidates (ms): {[round(x, 3) for x in ms]}")
    assert len(ms) >= 2 and wpb >= 1 and blocks >= 1
    # plan creation ran the sequence eagerly (autotuning); its outputs are results already
    for g, (name, h, p, kw, syn) in enumerate(data):
        osd = _check_group(plan, g, h, p, kw, syn, gl[g][2], True)
        _say(f"  {name} msg {kw['msg']}: {syn.shape[0]} shots, {osd} via OSD, equal to lbp_decode")


def test_plan_graph_replays_track_new_syndromes():
    import torch
    from workloads import sample
    groups = GROUPS[:3] + [("surface11_phen", 0.01, 0, dict(max_iter=100, msg=2, lottery=True, osd=1, seed=15))]
    plan, decs, data, gl = _make(groups, 5200, autotune=False)
    for rep in range(4):
        # new syndromes into the bound buffers, eager work of our own, then a replay
        fresh = []
        for g, (name, h, p, kw, syn) in enumerate(data):
            if syn.shape[0] == 0:
                fresh.append(syn)
                continue
            _, s2 = sample.make_batch(h, p, syn.shape[0], 9000 + 10 * rep + g)
            gl[g][1].copy_(torch.from_numpy(np.ascontiguousarray(s2).view(np.int32)))
            fresh.append(s2)
        junk = torch.randn(1 << 20, device="cuda").sum()   # unrelated eager work on the stream
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for g, (name, h, p, kw, syn) in enumerate(data):
            _check_group(plan, g, h, p, kw, fresh[g], gl[g][2], rep == 0)
        _say(f"  replay {rep}: every group equal to its eager decode")


def test_plan_rejects_bad_input():
    from paper_2605_00038_amd import Plan
    from paper_2605_00038_amd._lib import LbpError, LBP_EINVAL
    with pytest.raises(LbpError) as ei:
        Plan([])
    assert ei.value.status == LBP_EINVAL


@pytest.mark.parametrize("fmt", [2, 1], ids=["int8", "fp16"])
def test_batching_configuration_plan_matches_oracle(fmt):
    """The batching configuration's shape: BB144 code capacity at p = 0.01, 0.02,
    0.04, 0.06 (I=100, lottery, OSD-0) in one plan with rotated surface d=5
    code-capacity shots (FP32, constant scale 0.625, plain BP, I=50, OSD-0).
    Int3.4 groups bit-exact against the oracle on every shot; float groups
    identical corrections on >= 99.9% against the storage-matched oracle."""
    groups = [("bb144_cc", p, 2500, dict(max_iter=100, msg=fmt, lottery=True, osd=1, seed=2030 + j))
              for j, p in enumerate((0.01, 0.02, 0.04, 0.06))]
    groups.append(("surface5_cc", 0.05, 4000, dict(max_iter=50, msg=0, scale_mode=1, scale=0.625, lottery=False,
                                                     osd=1, seed=2001)))
    plan, decs, data, gl = _make(groups, 1030)
    from paper_2605_00038_amd import DecoderParams
    for g, (name, h, p, kw, syn) in enumerate(data):
        corr, flags, iters = (t.cpu().numpy() for t in plan.outputs[g])
        o = oracle.decode(h, p, oracle_params(DecoderParams(**kw)), syn, first_shot_id=gl[g][2], n_threads=8)
        same = (corr.view(np.uint32) == o["corr"]).all(axis=1)
        _say(f"  {name} p={p} msg {kw['msg']}: identical {same.mean():.4f}, OSD {int(((flags & 2) != 0).sum())}")
        if kw["msg"] == 2:
            assert same.all() and np.array_equal(flags, o["flags"]) and np.array_equal(iters, o["iters"])
        else:
            assert same.mean() >= 0.999
