"""Serving loop (lbp_server_*) and keyed decode on the GPU, through the C ABI.

The serving contract: a request's results depend only on (code, params,
request seed, shot ids, syndromes), never on what else was packed into the
same launch.  Every check compares against a lone lbp_decode of the request,
and the Int3.4 cases also against the oracle.
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


def _code(h, p):
    from paper_2605_00038_amd import Code
    return Code.from_scipy(h, p)


CODES = [
    # name, p, params
    ("bb144_phen", 0.003, dict(max_iter=200, lottery=True, osd=2, osd_order=10)),
    ("surface5_phen", 0.01, dict(max_iter=100, lottery=True, osd=1)),
    ("surface11_phen", 0.01, dict(max_iter=100, lottery=True, osd=1, msg=1)),
]


def test_keyed_decode_matches_first_shot_id_and_per_shot_seeds():
    import torch
    from paper_2605_00038_amd import Decoder
    h, e, syn = batch("bb144_phen", 0.006, 700, 77)
    prm = _params(max_iter=120, lottery=True, osd=2, osd_order=10, seed=9)
    dec = Decoder(_code(h, 0.006), prm, 700)
    s = torch.from_numpy(syn.view(np.int32)).cuda()
    keys = np.stack([np.full(700, 9, np.uint64), np.arange(1000, 1700, dtype=np.uint64)], 1)
    corr, flags, iters = dec.decode_keyed(s, torch.from_numpy(keys.view(np.int64)).cuda())
    c2, f2, i2, _ = dec.decode(s, first_shot_id=1000)
    torch.cuda.synchronize()
    assert np.array_equal(corr.cpu().numpy(), c2.cpu().numpy())
    assert np.array_equal(flags.cpu().numpy(), f2.cpu().numpy())
    assert np.array_equal(iters.cpu().numpy(), i2.cpu().numpy())
    # per-shot seeds: shot k with seed (k % 3) equals the oracle run with that seed
    keys[:, 0] = np.arange(700) % 3
    corr, flags, iters = dec.decode_keyed(s, torch.from_numpy(keys.view(np.int64)).cuda())
    torch.cuda.synchronize()
    corr, flags, iters = corr.cpu().numpy().view(np.uint32), flags.cpu().numpy(), iters.cpu().numpy()
    for sd in range(3):
        idx = np.nonzero(keys[:, 0] == sd)[0]
        o = oracle.decode(h, 0.006, oracle_params(prm, seed=sd), syn, first_shot_id=1000, n_threads=8)
        assert np.array_equal(corr[idx], o["corr"][idx]), sd
        assert np.array_equal(flags[idx], o["flags"][idx]), sd
        assert np.array_equal(iters[idx], o["iters"][idx]), sd


def test_server_mix_equals_lone_decodes():
    from paper_2605_00038_amd import Server
    rng = np.random.default_rng(5)
    srv = Server(max_slots=4)
    slots, data = [], []
    for j, (name, p, kw) in enumerate(CODES):
        h, e, syn = batch(name, p, 12000 if j == 0 else 3000, 500 + j)
        slots.append(srv.add_code(_code(h, p), _params(**kw)))
        data.append((h, p, kw, syn))
    info = srv.slot_info(slots[0])
    _say("bb144 slot", info)
    assert info["ring_items"] >= 1024
    # requests: sizes 1..40, one of 10123 shots, random codes, seeds, shot ids
    reqs = []
    big = 10123
    plan = [(0, big)] + [(int(rng.integers(0, 3)), int(rng.integers(1, 41))) for _ in range(300)]
    for k, (ci, size) in enumerate(plan):
        syn = data[ci][3]
        lo = int(rng.integers(0, syn.shape[0] - size + 1))
        seed = int(rng.integers(0, 1 << 62))
        first = int(rng.integers(0, 1 << 40))
        t = srv.submit(slots[ci], syn[lo:lo + size], seed, first)
        reqs.append((t, ci, lo, size, seed, first))
    got = []
    for t, ci, lo, size, seed, first in reqs:
        r = srv.wait(t, slots[ci], size, timeout_us=120_000_000)
        assert r is not None, "request did not complete"
        got.append(r)
    info = srv.slot_info(slots[0])
    _say("after", info)
    assert info["queued_shots"] == 0 and info["shots"] >= big
    # lone decodes, one per request (the big one included)
    for (t, ci, lo, size, seed, first), (corr, flags, iters) in zip(reqs, got):
        h, p, kw, syn = data[ci]
        ref = gpu_decode(h, p, _params(**kw, seed=seed), syn[lo:lo + size], first_shot_id=first)
        assert np.array_equal(corr, ref["corr"]), (ci, size)
        assert np.array_equal(flags, ref["flags"]), (ci, size)
        assert np.array_equal(iters, ref["iters"]), (ci, size)
    # Int3.4 requests also against the oracle
    for (t, ci, lo, size, seed, first), (corr, flags, iters) in list(zip(reqs, got))[1:60]:
        h, p, kw, syn = data[ci]
        if kw.get("msg", 2) != 2:
            continue
        o = oracle.decode(h, p, oracle_params(_params(**kw, seed=seed)), syn[lo:lo + size], first_shot_id=first)
        assert np.array_equal(corr, o["corr"]) and np.array_equal(flags, o["flags"]), (ci, size)
    srv.close()


def test_server_cancel_admission_and_tickets():
    from paper_2605_00038_amd import Server
    from paper_2605_00038_amd._lib import LbpError, LBP_EBUSY, LBP_EINVAL
    name, p, kw = CODES[1]
    h, e, syn = batch(name, p, 2000, 900)
    srv = Server(max_slots=1)
    slot = srv.add_code(_code(h, p), _params(**kw))
    ring = srv.slot_info(slot)["ring_items"]
    with pytest.raises(LbpError) as ei:   # more than the admission bound in one request
        srv.submit(slot, np.zeros((16 * ring + 1, syn.shape[1]), np.uint32), 1)
    assert ei.value.status == LBP_EBUSY
    with pytest.raises(LbpError) as ei:   # a second slot does not exist
        srv.add_code(_code(h, p), _params(**kw))
    assert ei.value.status == LBP_EBUSY
    tickets = [srv.submit(slot, syn[k * 10:(k + 1) * 10], 3, k * 10) for k in range(100)]
    for t in tickets[::3]:
        srv.cancel(t)
    for k, t in enumerate(tickets):
        if k % 3 == 0:
            with pytest.raises(LbpError) as ei:
                srv.poll(t, slot, 10)
            assert ei.value.status == LBP_EINVAL
            continue
        r = srv.wait(t, slot, 10, timeout_us=60_000_000)
        ref = gpu_decode(h, p, _params(**kw, seed=3), syn[k * 10:(k + 1) * 10], first_shot_id=k * 10)
        assert np.array_equal(r[0], ref["corr"]) and np.array_equal(r[1], ref["flags"])
        with pytest.raises(LbpError):      # released after the first successful wait
            srv.poll(t, slot, 10)
    srv.close()


def test_server_many_outstanding_tickets_out_of_order():
    """Tens of thousands of requests in flight before the first wait, collected
    in a shuffled order (a few cancelled, some polled first): the ticket table
    keeps every one until it is collected, and each result is the lone decode's."""
    from paper_2605_00038_amd import Server
    from paper_2605_00038_amd._lib import LbpError, LBP_EINVAL
    name, p, kw = CODES[1]
    n = 24000
    h, e, syn = batch(name, p, n, 920)
    srv = Server(max_slots=1)
    slot = srv.add_code(_code(h, p), _params(**kw))
    tickets = [srv.submit(slot, syn[k:k + 1], 5, k) for k in range(n)]
    ref = gpu_decode(h, p, _params(**kw, seed=5), syn)
    cancelled = set(range(7, n, 997))
    for k in cancelled:
        srv.cancel(tickets[k])
    order = np.random.default_rng(921).permutation(n)
    polled = 0
    for k in order[: n // 4]:
        if k in cancelled:
            continue
        r = srv.poll(tickets[k], slot, 1)
        if r is not None:
            polled += 1
            assert np.array_equal(r[0][0], ref["corr"][k]) and r[1][0] == ref["flags"][k]
        else:
            r = srv.wait(tickets[k], slot, 1, timeout_us=60_000_000)
            assert np.array_equal(r[0][0], ref["corr"][k]) and r[1][0] == ref["flags"][k]
    for k in order[n // 4:][::-1]:
        if k in cancelled:
            with pytest.raises(LbpError) as ei:
                srv.poll(tickets[k], slot, 1)
            assert ei.value.status == LBP_EINVAL
            continue
        r = srv.wait(tickets[k], slot, 1, timeout_us=60_000_000)
        assert np.array_equal(r[0][0], ref["corr"][k]) and r[1][0] == ref["flags"][k] and r[2][0] == ref["iters"][k]
    _say("outstanding tickets", n, "polled ready", polled)
    srv.close()


def test_server_memory_budget_limits_ring_size():
    from paper_2605_00038_amd import Server
    from paper_2605_00038_amd._lib import LbpError, LBP_ENOMEM
    name, p, kw = CODES[0]
    h, e, syn = batch(name, p, 64, 901)
    big = Server(device_mem_budget=16 << 30, max_slots=1)
    # Int3.4 stages 2n bytes of lambda per ring item: 65536 items of BB144 r=12 take 340 MB
    small = Server(device_mem_budget=200 << 20, max_slots=1)
    s1 = big.add_code(_code(h, p), _params(**kw))
    s2 = small.add_code(_code(h, p), _params(**kw))
    t1, t2 = big.slot_info(s1)["ring_items"], small.slot_info(s2)["ring_items"]
    _say("rings", t1, t2)
    assert t2 < t1
    r1 = big.wait(big.submit(s1, syn, 4), s1, 64)
    r2 = small.wait(small.submit(s2, syn, 4), s2, 64)
    assert all(np.array_equal(a, b) for a, b in zip(r1, r2))
    tiny = Server(device_mem_budget=1 << 20, max_slots=1)
    with pytest.raises(LbpError) as ei:
        tiny.add_code(_code(h, p), _params(**kw))
    assert ei.value.status == LBP_ENOMEM
    for s in (big, small, tiny):
        s.close()


def test_server_load_generator():
    from paper_2605_00038_amd import Server
    srv = Server(max_slots=2)
    pools, slots = [], []
    for j in (0, 1):
        name, p, kw = CODES[j]
        h, e, syn = batch(name, p, 4000, 910 + j)
        slots.append(srv.add_code(_code(h, p), _params(**kw)))
        pools.append(syn)
    lat, code, el = srv.run_load(slots, pools, 3000, 1, 0.0, 12)       # saturation
    _say("saturation", 3000 / el, "req/s; p50/p99 us", np.percentile(lat, [50, 99]))
    assert np.all(lat > 0) and el > 0 and set(np.unique(code)) == {0, 1}
    lat, code, el = srv.run_load(slots[:1], pools[:1], 2000, 4, 20000.0, 13)   # Poisson, 4-shot requests
    _say("poisson 20k/s", np.percentile(lat, [50, 99, 99.9]), el)
    assert np.all(lat > 0) and el >= 2000 / 20000.0 * 0.5
    srv.close()
