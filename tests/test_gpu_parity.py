"""GPU decoder (through the C ABI) against the CPU oracle on the same seeded inputs.

Bars: Int3.4 BP is bit-exact (corrections, flags, iteration counts, lambda);
OSD-0 / OSD-CS are bit-exact given the same lambda; float BP gives identical
corrections on >= 99.9% of shots against the oracle with the same storage
rounding.
"""
import sys

import numpy as np
import pytest

import oracle
from tests.gpu_util import batch, gpu_decode, oracle_params
from workloads import codes, sample

pytestmark = pytest.mark.gpu


def _params(**kw):
    from paper_2605_00038_amd import DecoderParams
    return DecoderParams(**kw)


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


INT8_CASES = [
    # name, p, shots, data seed, params
    ("surface5_cc", 0.05, 3000, 1001, dict(max_iter=50, scale_mode=1, scale=0.625, lottery=False, osd=1)),
    ("surface5_cc", 0.05, 3000, 1001, dict(max_iter=50, scale_mode=1, scale=0.625, lottery=True, osd=1, seed=2001)),
    ("bb144_cc", 0.06, 2000, 1033, dict(max_iter=100, lottery=True, osd=1, seed=2033)),
    ("surface11_phen", 0.01, 600, 1002, dict(max_iter=100, lottery=True, osd=1, seed=2002)),
    ("bb144_phen", 0.003, 3000, 1004, dict(max_iter=200, lottery=True, osd=2, osd_order=10, seed=2004)),
    ("bb144_phen", 0.01, 300, 1005, dict(max_iter=60, lottery=True, osd=2, osd_order=10, seed=7, flip=1)),
    ("surface5_phen", 0.02, 2000, 1006, dict(max_iter=40, lottery=True, lottery_skip=2, osd=0, seed=11)),
    # H_st with the noiseless final read-out: weight-1 rows, every measurement column of weight 2
    ("surface9_phenpf", 0.003, 2000, 1007, dict(max_iter=100, lottery=True, osd=2, osd_order=10, seed=12)),
    ("bb144_phenpf", 0.004, 1000, 1008, dict(max_iter=100, lottery=True, osd=1, seed=13)),
    # unrotated (planar) surface code, the layout of Table II: 720 x 1953 (d=9), 4896 x 13889 (d=17)
    ("usurface9_phenpf", 0.004, 2000, 1009, dict(max_iter=100, lottery=True, osd=2, osd_order=10, seed=14)),
    ("usurface17_phenpf", 0.002, 96, 1011, dict(max_iter=100, lottery=True, osd=1, seed=15)),
    # K = 0: the first lottery reads the estimate before iteration 0 (all zero); 20000
    # shots of a small code give every wave many shots, so a stale estimate would show
    ("surface5_phen", 0.02, 20000, 1014, dict(max_iter=60, lottery=True, lottery_skip=0, osd=1, seed=18)),
    ("bb144_phen", 0.006, 4000, 1015, dict(max_iter=100, lottery=True, lottery_skip=0, osd=1, seed=19)),
    ("surface13_phen", 0.003, 300, 1016, dict(max_iter=100, lottery=True, lottery_skip=0, osd=1, seed=20)),
]


@pytest.mark.parametrize("case", INT8_CASES, ids=[f"{c[0]}-{i}" for i, c in enumerate(INT8_CASES)])
def test_int8_bit_exact(case):
    name, p, shots, seed, kw = case
    _say("int8 parity", name, p, shots, kw)
    h, e, syn = batch(name, p, shots, seed)
    prm = _params(msg=2, **kw)
    g = gpu_decode(h, p, prm, syn, first_shot_id=5, want_llr=True)
    o = oracle.decode(h, p, oracle_params(prm), syn, first_shot_id=5, want_llr=True, n_threads=8)
    assert (g["flags"] == o["flags"]).all()
    assert (g["iters"] == o["iters"]).all()
    assert (g["llr"] == o["llr"]).all()
    assert (g["corr"] == o["corr"]).all()


def test_worked_example_gpu():
    h = codes.worked_example_h()
    e = np.zeros((64, 13), np.uint8)
    e[:, [2, 8, 9]] = 1
    import scipy.sparse as sp
    syn = sample.pack_bits(sample.syndromes(h, sp.csr_matrix(e)))
    for msg in (0, 1, 2):
        plain = gpu_decode(h, 0.05, _params(msg=msg, max_iter=100, lottery=False, osd=0), syn)
        assert (plain["flags"] & 1 == 0).all()
        lot = gpu_decode(h, 0.05, _params(msg=msg, max_iter=100, lottery=True, osd=0, seed=3), syn)
        assert (lot["flags"] & 1 == 1).all()
        o = oracle.decode(h, 0.05, oracle_params(_params(msg=msg, max_iter=100, lottery=True, osd=0, seed=3)), syn)
        assert (lot["corr"] == o["corr"]).all() and (lot["iters"] == o["iters"]).all()


FLOAT_CASES = [
    ("surface11_phen", 0.01, 3000, 1002, dict(max_iter=100, lottery=True, osd=1, seed=2002)),
    ("bb144_phen", 0.003, 3000, 1004, dict(max_iter=200, lottery=True, osd=2, seed=2004)),
    ("bb144_cc", 0.04, 3000, 1032, dict(max_iter=100, lottery=True, osd=1, seed=2032)),
    ("surface5_cc", 0.05, 3000, 1001, dict(max_iter=50, scale_mode=1, scale=0.625, lottery=False, osd=1)),
    ("surface9_phenpf", 0.003, 3000, 1007, dict(max_iter=100, lottery=True, osd=2, seed=12)),
    ("surface5_phen", 0.02, 20000, 1014, dict(max_iter=60, lottery=True, lottery_skip=0, osd=1, seed=18)),
]


@pytest.mark.parametrize("msg", [0, 1], ids=["fp32", "fp16"])
@pytest.mark.parametrize("case", FLOAT_CASES, ids=[c[0] for c in FLOAT_CASES])
def test_float_identity(case, msg):
    name, p, shots, seed, kw = case
    _say("float parity", msg, name, p, shots)
    h, e, syn = batch(name, p, shots, seed)
    prm = _params(msg=msg, **kw)
    g = gpu_decode(h, p, prm, syn, want_llr=True)
    o = oracle.decode(h, p, oracle_params(prm), syn, want_llr=True, n_threads=8)
    same = (g["corr"] == o["corr"]).all(axis=1)
    _say("  identical", same.mean(), "flags", (g["flags"] == o["flags"]).mean())
    assert same.mean() >= 0.999
    # OSD given the GPU's own lambda is bit-exact (fp16: lambda is exactly its fp32 value;
    # fp32 carries lambda as an exact pair, of which only the rounded part is exported)
    osd_shots = np.nonzero(g["flags"] & 2)[0][:40] if msg == 1 else []
    for k in osd_shots:
        c, f = oracle.osd(h, g["llr"][k].astype(np.float64), syn[k], prm.osd, prm.osd_order)
        assert f == g["flags"][k]
        if not f & 4:
            assert (c == g["corr"][k]).all()


def test_osd_all_shots_and_overflow():
    """max_iter=1 sends most shots to OSD; a tiny staging capacity forces the re-decode loop."""
    h, e, syn = batch("bb144_phen", 0.003, 700, 1004)
    for osd_mode in (1, 2):
        prm = _params(msg=2, max_iter=1, lottery=False, osd=osd_mode)
        ref = oracle.decode(h, 0.003, oracle_params(prm), syn, n_threads=8)
        assert (ref["flags"] & 2).sum() > 300
        for cap in (None, 37):
            g = gpu_decode(h, 0.003, prm, syn, max_batch=1024, osd_cap=cap)
            assert (g["flags"] == ref["flags"]).all()
            assert (g["corr"] == ref["corr"]).all()
        est = sample.unpack_bits(g["corr"], h.shape[1])
        import scipy.sparse as sp
        assert (sample.pack_bits(sample.syndromes(h, sp.csr_matrix(est))) == syn).all()


def test_inconsistent_syndromes_flagged():
    h, _, _ = codes.workload_matrices("bb144_cc")
    hd = h.toarray().astype(np.int64)
    left = codes.gf2_nullspace(hd.T)
    rng = np.random.default_rng(5)
    bad = []
    while len(bad) < 64:
        s = rng.integers(0, 2, 72)
        if ((left @ s) % 2).any():
            bad.append(s)
    syn = sample.pack_bits(np.array(bad, np.uint8))
    prm = _params(msg=2, max_iter=20, osd=1)
    g = gpu_decode(h, 0.01, prm, syn)
    o = oracle.decode(h, 0.01, oracle_params(prm), syn)
    assert (g["flags"] == 2 | 4).all()
    assert (g["corr"] == o["corr"]).all()


def test_edge_batches_and_composition():
    """Empty batch, one shot, ragged sizes; results depend only on (shot id, syndrome)."""
    import torch
    from paper_2605_00038_amd import Code, Decoder
    h, e, syn = batch("bb144_phen", 0.003, 1000, 1004)
    prm = _params(msg=2, max_iter=200, lottery=True, osd=2, seed=9)
    code = Code.from_scipy(h, 0.003)
    dec = Decoder(code, prm, 1000)
    s = torch.from_numpy(syn.view(np.int32)).cuda()
    full = [t.cpu().numpy() for t in dec.decode(s, first_shot_id=100)[:3]]
    empty = dec.decode(s[:0], first_shot_id=0)
    assert empty[0].shape == (0, 81)
    for lo, hi in ((0, 1), (1, 2), (333, 334), (17, 530), (999, 1000), (64, 129)):
        part = [t.cpu().numpy() for t in dec.decode(s[lo:hi].contiguous(), first_shot_id=100 + lo)[:3]]
        for a, b in zip(full, part):
            assert (a[lo:hi] == b).all()
    with pytest.raises(Exception):
        dec.decode(torch.zeros((1001, 27), dtype=torch.int32, device="cuda"))


def test_host_entry_point_matches_device():
    h, e, syn = batch("surface11_phen", 0.01, 500, 1002)
    from paper_2605_00038_amd import Code, Decoder
    prm = _params(msg=1, max_iter=100, osd=1, seed=4)
    dec = Decoder(Code.from_scipy(h, 0.01), prm, 500)
    c1, f1, i1, _ = dec.decode_host(syn, first_shot_id=3)
    g = gpu_decode(h, 0.01, prm, syn, first_shot_id=3)
    assert (c1 == g["corr"]).all() and (f1 == g["flags"]).all() and (i1 == g["iters"]).all()


def test_full_size_sampled_bb144():
    """The benchmark's workload size (65536-shot chunks of BB144 r=12): a random sample
    of shots decoded one by one by the oracle must match bit-exactly (Int3.4)."""
    h, e, syn = batch("bb144_phen", 0.003, 65536, 1004)
    prm = _params(msg=2, max_iter=200, lottery=True, osd=2, osd_order=10, seed=2004)
    g = gpu_decode(h, 0.003, prm, syn)
    rng = np.random.default_rng(0)
    idx = np.sort(np.concatenate([rng.choice(65536, 300, replace=False), np.nonzero(g["flags"] & 2)[0][:60]]))
    for k in idx:
        o = oracle.decode(h, 0.003, oracle_params(prm), syn[k:k + 1], first_shot_id=int(k))
        assert o["flags"][0] == g["flags"][k] and o["iters"][0] == g["iters"][k]
        assert (o["corr"][0] == g["corr"][k]).all(), k
    _say("  failed-BP shots", int((g["flags"] & 2).sum()), "of 65536")


@pytest.mark.parametrize("name", ["surface13_phen", "surface17_phen", "bb288_phen"])
def test_osd_large_codes(name):
    """Codes with m > 1024 run OSD with G in LDS (d=13, 1092 checks) or in global
    memory (d=17, 2448 checks; BB[[288,12,18]] r=18, 2592 checks); few BP
    iterations force many shots into OSD."""
    h, e, syn = batch(name, 0.01, 24, 1010)
    for osd_mode in (1, 2):
        prm = _params(msg=2, max_iter=3, lottery=False, osd=osd_mode, osd_order=6)
        g = gpu_decode(h, 0.01, prm, syn)
        o = oracle.decode(h, 0.01, oracle_params(prm), syn, n_threads=8)
        assert ((g["flags"] & 2) != 0).sum() >= 8
        assert (g["flags"] == o["flags"]).all()
        assert (g["corr"] == o["corr"]).all()


def test_code_released_before_decoder():
    """A decoder keeps its code alive: destroying the code handle first (as Python's
    cycle collector may do) leaves the decoder working and the HIP state clean."""
    import ctypes
    import torch
    from paper_2605_00038_amd import Code, Decoder
    h, e, syn = batch("surface5_cc", 0.05, 300, 1001)
    prm = _params(msg=2, max_iter=50, lottery=True, osd=1, seed=2001)
    code = Code.from_scipy(h, 0.05)
    dec = Decoder(code, prm, syn.shape[0])
    code.__del__()                                  # lbp_code_destroy while the decoder lives
    assert code.handle is None
    s = torch.from_numpy(np.ascontiguousarray(syn).view(np.int32)).cuda()
    corr, flags, iters, _ = dec.decode(s, first_shot_id=0)
    o = oracle.decode(h, 0.05, oracle_params(prm), syn, n_threads=8)
    assert (corr.cpu().numpy().view(np.uint32) == o["corr"]).all()
    del dec, code
    hip = ctypes.CDLL("libamdhip64.so")
    assert hip.hipPeekAtLastError() == 0
    t = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")  # a fresh segment from the allocator
    del t


def test_osd_staging_grows_for_high_invoke_rate():
    """When more shots fail BP than the OSD staging holds, the decoder grows the
    staging once instead of re-decoding the overflow pass after pass; results equal
    the pinned-capacity path and the oracle."""
    import torch
    from paper_2605_00038_amd import Code, Decoder
    h, e, syn = batch("surface17_phen", 0.01, 12000, 1011)
    prm = _params(msg=2, max_iter=3, lottery=False, osd=1)
    code = Code.from_scipy(h, 0.01)
    s = torch.from_numpy(np.ascontiguousarray(syn).view(np.int32)).cuda()
    grow = Decoder(code, prm, syn.shape[0])
    cap0 = grow.osd_capacity
    c1, f1, i1, _ = grow.decode(s)
    torch.cuda.synchronize()
    assert int(((f1.cpu().numpy() & 2) != 0).sum()) > 2 * cap0       # the overflow path ran
    assert grow.osd_capacity > cap0                                   # and the staging grew
    pinned = Decoder(code, prm, syn.shape[0])
    pinned.set_osd_capacity(cap0)
    c2, f2, i2, _ = pinned.decode(s)
    torch.cuda.synchronize()
    assert (c1.cpu().numpy() == c2.cpu().numpy()).all() and (f1.cpu().numpy() == f2.cpu().numpy()).all()
    idx = np.random.default_rng(5).choice(syn.shape[0], 300, replace=False)
    o = oracle.decode(h, 0.01, oracle_params(prm), syn[idx], n_threads=8)
    assert (c1.cpu().numpy().view(np.uint32)[idx] == o["corr"]).all()
    assert (f1.cpu().numpy()[idx] == o["flags"]).all()


@pytest.mark.parametrize("name,p,shots,osd", [("surface21_phenpf", 0.002, 64, 1), ("surface25_phenpf", 0.0015, 48, 1),
                                               ("surface21_phenpf", 0.002, 32, 2)])
def test_large_surface_codes(name, p, shots, osd):
    """The paper's scale on the general kernel: surface d=21 (4840 x 13881) and d=25
    (8112 x 23425) over d rounds with the final read-out, Int3.4 bit-exact against
    the oracle, OSD-0 or OSD-CS(10) with G in global memory."""
    h, e, syn = batch(name, p, shots, 1301)
    prm = _params(msg=2, max_iter=100, lottery=True, osd=osd, osd_order=10, seed=5)
    g = gpu_decode(h, p, prm, syn, want_llr=True)
    o = oracle.decode(h, p, oracle_params(prm), syn, want_llr=True, n_threads=8)
    assert ((g["flags"] & 2) != 0).sum() >= 8
    assert (g["flags"] == o["flags"]).all()
    assert (g["iters"] == o["iters"]).all()
    assert (g["llr"] == o["llr"]).all()
    assert (g["corr"] == o["corr"]).all()
