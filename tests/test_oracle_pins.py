"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each test compares the oracle with something it does not compute: a published
generator's known answers, numpy's IEEE conversions, brute-force enumeration,
hand-derived closed forms of special cases, and the paper's worked example.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from workloads import codes, sample
from workloads.logical import LogicalChecker, wilson

M256 = 1 << 256


def numpy_philox(ctr, key):
    """numpy.random.Philox is Philox4x64-10; it increments its counter before each block."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(ctr))
    c = (c - 1) % M256
    cw = np.array([(c >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=cw)
    return [int(x) for x in g.random_raw(4)]


# ----------------------------------------------------------------------------- RNG

def test_philox_published_zero_vector():
    # Random123 known-answer vector for Philox4x64-10, counter 0 and key 0
    out = oracle.philox4x64_10([0, 0, 0, 0], [0, 0])
    assert [int(x) for x in out] == [0x16554D9ECA36314C, 0xDB20FE9D672D0FDC,
                                     0xD7E772CEE186176B, 0x7E68B68AEC7BA23B]


def test_philox_matches_numpy():
    rng = np.random.default_rng(1)
    cases = [([0, 0, 0, 0], [0, 0]), ([2**64 - 1, 0, 0, 0], [5, 9]), ([1, 2**64 - 1, 3, 4], [2**63, 1])]
    for _ in range(20):
        cases.append((list(rng.integers(0, 2**63, 4, dtype=np.uint64)),
                      list(rng.integers(0, 2**63, 2, dtype=np.uint64))))
    for ctr, key in cases:
        assert [int(x) for x in oracle.philox4x64_10(ctr, key)] == numpy_philox(ctr, key)


# ------------------------------------------------------------------ storage rounding

def test_fp16_store_matches_ieee():
    rng = np.random.default_rng(2)
    xs = np.concatenate([rng.standard_normal(3000) * 10.0 ** rng.integers(-9, 5, 3000),
                         [1 + 2**-11, 1 + 3 * 2**-11, 2**-25, 3 * 2**-25, 65504.0, 65519.9, -0.0, 6e-8]])
    for x in xs:
        ref = float(np.float16(x))
        if abs(x) >= 65520:
            ref = np.copysign(65504.0, x)
        assert oracle.store(oracle.FP16, x) == ref, x
    assert oracle.store(oracle.FP16, 1e6) == 65504.0          # saturating, never inf


def test_fp32_store_matches_ieee():
    rng = np.random.default_rng(3)
    for x in rng.standard_normal(3000) * 10.0 ** rng.integers(-30, 30, 3000):
        assert oracle.store(oracle.FP32, x) == float(np.float32(x))
    assert oracle.store(oracle.FP32, 1e300) == float(np.finfo(np.float32).max)


def test_int34_priors():
    # 16 * ln((1-p)/p) to the nearest integer, saturated at 127
    assert [oracle.prior_int8(p) for p in (0.05, 0.01, 0.003, 0.001, 1e-4)] == [47, 74, 93, 111, 127]


def test_fixed_point_priors():
    """Int x.y: 2^y ln((1-p)/p) to the nearest integer, saturated at 2^(x+y) - 1.
    ln 9 = 2.1972, ln 99 = 4.5951, ln 999 = 6.9068; 7-bit formats saturate at 63,
    8-bit ones at 127."""
    table = {(2, 4): [35, 63, 63], (3, 3): [18, 37, 55], (4, 2): [9, 18, 28], (2, 5): [70, 127, 127],
             (4, 3): [18, 37, 55], (3, 4): [35, 74, 111]}
    for (x, y), want in table.items():
        assert [oracle.prior_fixed(p, x, y) for p in (0.1, 0.01, 0.001)] == want, (x, y)
    assert oracle.prior_fixed(0.001, 3, 4) == oracle.prior_int8(0.001)


# ---------------------------------------------------------- closed-form BP schedules

def _lam_after(h, prior, prm, s_bits, iters):
    prm.max_iter = iters
    prm.early_stop = False
    prm.lottery = False
    res = oracle.decode(h, prior, prm, sample.pack_bits(np.asarray([s_bits], np.uint8)), want_llr=True)
    return res["llr"][0]


def test_sigma_schedule_two_variable_check():
    """One check on two variables, s = 1: variable a only ever hears
    beta = -sigma_i * mu_b, so lambda_a = mu_a - sigma_i mu_b after iteration i."""
    h = sp.csr_matrix(np.array([[1, 1]], dtype=np.uint8))
    pa, pb = 0.1, 0.2
    mua, mub = np.log(0.9 / 0.1), np.log(0.8 / 0.2)
    for i, sig in [(0, 0.5), (1, 0.75), (2, 0.875), (9, 1 - 2.0**-10), (23, 1 - 2.0**-24), (24, 1.0), (40, 1.0)]:
        lam = _lam_after(h, [pa, pb], oracle.OracleParams(msg=oracle.FP64), [1], i + 1)
        assert lam[0] == pytest.approx(mua - sig * mub, abs=1e-15, rel=1e-15)
        assert lam[1] == pytest.approx(mub - sig * mua, abs=1e-15, rel=1e-15)
    # constant scale
    lam = _lam_after(h, [pa, pb], oracle.OracleParams(msg=oracle.FP64, scale_mode=1, scale=0.625), [0], 3)
    assert lam[0] == pytest.approx(mua + 0.625 * mub, rel=1e-15)


def test_sigma_schedule_int34():
    """Int3.4 magnitudes: |beta| = mag - (mag >> (i+1)); constant 5/8: (5 mag) >> 3."""
    h = sp.csr_matrix(np.array([[1, 1]], dtype=np.uint8))
    qa, qb = oracle.prior_int8(0.1), oracle.prior_int8(0.2)      # 35, 22
    assert (qa, qb) == (35, 22)
    for i in range(0, 9):
        lam = _lam_after(h, [0.1, 0.2], oracle.OracleParams(msg=oracle.INT8), [1], i + 1)
        assert lam[0] == qa - (qb - (qb >> (i + 1)))
        assert lam[1] == qb - (qa - (qa >> (i + 1)))
    lam = _lam_after(h, [0.1, 0.2], oracle.OracleParams(msg=oracle.INT8, scale_mode=1, scale=0.625), [1], 2)
    assert lam[0] == 35 - ((5 * 22) >> 3) and lam[1] == 22 - ((5 * 35) >> 3)


@pytest.mark.parametrize("fx", [(2, 4), (3, 3), (4, 3)])
def test_sigma_schedule_fixed_point(fx):
    """The Int3.4 schedule in other formats, with the 7-bit saturation at 63: one
    check on two variables (s = 1), lambda_a = q_a - (q_b - (q_b >> (i+1)))."""
    x, y = fx
    h = sp.csr_matrix(np.array([[1, 1]], dtype=np.uint8))
    qa, qb = oracle.prior_fixed(0.001, x, y), oracle.prior_fixed(0.1, x, y)   # 63/35, 55/18, 55/18
    for i in range(0, 8):
        lam = _lam_after(h, [0.001, 0.1], oracle.OracleParams(msg=oracle.INT8, fx_int=x, fx_frac=y), [1], i + 1)
        assert lam[0] == qa - (qb - (qb >> (i + 1)))
        assert lam[1] == qb - (qa - (qa >> (i + 1)))


@pytest.mark.parametrize("fx,qmax", [((3, 4), 127), ((3, 3), 63), ((2, 4), 63), ((1, 1), 3)])
def test_degree_one_check_sends_the_format_maximum(fx, qmax):
    """A check on one variable has no other input: it sends the largest magnitude
    of the format, scaled, with the sign of the syndrome bit:
    lambda = q - (qmax - (qmax >> 1)) after one iteration with s = 1."""
    x, y = fx
    h = sp.csr_matrix(np.array([[1]], dtype=np.uint8))
    q = oracle.prior_fixed(0.3, x, y)
    lam = _lam_after(h, [0.3], oracle.OracleParams(msg=oracle.INT8, fx_int=x, fx_frac=y), [1], 1)
    assert lam[0] == q - (qmax - (qmax >> 1))
    lam = _lam_after(h, [0.3], oracle.OracleParams(msg=oracle.INT8, fx_int=x, fx_frac=y), [0], 1)
    assert lam[0] == q + (qmax - (qmax >> 1))


def test_fixed_point_rejects_unsupported_formats():
    h = sp.csr_matrix(np.array([[1, 1]], dtype=np.uint8))
    syn = sample.pack_bits(np.asarray([[1]], np.uint8))
    for x, y in [(4, 4), (0, 0 + 8), (-1, 3)]:
        with pytest.raises(ValueError):
            oracle.decode(h, 0.1, oracle.OracleParams(msg=oracle.INT8, fx_int=x, fx_frac=y), syn)


# -------------------------------------------------------------- exactness on trees

def _random_tree(rng, n_target):
    """Bipartite tree: each new check joins one existing variable to 1-3 new ones."""
    rows = []
    n = 1
    while n < n_target:
        k = int(min(rng.integers(1, 4), n_target - n))
        anchor = int(rng.integers(0, n))
        rows.append([anchor] + list(range(n, n + k)))
        n += k
    data = [(r, c) for r, row in enumerate(rows) for c in row]
    h = sp.csr_matrix((np.ones(len(data), np.uint8), ([a for a, _ in data], [b for _, b in data])),
                      shape=(len(rows), n))
    h.sort_indices()
    return h


def _max_marginals(h, mu, s):
    """lambda_v = min cost with e_v = 1 minus min cost with e_v = 0, over He = s (brute force)."""
    hd = h.toarray().astype(np.int64)
    n = hd.shape[1]
    es = np.array(list(itertools.product([0, 1], repeat=n)), dtype=np.int64)
    ok = ((es @ hd.T) % 2 == s).all(axis=1)
    es = es[ok]
    cost = es @ mu
    out = np.empty(n)
    for v in range(n):
        out[v] = cost[es[:, v] == 1].min() - cost[es[:, v] == 0].min()
    return out


@pytest.mark.parametrize("seed", range(8))
def test_min_sum_is_exact_max_product_on_trees(seed):
    rng = np.random.default_rng(100 + seed)
    h = _random_tree(rng, int(rng.integers(5, 13)))
    m, n = h.shape
    p = rng.uniform(0.02, 0.3, n)
    mu = np.log((1 - p) / p)
    s = rng.integers(0, 2, m)
    lam = _lam_after(h, p, oracle.OracleParams(msg=oracle.FP64, scale_mode=1, scale=1.0), s, 2 * (n + m))
    np.testing.assert_allclose(lam, _max_marginals(h, mu, s), rtol=0, atol=1e-9)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("fx", [(3, 4), (3, 3), (2, 4)])
def test_int34_min_sum_is_exact_on_trees(seed, fx):
    """Integer min-sum on a tree is max-product exactly, in every Int x.y format
    (priors small enough that no sum saturates)."""
    x, y = fx
    rng = np.random.default_rng(200 + seed)
    h = _random_tree(rng, int(rng.integers(4, 9)))
    m, n = h.shape
    p = rng.uniform(0.36, 0.45, n)                              # priors 3..9 in Int3.4: no saturation
    muq = np.array([oracle.prior_fixed(v, x, y) for v in p], dtype=np.int64)
    s = rng.integers(0, 2, m)
    lam = _lam_after(h, p, oracle.OracleParams(msg=oracle.INT8, scale_mode=1, scale=1.0, fx_int=x, fx_frac=y), s,
                     2 * (n + m))
    assert (lam == _max_marginals(h, muq, s)).all()


# ------------------------------------------------------------- the worked example

@pytest.mark.parametrize("p", [0.01, 0.05, 0.1])
def test_worked_example_deadlock_and_lottery(p):
    """Fig. 4: errors {q2,q8,q9} deadlock plain NMS BP; Lottery BP breaks the tie."""
    h = codes.worked_example_h()
    e = np.zeros((1, 13), np.uint8)
    e[0, [2, 8, 9]] = 1
    syn = sample.pack_bits(sample.syndromes(h, sp.csr_matrix(e)))
    for msg in (oracle.FP64, oracle.FP32, oracle.INT8):
        plain = oracle.decode(h, p, oracle.OracleParams(max_iter=100, msg=msg, lottery=False), syn)
        assert plain["flags"][0] & oracle.FLAG_CONVERGED == 0
    sols = set()
    for seed in range(50):
        r = oracle.decode(h, p, oracle.OracleParams(max_iter=100, msg=oracle.FP64, seed=seed), syn,
                          first_shot_id=seed)
        assert r["flags"][0] & oracle.FLAG_CONVERGED
        est = sample.unpack_bits(r["corr"], 13)[0]
        assert (sample.syndromes(h, sp.csr_matrix(est[None]))[0] == sample.syndromes(h, sp.csr_matrix(e))[0]).all()
        sols.add(tuple(np.nonzero(est)[0]))
    assert sols <= {(2, 8, 9), (1, 3, 8)}                       # the two degenerate weight-3 solutions


# ----------------------------------------------------------- the lottery selection

def test_lottery_selection_hand_traced():
    """Checks: c0={0,1,2}, c1={1,3}, c2={2,3,4,5}, c3={5,6}; U = {c0,c1,c2}.
    Unsatisfied-neighbour counts and |lambda| (quantized to 2^-12) give:
      c* = c0 -> candidates {1,2} (count 2); |l1| = 1.5 > |l2| -> v* = 2
      c* = c1 -> candidates {1,3}; |l3| < |l1| -> v* = 3
      c* = c2 -> candidates {2,3} (4 and 5 see one unsatisfied check); |l2|, |l3| quantize
                 to the same level -> smaller column -> v* = 2 although |l3| < |l2|."""
    rows = [[0, 1, 2], [1, 3], [2, 3, 4, 5], [5, 6]]
    data = [(r, c) for r, row in enumerate(rows) for c in row]
    h = sp.csr_matrix((np.ones(len(data), np.uint8), ([a for a, _ in data], [b for _, b in data])), shape=(4, 7))
    s = [1, 0, 1, 0]
    sprev = [0, 1, 0, 0]                                        # U = {0, 1, 2}
    lam = [5.0, -1.5, 1.0002, 1.0001, 0.1, 0.2, 3.0]
    expect = {0: 2, 1: 3, 2: 2}
    seen = set()
    for shot in range(3):
        x = numpy_philox([shot, 7, 0, 0], [123, 0])[0]
        k = ((x >> 32) * 3) >> 32                               # floor(r N), r = (x >> 32) / 2^32
        seen.add(k)
        assert oracle.lottery_pick(h, 123, shot, 7, s, sprev, lam) == expect[k]
    assert seen == {0, 1, 2}
    # Int3.4 compares |lambda| itself
    assert oracle.lottery_pick(h, 123, 1, 7, s, sprev, [5, -3, 2, 2, 1, 1, 3], is_int8=True) == 3
    assert oracle.lottery_pick(h, 123, 0, 7, s, sprev, [5, -3, 2, 2, 1, 1, 3], is_int8=True) == 2
    assert oracle.lottery_pick(h, 123, 0, 7, s, sprev, [5, -3, 3, 2, 1, 1, 3], is_int8=True) == 1  # tie


def _pin_graph():
    rows = [[0, 1, 2], [1, 3], [2, 3, 4, 5], [5, 6]]
    data = [(r, c) for r, row in enumerate(rows) for c in row]
    return rows, sp.csr_matrix((np.ones(len(data), np.uint8), ([a for a, _ in data], [b for _, b in data])),
                               shape=(4, 7))


def test_lottery_worst_check_rule():
    """Worst check (Sec. III-B): among U, the check with the most neighbours in the
    current hard decision; checks outside U never count; equal counts -> smaller index.
    Same graph as above, U = {c0, c1, c2}; the VN rule then picks inside that check."""
    rows, h = _pin_graph()
    s, sprev = [1, 0, 1, 0], [0, 1, 0, 0]
    lam = [5.0, -1.5, 1.0002, 1.0001, 0.1, 0.2, 3.0]
    worst = oracle.policy_code(cn=oracle.CN_WORST)
    unrel = oracle.policy_code(cn=oracle.CN_WORST, vn=oracle.VN_UNRELIABLE)
    cases = [([0, 1, 0, 1, 1, 1, 0], 2),    # c0:1 c1:2 c2:3
             ([1, 1, 0, 0, 0, 0, 0], 0),    # c0:2 c1:1 c2:0
             ([0, 1, 0, 0, 0, 0, 0], 0),    # c0:1 c1:1 -> smaller index
             ([0, 0, 0, 0, 0, 1, 1], 2),    # c3 has two but is satisfied; c2:1
             ([0, 0, 0, 0, 0, 0, 0], 0)]    # all zero -> first check of U
    # the proposed key inside each check (counts: col 1,2,3 see two checks of U)
    vn_in = {0: 2, 1: 3, 2: 2}
    # unreliable inside each check: smallest quantized |lambda|, then column
    unrel_in = {0: 2, 1: 3, 2: 4}
    for ehat, c in cases:
        for shot in range(4):               # the draw must not matter
            assert oracle.lottery_pick(h, 9, shot, 7, s, sprev, lam, policy=worst, ehat=ehat) == vn_in[c]
            assert oracle.lottery_pick(h, 9, shot, 7, s, sprev, lam, policy=unrel, ehat=ehat) == unrel_in[c]


def test_lottery_neighbour_rules():
    """The neighbour rules on c2 = {2,3,4,5} with U = all four checks, so the
    unsatisfied counts of columns 2..5 are 2, 2, 1, 2 (c3 now counts for column 5):
      A: Q = 4096, 2048, 204, 409 -> proposed (count, then Q) picks 5; Q-first and
         unreliable pick 4 (smallest Q).
      B: Q = 4096, 2048, 409, 409 -> proposed 5; Q-first breaks the Q tie by the
         larger count -> 5; unreliable breaks it by the smaller column -> 4.
    Worst-check rule with ehat on columns 3,4,5 fixes c* = c2."""
    rows, h = _pin_graph()
    s, sprev = [1, 0, 1, 0], [0, 1, 0, 1]
    ehat = [0, 0, 0, 1, 1, 1, 0]
    lam_a = [5.0, -1.5, 1.0, 0.5, 0.05, 0.1, 3.0]
    lam_b = [5.0, -1.5, 1.0, 0.5, 0.1, -0.1, 3.0]
    expect = {oracle.VN_PROPOSED: (5, 5), oracle.VN_Q_FIRST: (4, 5), oracle.VN_UNRELIABLE: (4, 4)}
    for vn, (ea, eb) in expect.items():
        pol = oracle.policy_code(cn=oracle.CN_WORST, vn=vn)
        assert oracle.lottery_pick(h, 5, 0, 9, s, sprev, lam_a, policy=pol, ehat=ehat) == ea
        assert oracle.lottery_pick(h, 5, 0, 9, s, sprev, lam_b, policy=pol, ehat=ehat) == eb
    # Int3.4: the same comparisons on |lambda| itself
    pol = oracle.policy_code(cn=oracle.CN_WORST, vn=oracle.VN_Q_FIRST)
    assert oracle.lottery_pick(h, 5, 0, 9, s, sprev, [80, -24, 16, 8, 2, -2, 48], is_int8=True,
                               policy=pol, ehat=ehat) == 5
    pol = oracle.policy_code(cn=oracle.CN_WORST, vn=oracle.VN_UNRELIABLE)
    assert oracle.lottery_pick(h, 5, 0, 9, s, sprev, [80, -24, 16, 8, 2, -2, 48], is_int8=True,
                               policy=pol, ehat=ehat) == 4


def test_lottery_random_neighbour_draw():
    """Random neighbour: word 1 of the same Philox block, r1 = (w1 >> 32) / 2^32,
    picks column floor(r1 deg) of the check in ascending order; the check comes from
    word 0 (random rule) or from the worst-check rule.  Every neighbour must occur."""
    rows, h = _pin_graph()
    s, sprev = [1, 0, 1, 0], [0, 1, 0, 0]
    lam = [5.0, -1.5, 1.0002, 1.0001, 0.1, 0.2, 3.0]
    seen = set()
    for shot in range(64):
        w = numpy_philox([shot, 4, 0, 0], [77, 0])
        c = [0, 1, 2][((w[0] >> 32) * 3) >> 32]
        v = rows[c][((w[1] >> 32) * len(rows[c])) >> 32]
        seen.add(v)
        pol = oracle.policy_code(cn=oracle.CN_RANDOM, vn=oracle.VN_RANDOM)
        assert oracle.lottery_pick(h, 77, shot, 4, s, sprev, lam, policy=pol) == v
        ehat = [0, 0, 0, 1, 1, 1, 0]                              # worst check c2
        v2 = rows[2][((w[1] >> 32) * 4) >> 32]
        pol = oracle.policy_code(cn=oracle.CN_WORST, vn=oracle.VN_RANDOM)
        assert oracle.lottery_pick(h, 77, shot, 4, s, sprev, lam, policy=pol, ehat=ehat) == v2
    assert seen == {0, 1, 2, 3, 4, 5}
    # no unsatisfied check: no flip under every rule
    for pol in range(0, 0x40, 0x10):
        for cn in (0, 1):
            assert oracle.lottery_pick(h, 77, 0, 4, s, s, lam, policy=pol | cn, ehat=[1] * 7) == -1


@pytest.mark.parametrize("msg", [oracle.FP64, oracle.INT8])
def test_lottery_policies_keep_decoder_outputs_valid(msg):
    """Every rule runs through the whole decoder: a shot flagged converged has a
    correction whose syndrome matches, and each rule other than the proposed one
    changes some shot's iteration count (so the policy reaches the lottery)."""
    h, _, _ = codes.workload_matrices("bb144_cc")
    _, syn = sample.make_batch(h, 0.05, 96, seed=11)
    n = h.shape[1]
    base = None
    for pol in [0, 0x01, 0x10, 0x20, 0x30, 0x21]:
        r = oracle.decode(h, 0.05, oracle.OracleParams(max_iter=40, msg=msg, policy=pol, seed=2), syn)
        corr = sample.unpack_bits(r["corr"], n)
        ok = (r["flags"] & oracle.FLAG_CONVERGED) != 0
        assert ok.sum() > 10
        assert np.array_equal(sample.pack_bits((corr[ok].astype(np.int64) @ h.T.toarray()) % 2), syn[ok])
        if base is None:
            base = r["iters"]
        else:
            assert not np.array_equal(r["iters"], base), pol


# ------------------------------------------------------------------------ OSD

def _span_rank(cols):
    """GF(2) rank by enumerating the span of the given column vectors."""
    span = {0}
    for c in cols:
        v = int("".join(map(str, c)), 2)
        span |= {x ^ v for x in span}
    return int(np.log2(len(span)))


def _brute_solve(hS, rhs):
    sols = [e for e in itertools.product([0, 1], repeat=hS.shape[1])
            if ((hS @ np.array(e, dtype=np.int64)) % 2 == rhs).all()]
    return sols


def _brute_osd(hd, lam, s, order, cs):
    m, n = hd.shape
    pi = np.lexsort((np.arange(n), lam))
    S = []
    for j in pi:
        if _span_rank([hd[:, c] for c in S + [j]]) > len(S):
            S.append(int(j))
    T = [int(j) for j in pi if j not in S]
    cands = [()]
    if cs:
        cands += [(t,) for t in T] + [(T[a], T[b]) for a in range(min(order, len(T)))
                                       for b in range(a + 1, min(order, len(T)))]
    best, best_cost = None, None
    for t in cands:
        rhs = (s + hd[:, list(t)].sum(axis=1)) % 2 if t else s % 2
        sols = _brute_solve(hd[:, S], rhs)
        if not sols:
            return None
        assert len(sols) == 1                                   # unique on the basis
        cost = sum(sols[0]) + len(t)
        if best_cost is None or cost < best_cost:
            best_cost = cost
            e = np.zeros(n, np.uint8)
            e[S] = sols[0]
            e[list(t)] = 1
            best = e
    return best


@pytest.mark.parametrize("seed", range(30))
def test_osd_matches_brute_force(seed):
    rng = np.random.default_rng(300 + seed)
    m, n = int(rng.integers(3, 7)), int(rng.integers(6, 12))
    hd = (rng.random((m, n)) < 0.35).astype(np.int64)
    hd[:, 0] |= 0
    for r in range(m):
        if not hd[r].any():
            hd[r, rng.integers(0, n)] = 1
    h = sp.csr_matrix(hd.astype(np.uint8))
    lam = np.round(rng.normal(0, 2, n), 1)                      # rounding creates ties
    if seed % 3 == 0:
        e = (rng.random(n) < 0.3).astype(np.int64)
        s = hd @ e % 2                                          # consistent
    else:
        s = rng.integers(0, 2, m)                               # may be inconsistent
    syn = sample.pack_bits(s[None].astype(np.uint8))[0]
    for mode, order in ((oracle.OSD_0, 0), (oracle.OSD_CS, 3), (oracle.OSD_CS, 10)):
        corr, flag = oracle.osd(h, lam, syn, mode, order)
        ref = _brute_osd(hd, lam, s, order, mode == oracle.OSD_CS)
        if ref is None:
            assert flag & oracle.FLAG_OSD_INCONSISTENT
        else:
            assert not flag & oracle.FLAG_OSD_INCONSISTENT
            got = sample.unpack_bits(corr[None], n)[0]
            assert (got == ref).all()
            assert ((hd @ got) % 2 == s).all()                  # H e = s


def test_osd_cs_never_worse_than_osd0():
    h, _, _ = codes.workload_matrices("bb144_cc")
    e, syn = sample.make_batch(h, 0.06, 60, seed=9)
    rng = np.random.default_rng(4)
    for k in range(60):
        lam = rng.normal(2, 2, 144)
        c0, f0 = oracle.osd(h, lam, syn[k], oracle.OSD_0)
        c1, f1 = oracle.osd(h, lam, syn[k], oracle.OSD_CS, 10)
        assert f0 == f1 == oracle.FLAG_OSD
        w0 = sample.unpack_bits(c0[None], 144).sum()
        w1 = sample.unpack_bits(c1[None], 144).sum()
        assert w1 <= w0


def test_rank_deficient_inconsistent_syndrome_flags():
    """BB144 code capacity: H_X has rank 66 < 72, so some syndromes are not H e for any e."""
    h, _, _ = codes.workload_matrices("bb144_cc")
    hd = h.toarray().astype(np.int64)
    null_left = codes.gf2_nullspace(hd.T)                       # y with y H = 0
    assert null_left.shape[0] == 6
    rng = np.random.default_rng(5)
    bad = []
    while len(bad) < 5:
        s = rng.integers(0, 2, 72)
        if ((null_left @ s) % 2).any():
            bad.append(s)
    syn = sample.pack_bits(np.array(bad, np.uint8))
    prm = oracle.OracleParams(max_iter=20, msg=oracle.FP32, osd=oracle.OSD_0)
    r = oracle.decode(h, 0.01, prm, syn)
    assert (r["flags"] == oracle.FLAG_OSD | oracle.FLAG_OSD_INCONSISTENT).all()
    prm.osd = oracle.OSD_NONE
    r2 = oracle.decode(h, 0.01, prm, syn)
    assert (r2["corr"] == r["corr"]).all()                      # BP hard decision is kept


def test_osd_outputs_satisfy_syndrome():
    h, _, _ = codes.workload_matrices("bb144_phen")
    e, syn = sample.make_batch(h, 0.003, 64, seed=11)
    for osd_mode in (oracle.OSD_0, oracle.OSD_CS):
        r = oracle.decode(h, 0.003, oracle.OracleParams(max_iter=1, msg=oracle.INT8, osd=osd_mode), syn,
                          n_threads=4)
        est = sample.unpack_bits(r["corr"], h.shape[1])
        sh = sample.pack_bits(sample.syndromes(h, sp.csr_matrix(est)))
        osd_done = (r["flags"] & oracle.FLAG_OSD) > 0
        assert osd_done.sum() > 10
        assert (sh[osd_done] == syn[osd_done]).all()


# ----------------------------------------------- the whole decoder vs maximum likelihood

def _d3_enumeration(p):
    h, hc, _ = codes.workload_matrices("surface3_cc")
    hd = h.toarray().astype(np.int64)
    errs = np.array(list(itertools.product([0, 1], repeat=9)), dtype=np.int64)
    w = errs.sum(axis=1)
    prob = p**w * (1 - p) ** (9 - w)
    synd = errs @ hd.T % 2
    logical = codes.gf2_nullspace(hc.toarray())                 # ker(H_X): stabilizers + logical Z
    cls = ((errs @ logical.T) % 2 != 0).astype(np.int64) @ (1 << np.arange(logical.shape[0]))
    return h, hd, errs, prob, synd, cls


def test_decoder_not_better_than_maximum_likelihood():
    """d=3 rotated code, code capacity, all 2^9 errors: exact LER of the decoder
    (deterministic: every syndrome decoded with the same lottery key) >= exact ML LER."""
    p = 0.05
    h, hd, errs, prob, synd, cls = _d3_enumeration(p)
    keys = [tuple(s) for s in synd]
    uniq = sorted(set(keys))
    syn = sample.pack_bits(np.array(uniq, np.uint8))
    prm = oracle.OracleParams(max_iter=50, msg=oracle.FP64, osd=oracle.OSD_0, seed=3)
    corr = np.stack([oracle.decode(h, p, prm, syn[k:k + 1])["corr"][0] for k in range(len(uniq))])
    est = {u: sample.unpack_bits(corr[k:k + 1], 9)[0].astype(np.int64) for k, u in enumerate(uniq)}
    hc = codes.workload_matrices("surface3_cc")[1].toarray()
    logical = codes.gf2_nullspace(hc)
    ler_dec = 0.0
    ml = {}
    for e, pr, key, c in zip(errs, prob, keys, cls):
        r = (e + est[key]) % 2
        assert ((hd @ r) % 2 == 0).all()                        # OSD / BP output satisfies s
        if ((logical @ r) % 2).any():
            ler_dec += pr
        ml.setdefault(key, {}).setdefault(c, 0.0)
        ml[key][c] += pr
    ler_ml = sum(sum(v.values()) - max(v.values()) for v in ml.values())
    assert ler_dec >= ler_ml - 1e-15
    assert ler_ml > 0


def test_monte_carlo_ler_agrees_with_enumeration():
    """Sampler + logical check vs exact enumeration of the same deterministic decoder."""
    p = 0.05
    h, hd, errs, prob, synd, cls = _d3_enumeration(p)
    hx, hz = codes.rotated_surface(3)
    prm = oracle.OracleParams(max_iter=50, msg=oracle.FP64, osd=oracle.OSD_0, seed=3, lottery=False)
    uniq = sorted(set(tuple(s) for s in synd))
    table = {}
    for u in uniq:
        table[u] = oracle.decode(h, p, prm, sample.pack_bits(np.array([u], np.uint8)))["corr"][0]
    chk = LogicalChecker(hz, hx, 1)
    corr_all = np.stack([table[tuple(s)] for s in synd])
    sf, lf = chk.failures(sp.csr_matrix(errs.astype(np.uint8)), corr_all, 9)
    exact = float((prob * (sf | lf)).sum())
    shots = 200_000
    e, syn = sample.make_batch(h, p, shots, seed=77)
    r = oracle.decode(h, p, prm, syn, n_threads=4)
    sf, lf = chk.failures(e, r["corr"], 9)
    k = int((sf | lf).sum())
    lo, hi = wilson(k, shots, z=3.5)
    assert lo <= exact <= hi, (k / shots, exact)
