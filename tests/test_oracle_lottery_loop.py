"""Pins of the lottery inside the BP loop, the LLR-flip arithmetic and the
saturation of alpha in Int x.y, against hand-derived trajectories.

Every expected value below is worked out by hand in the comments (tiny graphs,
no early stop), not recomputed by a formula in the test.  Together they fix:
  * when the lottery runs: after iterations K..I-2, 0-based (Sec. III-B skips
    the first K = 6 iterations; Algorithm 3 runs after the termination test);
  * that U is built from the previous iteration's syndrome estimate (Algorithm
    3 and the delayed-syndrome selector of Sec. IV-B), with the estimate before
    iteration 0 equal to H * 0 = 0 (the hard decision of the prior);
  * that the message flip negates the V2C messages of v* for exactly one
    check-node update (the sign-flip stage in front of the CNU, Sec. IV-B);
  * that the LLR flip negates lambda_v* before the next VN update, whose
    alpha = lambda - beta then reads -lambda - beta (Algorithm 3, last step);
  * that alpha saturates at +-qmax = +-(2^(x+y) - 1) in Int x.y (Sec. VII-A)
    before the check-node minimum.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from workloads import sample


def _trajectory(h, prior, s_bits, upto, **kw):
    """lambda^(j) for j = 0..upto: a run of j+1 iterations without early stop
    returns the lambda of its last iteration (the lottery never runs after the
    last one, so lambda^(j) is the same as in any longer run)."""
    syn = sample.pack_bits(np.asarray([s_bits], np.uint8))
    out = []
    for j in range(upto + 1):
        prm = oracle.OracleParams(max_iter=j + 1, early_stop=False, **kw)
        out.append(oracle.decode(h, prior, prm, syn, want_llr=True)["llr"][0])
    return np.array(out)


# One check on two columns, s = 1, both priors p = 0.003 (Int3.4: mu_q = 93).
# Each column sits in this check only, so its extrinsic sum is its prior:
# alpha = (93, 93) in every iteration without a flip, and the check answers
# each column with beta = -sigma_i(93) (s = 1, no negative input), where
# sigma_i(x) = x - (x >> (i+1)).  So lambda = 93 - sigma_i(93) = 93 >> (i+1):
# 46, 23, 11, 5, 2, 1, then 0 from i = 6 on.  The hard decision is (0,0) while
# lambda > 0 and (1,1) at lambda = 0; both give H e = 0 != s: plain BP is
# stuck for ever (a degenerate pair of weight-1 columns).
PAIR = sp.csr_matrix(np.array([[1, 1]], np.uint8))
PLAIN_INT = [(46, 46), (23, 23), (11, 11), (5, 5), (2, 2), (1, 1)] + [(0, 0)] * 9


def test_plain_bp_deadlocks_on_the_pair():
    t = _trajectory(PAIR, 0.003, [1], 14, msg=oracle.INT8, lottery=False)
    assert [tuple(int(x) for x in r) for r in t] == PLAIN_INT


def test_lottery_starts_after_iteration_k_and_flips_one_update():
    """K = 6, message flip.
    * i <= 6: no lottery has acted yet -> identical to plain BP (pins that the
      first lottery runs at the end of iteration K, not K-1).
    * end of i = 6: U = {c0} (estimate of i = 5 is 0 != 1); both columns see
      one unsatisfied check and |lambda| = 0 -> smaller column: v* = 0.
      i = 7: alpha = (-93, 93); parity 1; beta_0 = -(93 - (93 >> 8)) = -93,
      beta_1 = +93 -> lambda^(7) = (0, 186): e = (1, 0), H e = 1 = s.
    * end of i = 7: U uses the estimate of i = 6 (0 != s) -> flip again:
      lambda^(8) = (0, 186).  (With the estimate of i = 7, U would be empty
      and lambda^(8) would be (0, 0): this pins the delayed syndrome.)
    * end of i = 8: estimate of i = 7 equals s -> U empty, no flip:
      lambda^(9) = (0, 0) (pins that a flip lasts one CN update).
    * end of i = 9: estimate of i = 8 = s -> no flip: lambda^(10) = (0, 0).
    * end of i = 10: estimate of i = 9 is 0 -> flip: lambda^(11) = (0, 186);
      the pattern repeats with period 4."""
    t = _trajectory(PAIR, 0.003, [1], 14, msg=oracle.INT8, lottery=True, lottery_skip=6)
    flip = (0, 186)
    want = PLAIN_INT[:7] + [flip, flip, (0, 0), (0, 0), flip, flip, (0, 0), (0, 0)]
    assert [tuple(int(x) for x in r) for r in t] == want


def test_lottery_converged_shot_reports_the_flipped_iteration():
    """With early stop, the same shot converges in iteration 7: 8 iterations,
    correction e = (1, 0) (the flipped column is the error)."""
    syn = sample.pack_bits(np.asarray([[1]], np.uint8))
    r = oracle.decode(PAIR, 0.003, oracle.OracleParams(max_iter=50, msg=oracle.INT8, lottery_skip=6), syn)
    assert r["flags"][0] & oracle.FLAG_CONVERGED
    assert r["iters"][0] == 8
    assert sample.unpack_bits(r["corr"], 2)[0].tolist() == [1, 0]


def test_lottery_skip_zero_uses_the_all_zero_previous_estimate():
    """K = 0: the lottery after iteration 0 takes U from the estimate before
    iteration 0, H * 0 = 0 != s -> U = {c0}; lambda^(0) = (46, 46) -> v* = 0.
    i = 1: alpha = (-93, 93), beta magnitudes sigma_1(93) = 93 - 23 = 70:
    beta_0 = -70 (s=1, parity 1, own sign negative), beta_1 = +70 ->
    lambda^(1) = (23, 163).  End of i = 1: estimate of i = 0 is 0 -> U = {c0};
    |lambda| 23 < 163 -> v* = 0 again: i = 2, sigma_2(93) = 93 - 11 = 82 ->
    lambda^(2) = (11, 175)."""
    t = _trajectory(PAIR, 0.003, [1], 2, msg=oracle.INT8, lottery=True, lottery_skip=0)
    assert [tuple(int(x) for x in r) for r in t] == [(46, 46), (23, 163), (11, 175)]


def test_llr_flip_reads_minus_lambda_minus_beta():
    """K = 5, LLR flip.  End of i = 5: lambda^(5) = (1, 1), U = {c0}, equal
    counts and |lambda| -> v* = 0; lambda_0 := -1.
    i = 6 uses alpha = lambda - beta^(5) with beta^(5) = -(93 - (93 >> 6)) = -92:
    alpha_0 = -1 + 92 = 91 (the flipped lambda), alpha_1 = 1 + 92 = 93.
    Check: parity 0, s = 1 -> every beta negative; sigma_6(x) = x - (x >> 7) = x
    for x < 128: beta_0 = -93 (from alpha_1), beta_1 = -91 (from alpha_0)
    -> lambda^(6) = mu + beta = (0, 2).  Without the flip alpha_0 would be 93
    and lambda^(6) = (0, 0); a message flip (alpha_0 = -93) would give
    lambda^(6) = (0, 186).
    End of i = 6: U = {c0}, |lambda| 0 < 2 -> v* = 0, and -0 = 0: i = 7 reads
    alpha = (0 + 93, 2 + 91) = (93, 93) -> lambda^(7) = (0, 0)."""
    t = _trajectory(PAIR, 0.003, [1], 7, msg=oracle.INT8, lottery=True, lottery_skip=5, flip=oracle.FLIP_LLR)
    assert [tuple(int(x) for x in r) for r in t] == PLAIN_INT[:6] + [(0, 2), (0, 0)]
    t = _trajectory(PAIR, 0.003, [1], 6, msg=oracle.INT8, lottery=True, lottery_skip=5, flip=oracle.FLIP_MSG)
    assert tuple(int(x) for x in t[6]) == (0, 186)


def test_float_lottery_trajectory_in_closed_form():
    """The float loop (FP64) on the same pair, K = 6.  mu = ln(997/3); without a
    flip lambda = mu - sigma_i mu = mu 2^-(i+1) (sigma_i = 1 - 2^-(i+1) exactly
    in fp32 for i < 24), above tau = 2^-12 while mu 2^-(i+1) > 2^-12, i.e.
    until i = 13: e = (0, 0), estimate 0 != s.
    From the end of i = 6 the lottery flips v* = 0 (smaller |lambda|, then
    smaller column): alpha = (-mu, mu), beta = (-sigma mu, +sigma mu) ->
    lambda^(i) = (mu 2^-(i+1), mu (2 - 2^-(i+1))) for i = 7..15, the estimate
    staying 0 until i = 14 (mu 2^-15 <= 2^-12 -> e = (1, 0), estimate = s).
    End of i = 14 still flips (estimate of i = 13 is 0); end of i = 15 does
    not (estimate of i = 14 = s): lambda^(16) = mu 2^-17 (1, 1) -> e = (1, 1),
    estimate 0.  End of i = 16: estimate of i = 15 = s -> no flip:
    lambda^(17) = mu 2^-18 (1, 1).  End of i = 17: estimate of 16 is 0 ->
    flips at i = 18 and i = 19; none at i = 20."""
    mu = np.log(997 / 3)
    t = _trajectory(PAIR, 0.003, [1], 20, msg=oracle.FP64, lottery=True, lottery_skip=6)
    flipped = {7, 8, 9, 10, 11, 12, 13, 14, 15, 18, 19}
    for i in range(21):
        lo = mu * 2.0 ** -(i + 1)
        want = (lo, 2 * mu - lo) if i in flipped else (lo, lo)
        # mu - sigma mu cancels: the small value carries a few ulps of mu (~1e-15)
        np.testing.assert_allclose(t[i], want, rtol=1e-13, atol=1e-14, err_msg=f"iteration {i}")


# Saturation of alpha.  A star: column 0 in three checks {0,k}, k = 1..3, s = 0,
# every prior p.  Iteration 0: alpha = mu everywhere, beta = sigma_0(mu) =
# mu - (mu >> 1) on every edge.  Iteration 1: column 0 sends check k its
# extrinsic sum mu + 2 beta, which exceeds qmax, so it is sent as qmax; column k
# (in one check only) then receives sigma_1(qmax) = qmax - (qmax >> 2), and
# lambda^(1)_k = mu + qmax - (qmax >> 2).  Unsaturated it would be
# mu + (mu + 2 beta) - ((mu + 2 beta) >> 2).
STAR = sp.csr_matrix(np.array([[1, 1, 0, 0], [1, 0, 1, 0], [1, 0, 0, 1]], np.uint8))


@pytest.mark.parametrize("fx,p,expect", [
    # Int3.4, mu 93 (qmax 127): beta^(0) 47, lambda^(0) = (93+141, 140) = (234, 140);
    # alpha_0 = 93 + 94 = 187 -> 127, sigma_1(127) = 96 -> lambda_k = 189
    # (unsaturated: 187 - 46 = 141 -> 234); column 0: 93 + 3 (93 - 23) = 303.
    ((3, 4), 0.003, [(234, 140), (303, 189)]),
    # Int3.3, mu rne(8 * 5.806) = 46 (qmax 63): beta^(0) 23, lambda^(0) = (115, 69);
    # alpha_0 = 92 -> 63, sigma_1(63) = 48 -> 94 (unsaturated 92 - 23 = 69 -> 115); 46 + 3*35 = 151.
    ((3, 3), 0.003, [(115, 69), (151, 94)]),
    # Int2.4, mu rne(16 * 5.806) = 93 -> 63 (qmax 63): beta^(0) 32, lambda^(0) = (159, 95);
    # alpha_0 = 127 -> 63, sigma_1(63) = 48 -> 111; 63 + 3*48 = 207.
    ((2, 4), 0.003, [(159, 95), (207, 111)]),
    # Int4.3 at p = 1e-4, mu rne(8 * 9.21) = 74 (qmax 127): beta^(0) 37, lambda^(0) = (185, 111);
    # alpha_0 = 148 -> 127, sigma_1(127) = 96 -> 170 (unsaturated 148 - 37 = 111 -> 185); 74 + 3*56 = 242.
    ((4, 3), 1e-4, [(185, 111), (242, 170)]),
])
def test_alpha_saturates_at_qmax(fx, p, expect):
    t = _trajectory(STAR, p, [0, 0, 0], 1, msg=oracle.INT8, lottery=False, fx_int=fx[0], fx_frac=fx[1])
    for i, (l0, lk) in enumerate(expect):
        assert [int(x) for x in t[i]] == [l0, lk, lk, lk], f"iteration {i}"


# Negative saturation: column 0 (p = 0.45) in four checks {0,k} with s = 1 and
# p = 0.003 on the columns k.  Iteration 0: beta to column 0 is -sigma_0(mu_k),
# to column k -sigma_0(mu_0).  Iteration 1: column 0 sends mu_0 - 3 sigma_0(mu_k),
# below -qmax where the format saturates; each check then has parity 1, so
# column k receives +sigma_1(|alpha_0|).
FAN = sp.csr_matrix(np.array([[1, 1, 0, 0, 0], [1, 0, 1, 0, 0], [1, 0, 0, 1, 0], [1, 0, 0, 0, 1]], np.uint8))


@pytest.mark.parametrize("fx,expect", [
    # Int3.4: mu_0 = rne(16 * 0.2007) = 3, mu_k = 93.  i=0: beta_0 = -47, beta_k = -(3 - 1) = -2:
    # lambda^(0) = (3 - 188, 91) = (-185, 91).  i=1: alpha_0 = 3 - 141 = -138 -> -127;
    # beta_k = +(127 - 31) = 96 -> 189 (unsaturated 138 - 34 = 104 -> 197);
    # beta_0 = -(93 - 23) = -70 -> 3 - 280 = -277.
    ((3, 4), [(-185, 91), (-277, 189)]),
    # Int3.3: mu_0 = 2, mu_k = 46, qmax 63.  i=0: beta_0 = -23, beta_k = -1: (-90, 45).
    # i=1: alpha_0 = 2 - 69 = -67 -> -63; beta_k = 63 - 15 = 48 -> 94; beta_0 = -(46 - 11) -> 2 - 140 = -138.
    ((3, 3), [(-90, 45), (-138, 94)]),
    # Int2.4: mu_0 = 3, mu_k = 93 -> 63, qmax 63.  i=0: beta_0 = -32, beta_k = -2: (-125, 61).
    # i=1: alpha_0 = 3 - 96 = -93 -> -63; beta_k = 48 -> 111; beta_0 = -48 -> 3 - 192 = -189.
    ((2, 4), [(-125, 61), (-189, 111)]),
    # Int4.3 (qmax 127), control without saturation: mu_0 = 2, mu_k = 46; i=1: alpha_0 = -67
    # passes unchanged, beta_k = 67 - 16 = 51 -> 97.
    ((4, 3), [(-90, 45), (-138, 97)]),
])
def test_alpha_saturates_at_minus_qmax(fx, expect):
    pr = [0.45, 0.003, 0.003, 0.003, 0.003]
    t = _trajectory(FAN, pr, [1, 1, 1, 1], 1, msg=oracle.INT8, lottery=False, fx_int=fx[0], fx_frac=fx[1])
    for i, (l0, lk) in enumerate(expect):
        assert [int(x) for x in t[i]] == [l0, lk, lk, lk, lk], f"iteration {i}"
