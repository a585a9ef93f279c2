"""Logical-failure check and error-rate statistics for decoded shots (harness).

For a decoding matrix H_dec built from a single-round matrix H (code capacity:
H_dec = H; phenomenological: H_dec = H_st over r rounds, data columns first),
the residual on the data qubits is R = XOR over rounds of (e_t XOR e_hat_t).
A shot fails when
  * H R != 0 (the residual leaves a non-trivial syndrome, e.g. when a last-round
    measurement flip was explained by a data flip or the reverse), or
  * K R != 0, where the rows of K span ker(H_conj) and H_conj is the other
    stabilizer type (R then acts as a non-trivial logical operator).
The two causes are reported separately.  The paper states only that a trial
fails when the logical measurement differs from the initial state
(Section VI); this rule is its phenomenological analogue.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .codes import gf2_nullspace
from .sample import unpack_bits


class LogicalChecker:
    def __init__(self, h_single: sp.csr_matrix, h_conj: sp.csr_matrix, rounds: int):
        self.h = sp.csr_matrix(h_single, dtype=np.int32)
        self.n = self.h.shape[1]
        self.r = rounds
        k = gf2_nullspace(h_conj)
        self.k = sp.csr_matrix(k.astype(np.int32))

    def residual(self, errors: sp.csr_matrix, corr_packed: np.ndarray, n_dec: int) -> np.ndarray:
        ehat = unpack_bits(corr_packed, n_dec).astype(np.uint8)
        e = errors.toarray().astype(np.uint8) if sp.issparse(errors) else np.asarray(errors, np.uint8)
        diff = e[:, : self.r * self.n] ^ ehat[:, : self.r * self.n]
        return np.bitwise_xor.reduce(diff.reshape(diff.shape[0], self.r, self.n), axis=1)

    def failures(self, errors, corr_packed, n_dec):
        """Return (syndrome_fail[bool], logical_fail[bool]) per shot."""
        R = sp.csr_matrix(self.residual(errors, corr_packed, n_dec).astype(np.int32))
        synd_fail = np.asarray(((R @ self.h.T).toarray() & 1).any(axis=1)).ravel()
        log_fail = np.asarray(((R @ self.k.T).toarray() & 1).any(axis=1)).ravel()
        return synd_fail, log_fail & ~synd_fail


def failures_packed(checker: "LogicalChecker", err_packed: np.ndarray, corr_packed: np.ndarray, n_dec: int,
                    chunk: int = 32768):
    """Same as LogicalChecker.failures for packed error words (dense, chunked)."""
    hT = checker.h.toarray().T.astype(np.float32)
    kT = checker.k.toarray().T.astype(np.float32)
    S = err_packed.shape[0]
    sf = np.zeros(S, bool)
    lf = np.zeros(S, bool)
    span = checker.r * checker.n
    for lo in range(0, S, chunk):
        hi = min(S, lo + chunk)
        diff = np.ascontiguousarray(err_packed[lo:hi] ^ corr_packed[lo:hi], dtype="<u4")
        nz = diff.any(axis=1)
        if not nz.any():
            continue
        bits = unpack_bits(diff[nz], n_dec)[:, :span]
        R = np.bitwise_xor.reduce(bits.reshape(bits.shape[0], checker.r, checker.n), axis=1).astype(np.float32)
        s_bad = (np.rint(R @ hT).astype(np.int64) & 1).any(axis=1)
        l_bad = (np.rint(R @ kT).astype(np.int64) & 1).any(axis=1) & ~s_bad
        idx = np.nonzero(nz)[0] + lo
        sf[idx] = s_bad
        lf[idx] = l_bad
    return sf, lf


def wilson(k: int, n: int, z: float = 1.959963984540054) -> tuple[float, float]:
    """Wilson score interval for a binomial proportion k/n (95% by default)."""
    if n == 0:
        return (0.0, 1.0)
    ph = k / n
    den = 1 + z * z / n
    c = (ph + z * z / (2 * n)) / den
    half = z * math.sqrt(ph * (1 - ph) / n + z * z / (4 * n * n)) / den
    return (max(0.0, c - half), min(1.0, c + half))
