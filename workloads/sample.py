"""Seeded synthetic decoding workloads: errors, syndromes and bit packing.

Recipe (shared by the oracle and the GPU path; it holds none of the decoding
method's arithmetic):

* shots are produced in chunks of ``CHUNK`` = 65536; chunk k of seed S uses
  ``numpy.random.Generator(PCG64(SeedSequence([S, k])))``;
* every column of the decoding matrix flips independently with probability p:
  ``rng.random((rows, n), dtype=float32) < p`` (data and measurement flips of a
  phenomenological model, or data flips only for code capacity);
* the syndrome is s = H e mod 2;
* bit vectors are packed LSB-first into little-endian uint32 words, each shot
  padded to whole words: word w, bit b holds element 32*w + b.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

CHUNK = 65536


def words(nbits: int) -> int:
    return (nbits + 31) // 32


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """[shots, nbits] of {0,1} -> [shots, words(nbits)] uint32, LSB-first."""
    bits = np.ascontiguousarray(bits, dtype=np.uint8)
    shots, nbits = bits.shape
    nw = words(nbits)
    padded = np.zeros((shots, nw * 32), dtype=np.uint8)
    padded[:, :nbits] = bits
    by = np.packbits(padded, axis=1, bitorder="little")
    return np.ascontiguousarray(by).view("<u4").reshape(shots, nw).astype(np.uint32)


def unpack_bits(packed: np.ndarray, nbits: int) -> np.ndarray:
    """Inverse of :func:`pack_bits`."""
    packed = np.ascontiguousarray(packed, dtype="<u4")
    shots = packed.shape[0]
    by = packed.view(np.uint8).reshape(shots, -1)
    return np.unpackbits(by, axis=1, bitorder="little")[:, :nbits]


def sample_errors(n: int, p: float, shots: int, seed: int, first_shot: int = 0) -> sp.csr_matrix:
    """Errors of shots [first_shot, first_shot + shots) as a sparse 0/1 matrix [shots, n]."""
    out_rows = []
    k0 = first_shot // CHUNK
    k1 = (first_shot + shots + CHUNK - 1) // CHUNK
    for k in range(k0, k1):
        lo = max(first_shot, k * CHUNK)
        hi = min(first_shot + shots, (k + 1) * CHUNK)
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, k])))
        # draw the whole chunk so shot i's error never depends on the requested range
        rows_needed = hi - k * CHUNK
        e = rng.random((rows_needed, n), dtype=np.float32) < np.float32(p)
        e = e[lo - k * CHUNK:hi - k * CHUNK]
        r, c = np.nonzero(e)
        indptr = np.zeros(e.shape[0] + 1, dtype=np.int64)
        np.cumsum(np.bincount(r, minlength=e.shape[0]), out=indptr[1:])
        out_rows.append(sp.csr_matrix((np.ones(r.size, np.uint8), c, indptr), shape=e.shape))
    if not out_rows:
        return sp.csr_matrix((0, n), dtype=np.uint8)
    return sp.vstack(out_rows, format="csr").astype(np.uint8)


def syndromes(h: sp.csr_matrix, errors: sp.csr_matrix) -> np.ndarray:
    """s = H e mod 2 for each row of ``errors``; returns [shots, m] uint8."""
    s = (errors.astype(np.int32) @ sp.csr_matrix(h, dtype=np.int32).T)
    return (s.toarray() & 1).astype(np.uint8)


def make_batch(h: sp.csr_matrix, p: float, shots: int, seed: int, first_shot: int = 0):
    """Return (errors sparse [shots,n], packed syndromes [shots, words(m)] uint32)."""
    e = sample_errors(h.shape[1], p, shots, seed, first_shot)
    s = syndromes(h, e)
    return e, pack_bits(s)


def pack_sparse(errors: sp.csr_matrix) -> np.ndarray:
    """Sparse 0/1 rows -> packed uint32 words (same layout as pack_bits)."""
    e = sp.csr_matrix(errors)
    out = np.zeros((e.shape[0], words(e.shape[1])), dtype=np.uint32)
    rows = np.repeat(np.arange(e.shape[0]), np.diff(e.indptr))
    cols = e.indices.astype(np.int64)
    np.bitwise_or.at(out, (rows, cols >> 5), (np.uint32(1) << (cols & 31).astype(np.uint32)))
    return out
