"""Parity-check matrices of the codes the decoder is exercised on.

Seeded-input side of the test harness: nothing here performs any step of the
decoding method.  Matrices are returned as ``scipy.sparse.csr_matrix`` with
uint8 entries and sorted, unique column indices.

* Rotated surface code (data qubits on a d x d grid, checkerboard weight-4
  plaquettes, weight-2 plaquettes on two opposite boundaries per type).
* Bivariate bicycle (BB) codes H_X = [A | B], H_Z = [B^T | A^T] with
  A, B polynomials in the commuting shifts x = S_l (x) I_m, y = I_l (x) S_m.
* The space-time (phenomenological) matrix of the paper's Eq. 1:
  H_st = [I_r (x) H | D (x) I_m] with D the r x r lower-bidiagonal
  differencing matrix (Section IV-A).
* The unrotated surface code of the paper's worked example (Fig. 4) and of
  Table II, with checks on vertices and qubits on edges.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _csr(rows: list[list[int]], n: int) -> sp.csr_matrix:
    indptr = np.zeros(len(rows) + 1, dtype=np.int64)
    indices = []
    for i, r in enumerate(rows):
        r = sorted(set(int(x) for x in r))
        indices.extend(r)
        indptr[i + 1] = indptr[i] + len(r)
    data = np.ones(len(indices), dtype=np.uint8)
    return sp.csr_matrix((data, np.asarray(indices, dtype=np.int64), indptr), shape=(len(rows), n))


def rotated_surface(d: int) -> tuple[sp.csr_matrix, sp.csr_matrix]:
    """Return (H_X, H_Z) of the distance-d rotated surface code, each (d^2-1)/2 x d^2.

    Qubit (a, b) of the grid has index a*d + b.  Face (a, b), a, b in [-1, d-1],
    touches qubits (a,b), (a+1,b), (a,b+1), (a+1,b+1) clipped to the grid.
    Interior faces alternate X/Z by the parity of a+b; X-type weight-2 faces sit
    on the top/bottom boundaries, Z-type on the left/right ones.
    """
    if d < 2:
        raise ValueError("d >= 2")
    hx, hz = [], []
    for a in range(-1, d):
        for b in range(-1, d):
            qs = [(a + da) * d + (b + db) for da in (0, 1) for db in (0, 1)
                  if 0 <= a + da < d and 0 <= b + db < d]
            interior = 0 <= a <= d - 2 and 0 <= b <= d - 2
            is_x = (a + b) % 2 == 0
            if interior:
                (hx if is_x else hz).append(qs)
            elif len(qs) == 2:
                top_bottom = (a == -1 or a == d - 1) and 0 <= b <= d - 2
                left_right = (b == -1 or b == d - 1) and 0 <= a <= d - 2
                if top_bottom and is_x:
                    hx.append(qs)
                elif left_right and not is_x:
                    hz.append(qs)
    return _csr(hx, d * d), _csr(hz, d * d)


def _shift(k: int) -> np.ndarray:
    return np.roll(np.eye(k, dtype=np.uint8), 1, axis=1)


def bb_code(l: int, m: int, a_terms: list[tuple[int, int]], b_terms: list[tuple[int, int]]
            ) -> tuple[sp.csr_matrix, sp.csr_matrix]:
    """Bivariate bicycle code.  Each term (i, j) stands for x^i y^j.

    Returns (H_X, H_Z) with H_X = [A | B] and H_Z = [B^T | A^T], both lm x 2lm.
    """
    x = np.kron(_shift(l), np.eye(m, dtype=np.uint8))
    y = np.kron(np.eye(l, dtype=np.uint8), _shift(m))

    def poly(terms):
        acc = np.zeros((l * m, l * m), dtype=np.int64)
        for i, j in terms:
            acc += np.linalg.matrix_power(x.astype(np.int64), i) @ np.linalg.matrix_power(y.astype(np.int64), j)
        return (acc % 2).astype(np.uint8)

    A, B = poly(a_terms), poly(b_terms)
    hx = np.hstack([A, B])
    hz = np.hstack([B.T, A.T])
    return sp.csr_matrix(hx), sp.csr_matrix(hz)


def bb144() -> tuple[sp.csr_matrix, sp.csr_matrix]:
    """[[144,12,12]]: l=12, m=6, A = x^3 + y + y^2, B = y^3 + x + x^2."""
    return bb_code(12, 6, [(3, 0), (0, 1), (0, 2)], [(0, 3), (1, 0), (2, 0)])


def bb288() -> tuple[sp.csr_matrix, sp.csr_matrix]:
    """[[288,12,18]]: l=m=12, A = x^3 + y^2 + y^7, B = y^3 + x + x^2."""
    return bb_code(12, 12, [(3, 0), (0, 2), (0, 7)], [(0, 3), (1, 0), (2, 0)])


def spacetime(h: sp.csr_matrix, r: int, final_round: bool = False) -> sp.csr_matrix:
    """H_st = [I_r (x) H | D (x) I_m] of Eq. 1; D[t][t] = D[t][t-1] = 1.

    Columns: r blocks of n data columns (round t), then r blocks of m
    measurement columns.  Shape (r*m) x (r*n + r*m).

    final_round=True appends the detectors of a noiseless final read-out of
    the data qubits: m more rows [0 | 0 ... 0 I], which compare that read-out
    with round r-1 and so see only round r-1's measurement errors.  Every
    measurement column then has weight 2, the structure whose nonzero counts
    Table II lists.
    """
    h = sp.csr_matrix(h, dtype=np.uint8)
    mm = h.shape[0]
    D = sp.eye(r, dtype=np.uint8, format="csr") + sp.eye(r, k=-1, dtype=np.uint8, format="csr")
    left = sp.kron(sp.eye(r, dtype=np.uint8), h, format="csr")
    right = sp.kron(D, sp.eye(mm, dtype=np.uint8), format="csr")
    if final_round:
        last = sp.csr_matrix((np.ones(mm, np.uint8), (np.arange(mm), (r - 1) * mm + np.arange(mm))),
                             shape=(mm, r * mm))
        left = sp.vstack([left, sp.csr_matrix((mm, left.shape[1]), dtype=np.uint8)], format="csr")
        right = sp.vstack([right, last], format="csr")
    out = sp.hstack([left, right], format="csr").astype(np.uint8)
    out.sort_indices()
    out.sum_duplicates()
    return out


def unrotated_surface_x(d: int) -> sp.csr_matrix:
    """X-check matrix of the unrotated (planar) surface code, d(d-1) x (d^2 + (d-1)^2).

    Qubits are the edges of a grid as in the paper's Fig. 4: d rows of d
    horizontal edges (index row*d + col), then d-1 rows of d-1 vertical edges.
    X checks sit on the d x (d-1) interior vertices; the left and right
    boundaries carry no checks.
    """
    nh = d * d
    n = nh + (d - 1) * (d - 1)
    rows = []
    for y in range(d):            # vertex row (top = 0)
        for x in range(1, d):     # interior vertex column
            qs = [y * d + (x - 1), y * d + x]
            if y > 0:
                qs.append(nh + (y - 1) * (d - 1) + (x - 1))
            if y < d - 1:
                qs.append(nh + y * (d - 1) + (x - 1))
            rows.append(qs)
    return _csr(rows, n)


def unrotated_surface_z(d: int) -> sp.csr_matrix:
    """Z-check matrix of the same unrotated surface code, (d-1)d x (d^2 + (d-1)^2):
    one check per face between vertex rows y and y+1 and vertex columns x and x+1
    (two horizontal edges, and the vertical edges that are not on the left or
    right boundary)."""
    nh = d * d
    n = nh + (d - 1) * (d - 1)
    rows = []
    for y in range(d - 1):
        for x in range(d):
            qs = [y * d + x, (y + 1) * d + x]
            if x >= 1:
                qs.append(nh + y * (d - 1) + (x - 1))
            if x <= d - 2:
                qs.append(nh + y * (d - 1) + x)
            rows.append(sorted(qs))
    return _csr(rows, n)


def worked_example_h() -> sp.csr_matrix:
    """The 6 x 13 X-check matrix of the paper's Fig. 4 ([[13,1,3]] surface code).

    Read off the figure: horizontal edges q0..q8 (three rows of three), vertical
    edges q9..q12, checks X0..X5 on the interior vertices.
    """
    rows = [[0, 1, 9], [1, 2, 10], [3, 4, 9, 11], [4, 5, 10, 12], [6, 7, 11], [7, 8, 12]]
    return _csr(rows, 13)


def gf2_rank(h) -> int:
    """Rank over GF(2) (dense elimination on packed rows; harness helper)."""
    a = np.asarray(h.todense() if sp.issparse(h) else h, dtype=np.uint8) & 1
    a = a.copy()
    rank = 0
    rows, cols = a.shape
    for c in range(cols):
        piv = np.nonzero(a[rank:, c])[0]
        if piv.size == 0:
            continue
        p = rank + piv[0]
        if p != rank:
            a[[rank, p]] = a[[p, rank]]
        hit = np.nonzero(a[:, c])[0]
        hit = hit[hit != rank]
        a[hit] ^= a[rank]
        rank += 1
        if rank == rows:
            break
    return rank


def gf2_nullspace(h) -> np.ndarray:
    """Basis of {x : h x = 0} over GF(2), one vector per row (harness helper)."""
    a = np.asarray(h.todense() if sp.issparse(h) else h, dtype=np.uint8) & 1
    a = a.copy()
    rows, cols = a.shape
    pivots = []
    r = 0
    for c in range(cols):
        if r == rows:
            break
        piv = np.nonzero(a[r:, c])[0]
        if piv.size == 0:
            continue
        p = r + piv[0]
        if p != r:
            a[[r, p]] = a[[p, r]]
        hit = np.nonzero(a[:, c])[0]
        hit = hit[hit != r]
        a[hit] ^= a[r]
        pivots.append(c)
        r += 1
    free = [c for c in range(cols) if c not in set(pivots)]
    basis = np.zeros((len(free), cols), dtype=np.uint8)
    for k, f in enumerate(free):
        basis[k, f] = 1
        for i, pc in enumerate(pivots):
            basis[k, pc] = a[i, f]
    return basis


# The named workloads: (matrix used for decoding, conjugate matrix for the logical check, rounds)
def workload_matrices(name: str) -> tuple[sp.csr_matrix, sp.csr_matrix, int]:
    """Return (H_dec, H_conj, r) for a named workload.

    H_dec is the matrix the decoder sees; H_conj is the other stabilizer type of
    the single-round code (used only by the logical-failure check); r is the
    number of rounds (1 = code capacity).
    """
    if name == "surface5_cc":
        hx, hz = rotated_surface(5)
        return hz, hx, 1
    if name == "surface3_cc":
        hx, hz = rotated_surface(3)
        return hz, hx, 1
    if name.startswith("surface") and name.endswith("_phen"):
        d = int(name[len("surface"):-len("_phen")])
        hx, hz = rotated_surface(d)
        return spacetime(hz, d), hx, d
    if name.startswith("surface") and name.endswith("_phenpf"):
        d = int(name[len("surface"):-len("_phenpf")])
        hx, hz = rotated_surface(d)
        return spacetime(hz, d, final_round=True), hx, d
    if name.startswith("usurface") and (name.endswith("_phen") or name.endswith("_phenpf")):
        # unrotated (planar) surface code, X checks decoded, d rounds
        final = name.endswith("_phenpf")
        d = int(name[len("usurface"):name.index("_")])
        return spacetime(unrotated_surface_x(d), d, final_round=final), unrotated_surface_z(d), d
    if name == "bb144_cc":
        hx, hz = bb144()
        return hx, hz, 1
    if name == "bb144_phen":
        hx, hz = bb144()
        return spacetime(hx, 12), hz, 12
    if name == "bb288_phen":
        hx, hz = bb288()
        return spacetime(hx, 18), hz, 18
    if name == "bb144_phenpf":
        hx, hz = bb144()
        return spacetime(hx, 12, final_round=True), hz, 12
    raise KeyError(name)
