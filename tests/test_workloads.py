"""Shapes and invariants of the synthetic workloads (harness, no decoding)."""
import math

import numpy as np
import scipy.sparse as sp

from workloads import codes, sample


def _rank(h):
    return codes.gf2_rank(h)


def test_rotated_surface_invariants():
    for d in (3, 5, 7, 11):
        hx, hz = codes.rotated_surface(d)
        assert hx.shape == hz.shape == ((d * d - 1) // 2, d * d)
        assert not ((hx @ hz.T).toarray() % 2).any()
        assert d * d - _rank(hx) - _rank(hz) == 1            # one logical qubit
        assert hx.nnz == hz.nnz == 2 * d * (d - 1)
        assert set(np.diff(hz.indptr)) == {2, 4}


def test_bb_codes():
    hx, hz = codes.bb144()
    assert hx.shape == (72, 144)
    assert not ((hx @ hz.T).toarray() % 2).any()
    assert _rank(hx) == 66 and _rank(hz) == 66               # k = 144 - 132 = 12
    assert set(np.diff(hx.indptr)) == {6}
    assert set(np.asarray(hx.sum(0)).ravel()) == {3}
    gx, gz = codes.bb288()
    assert gx.shape == (144, 288)
    assert not ((gx @ gz.T).toarray() % 2).any()
    assert 288 - _rank(gx) - _rank(gz) == 12


def test_spacetime_shapes_match_configs():
    expect = {"surface11_phen": (660, 1991, 3680), "bb144_phen": (864, 2592, 6840),
              "surface5_phen": (60, 185, 308), "surface9_phen": (360, 1089, 1976),
              "surface13_phen": (1092, 3289, 6156)}
    for name, (m, n, e) in expect.items():
        h, _, r = codes.workload_matrices(name)
        assert h.shape == (m, n) and h.nnz == e, name
    h, _, _ = codes.workload_matrices("bb144_phen")
    assert set(np.diff(h.indptr)) == {7, 8}
    assert _rank(h) == 864                                      # D invertible: full row rank


def test_eq1_block_structure():
    h1 = sp.csr_matrix(np.array([[1, 1, 0], [0, 1, 1]], dtype=np.uint8))
    st = codes.spacetime(h1, 3).toarray()
    # round 0 sees its data block and its own measurement; later rounds the previous one too
    assert st.shape == (6, 9 + 6)
    assert (st[0:2, 0:3] == h1.toarray()).all() and (st[2:4, 3:6] == h1.toarray()).all()
    meas = st[:, 9:]
    assert (meas[0:2, 0:2] == np.eye(2)).all() and not meas[0:2, 2:].any()
    assert (meas[2:4, 0:2] == np.eye(2)).all() and (meas[2:4, 2:4] == np.eye(2)).all()


def test_worked_example_matrix():
    h = codes.worked_example_h()
    assert (h != codes.unrotated_surface_x(3)).nnz == 0
    e = np.zeros((1, 13), np.uint8)
    e[0, [2, 8, 9]] = 1                                          # Fig. 4: errors {q2, q8, q9}
    s = sample.syndromes(h, sp.csr_matrix(e))[0]
    assert list(np.nonzero(s)[0]) == [0, 1, 2, 5]                # triggers {X0, X1, X2, X5}


def test_table2_column_counts():
    # Table II: H_st columns of the d-round unrotated code
    for d, cols in ((3, 57), (9, 1953)):
        h = codes.unrotated_surface_x(d)
        st = codes.spacetime(h, d)
        assert st.shape[1] == cols
    # Table II's nonzero counts equal r*nnz(H) + 2*r*m (a weight-2 measurement
    # column per round), while Eq. 1 with a bidiagonal D gives (2r-1)*m.
    h = codes.unrotated_surface_x(9)
    assert 9 * h.nnz + 2 * 9 * h.shape[0] == 3744
    assert codes.spacetime(h, 9).nnz == 9 * h.nnz + 17 * h.shape[0]


def test_table2_with_final_round():
    """Table II, d = 3 ... 27 (columns, nonzeros as printed, K = 10^3 rounded to three
    figures): reproduced by the d-round H_st with the noiseless final read-out rows."""
    table = {3: (57, 96), 9: (1.95e3, 3.74e3), 15: (9.47e3, 18.5e3), 21: (26.5e3, 52.1e3), 27: (56.9e3, 112e3)}
    for d, (cols, nnz) in table.items():
        h = codes.unrotated_surface_x(d)
        st = codes.spacetime(h, d, final_round=True)
        for got, printed in ((st.shape[1], cols), (st.nnz, nnz)):   # three figures, half rounded up
            half = 0.5 * 10 ** (math.floor(math.log10(printed)) - 2)
            assert printed - half <= got < printed + half, (d, got, printed)
        assert st.shape[0] == (d + 1) * h.shape[0]
        assert st.sum(axis=0).max() == 2 and st[: d * h.shape[0]].nnz + h.shape[0] == st.nnz


def test_final_round_makes_last_measurement_errors_visible():
    """A lone measurement error in the last round has a zero syndrome on the r-row
    H_st only through its one row, while the final read-out adds a second one; a
    decoder matching every detector then leaves a residual with no data syndrome."""
    hx, hz = codes.rotated_surface(3)
    r, m, n = 3, hz.shape[0], hz.shape[1]
    plain, pf = codes.spacetime(hz, r), codes.spacetime(hz, r, final_round=True)
    col = r * n + (r - 1) * m                                   # measurement column of round r-1, check 0
    assert plain[:, col].nnz == 1 and pf[:, col].nnz == 2
    assert pf[r * m, col] == 1                                   # the final read-out row of check 0


def test_pack_roundtrip_and_chunk_independence():
    rng = np.random.default_rng(0)
    bits = (rng.random((7, 77)) < 0.3).astype(np.uint8)
    packed = sample.pack_bits(bits)
    assert packed.shape == (7, 3) and packed.dtype == np.uint32
    assert (sample.unpack_bits(packed, 77) == bits).all()
    assert packed[0, 0] == int("".join(str(b) for b in bits[0, :32][::-1]), 2)
    h, _, _ = codes.workload_matrices("surface5_cc")
    e_all = sample.sample_errors(25, 0.1, 70000, seed=5)
    e_part = sample.sample_errors(25, 0.1, 1000, seed=5, first_shot=65000)
    assert (e_all[65000:66000] != e_part).nnz == 0


def test_unrotated_surface_code():
    """Planar (unrotated) surface code: checks commute, one logical qubit, weights
    <= 4 / <= 2, d = 3 is the paper's Fig. 4 matrix, and its distance is 3 by
    enumeration of every Z-type vector."""
    for d in (3, 5, 7, 9):
        hx, hz = codes.unrotated_surface_x(d), codes.unrotated_surface_z(d)
        n = d * d + (d - 1) ** 2
        assert hx.shape == (d * (d - 1), n) and hz.shape == (d * (d - 1), n)
        assert not ((hx @ hz.T).toarray() % 2).any()
        assert n - codes.gf2_rank(hx) - codes.gf2_rank(hz) == 1
        assert hx.sum(axis=1).max() == 4 and hx.sum(axis=0).max() == 2
    assert (codes.unrotated_surface_x(3) != codes.worked_example_h()).nnz == 0
    hx, hz = codes.unrotated_surface_x(3), codes.unrotated_surface_z(3)
    xs = ((np.arange(1 << 13)[:, None] >> np.arange(13)) & 1).astype(np.int64)
    in_ker = ~((xs @ hx.toarray().T.astype(np.int64)) % 2).any(axis=1)
    rank_z = codes.gf2_rank(hz)
    logical = [x for x in xs[in_ker] if x.any() and codes.gf2_rank(np.vstack([hz.toarray(), x])) > rank_z]
    assert min(int(x.sum()) for x in logical) == 3
    h, hc, r = codes.workload_matrices("usurface9_phenpf")
    assert h.shape == (10 * 72, 9 * (145 + 72)) and r == 9 and hc.shape == (72, 145)
