"""Pins of the oracle's per-row-block tables (Section III-B.1, sampling).

The matrix is cut into blocks of ``block_rows`` rows; each block gets its own
table, chosen from the exponents of one drawn row of the block (or of the
whole block), with the block's own largest exponent added when the sample
misses it.  The checks come from outside the oracle's code:

  * a brute-force table choice written here from the description (count the
    exponent fields, take the k most frequent, larger exponent on ties, the
    sample's maximum forced in, then the block's maximum);
  * the format's definition per value (magnitude on the grid of the nearest
    shared exponent above, truncated), in exact rational arithmetic;
  * reductions to the global encoder: one block covering every row is the
    global table; and every block of an exact-histogram encode is the
    global encode of that block's rows alone;
  * the SpMV of the block planes against an exactly rounded sum of the
    block-decoded products, and eta against its definition;
  * argument errors, and that every value of a block is representable even
    when the drawn row misses the block's maximum exponent.

The other reading, one table for the whole matrix from the drawn rows'
counts pooled, is pinned the same way: brute force over the pooled rows,
every row drawn reduces to the exact global encode, and its planes are the
global encoder's with that table reused.
"""
import collections
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from workloads import CSR, block_sample_rows, diffusion3d, layered3d, random_sparse


def field(v: float) -> int:
    if v == 0.0:
        return 0
    _, ex = math.frexp(abs(v))
    f = ex - 1 + 1023
    return f if f >= 1 else 0


def brute_table(sample_vals, block_vals, k):
    """The table (biased exponent + 1 per slot) from the sample's exponent
    fields, with the block's maximum added when missing."""
    cnt = collections.Counter(field(v) for v in sample_vals if field(v) >= 1)
    order = sorted(cnt.items(), key=lambda kv: (-kv[1], -kv[0]))
    chosen = [e for e, _ in order[:k]]
    if not chosen:
        chosen = [1023]
    elif max(cnt) not in chosen:
        chosen[-1] = max(cnt)
    bmax = max([field(v) for v in block_vals] + [0])
    if bmax >= 1 and bmax not in chosen:
        if len(chosen) < k:
            chosen.append(bmax)
        else:
            chosen[-1] = bmax
    return [e + 1 for e in chosen]


def blocks_of(A: CSR, R: int):
    for b in range(-(-A.n_rows // R)):
        r0, r1 = b * R, min((b + 1) * R, A.n_rows)
        yield b, r0, r1, int(A.indptr[r0]), int(A.indptr[r1])


def small_cases():
    return [
        (random_sparse(700, 500, 3, mean_row=5, exp_spread=30.0), 128),
        (random_sparse(1000, 1000, 4, mean_row=7, empty_frac=0.2, exp_spread=12.0), 130),
        (layered3d(10, 5, contrast=12.0), 200),
    ]


@pytest.mark.parametrize("k", [1, 3, 8, 64])
@pytest.mark.parametrize("sampled", [False, True])
def test_tables_match_brute_force(k, sampled):
    for A, R in small_cases():
        sr = block_sample_rows(A.n_rows, R, 11) if sampled else None
        enc = O.encode_blocks(A.indptr, A.indices, A.data, A.n_cols, num_exp=k, block_rows=R,
                              sample_rows=sr)
        assert enc.block_sem.shape == (-(-A.n_rows // R), 64)
        for b, r0, r1, j0, j1 in blocks_of(A, R):
            if sampled:
                s = int(sr[b])
                assert r0 <= s < r1
                sample = A.data[A.indptr[s]:A.indptr[s + 1]]
            else:
                sample = A.data[j0:j1]
            want = brute_table(sample, A.data[j0:j1], k)
            got = [int(t) for t in enc.block_sem[b]]
            assert got[:len(want)] == want, (A.name, b)
            assert all(t == 0 for t in got[len(want):])


@pytest.mark.parametrize("sampled", [False, True])
def test_values_follow_the_definition(sampled):
    A, R = small_cases()[0]
    sr = block_sample_rows(A.n_rows, R, 2) if sampled else None
    enc = O.encode_blocks(A.indptr, A.indices, A.data, A.n_cols, block_rows=R, sample_rows=sr)
    tables = enc.table_of_rows(A.indptr)
    slots = enc.slot()
    cols = enc.column()
    rng = np.random.default_rng(0)
    for j in rng.choice(A.nnz, size=400, replace=False):
        v = float(A.data[j])
        sem = [int(t) for t in tables[j]]
        above = [(S, i) for i, S in enumerate(sem) if S > field(v)]
        S, slot = min(above)  # nearest shared exponent above the value's own
        assert int(slots[j]) == slot and int(cols[j]) == int(A.indices[j])
        F = math.floor(abs(Fraction(v)) * Fraction(2) ** (1086 - S))
        word = (int(enc.head[j]) & 0x7FFF) << 48 | int(enc.tail1[j]) << 32 | int(enc.tail2[j])
        assert word == F and (int(enc.head[j]) >> 15) == (v < 0 or (v == 0 and math.copysign(1, v) < 0))
    # s = 3 reads the value exactly whenever no bit was shifted out
    d3 = O.decode_blocks(A.indptr, enc, 3)
    for j in rng.choice(A.nnz, size=200, replace=False):
        S = int(tables[j][int(slots[j])])
        if (S - field(A.data[j])) <= 11:
            assert d3[j] == A.data[j]


def test_one_block_is_the_global_table():
    A = diffusion3d(12, 1)
    g = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    b = O.encode_blocks(A.indptr, A.indices, A.data, A.n_cols, block_rows=A.n_rows)
    assert np.array_equal(b.block_sem[0][:8], g.table[:8])
    for a, c in ((b.col_idx, g.col_idx), (b.head, g.head), (b.tail1, g.tail1), (b.tail2, g.tail2)):
        assert np.array_equal(a, c)
    assert np.array_equal(b.eta, g.eta) and b.exact_frac == g.exact_frac


@pytest.mark.parametrize("layout", [0, 1])
def test_exact_blocks_are_the_global_encode_of_each_block(layout):
    A, R = small_cases()[2]
    enc = O.encode_blocks(A.indptr, A.indices, A.data, A.n_cols, num_exp=8, block_rows=R,
                          layout=layout)
    assert enc.layout == layout
    covered = 0
    for b, r0, r1, j0, j1 in blocks_of(A, R):
        sub_ptr = A.indptr[r0:r1 + 1] - A.indptr[r0]
        g = O.encode(sub_ptr, A.indices[j0:j1], A.data[j0:j1], A.n_cols, num_exp=8, layout=layout)
        assert np.array_equal(enc.block_sem[b][:8], g.table[:8])
        for a, c in ((enc.col_idx, g.col_idx), (enc.head, g.head), (enc.tail1, g.tail1),
                     (enc.tail2, g.tail2)):
            assert np.array_equal(a[j0:j1], c)
        covered += round(g.exact_frac * (j1 - j0))
    assert enc.exact_frac == pytest.approx(covered / A.nnz, abs=1e-15)


def test_eta_and_spmv_against_their_definitions():
    A, R = small_cases()[1]
    sr = block_sample_rows(A.n_rows, R, 5)
    enc = O.encode_blocks(A.indptr, A.indices, A.data, A.n_cols, block_rows=R, sample_rows=sr)
    x = np.random.default_rng(1).uniform(-1, 1, A.n_cols)
    absrow = np.array([math.fsum(abs(A.data[A.indptr[r]:A.indptr[r + 1]]))
                       for r in range(A.n_rows)])
    for s in (1, 2, 3):
        d = O.decode_blocks(A.indptr, enc, s)
        err = np.array([math.fsum(abs(A.data[A.indptr[r]:A.indptr[r + 1]] -
                                      d[A.indptr[r]:A.indptr[r + 1]]))
                        for r in range(A.n_rows)])
        assert enc.eta[s - 1] == pytest.approx(err.max() / absrow.max(), rel=1e-13)
        y = O.gse_spmv(A.indptr, enc, s, x)
        for r in range(A.n_rows):
            lo, hi = A.indptr[r], A.indptr[r + 1]
            terms = d[lo:hi] * x[A.indices[lo:hi]]
            exact = math.fsum(terms)
            bound = 2 * (hi - lo + 1) * np.finfo(float).eps * math.fsum(abs(terms))
            assert abs(y[r] - exact) <= bound
    # the solvers' operator is the same product
    res = O.cg(A.indptr, np.ones(A.n_rows), O.make_params(max_iter=0, fixed_segments=1),
               enc=enc)
    assert res.status in (O.OK, O.NOT_CONVERGED)


def test_sample_missing_the_block_maximum_still_covers_every_value():
    # one huge value in row 1 of each block; the drawn row is row 0
    n, R = 512, 128
    rng = np.random.default_rng(3)
    indptr = np.arange(0, 4 * n + 1, 4, dtype=np.int32)
    indices = np.tile(np.arange(4, dtype=np.int32), n)
    data = rng.uniform(1.0, 2.0, 4 * n)
    data[4 * np.arange(1, n, R)] = 3.0e30
    A = CSR(n, 4, indptr, indices, data, "spike")
    sr = np.arange(0, n, R, dtype=np.int32)
    enc = O.encode_blocks(A.indptr, A.indices, A.data, 4, num_exp=2, block_rows=R, sample_rows=sr)
    for b in range(n // R):
        assert field(3.0e30) + 1 in [int(t) for t in enc.block_sem[b][:2]]
    d3 = O.decode_blocks(A.indptr, enc, 3)
    assert np.all(d3[4 * np.arange(1, n, R)] == 3.0e30)
    assert np.all(np.abs(d3 - data) <= np.abs(data) * 2.0 ** -40)


def test_argument_errors():
    A, R = small_cases()[0]
    with pytest.raises(O.OracleError) as e:
        O.encode_blocks(A.indptr, A.indices, A.data, A.n_cols, block_rows=0)
    assert e.value.code == O.ERR_ARG
    sr = block_sample_rows(A.n_rows, R, 0)
    sr[1] = sr[1] + R  # a row of the next block
    with pytest.raises(O.OracleError) as e:
        O.encode_blocks(A.indptr, A.indices, A.data, A.n_cols, block_rows=R, sample_rows=sr)
    assert e.value.code == O.ERR_ARG
    bad = A.data.copy()
    bad[5] = np.inf
    with pytest.raises(O.OracleError) as e:
        O.encode_blocks(A.indptr, A.indices, bad, A.n_cols, block_rows=R)
    assert e.value.code == O.ERR_NONFINITE


def test_block_sample_rows_draws_one_row_per_block():
    for n, R in ((1000, 128), (1024, 256), (5, 128), (129, 128)):
        sr = block_sample_rows(n, R, 7)
        assert sr.dtype == np.int32 and sr.size == -(-n // R)
        b = np.arange(sr.size)
        assert np.all(sr >= b * R) and np.all(sr < np.minimum((b + 1) * R, n))


def test_layered_medium_blocks_beat_the_global_table():
    # each slab's coefficients sit within a decade: a block's own table
    # covers its exponents where one table for eight decades cannot
    A = layered3d(16, 0, contrast=8.0, layers=4)
    g = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    b = O.encode_blocks(A.indptr, A.indices, A.data, A.n_cols, block_rows=256)
    assert b.exact_frac > g.exact_frac + 0.2
    assert b.eta[0] < g.eta[0]


# ---- one table for the matrix from the pooled drawn rows (the other reading) ----

@pytest.mark.parametrize("k", [1, 3, 8, 64])
def test_pooled_sample_table_matches_brute_force(k):
    for A, R in small_cases():
        sr = block_sample_rows(A.n_rows, R, 21)
        enc = O.encode_sampled(A.indptr, A.indices, A.data, A.n_cols, num_exp=k, block_rows=R,
                               sample_rows=sr)
        pooled = np.concatenate([A.data[A.indptr[s]:A.indptr[s + 1]] for s in sr])
        want = brute_table(pooled, A.data, k)
        got = [int(t) for t in enc.table]
        assert got[:len(want)] == want and not any(got[len(want):]), A.name
        # exact_frac is measured on all values
        fields = np.array([field(v) for v in A.data])
        assert enc.exact_frac == pytest.approx(np.isin(fields + 1, want).mean(), abs=1e-15)


def test_every_row_drawn_is_the_global_encode():
    for A, _ in small_cases():
        enc = O.encode_sampled(A.indptr, A.indices, A.data, A.n_cols, block_rows=1,
                               sample_rows=np.arange(A.n_rows, dtype=np.int32))
        g = O.encode(A.indptr, A.indices, A.data, A.n_cols)
        assert np.array_equal(enc.table, g.table)
        for a, c in ((enc.col_idx, g.col_idx), (enc.head, g.head), (enc.tail1, g.tail1),
                     (enc.tail2, g.tail2)):
            assert np.array_equal(a, c)
        assert np.array_equal(enc.eta, g.eta) and enc.exact_frac == g.exact_frac


def test_pooled_sample_planes_are_the_encode_of_that_table():
    A, R = small_cases()[0]
    sr = block_sample_rows(A.n_rows, R, 4)
    enc = O.encode_sampled(A.indptr, A.indices, A.data, A.n_cols, block_rows=R, sample_rows=sr)
    again = O.encode(A.indptr, A.indices, A.data, A.n_cols, sem_in=enc.table[:8])
    for a, c in ((enc.col_idx, again.col_idx), (enc.head, again.head), (enc.tail1, again.tail1),
                 (enc.tail2, again.tail2)):
        assert np.array_equal(a, c)
    assert np.allclose(enc.eta, again.eta, rtol=0, atol=0)
    bad = sr.copy()
    bad[0] = R  # a row of the next block
    with pytest.raises(O.OracleError) as e:
        O.encode_sampled(A.indptr, A.indices, A.data, A.n_cols, block_rows=R, sample_rows=bad)
    assert e.value.code == O.ERR_ARG


def test_added_maximum_below_the_normal_grid_is_a_range_error():
    # the drawn row holds only zeros; the block's largest value has exponent
    # field 10, whose shared exponent 11 would leave the normal range
    indptr = np.array([0, 2, 4] + [4] * 127, dtype=np.int32)
    data = np.array([0.0, 0.0, 2.0 ** -1013, 2.0 ** -1014])
    A = CSR(129, 2, indptr, np.array([0, 1, 0, 1], np.int32), data, "tiny")
    sr = np.array([0, 128], np.int32)
    with pytest.raises(O.OracleError) as e:
        O.encode_blocks(A.indptr, A.indices, A.data, 2, block_rows=128, sample_rows=sr)
    assert e.value.code == O.ERR_RANGE
    with pytest.raises(O.OracleError) as e:
        O.encode_sampled(A.indptr, A.indices, A.data, 2, block_rows=128, sample_rows=sr)
    assert e.value.code == O.ERR_RANGE
