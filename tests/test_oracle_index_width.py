"""Pins of the oracle's variable slot-index width (Section III-B.1: the number
of shared exponents k sets the width of the exponent index; Section III-C.1:
the index sits in the top bits of the column word) and of its k sweep
(Section IV-B, k = 2 ... 64).

Independent checks only: exact rational arithmetic of the format's definition
(the magnitude is the value on its slot's fixed-point grid, truncated toward
zero), integer splitting of the column word, the refinement of power-of-two
grids (a table that contains another gives every value a grid at least as
fine, so its truncation error cannot grow), and the all-exponents-shared
special case.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

KS = [1, 2, 3, 4, 5, 8, 9, 16, 17, 32, 33, 64]


def field(v: float) -> int:
    if v == 0.0:
        return 0
    m, ex = math.frexp(abs(v))
    f = ex - 1 + 1023
    return f if f >= 1 else 0


def wide_values(rng, n, binades):
    ex = rng.integers(-binades // 2, binades // 2, size=n)
    v = rng.uniform(1.0, 2.0, size=n) * np.exp2(ex.astype(float))
    v *= np.where(rng.random(n) < 0.5, -1.0, 1.0)
    v[rng.random(n) < 0.01] = 0.0
    return v


@pytest.mark.parametrize("k", KS)
def test_index_width_numbers_every_slot_and_no_more_bits(k):
    b = O.index_bits(k)
    assert 2 ** b >= k
    assert b == 0 or 2 ** (b - 1) < k


@pytest.mark.parametrize("k", [16, 64])
def test_encoder_against_exact_rationals_with_wide_tables(k):
    """Values over 80 binades fill a table of k; every word is the
    definition: slot of the smallest shared exponent above the value's field,
    F = floor(|v| 2^(1086 - SEM)) exactly, column word = col + slot 2^(32-b)."""
    rng = np.random.default_rng(k)
    n = 6000
    v = wide_values(rng, n, 80)
    rows = n // 10
    indptr = np.arange(0, n + 1, 10, dtype=np.int32)
    n_cols = 5000
    col = rng.integers(0, n_cols, size=n).astype(np.int32)
    for r in range(rows):  # CSR columns ascending within a row
        col[indptr[r]:indptr[r + 1]].sort()
    enc = O.encode(indptr, col, v, n_cols, num_exp=k)
    b = O.index_bits(k)
    assert enc.idx_bits == b
    sem = [int(s) for s in enc.sem[:k]]
    assert all(s > 0 for s in sem) and len(set(sem)) == k  # 80 binades: the table is full
    for i in range(n):
        e = field(float(v[i]))
        above = [(s, j) for j, s in enumerate(sem) if s > e]
        S, slot = min(above)
        word = int(enc.col_idx[i])
        assert word // 2 ** (32 - b) == slot and word % 2 ** (32 - b) == int(col[i])
        F = math.floor(abs(Fraction(float(v[i]))) * Fraction(2) ** (1086 - S))
        got = ((int(enc.head[i]) & 0x7FFF) << 48) | (int(enc.tail1[i]) << 32) | int(enc.tail2[i])
        assert got == F, (i, v[i], S)
        assert (int(enc.head[i]) >> 15) == (1 if math.copysign(1.0, v[i]) < 0 else 0)


@pytest.mark.parametrize("k", [1, 2, 4, 16, 64])
def test_column_field_limit_follows_the_index_width(k):
    b = O.index_bits(k)
    limit = min(2 ** (32 - b), 2 ** 31 - 1)  # int32 columns bound b = 0 and b = 1
    indptr = np.array([0, 1], np.int32)
    col = np.array([limit - 1], np.int32)
    enc = O.encode(indptr, col, np.array([3.0]), limit, num_exp=k)
    assert int(enc.column()[0]) == limit - 1 and int(enc.slot()[0]) == 0
    assert O.decode(enc, 3)[0] == 3.0
    if b > 1:
        # forced into the column word it no longer fits ...
        with pytest.raises(O.OracleError) as ei:
            O.encode(indptr, col, np.array([3.0]), limit + 1, num_exp=k, layout=0)
        assert ei.value.code == O.ERR_RANGE
        # ... so by default the index moves into the value (Section III-C.1)
        enc = O.encode(indptr, col, np.array([3.0]), limit + 1, num_exp=k)
        assert enc.layout == 1 and int(enc.column()[0]) == limit - 1
        assert O.decode(enc, 3)[0] == 3.0


def test_truncation_error_never_grows_with_k():
    """Tables of growing k contain each other (the k most frequent plus the
    forced maximum), so each value's grid only gets finer; truncation onto a
    finer power-of-two grid loses no more.  Per value and per segment count,
    |v - dec_s(v)| is non-increasing in k, and the exactly represented share
    is non-decreasing (Section IV-B's error trend)."""
    rng = np.random.default_rng(5)
    n = 20000
    v = wide_values(rng, n, 70)
    indptr = np.array([0, n], np.int32)
    col = np.arange(n, dtype=np.int32)
    prev_err = None
    prev_exact = -1
    prev_table = set()
    for k in (1, 2, 4, 8, 16, 32, 64):
        enc = O.encode(indptr, col, v, n, num_exp=k)
        table = {int(s) for s in enc.sem if s}
        assert prev_table <= table
        prev_table = table
        err = np.stack([np.abs(v - O.decode(enc, s)) for s in (1, 2, 3)])
        if prev_err is not None:
            assert np.all(err <= prev_err)
        exact = int(np.sum(err[2] == 0))
        assert exact >= prev_exact
        prev_err, prev_exact = err, exact
    assert prev_exact > 0.9 * n  # 64 slots cover 64 of the 70 binades


def test_all_exponents_shared_at_k64():
    """k at least the number of distinct exponents: every value's own field
    + 1 is shared, so the head is the value with its fraction cut to 14 bits
    and three segments give it back exactly."""
    rng = np.random.default_rng(9)
    v = wide_values(rng, 5000, 50)
    v = v[v != 0.0]
    indptr = np.array([0, v.size], np.int32)
    enc = O.encode(indptr, np.arange(v.size, dtype=np.int32), v, v.size, num_exp=64)
    cut = np.array([np.frombuffer(np.float64(x).tobytes(), np.uint64)[0] for x in v])
    cut &= ~np.uint64((1 << 38) - 1)
    assert np.array_equal(O.decode(enc, 1), cut.view(np.float64))
    assert np.array_equal(O.decode(enc, 3), v)
