"""Pins of the oracle's index-in-value layout (Algorithm 1 with EI_bit = b,
the fallback of Section III-C.1 when the column field is too narrow): the
64-bit word is sign | slot (b bits) | magnitude on a 63 - b bit field, so the
head keeps 15 - b magnitude bits and the column word is the bare column.

Independent checks: exact rational arithmetic of the definition, the
properties Algorithm 1 states for its 16-bit word (the hidden one made
explicit at bit 15 - EI_bit - minDiff, the fraction below it truncated, the
index in the bits under the sign), the identity between the two layouts
(truncating the column-layout field by b more bits gives the value-layout
field: floor(floor(x) / 2^b) = floor(x / 2^b)), and the truncation bound.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def field(v: float) -> int:
    if v == 0.0:
        return 0
    m, ex = math.frexp(abs(v))
    f = ex - 1 + 1023
    return f if f >= 1 else 0


def matrix(k, seed=0, n=4000, binades=40):
    rng = np.random.default_rng(seed)
    ex = rng.integers(-binades // 2, binades // 2, size=n)
    v = rng.uniform(1.0, 2.0, size=n) * np.exp2(ex.astype(float))
    v *= np.where(rng.random(n) < 0.5, -1.0, 1.0)
    v[rng.random(n) < 0.01] = 0.0
    indptr = np.arange(0, n + 1, 8, dtype=np.int32)
    col = np.tile(np.arange(8, dtype=np.int32), n // 8) * 97
    return indptr, col, v


@pytest.mark.parametrize("k", [2, 8, 16, 64])
def test_value_layout_against_exact_rationals(k):
    indptr, col, v = matrix(k)
    enc = O.encode(indptr, col, v, 1000, num_exp=k, layout=1)
    b = O.index_bits(k)
    assert enc.layout == 1 and enc.idx_bits == b
    assert np.array_equal(enc.col_idx, col.astype(np.uint32))  # the bare column
    sem = [int(s) for s in enc.sem[:k]]
    for i in range(v.size):
        e = field(float(v[i]))
        S, slot = min((s, j) for j, s in enumerate(sem) if s > e)
        F = math.floor(abs(Fraction(float(v[i]))) * Fraction(2) ** (1086 - b - S))
        h = int(enc.head[i])
        assert h >> 15 == (1 if math.copysign(1.0, v[i]) < 0 else 0)
        if b:
            assert (h >> (15 - b)) & ((1 << b) - 1) == slot
        mag = ((h & (0x7FFF >> b)) << 48) | (int(enc.tail1[i]) << 32) | int(enc.tail2[i])
        assert mag == F, (i, v[i])


@pytest.mark.parametrize("b_k", [(1, 2), (3, 8), (4, 16)])
def test_head_has_algorithm1_properties(b_k):
    """For each non-zero value the 16-bit head is Algorithm 1's word with
    EI_bit = b: sign at bit 15, the index in bits 14 .. 15 - b, and -- when
    minDiff <= 15 - b -- the explicit one at bit 15 - b - minDiff with the
    value's leading fraction bits below it, cut toward zero."""
    b, k = b_k
    indptr, col, v = matrix(k, seed=b)
    enc = O.encode(indptr, col, v, 1000, num_exp=k, layout=1)
    sem = [int(s) for s in enc.sem[:k]]
    checked = 0
    for i in range(v.size):
        if v[i] == 0.0:
            continue
        e = field(float(v[i]))
        S = min(s for s in sem if s > e)
        min_diff = S - e
        h = int(enc.head[i])
        mag = h & (0x7FFF >> b)
        if min_diff > 15 - b:
            assert mag == 0  # the explicit one shifted out of the head
            continue
        lead = 15 - b - min_diff
        assert mag >> lead == 1  # explicit one, nothing above it
        frac_bits = lead  # fraction bits the head keeps below the one
        m, _ = math.frexp(abs(float(v[i])))  # 0.5 <= m < 1: m * 2 = 1.f
        frac = Fraction(m) * 2 - 1
        assert mag & ((1 << frac_bits) - 1) == math.floor(frac * 2 ** frac_bits)
        checked += 1
    assert checked > 1000


@pytest.mark.parametrize("k", [2, 8, 64])
def test_value_layout_field_is_the_column_layout_field_cut_by_b_bits(k):
    indptr, col, v = matrix(k, seed=7)
    e0 = O.encode(indptr, col, v, 1000, num_exp=k, layout=0)
    e1 = O.encode(indptr, col, v, 1000, num_exp=k, layout=1)
    b = O.index_bits(k)
    assert np.array_equal(e0.sem, e1.sem)
    f0 = ((e0.head.astype(np.uint64) & 0x7FFF) << 48) | (e0.tail1.astype(np.uint64) << 32) | \
        e0.tail2.astype(np.uint64)
    f1 = ((e1.head.astype(np.uint64) & np.uint64(0x7FFF >> b)) << 48) | \
        (e1.tail1.astype(np.uint64) << 32) | e1.tail2.astype(np.uint64)
    assert np.array_equal(f1, f0 >> np.uint64(b))
    assert np.array_equal(e1.slot(), e0.slot())


@pytest.mark.parametrize("k", [8, 64])
def test_value_layout_nesting_and_bound(k):
    indptr, col, v = matrix(k, seed=11)
    enc = O.encode(indptr, col, v, 1000, num_exp=k, layout=1)
    b = O.index_bits(k)
    d = [np.abs(O.decode(enc, s)) for s in (1, 2, 3)]
    a = np.abs(v)
    assert np.all(d[0] <= d[1]) and np.all(d[1] <= d[2]) and np.all(d[2] <= a)
    table = enc.table
    S = table[enc.slot()].astype(float)
    for s, W in ((1, 15 - b), (2, 31 - b), (3, 63 - b)):
        grid = np.exp2(S - 1023 - W)
        assert np.all(a - d[s - 1] < grid)
    # each segment count reads the truncated value: s = 3 is exact whenever
    # minDiff + b <= 11 (no significand bit leaves the 63 - b bit field)
    e = np.array([field(float(x)) for x in v])
    md = S - np.maximum(e, 1)
    exact = (md + b <= 11) & (v != 0.0)
    assert np.all(d[2][exact] == a[exact])


def test_spmv_and_cg_read_the_value_layout():
    """The oracle's SpMV on a value-layout encoding keeps the componentwise
    format bound |y_s,i - (Ax)_i| <= sum_j 2^(SEM_j - 1023 - W_s) |x_j|
    (+ FP64 rounding) with the layout's W_s = 15 - b, 31 - b, 63 - b, and its
    stepped CG reaches 1e-10 on it."""
    from workloads import diffusion3d, rhs_from_solution
    A = diffusion3d(8, 2)
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols, layout=1)
    b = enc.idx_bits
    x = np.random.default_rng(1).uniform(-1, 1, A.n_cols)
    exact = A.to_scipy() @ x
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.indptr))
    S = enc.table[enc.slot()].astype(float)
    absum = np.zeros(A.n_rows)
    np.add.at(absum, rows, np.abs(A.data * x[A.indices]))
    for s, W in ((1, 15 - b), (2, 31 - b), (3, 63 - b)):
        y = O.gse_spmv(A.indptr, enc, s, x)
        bound = np.zeros(A.n_rows)
        np.add.at(bound, rows, np.exp2(S - 1023 - W) * np.abs(x[A.indices]))
        assert np.all(np.abs(y - exact) <= bound + 1e-14 * absum)
    _, rhs = rhs_from_solution(A, 2)
    prm = O.make_params(tol=1e-10, max_iter=5000, switch_mode=0, orth=1)
    r = O.cg(A.indptr, rhs, prm, A.indices, A.data, enc)
    assert r.status == O.OK and r.relres_true <= 1e-10
