"""Pins of the oracle's GSE-SEM encoder and decoder.

Nothing here re-runs the oracle's own arithmetic.  The checks come from:
  * the format's definition (Section III-B.2): the stored magnitude is the
    value on its slot's fixed-point grid, truncated toward zero -- computed
    here with exact rational arithmetic (``fractions.Fraction``);
  * the 16-bit SEM word's stated properties (Section III-B.2: sign, exponent
    index, magnitude on the shared exponent's grid with the hidden one minDiff
    places down, truncated), which the head segment must have;
  * Algorithm 2's leading-one reconstruction of an FP64 value from the head,
    rebuilt here from IEEE fields, which must agree with the decoder on every
    head pattern;
  * IEEE special cases (all exponents shared: the head is the value with its
    fraction cut to 14 bits), hand-derived words, and invariants (nesting,
    the truncation bound, exact round trip iff no significand bit is shifted
    out).
"""
import collections
import json
import math
import os
import struct
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
W = {1: 15, 2: 31, 3: 63}


def field(v: float) -> int:
    """Biased exponent field via frexp (no bit operations)."""
    if v == 0.0:
        return 0
    m, ex = math.frexp(abs(v))  # |v| = m 2^ex, 0.5 <= m < 1
    f = ex - 1 + 1023
    return f if f >= 1 else 0


def slot_of(v: float, sem) -> int:
    e = field(v)
    cands = [(s, i) for i, s in enumerate(sem) if s > e and s != 0]
    return min(cands)[1]


def exact_F63(v: float, S: int) -> int:
    """floor(|v| * 2^(1086 - SEM)) with exact rationals."""
    return math.floor(abs(Fraction(v)) * Fraction(2) ** (1086 - S))


def bits(v: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", v))[0]


def from_bits(u: int) -> float:
    return struct.unpack("<d", struct.pack("<Q", u))[0]


def random_values(rng, n, spread=40):
    ex = rng.integers(-spread // 2, spread // 2, size=n)
    v = rng.uniform(1.0, 2.0, size=n) * np.exp2(ex.astype(float))
    v *= np.where(rng.random(n) < 0.5, -1.0, 1.0)
    v[rng.random(n) < 0.02] = 0.0
    return v


# ----------------------------------------------------------------------------
def test_golden_hand_encodings():
    rows = []
    with open(os.path.join(GOLDEN, "hand_encodings.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    assert len(rows) == 10
    for v, table, slot, h, t1, t2 in rows:
        sem = np.zeros(8, np.int16)
        tab = [int(s) for s in table.split(",")]
        sem[: len(tab)] = tab
        ci, hh, tt1, tt2 = O.encode_values(np.array([float(v)]), np.array([5]), sem)
        assert int(ci[0]) == (5 | (int(slot) << 29)), v
        assert int(hh[0]) == int(h, 16), (v, hex(hh[0]))
        assert int(tt1[0]) == int(t1, 16), (v, hex(tt1[0]))
        assert int(tt2[0]) == int(t2, 16), (v, hex(tt2[0]))


def test_paper_parameters_golden():
    g = json.load(open(os.path.join(GOLDEN, "paper_parameters.json")))
    for name, key in (("paper_cg", "cg"), ("paper_gmres", "gmres")):
        for k in ("l", "t", "m", "rsd_limit", "ndec_limit", "reldec_limit"):
            assert O.PRESETS[name][k] == g[key][k]
    p = O.make_params(preset="paper_gmres")
    assert p.restart == g["gmres_restart"]["value"]


def test_encoder_matches_exact_rational_definition():
    rng = np.random.default_rng(11)
    vals = random_values(rng, 4000, spread=60)
    sem = np.array([1024, 1020, 1030, 1012, 1003, 1040, 1000, 1060], np.int16)
    col = rng.integers(0, 2**29, size=vals.size).astype(np.int32)
    ci, h, t1, t2 = O.encode_values(vals, col, sem)
    for i, v in enumerate(vals):
        k = slot_of(v, sem)
        F = exact_F63(float(v), int(sem[k]))
        assert int(ci[i]) >> 29 == k
        assert int(ci[i]) & 0x1FFFFFFF == int(col[i])
        assert (int(h[i]) & 0x7FFF) == F >> 48
        assert int(t1[i]) == (F >> 32) & 0xFFFF
        assert int(t2[i]) == F & 0xFFFFFFFF
        assert (int(h[i]) >> 15) == (1 if math.copysign(1.0, v) < 0 else 0)


def test_encoder_subnormals_and_zero_match_definition():
    tiny = [5e-324, -5e-324, 2.2250738585072009e-308, 1e-310, 0.0, -0.0]
    sem = np.array([64, 1024, 0, 0, 0, 0, 0, 0], np.int16)
    ci, h, t1, t2 = O.encode_values(np.array(tiny), np.zeros(len(tiny), np.int32), sem)
    for i, v in enumerate(tiny):
        assert int(ci[i]) >> 29 == 0  # smallest shared exponent above field 0
        F = exact_F63(v, 64)
        got = ((int(h[i]) & 0x7FFF) << 48) | (int(t1[i]) << 32) | int(t2[i])
        assert got == F


@pytest.mark.parametrize("ei_bit", [0, 3])
def test_head_is_the_16_bit_sem_of_section_3b2(ei_bit):
    """The 16-bit SEM word of Section III-B.2 from the format's stated
    properties: the sign on top, an EI_bit-bit exponent index below it, and
    15 - EI_bit magnitude bits holding |v| on the grid of its shared exponent
    -- the hidden one made explicit minDiff places below the field's top
    (minDiff = SEM - exponent field, at least 1), the bits below the field
    dropped (truncation toward zero).  Checked against the head of the
    oracle's 64-bit words (the index in the value word when EI_bit > 0):
    magnitude by exact rationals, the leading one's position, the index."""
    rng = np.random.default_rng(3)
    vals = random_values(rng, 3000, spread=24)
    vals = vals[vals != 0]
    sem = np.array([1024, 1027, 1021, 1030, 1017, 1034, 1014, 1036], np.int16)
    ci, h, _, _ = O.encode_values(vals, np.zeros(vals.size, np.int32), sem,
                                  idx_bits=3, layout=1 if ei_bit else 0)
    width = 15 - ei_bit  # magnitude bits of the 16-bit word
    checked = 0
    for i, v in enumerate(vals):
        slot = slot_of(float(v), [int(t) for t in sem])
        S = int(sem[slot])
        min_diff = S - field(float(v))
        head = int(h[i])
        mag = head & ((1 << width) - 1)
        # |v| on the grid 2^(S - 1023 - width), truncated
        want = math.floor(abs(Fraction(float(v))) * Fraction(2) ** (width - (S - 1023)))
        assert mag == want, (v, S)
        assert head >> 15 == (1 if v < 0 else 0)
        if ei_bit:
            assert (head >> width) & ((1 << ei_bit) - 1) == slot
        else:
            assert int(ci[i]) >> 29 == slot
        if min_diff <= width:  # the hidden one is still inside the field
            assert mag.bit_length() == width - min_diff + 1
            checked += 1
        else:
            assert mag == 0
    assert checked > 1000


def test_decoder_agrees_with_algorithm2_on_every_head():
    """Algorithm 2 rebuilds the FP64 value from the head by the position of
    its leading one: exponent field SEM - (15 - pos), fraction = bits below
    the leading one.  Built here from IEEE fields for all 2^15 heads, both
    signs and several shared exponents."""
    sem = np.array([1024, 1100, 900, 64, 2047, 1500, 600, 1030], np.int16)
    hm = np.arange(1 << 15, dtype=np.int64)
    for slot in range(8):
        S = int(sem[slot])
        for sign in (0, 1):
            got = np.array([O.decode_one(slot << 29, int((sign << 15) | m), 0, 0, sem, 1)
                            for m in hm[:: 1 if slot in (0, 3) else 97]])
            ms = hm[:: 1 if slot in (0, 3) else 97]
            for m, g in zip(ms, got):
                m = int(m)
                if m == 0:
                    assert g == 0.0
                    continue
                pos = m.bit_length() - 1
                fld = S - (15 - pos)
                fracbits = (m - (1 << pos)) << (52 - pos)
                want = from_bits((sign << 63) | (fld << 52) | fracbits)
                assert g == want, (slot, sign, m)


def test_all_exponents_shared_is_ieee_truncation():
    """With every exponent in the table each value is an exact match: the
    head reads the value with its fraction cut to 14 bits, head+tail1 to 30
    bits, all three segments reproduce it."""
    rng = np.random.default_rng(5)
    v = rng.uniform(1.0, 2.0, 2000) * np.exp2(rng.integers(-3, 4, 2000).astype(float))
    v *= np.where(rng.random(2000) < 0.5, -1, 1)
    indptr = np.array([0, v.size], np.int32)
    enc = O.encode(indptr, np.zeros(v.size, np.int32), v, 1)
    assert enc.exact_frac == 1.0
    for s, keep in ((1, 14), (2, 30), (3, 52)):
        d = O.decode(enc, s)
        mask = ~((1 << (52 - keep)) - 1) & 0xFFFFFFFFFFFFFFFF
        want = np.array([from_bits(bits(float(x)) & mask) for x in v])
        assert np.array_equal(d, want), s
    assert np.all(enc.eta[2] == 0.0)


def test_nesting_bound_and_roundtrip():
    rng = np.random.default_rng(7)
    v = random_values(rng, 6000, spread=50)
    indptr = np.array([0, v.size], np.int32)
    enc = O.encode(indptr, np.zeros(v.size, np.int32), v, 1)
    sem = [int(s) for s in enc.sem]
    d = {s: O.decode(enc, s) for s in (1, 2, 3)}
    for i, x in enumerate(v):
        k = int(enc.col_idx[i]) >> 29
        S = sem[k]
        a = abs(Fraction(float(x)))
        prev = Fraction(0)
        for s in (1, 2, 3):
            ds = abs(Fraction(float(d[s][i])))
            assert ds <= a
            assert ds >= prev
            assert a - ds < Fraction(2) ** (S - 1023 - W[s])
            if ds != 0:
                assert math.copysign(1, d[s][i]) == math.copysign(1, x)
            prev = ds
        e = field(float(x))
        min_diff = S - max(e, 1)
        if x != 0 and e >= 1:
            # all segments reproduce v exactly iff no significand bit is
            # shifted out: minDiff <= 11, or the dropped low bits are zero
            sig = (1 << 52) | (bits(float(x)) & ((1 << 52) - 1))
            lossless = min_diff <= 11 or sig % (1 << (min_diff - 11)) == 0
            assert (d[3][i] == x) == lossless, (x, min_diff)


def test_table_selection_against_counter():
    rng = np.random.default_rng(9)
    for trial in range(60):
        n = int(rng.integers(1, 400))
        spread = int(rng.integers(1, 30))
        v = random_values(rng, n, spread=spread)
        hist, nf = O.exponent_histogram(v)
        assert nf == 0
        cnt = collections.Counter(field(float(x)) for x in v)
        assert all(hist[e] == c for e, c in cnt.items())
        k = int(rng.integers(1, 9))
        sem = O.select_shared_exponents(hist, k)
        cands = sorted(((c, e) for e, c in cnt.items() if e != 0), reverse=True)
        top = [e for c, e in cands[:k]]
        if not top:
            assert list(sem) == [1024] + [0] * 7
            continue
        emax = max(e for e in cnt if e != 0)
        if emax not in top:
            top[-1] = emax
        assert [int(s) for s in sem[: len(top)]] == [e + 1 for e in top]
        assert all(s == 0 for s in sem[len(top):])
        # every value has a shared exponent above its own
        assert all(any(s > field(float(x)) for s in sem) for x in v)


def test_table_ties_and_max_rule():
    hist = np.zeros(2048, np.uint32)
    hist[1000] = 5
    hist[1001] = 5
    hist[1002] = 9
    hist[1010] = 1
    sem = O.select_shared_exponents(hist, 2)
    assert list(sem[:2]) == [1003, 1011]  # 1002 first; max rule replaces slot 1
    sem = O.select_shared_exponents(hist, 3)
    assert list(sem[:3]) == [1003, 1002, 1011]  # tie 1000/1001 -> larger; then max rule
    sem = O.select_shared_exponents(hist, 8)
    assert list(sem[:4]) == [1003, 1002, 1001, 1011]
    hist[0] = 1000  # zeros never enter the table
    assert 1 not in list(O.select_shared_exponents(hist, 8))
    hist2 = np.zeros(2048, np.uint32)
    hist2[40] = 3
    with pytest.raises(O.OracleError):
        O.select_shared_exponents(hist2, 8)


def test_nonfinite_rejected():
    indptr = np.array([0, 2], np.int32)
    for bad in (np.inf, -np.inf, np.nan):
        with pytest.raises(O.OracleError) as ei:
            O.encode(indptr, np.array([0, 1], np.int32), np.array([1.0, bad]), 2)
        assert ei.value.code == O.ERR_NONFINITE


def test_reused_table_must_cover():
    indptr = np.array([0, 2], np.int32)
    sem = np.array([1024] + [0] * 7, np.int16)
    e = O.encode(indptr, np.array([0, 1], np.int32), np.array([1.5, -0.25]), 2, sem_in=sem)
    assert list(e.sem) == list(sem)
    with pytest.raises(O.OracleError) as ei:
        O.encode(indptr, np.array([0, 1], np.int32), np.array([1.5, 4.0]), 2, sem_in=sem)
    assert ei.value.code == O.ERR_RANGE


def test_eta_definition_small():
    """eta_s = ||A - A_s||_inf / ||A||_inf computed from the exact decodes."""
    rng = np.random.default_rng(2)
    from workloads import random_sparse
    A = random_sparse(60, 50, 4, mean_row=5, exp_spread=30)
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    for s in (1, 2, 3):
        d = O.decode(enc, s)
        num = max((sum(abs(Fraction(float(A.data[j])) - Fraction(float(d[j])))
                       for j in range(A.indptr[r], A.indptr[r + 1])) for r in range(A.n_rows)))
        den = max((sum(abs(Fraction(float(A.data[j])))
                       for j in range(A.indptr[r], A.indptr[r + 1])) for r in range(A.n_rows)))
        assert enc.eta[s - 1] == pytest.approx(float(num / den), rel=1e-12, abs=1e-300)
