"""Host model of the SpMV tile schedule (no GPU).

Replays, in Python, the index arithmetic of the tiled SpMV kernel (tile
ranges, the row range each tile writes, the staged non-zero window, the
vector-load groups of phase 1, the LDS product slots, the deferred-row list
and the long-row tail) and checks on the test matrices and the full-size
operators that every access stays inside its buffer and every row is written
by exactly one tile.  The constants mirror csrc/gse_internal.h.
"""
import numpy as np
import pytest

from workloads import (diagonal, diffusion3d, convdiff2d, fixed_rows, poisson2d, powerlaw,
                       random_sparse)

WG, EXTRA, SHORT, PAD, SPEC = 256, 256, 24, 16, 16


def lower_bound(a, v):
    return int(np.searchsorted(a, v, side="left"))


def walk(n_tiles, g):
    """Tiles visited by each persistent workgroup (mirrors TileWalk)."""
    seen = []
    for wg in range(g):
        xcd, local = wg & 7, wg >> 3
        nx = (g >> 3) + (1 if (g & 7) > xcd else 0)
        tb, te = (n_tiles * xcd) >> 3, (n_tiles * (xcd + 1)) >> 3
        seen += list(range(tb + local, te, nx))
    return seen


@pytest.mark.parametrize("n_tiles", [1, 5, 8, 9, 63, 1000, 7121])
@pytest.mark.parametrize("resident", [8, 1536, 2048])
def test_persistent_walk_covers_every_tile_once(n_tiles, resident):
    g = min(resident, (n_tiles + 7) // 8 * 8)
    g = max(g, 8)
    seen = walk(n_tiles, g)
    assert sorted(seen) == list(range(n_tiles))


def check(indptr, n_cols, cols, E):
    T = WG * E
    n_rows = indptr.size - 1
    nnz = int(indptr[-1])
    pad = (nnz + PAD - 1) // PAD * PAD
    n_tiles = max(1, -(-nnz // T))
    starts = indptr[:n_rows]
    tile_row = [lower_bound(starts, t * T) for t in range(n_tiles)] + [n_rows]
    nprod = (T + EXTRA) + (T + EXTRA) // 8
    ndef_cap = (T + EXTRA) // (SHORT + 1) + 2
    written = np.zeros(n_rows, np.int32)
    assert tile_row[0] == 0 or n_rows == 0
    for t in range(n_tiles):
        j0, j1 = t * T, min(t * T + T, nnz)
        ra, rb = tile_row[t], tile_row[t + 1]
        assert ra <= rb
        if ra == rb:
            continue
        js, je = int(indptr[ra]), int(indptr[rb])
        assert j0 <= js <= j1 and je >= j1 or rb == n_rows
        tail = (je - j1) <= EXTRA
        jl = je if tail else j1
        assert jl <= nnz and jl <= j1 + EXTRA
        # plane loads issued before the row lookup (main vector groups, bounded
        # by nnz only) and the one-element look-ahead of lanes < SPEC
        for b in [j0 + tid * E for tid in range(WG)]:
            if b < nnz:
                assert b % E == 0 and b + E <= pad
        # every staged non-zero [js, jl) lands in a valid LDS slot
        if jl > js:
            li = np.arange(js, jl) - j0
            slot = li + li // 8
            assert slot.min() >= 0 and slot.max() < nprod
            assert cols[js:jl].max() < n_cols
        # row pointers staged for rows ra .. ra + min(nr, 511)
        nr = rb - ra
        nstage = min(nr, 2 * WG - 1)
        assert ra + nstage <= n_rows
        ndef = 0
        for r in range(ra, rb):
            written[r] += 1
            s0, s1 = int(indptr[r]), int(indptr[r + 1])
            if not tail and r == rb - 1:
                assert s1 > j1 + EXTRA and s0 >= js
                continue
            assert js <= s0 <= s1 <= jl
            if s1 - s0 > SHORT:
                ndef += 1
        assert ndef <= ndef_cap
    assert np.all(written == 1)
    return n_tiles


MATS = {
    "poisson2d_64": lambda: poisson2d(64),
    "diffusion3d_24": lambda: diffusion3d(24, 0),
    "convdiff2d_64": lambda: convdiff2d(64, 1),
    "powerlaw_20k": lambda: powerlaw(20_000, 2),
    "random_empty_long": lambda: random_sparse(3000, 2500, 5, mean_row=4, empty_frac=0.2,
                                               long_rows=6, long_len=2400, exp_spread=60),
    "random_ragged": lambda: random_sparse(1777, 1901, 6, mean_row=9, exp_spread=20),
    "one_row_long": lambda: random_sparse(1, 9000, 7, mean_row=1, long_rows=1, long_len=8999),
    "tiny": lambda: random_sparse(3, 3, 8, mean_row=2),
    "empty": lambda: random_sparse(5, 5, 9, mean_row=0),
    "diagonal_3000": lambda: diagonal(3000, 10),
    "sparse_many_empty": lambda: random_sparse(6000, 6000, 9, mean_row=0.6, exp_spread=12),
    "fixed_rows_512x8": lambda: fixed_rows(512, 700, 8, 11),
    "fixed_rows_1000x3": lambda: fixed_rows(1000, 1200, 3, 12),
    "fixed_rows_777x5": lambda: fixed_rows(777, 800, 5, 13),
    "fixed_rows_1111x7": lambda: fixed_rows(1111, 1500, 7, 14),
    "fixed_rows_500x6": lambda: fixed_rows(500, 640, 6, 15),
    "random_rows_max7": lambda: random_sparse(2023, 2100, 23, mean_row=1.5, empty_frac=0.3,
                                              exp_spread=30),
    "random_rows_max9": lambda: random_sparse(2021, 2100, 21, mean_row=2, empty_frac=0.2,
                                              exp_spread=30),
}


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("E", [4, 8, 16])
def test_schedule_in_bounds(name, E):
    A = MATS[name]()
    check(A.indptr.astype(np.int64), A.n_cols, A.indices, E)


@pytest.mark.parametrize("E", [8])
def test_schedule_full_size_diffusion3d_128(E):
    A = diffusion3d(128, 0)
    assert check(A.indptr.astype(np.int64), A.n_cols, A.indices, E) == -(-A.nnz // (WG * E))


def check_short(indptr, n_cols, cols, E, look=32):
    """Index model of the short-row tile kernel (rows of at most 24)."""
    T = WG * E
    n_rows = indptr.size - 1
    nnz = int(indptr[-1])
    pad = (nnz + PAD - 1) // PAD * PAD
    lens = np.diff(indptr)
    assert lens.max(initial=0) <= SHORT
    n_tiles = max(1, -(-nnz // T))
    tile_row = [lower_bound(indptr[:n_rows], t * T) for t in range(n_tiles)] + [n_rows]
    ns = T + look + 8
    for t in range(n_tiles):
        j0, j1 = t * T, min(t * T + T, nnz)
        ra, rb = tile_row[t], tile_row[t + 1]
        for tid in range(WG):
            b = j0 + tid * E
            if b < nnz:
                assert b + E <= pad
            lb = j1 + tid * E
            if tid < look // E and lb < nnz:
                assert lb + E <= pad and T + tid * E + E <= ns
        for r in range(ra, rb):
            s0, s1 = int(indptr[r]), int(indptr[r + 1])
            o = s0 - j0
            assert 0 <= o < T
            # staged: main [0, T) and look-ahead [T, T + look); reads up to o+len-1
            assert o + (s1 - s0) <= T + look
            # unconditional 8-wide reads stay inside the LDS arrays
            last_read = o + ((max(s1 - s0, 1) - 1) // 8) * 8 + 7
            assert last_read < ns
            if s1 > s0:
                assert cols[s0:s1].max() < n_cols


@pytest.mark.parametrize("E", [4, 8, 16])
@pytest.mark.parametrize("name", ["poisson2d_64", "diffusion3d_24", "convdiff2d_64", "tiny",
                                  "empty", "random_ragged"])
def test_short_row_kernel_in_bounds(name, E):
    A = MATS[name]()
    if np.diff(A.indptr).max(initial=0) > SHORT:
        pytest.skip("rows longer than the short-row limit use the general kernel")
    check_short(A.indptr.astype(np.int64), A.n_cols, A.indices, E)


def test_short_row_kernel_full_size_diffusion3d_128():
    A = diffusion3d(128, 0)
    check_short(A.indptr.astype(np.int64), A.n_cols, A.indices, 4)


# ---- ring schedule (producer wave + LDS ring), short rows, 1024-nnz tiles ----
RING_T, RING_LOOK, RING_RP, RING_CONS = 1024, 32, 256, 192


def ring_layout(fmt, TL=RING_T + RING_LOOK, D=3):
    off_head = TL * 4
    off_t1 = off_head + TL * 2
    off_t2 = off_t1 + TL * 2
    off_val = TL * 4
    end = {0: off_val + TL * 8, 1: off_head + TL * 2, 2: off_t1 + TL * 2, 3: off_t2 + TL * 4}[fmt]
    stage = (end + RING_RP * 4 + 15) // 16 * 16
    # regions in the order the producer loads them: (name, offset, bytes,
    # elements per 16-byte chunk)
    order = [("col", 0, TL * 4, 4)]
    if fmt == 0:
        order.append(("val", off_val, TL * 8, 2))
    else:
        order.append(("head", off_head, TL * 2, 8))
        if fmt >= 2:
            order.append(("tail1", off_t1, TL * 2, 8))
        if fmt == 3:
            order.append(("tail2", off_t2, TL * 4, 4))
    loads = [(name, off, size, per, -(-size // 1024)) for name, off, size, per in order]
    ni = sum(n for *_, n in loads) + RING_RP // 64
    return dict(TL=TL, D=D, stage=stage, ni=ni, loads=loads, rps=end)


def window_limit(j0, jend, pad):
    """Exclusive chunk limit of a staged window (the producer's clamp)."""
    return min(max((jend + 15) // 16 * 16, j0 + 16), pad)


def check_ring(indptr, n_cols, cols, fmt):
    L = ring_layout(fmt)
    TL, T = L["TL"], RING_T
    n_rows = indptr.size - 1
    nnz = int(indptr[-1])
    assert nnz >= T  # the launcher's condition
    pad = (nnz + 15) // 16 * 16
    n_tiles = -(-nnz // T)
    # the producer's waits stay inside the 6-bit counter
    assert (L["D"] - 1) * L["ni"] < 64
    # every lane of every load writes 16 bytes at region + 1024 i + 16 l: the
    # bytes past a region's end land in the region loaded next (overwritten
    # later by the same wave); the row pointers, loaded last, fit exactly
    regions = L["loads"] + [("rps", L["rps"], RING_RP * 4, None, RING_RP // 64)]
    for k, (name, off, size, per, n) in enumerate(L["loads"]):
        spill_end = off + n * 1024
        nxt = regions[k + 1]
        assert nxt[1] == off + size, "regions are contiguous in load order"
        assert spill_end <= nxt[1] + nxt[2], name
    assert L["rps"] + (RING_RP // 64) * 256 == L["rps"] + RING_RP * 4 <= L["stage"]
    tile_row = [lower_bound(indptr[:n_rows], t * T) for t in range(n_tiles)] + [n_rows]
    for t in range(n_tiles):
        j0 = t * T
        ra, rb = tile_row[t], tile_row[t + 1]
        # chunks are clamped to the last one before the window's limit
        jlim = window_limit(j0, j0 + TL, pad)
        for name, off, size, per, n in L["loads"]:
            e = np.minimum(j0 + per * np.arange(n * 64), jlim - per)
            assert e.min() >= 0 and (e + per).max() <= pad
            # every position a consumer may read comes from its own chunk
            used = np.arange(min(TL, pad - j0))
            assert np.all(j0 + used // per * per <= jlim - per)
        if t < 1 or t >= n_tiles - 2:  # only the first and the last tiles clamp rows
            for i in range(RING_RP):
                assert 0 <= min(ra + i, n_rows) <= n_rows
        # consumers: staged positions read by each row (eight-wide batches)
        if rb > ra:
            s0 = indptr[ra:rb]
            ln = indptr[ra + 1:rb + 1] - s0
            o = s0 - j0
            assert o.min() >= 0 and o.max() < T and (o + ln).max() <= TL
            assert (o + (np.maximum(ln, 1) - 1) // 8 * 8 + 7).max() < TL
    assert int(cols.max(initial=0)) < n_cols
    assert L["D"] * L["stage"] <= 64 * 1024


@pytest.mark.parametrize("fmt", [0, 1, 2, 3])
@pytest.mark.parametrize("name", ["poisson2d_64", "diffusion3d_24", "convdiff2d_64", "random_ragged",
                                  "diagonal_3000", "sparse_many_empty", "fixed_rows_512x8",
                                  "random_rows_max9"])
def test_ring_kernel_in_bounds(name, fmt):
    A = MATS[name]()
    if np.diff(A.indptr).max(initial=0) > SHORT or A.indptr[-1] < RING_T:
        pytest.skip("the ring serves short rows in at least one full tile")
    check_ring(A.indptr.astype(np.int64), A.n_cols, A.indices, fmt)


def test_ring_kernel_full_size_diffusion3d_128():
    A = diffusion3d(128, 0)
    for fmt in (0, 1, 2, 3):
        check_ring(A.indptr.astype(np.int64), A.n_cols, A.indices, fmt)


# ---- row-tile ring (rows of at most B <= 8 non-zeros, 192 rows per tile) ----
ROW_TILE = RING_CONS


def batch_width(max_row):
    return 3 if max_row <= 3 else 5 if max_row <= 5 else 7 if max_row <= 7 else 8


def check_rows(indptr, n_cols, cols, fmt, D=2):
    n_rows = indptr.size - 1
    nnz = int(indptr[-1])
    lens = np.diff(indptr)
    B = batch_width(int(lens.max(initial=0)))
    assert lens.max(initial=0) <= B <= 8
    TL = ROW_TILE * B + 16
    L = ring_layout(fmt, TL, D)
    pad = (nnz + 15) // 16 * 16
    assert nnz >= RING_T  # the launcher's condition
    assert (L["D"] - 1) * L["ni"] < 64
    assert L["D"] * L["stage"] <= 64 * 1024
    regions = L["loads"] + [("rps", L["rps"], RING_RP * 4, None, RING_RP // 64)]
    for k, (name, off, size, per, n) in enumerate(L["loads"]):
        nxt = regions[k + 1]
        assert nxt[1] == off + size
        assert off + n * 1024 <= nxt[1] + nxt[2], name
        assert n * 1024 >= size  # the loads cover the region
    n_rt = -(-n_rows // ROW_TILE)
    covered = np.zeros(n_rows, np.int32)
    for t in range(n_rt):
        ra, rb = t * ROW_TILE, min(t * ROW_TILE + ROW_TILE, n_rows)
        ja = int(indptr[ra]) & ~15
        # exactly the tile's window: chunks clamped to the last one before
        # jlim, row pointers to rb
        jlim = window_limit(ja, int(indptr[rb]), pad)
        for name, off, size, per, n in L["loads"]:
            e = np.minimum(ja + per * np.arange(n * 64), jlim - per)
            assert e.min() >= 0 and (e + per).max() <= pad
            assert np.all(e % per == 0)
            # the tile's non-zeros come from their own (unclamped) chunks
            need = np.arange(int(indptr[ra]), int(indptr[rb]))
            if need.size:
                assert np.all(ja + (need - ja) // per * per <= jlim - per)
        staged_rows = np.minimum(ra + np.arange(RING_RP), rb)
        assert np.array_equal(staged_rows[:rb - ra + 1], np.arange(ra, rb + 1))
        assert ra + RING_RP - 1 >= rb  # staged row pointers ra .. rb
        s0 = indptr[ra:rb].astype(np.int64)
        ln = indptr[ra + 1:rb + 1] - s0
        o = s0 - ja
        covered[ra:rb] += 1
        if rb > ra:
            assert o.min() >= 0
            # every lane reads B staged entries from o, inside the stage
            assert (o + B - 1).max() < TL
            # the entries a row uses lie in chunks loaded from inside the planes
            assert (s0 + ln).max() <= nnz
    assert np.all(covered == 1)
    assert int(cols.max(initial=0)) < n_cols


@pytest.mark.parametrize("fmt", [0, 1, 2, 3])
@pytest.mark.parametrize("name", ["poisson2d_64", "diffusion3d_24", "convdiff2d_64", "diagonal_3000",
                                  "sparse_many_empty", "fixed_rows_512x8", "fixed_rows_1000x3",
                                  "fixed_rows_777x5", "fixed_rows_1111x7", "fixed_rows_500x6",
                                  "random_rows_max7"])
def test_row_ring_kernel_in_bounds(name, fmt):
    A = MATS[name]()
    if np.diff(A.indptr).max(initial=0) > 8 or A.indptr[-1] < RING_T:
        pytest.skip("the row-tile ring serves rows of at most eight in at least one full tile")
    check_rows(A.indptr.astype(np.int64), A.n_cols, A.indices, fmt)


def test_row_ring_kernel_full_size_operators():
    for A in (diffusion3d(128, 0), convdiff2d(1024, 0)):
        for fmt in (0, 1, 2, 3):
            check_rows(A.indptr.astype(np.int64), A.n_cols, A.indices, fmt)


def _random_structure(seed, n_rows, max_len, empty_frac):
    """Row lengths drawn from 0..max_len (a share of empty rows and of rows
    at the maximum), sorted random columns; only the index structure."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, max_len + 1, size=n_rows)
    lens[rng.random(n_rows) < empty_frac] = 0
    lens[rng.random(n_rows) < 0.2] = max_len
    indptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    n_cols = max(n_rows, max_len)
    cols = np.concatenate([np.sort(rng.choice(n_cols, size=l, replace=False)) for l in lens]
                          + [np.zeros(0, np.int64)]).astype(np.int32)
    return indptr, n_cols, cols


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("max_len", [1, 3, 4, 5, 6, 7, 8])
def test_row_ring_random_structures(seed, max_len):
    n_rows = (2500 if max_len == 1 else 700) + 97 * seed  # never a multiple of 192
    indptr, n_cols, cols = _random_structure(seed, n_rows, max_len, 0.1 * (seed % 3))
    if indptr[-1] < RING_T:
        pytest.skip("fewer non-zeros than one ring tile")
    for fmt in (0, 1, 2, 3):
        check_rows(indptr, n_cols, cols, fmt)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("max_len", [9, 16, 24])
def test_ring_random_structures(seed, max_len):
    indptr, n_cols, cols = _random_structure(seed, 900 + 131 * seed, max_len, 0.15)
    for fmt in (0, 1, 2, 3):
        check_ring(indptr, n_cols, cols, fmt)
