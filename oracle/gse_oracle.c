/*
 * gse_oracle.c -- sequential CPU oracle (TEST INFRASTRUCTURE; see header).
 *
 * Each function names the passage of the paper it restates.  Everything is
 * FP64 and sequential; sums run in row order, exactly as written in the
 * definitions.  Build: gcc -O2 -std=c99 -ffp-contract=off -fPIC -shared.
 */
#include "gse_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static uint64_t bits_of(double v) { uint64_t u; memcpy(&u, &v, sizeof u); return u; }

/* Section III-B.1: the number of shared exponents sets the width of the
 * exponent index -- the fewest bits that number k slots, ceil(log2 k)
 * (0 bits for a single shared exponent). */
int or_index_bits(int num_exp) {
    int b = 0;
    while ((1 << b) < num_exp) b += 1;
    return b;
}

/* Where the slot index lives (Section III-C.1): in the top idx_bits bits
 * of the column word (layout 0), or -- Algorithm 1's EI_bit, the fallback
 * when the column field is too narrow -- in the top idx_bits bits of the
 * value word below its sign (layout 1), where it takes magnitude bits. */
static uint32_t column_of(uint32_t word, int idx_bits, int layout) {
    if (layout == 1 || idx_bits == 0) return word;
    return word & (0xFFFFFFFFu >> idx_bits);
}

static int slot_of(uint32_t word, uint16_t head, int idx_bits, int layout) {
    if (idx_bits == 0) return 0;
    if (layout == 1) return (int)((head >> (15 - idx_bits)) & ((1u << idx_bits) - 1u));
    return (int)(word >> (32 - idx_bits));
}

/* Bits of the magnitude field: 63, less the index when it sits in the value. */
static int field_bits(int idx_bits, int layout) { return layout == 1 ? 63 - idx_bits : 63; }

/* ------------------------------------------------------------------------ */
/* Section III-B.1: occurrences N_i of every distinct exponent e_i.  The    */
/* 11-bit biased exponent field is the key; field 2047 (Inf/NaN) is counted */
/* and reported so the caller can reject the input.                         */
int64_t or_exponent_histogram(const double* val, int64_t nnz, uint32_t* hist) {
    int64_t nonfinite = 0;
    memset(hist, 0, 2048 * sizeof(uint32_t));
    for (int64_t i = 0; i < nnz; ++i) {
        unsigned e = (unsigned)((bits_of(val[i]) >> 52) & 0x7FF);
        hist[e] += 1;
        if (e == 2047) nonfinite += 1;
    }
    return nonfinite;
}

/* Section III-B.1 (sort exponents by occurrence, descending; keep the k most
 * frequent) and Section III-B.2 (store each shared exponent incremented by
 * one; the maximum exponent must be one of them so every value has a shared
 * exponent above its own).
 * Readings: field 0 (zero / subnormal) is never a candidate; ties in count go
 * to the larger exponent; when the maximum exponent is not among the k most
 * frequent it replaces the last (least frequent) slot; unused slots are 0; a
 * set without any normal value gets the single slot 1023+1.
 * Returns the number of slots used, or OR_ERR_RANGE when a shared exponent is
 * below 63 (its fixed-point grid would leave the normal FP64 range). */
int or_select_shared_exponents(const uint32_t* hist, int num_exp, int16_t* sem) {
    if (num_exp < 1 || num_exp > OR_MAX_EXP) return OR_ERR_ARG;
    unsigned char taken[2048];
    memset(taken, 0, sizeof taken);
    int chosen[OR_MAX_EXP];
    int used = 0;
    for (int slot = 0; slot < num_exp; ++slot) {
        int best = -1;
        for (int e = 2046; e >= 1; --e) {  /* high to low: ties keep the larger e */
            if (taken[e] || hist[e] == 0) continue;
            if (best < 0 || hist[e] > hist[best]) best = e;
        }
        if (best < 0) break;
        taken[best] = 1;
        chosen[used++] = best;
    }
    int max_e = 0;
    for (int e = 2046; e >= 1; --e)
        if (hist[e] > 0) { max_e = e; break; }
    if (used == 0) {
        chosen[0] = 1023;
        used = 1;
    } else if (!taken[max_e]) {
        chosen[used - 1] = max_e;
    }
    for (int i = 0; i < OR_MAX_EXP; ++i) sem[i] = 0;
    for (int i = 0; i < used; ++i) {
        if (chosen[i] < 63) return OR_ERR_RANGE;
        sem[i] = (int16_t)(chosen[i] + 1);
    }
    return used;
}

/* Algorithm 1 restated for the 64-bit SEM word with the index kept in the
 * column (Section III-C.1).  Steps, in the paper's order:
 *   sign and exponent field of the value;
 *   if exp+1 is a shared exponent, that slot, with minDiff = 1;
 *   otherwise the slot whose shared exponent is the nearest one above exp,
 *   minDiff = SEM - exp;
 *   the significand with its hidden one made explicit is shifted right by
 *   minDiff (denormalisation) -- here onto a 63-bit field, so the field is
 *   (hidden|fraction) << (11 - minDiff), truncated toward zero when the
 *   shift is to the right;
 *   sign, index and magnitude are packed.
 * A subnormal or zero value has no hidden one and the exponent of the
 * smallest normal (1) for the shift.  Returns OR_ERR_RANGE if a value has no
 * shared exponent above its own (possible only with a reused table). */
int or_encode_values(const double* val, const int32_t* col, int64_t nnz,
                     const int16_t* sem, int idx_bits, int layout, uint32_t* col_idx,
                     uint16_t* head, uint16_t* tail1, uint32_t* tail2) {
    if (idx_bits < 0 || idx_bits > 6 || (layout != 0 && layout != 1)) return OR_ERR_ARG;
    const int fb = field_bits(idx_bits, layout);
    for (int64_t i = 0; i < nnz; ++i) {
        uint64_t u = bits_of(val[i]);
        unsigned sign = (unsigned)(u >> 63);
        int e = (int)((u >> 52) & 0x7FF);
        uint64_t frac = u & ((1ull << 52) - 1);
        int slot = -1;
        int min_diff = 0;
        for (int k = 0; k < OR_MAX_EXP; ++k) {
            if (sem[k] != 0 && sem[k] == e + 1) { slot = k; min_diff = 1; break; }
        }
        if (slot < 0) {
            int best = 1 << 30;
            for (int k = 0; k < OR_MAX_EXP; ++k) {
                int d = (int)sem[k] - e;
                if (sem[k] != 0 && d > 0 && d < best) { best = d; slot = k; }
            }
            if (slot < 0) return OR_ERR_RANGE;
            min_diff = best;
        }
        uint64_t sig = (e > 0) ? ((1ull << 52) | frac) : frac;
        int shift_exp = (e > 0) ? e : 1;
        /* the field holds fb bits: the hidden one of a value with minDiff = 1
         * lands on its top bit (bit fb - 1) */
        int sh = (fb - 52) - ((int)sem[slot] - shift_exp);
        uint64_t F;
        if (sh >= 0) F = sig << sh;
        else if (-sh >= 64) F = 0;
        else F = sig >> (-sh);
        (void)min_diff;
        if (slot >= (1 << idx_bits)) return OR_ERR_ARG;
        unsigned idx_in_head = 0;
        if (layout == 1) {
            col_idx[i] = (uint32_t)col[i];
            if (idx_bits > 0) idx_in_head = (unsigned)slot << (15 - idx_bits);
        } else {
            col_idx[i] = (uint32_t)col[i] |
                         (idx_bits == 0 ? 0u : ((uint32_t)slot << (32 - idx_bits)));
        }
        head[i] = (uint16_t)((sign << 15) | idx_in_head | (unsigned)(F >> 48));
        tail1[i] = (uint16_t)((F >> 32) & 0xFFFF);
        tail2[i] = (uint32_t)(F & 0xFFFFFFFFu);
    }
    return OR_OK;
}

/* Algorithm 2 and its two wider variants (Section III-C.2): the value read
 * with s segments is +-F_W * 2^(SEM - 1023 - W), W = 15, 31, 63, where F_W is
 * the top W magnitude bits of the SEM word; a zero field reads as 0. */
double or_decode_one(uint32_t col_word, uint16_t h, uint16_t t1, uint32_t t2,
                     const int16_t* sem, int idx_bits, int layout, int s) {
    int slot = slot_of(col_word, h, idx_bits, layout);
    int fb = field_bits(idx_bits, layout);
    /* s segments keep the head's magnitude bits, then 16 and 32 more */
    int W = fb - ((s == 1) ? 48 : (s == 2) ? 32 : 0);
    uint64_t head_mag = (uint64_t)(h & (0x7FFFu >> (63 - fb)));
    uint64_t Ff = (head_mag << 48) | ((uint64_t)t1 << 32) | (uint64_t)t2;
    uint64_t F = Ff >> (fb - W);
    if (F == 0) return 0.0;
    double mag = ldexp((double)F, (int)sem[slot] - 1023 - W);
    return (h >> 15) ? -mag : mag;
}

void or_decode(const uint32_t* col_idx, const uint16_t* head, const uint16_t* tail1,
               const uint32_t* tail2, int64_t nnz, const int16_t* sem, int idx_bits,
               int layout, int s, double* out) {
    for (int64_t i = 0; i < nnz; ++i)
        out[i] = or_decode_one(col_idx[i], head[i], tail1[i], tail2[i], sem, idx_bits, layout,
                               s);
}

/* Whole conversion: histogram, table, per-value words, and the relative
 * perturbation eta_s = ||A - A_s||_inf / ||A||_inf of each segment count. */
int or_encode(const int32_t* row_ptr, const int32_t* col, const double* val,
              int32_t n_rows, int32_t n_cols, int64_t nnz, int num_exp, int layout,
              const int16_t* sem_in, int16_t* sem_out, uint32_t* col_idx,
              uint16_t* head, uint16_t* tail1, uint32_t* tail2, double* eta3,
              double* exact_frac, int* layout_out) {
    if (n_rows < 0 || n_cols < 0 || nnz < 0 || num_exp < 1 || num_exp > OR_MAX_EXP)
        return OR_ERR_ARG;
    int idx_bits = or_index_bits(num_exp);
    /* the column field keeps 32 - idx_bits bits; past that the index moves
     * into the value (layout -1 chooses so, Section III-C.1) */
    if (layout < 0) layout = ((int64_t)n_cols > (1ll << (32 - idx_bits))) ? 1 : 0;
    if (layout != 0 && layout != 1) return OR_ERR_ARG;
    if (layout_out) *layout_out = layout;
    if ((layout == 0 && (int64_t)n_cols > (1ll << (32 - idx_bits))) || nnz >= (1ll << 31))
        return OR_ERR_RANGE;
    uint32_t* hist = (uint32_t*)malloc(2048 * sizeof(uint32_t));
    if (!hist) return OR_ERR_ARG;
    if (or_exponent_histogram(val, nnz, hist) > 0) { free(hist); return OR_ERR_NONFINITE; }
    int rc;
    if (sem_in) {
        for (int i = 0; i < OR_MAX_EXP; ++i) sem_out[i] = (i < num_exp) ? sem_in[i] : 0;
        for (int i = 0; i < OR_MAX_EXP; ++i) {
            if (sem_out[i] != 0 && sem_out[i] < 64) { free(hist); return OR_ERR_RANGE; }
            for (int k = 0; k < i; ++k)
                if (sem_out[i] != 0 && sem_out[k] == sem_out[i]) { free(hist); return OR_ERR_ARG; }
        }
    } else {
        rc = or_select_shared_exponents(hist, num_exp, sem_out);
        if (rc < 0) { free(hist); return rc; }
    }
    uint64_t covered = 0;
    for (int i = 0; i < OR_MAX_EXP; ++i)
        if (sem_out[i] > 0) covered += hist[sem_out[i] - 1];
    if (exact_frac) *exact_frac = nnz ? (double)covered / (double)nnz : 1.0;
    free(hist);
    rc = or_encode_values(val, col, nnz, sem_out, idx_bits, layout, col_idx, head, tail1, tail2);
    if (rc != OR_OK) return rc;
    if (eta3) {
        double amax = 0.0, emax[3] = {0.0, 0.0, 0.0};
        for (int32_t r = 0; r < n_rows; ++r) {
            double a = 0.0, es[3] = {0.0, 0.0, 0.0};
            for (int32_t j = row_ptr[r]; j < row_ptr[r + 1]; ++j) {
                a += fabs(val[j]);
                for (int s = 1; s <= 3; ++s)
                    es[s - 1] += fabs(val[j] - or_decode_one(col_idx[j], head[j], tail1[j],
                                                             tail2[j], sem_out, idx_bits, layout,
                                                             s));
            }
            if (a > amax) amax = a;
            for (int s = 0; s < 3; ++s) if (es[s] > emax[s]) emax[s] = es[s];
        }
        for (int s = 0; s < 3; ++s) eta3[s] = amax > 0.0 ? emax[s] / amax : 0.0;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Section III-B.1, last part: for a low preprocessing cost the matrix is cut
 * into row blocks and the exponent distribution of one randomly drawn row of
 * each block stands for the distribution of that block.  Reading taken: every
 * block of block_rows rows (the last one may be shorter) gets a table of its
 * own, of the same size k and index width as a global table.  The table is
 * selected as for the whole matrix (count descending, ties to the larger
 * exponent, the sample's maximum forced in) from the histogram of the sample:
 * the drawn row (sample_rows[b], a row of block b) or, with sample_rows NULL,
 * every value of the block.  A drawn row need not hold the block's largest
 * exponent, which every value of the block needs a shared exponent above
 * (Section III-B.2): when the table misses it, it takes the next free slot,
 * or the last slot when all k are in use.  Tables are written to
 * block_sem[b * OR_MAX_EXP + i]; row r reads the table of block r / block_rows. */
static int block_table(const uint32_t* sample_hist, int block_max_e, int num_exp,
                       int16_t* sem) {
    int used = or_select_shared_exponents(sample_hist, num_exp, sem);
    if (used < 0) return used;
    if (block_max_e <= 0) return used;
    for (int i = 0; i < used; ++i)
        if (sem[i] == block_max_e + 1) return used;
    /* a shared exponent below 63 would put its grid below the normal range
     * (the same rule as for the sample's own choice) */
    if (block_max_e < 63) return OR_ERR_RANGE;
    if (used < num_exp) used += 1;
    sem[used - 1] = (int16_t)(block_max_e + 1);
    return used;
}

static const int16_t* table_of_row(const int16_t* block_sem, int32_t block_rows, int32_t r) {
    return block_sem + (int64_t)(r / block_rows) * OR_MAX_EXP;
}

int or_encode_blocks(const int32_t* row_ptr, const int32_t* col, const double* val,
                     int32_t n_rows, int32_t n_cols, int64_t nnz, int num_exp, int layout,
                     int32_t block_rows, const int32_t* sample_rows, int16_t* block_sem,
                     uint32_t* col_idx, uint16_t* head, uint16_t* tail1, uint32_t* tail2,
                     double* eta3, double* exact_frac, int* layout_out) {
    if (n_rows < 0 || n_cols < 0 || nnz < 0 || num_exp < 1 || num_exp > OR_MAX_EXP ||
        block_rows < 1)
        return OR_ERR_ARG;
    int idx_bits = or_index_bits(num_exp);
    if (layout < 0) layout = ((int64_t)n_cols > (1ll << (32 - idx_bits))) ? 1 : 0;
    if (layout != 0 && layout != 1) return OR_ERR_ARG;
    if (layout_out) *layout_out = layout;
    if ((layout == 0 && (int64_t)n_cols > (1ll << (32 - idx_bits))) || nnz >= (1ll << 31))
        return OR_ERR_RANGE;
    uint32_t* own = (uint32_t*)malloc(2048 * sizeof(uint32_t));
    uint32_t* sample = (uint32_t*)malloc(2048 * sizeof(uint32_t));
    if (!own || !sample) { free(own); free(sample); return OR_ERR_ARG; }
    int32_t n_blocks = (int32_t)(((int64_t)n_rows + block_rows - 1) / block_rows);
    uint64_t covered = 0;
    int rc = OR_OK;
    for (int32_t bk = 0; bk < n_blocks && rc == OR_OK; ++bk) {
        int32_t r0 = bk * block_rows;
        int32_t r1 = (int32_t)((int64_t)r0 + block_rows < n_rows ? r0 + block_rows : n_rows);
        int64_t j0 = row_ptr[r0], j1 = row_ptr[r1];
        /* the block's own exponents: for the coverage count and its maximum */
        if (or_exponent_histogram(val + j0, j1 - j0, own) > 0) { rc = OR_ERR_NONFINITE; break; }
        int max_e = 0;
        for (int e = 2046; e >= 1; --e)
            if (own[e] > 0) { max_e = e; break; }
        const uint32_t* hist = own;
        if (sample_rows) {
            int32_t sr = sample_rows[bk];
            if (sr < r0 || sr >= r1) { rc = OR_ERR_ARG; break; }
            or_exponent_histogram(val + row_ptr[sr], row_ptr[sr + 1] - row_ptr[sr], sample);
            hist = sample;
        }
        int16_t* sem = block_sem + (int64_t)bk * OR_MAX_EXP;
        int used = block_table(hist, max_e, num_exp, sem);
        if (used < 0) { rc = used; break; }
        for (int i = 0; i < used; ++i) covered += own[sem[i] - 1];
        rc = or_encode_values(val + j0, col + j0, j1 - j0, sem, idx_bits, layout, col_idx + j0,
                              head + j0, tail1 + j0, tail2 + j0);
    }
    free(own);
    free(sample);
    if (rc != OR_OK) return rc;
    if (exact_frac) *exact_frac = nnz ? (double)covered / (double)nnz : 1.0;
    if (eta3) {
        double amax = 0.0, emax[3] = {0.0, 0.0, 0.0};
        for (int32_t r = 0; r < n_rows; ++r) {
            const int16_t* sem = table_of_row(block_sem, block_rows, r);
            double a = 0.0, es[3] = {0.0, 0.0, 0.0};
            for (int32_t j = row_ptr[r]; j < row_ptr[r + 1]; ++j) {
                a += fabs(val[j]);
                for (int s = 1; s <= 3; ++s)
                    es[s - 1] += fabs(val[j] - or_decode_one(col_idx[j], head[j], tail1[j],
                                                             tail2[j], sem, idx_bits, layout, s));
            }
            if (a > amax) amax = a;
            for (int s = 0; s < 3; ++s) if (es[s] > emax[s]) emax[s] = es[s];
        }
        for (int s = 0; s < 3; ++s) eta3[s] = amax > 0.0 ? emax[s] / amax : 0.0;
    }
    return OR_OK;
}

/* Section III-B.1, sampling, the other reading: ONE table for the matrix,
 * chosen from the exponent counts of the drawn rows pooled (each block of
 * block_rows rows contributes the counts of its drawn row, which stands
 * for every row of the block; blocks hold equally many rows except the
 * last, so this weights the blocks by their rows up to the last one), by
 * the global rules, and then the matrix's own largest exponent added when
 * the pool misses it, as for a block table.  Encoding, eta and exact_frac
 * (measured on all values) as or_encode with that table. */
int or_encode_sampled(const int32_t* row_ptr, const int32_t* col, const double* val,
                      int32_t n_rows, int32_t n_cols, int64_t nnz, int num_exp, int layout,
                      int32_t block_rows, const int32_t* sample_rows, int16_t* sem_out,
                      uint32_t* col_idx, uint16_t* head, uint16_t* tail1, uint32_t* tail2,
                      double* eta3, double* exact_frac, int* layout_out) {
    if (n_rows < 0 || n_cols < 0 || nnz < 0 || num_exp < 1 || num_exp > OR_MAX_EXP ||
        block_rows < 1 || !sample_rows)
        return OR_ERR_ARG;
    int idx_bits = or_index_bits(num_exp);
    if (layout < 0) layout = ((int64_t)n_cols > (1ll << (32 - idx_bits))) ? 1 : 0;
    if (layout != 0 && layout != 1) return OR_ERR_ARG;
    if (layout_out) *layout_out = layout;
    if ((layout == 0 && (int64_t)n_cols > (1ll << (32 - idx_bits))) || nnz >= (1ll << 31))
        return OR_ERR_RANGE;
    uint32_t* all = (uint32_t*)malloc(2048 * sizeof(uint32_t));
    uint32_t* pool = (uint32_t*)malloc(2048 * sizeof(uint32_t));
    uint32_t* one = (uint32_t*)malloc(2048 * sizeof(uint32_t));
    if (!all || !pool || !one) { free(all); free(pool); free(one); return OR_ERR_ARG; }
    int rc = OR_OK;
    if (or_exponent_histogram(val, nnz, all) > 0) rc = OR_ERR_NONFINITE;
    int max_e = 0;
    for (int e = 2046; e >= 1 && rc == OR_OK; --e)
        if (all[e] > 0) { max_e = e; break; }
    memset(pool, 0, 2048 * sizeof(uint32_t));
    int32_t n_blocks = (int32_t)(((int64_t)n_rows + block_rows - 1) / block_rows);
    for (int32_t bk = 0; bk < n_blocks && rc == OR_OK; ++bk) {
        int32_t r0 = bk * block_rows;
        int32_t r1 = (int32_t)((int64_t)r0 + block_rows < n_rows ? r0 + block_rows : n_rows);
        int32_t sr = sample_rows[bk];
        if (sr < r0 || sr >= r1) { rc = OR_ERR_ARG; break; }
        or_exponent_histogram(val + row_ptr[sr], row_ptr[sr + 1] - row_ptr[sr], one);
        for (int e = 0; e < 2048; ++e) pool[e] += one[e];
    }
    if (rc == OR_OK) {
        int used = block_table(pool, max_e, num_exp, sem_out);
        if (used < 0) rc = used;
        else {
            uint64_t covered = 0;
            for (int i = 0; i < used; ++i) covered += all[sem_out[i] - 1];
            if (exact_frac) *exact_frac = nnz ? (double)covered / (double)nnz : 1.0;
            rc = or_encode_values(val, col, nnz, sem_out, idx_bits, layout, col_idx, head, tail1,
                                  tail2);
        }
    }
    free(all);
    free(pool);
    free(one);
    if (rc != OR_OK) return rc;
    if (eta3) {
        double amax = 0.0, emax[3] = {0.0, 0.0, 0.0};
        for (int32_t r = 0; r < n_rows; ++r) {
            double a = 0.0, es[3] = {0.0, 0.0, 0.0};
            for (int32_t j = row_ptr[r]; j < row_ptr[r + 1]; ++j) {
                a += fabs(val[j]);
                for (int s = 1; s <= 3; ++s)
                    es[s - 1] += fabs(val[j] - or_decode_one(col_idx[j], head[j], tail1[j],
                                                             tail2[j], sem_out, idx_bits, layout,
                                                             s));
            }
            if (a > amax) amax = a;
            for (int s = 0; s < 3; ++s) if (es[s] > emax[s]) emax[s] = es[s];
        }
        for (int s = 0; s < 3; ++s) eta3[s] = amax > 0.0 ? emax[s] / amax : 0.0;
    }
    return OR_OK;
}

/* Algorithm 2 and its wider variants with per-block tables: row r decodes
 * its values with the table of its block. */
void or_gse_spmv_blocks(int32_t n_rows, const int32_t* row_ptr, const uint32_t* col_idx,
                        const uint16_t* head, const uint16_t* tail1, const uint32_t* tail2,
                        const int16_t* block_sem, int32_t block_rows, int idx_bits, int layout,
                        int s, const double* x, double* y) {
    for (int32_t r = 0; r < n_rows; ++r) {
        const int16_t* sem = table_of_row(block_sem, block_rows, r);
        double sum = 0.0;
        for (int32_t j = row_ptr[r]; j < row_ptr[r + 1]; ++j) {
            double v = or_decode_one(col_idx[j], head[j], tail1[j], tail2[j], sem, idx_bits,
                                     layout, s);
            sum += v * x[column_of(col_idx[j], idx_bits, layout)];
        }
        y[r] = sum;
    }
}

/* ------------------------------------------------------------------------ */
/* Section IV-C: the FP16 and BF16 comparators.  Every value is rounded once,
 * to nearest with ties to even, into a binary format with `ebits` exponent
 * bits and `mbits` fraction bits (IEEE binary16: 5 and 10; bfloat16: 8 and
 * 7); a magnitude that rounds beyond the largest finite value becomes an
 * infinity (the overflow the paper reports for FP16).  Written from the
 * formats' definitions: the value is a multiple of its quantum 2^(e - mbits)
 * (2^(emin - mbits) below the normal range), rounded to the nearest one. */
static uint16_t round_to_small(double v, int ebits, int mbits, int* overflow) {
    const unsigned sign = signbit(v) ? 1u : 0u;
    const int emax = (1 << (ebits - 1)) - 1, emin = 1 - emax;
    const unsigned inf_bits = ((1u << ebits) - 1u) << mbits;
    double a = fabs(v);
    unsigned mag;
    if (a == 0.0) {
        mag = 0;
    } else {
        int ex;
        frexp(a, &ex);              /* a = m 2^ex, 1/2 <= m < 1 */
        int e = ex - 1;             /* a in [2^e, 2^(e+1)) */
        int qe = (e < emin ? emin : e) - mbits;
        double n = ldexp(a, -qe);   /* exact: a power-of-two scaling */
        double fl = floor(n), d = n - fl;
        double r = (d > 0.5 || (d == 0.5 && fmod(fl, 2.0) != 0.0)) ? fl + 1.0 : fl;
        double rq = ldexp(r, qe);   /* the rounded magnitude */
        double max_finite = ldexp(2.0 - ldexp(1.0, -mbits), emax);
        if (rq > max_finite) {
            mag = inf_bits;
            if (overflow) *overflow += 1;
        } else if (rq < ldexp(1.0, emin)) {
            mag = (unsigned)r;      /* subnormal: the multiple of 2^(emin - mbits) */
        } else {
            int ex2;
            frexp(rq, &ex2);
            int E = ex2 - 1;
            double frac = ldexp(rq, -E) - 1.0;  /* in [0, 1) */
            mag = ((unsigned)(E + emax) << mbits) | (unsigned)ldexp(frac, mbits);
        }
    }
    return (uint16_t)((sign << (ebits + mbits)) | mag);
}

static double widen_small(uint16_t h, int ebits, int mbits) {
    const int emax = (1 << (ebits - 1)) - 1;
    const unsigned sign = (unsigned)h >> (ebits + mbits);
    const unsigned E = ((unsigned)h >> mbits) & ((1u << ebits) - 1u);
    const unsigned F = (unsigned)h & ((1u << mbits) - 1u);
    double mag;
    if (E == 0) mag = ldexp((double)F, 1 - emax - mbits);
    else if (E == (1u << ebits) - 1u) mag = F ? NAN : INFINITY;
    else mag = ldexp(1.0 + ldexp((double)F, -mbits), (int)E - emax);
    return sign ? -mag : mag;
}

static int lp_ebits(int fmt) { return fmt == OR_LP_FP16 ? 5 : 8; }
static int lp_mbits(int fmt) { return fmt == OR_LP_FP16 ? 10 : 7; }

uint16_t or_lp_round(double v, int fmt, int* overflow) {
    return round_to_small(v, lp_ebits(fmt), lp_mbits(fmt), overflow);
}

double or_lp_widen(uint16_t h, int fmt) { return widen_small(h, lp_ebits(fmt), lp_mbits(fmt)); }

int64_t or_lp_convert(const double* val, int64_t nnz, int fmt, uint16_t* out) {
    int over = 0;
    int64_t total = 0;
    for (int64_t i = 0; i < nnz; ++i) {
        over = 0;
        out[i] = or_lp_round(val[i], fmt, &over);
        total += over;
    }
    return total;
}

/* FP16- / BF16-SpMV: each stored value widened to FP64, FP64 multiply and
 * accumulate in row order (Section IV-C). */
void or_lp_spmv(int32_t n_rows, const int32_t* row_ptr, const int32_t* col,
                const uint16_t* val16, int fmt, const double* x, double* y) {
    for (int32_t r = 0; r < n_rows; ++r) {
        double sum = 0.0;
        for (int32_t j = row_ptr[r]; j < row_ptr[r + 1]; ++j)
            sum += or_lp_widen(val16[j], fmt) * x[col[j]];
        y[r] = sum;
    }
}

/* ------------------------------------------------------------------------ */
/* FP64 CSR SpMV (the baseline the paper compares against, Section IV-A).    */
void or_csr_spmv(int32_t n_rows, const int32_t* row_ptr, const int32_t* col,
                 const double* val, const double* x, double* y) {
    for (int32_t r = 0; r < n_rows; ++r) {
        double sum = 0.0;
        for (int32_t j = row_ptr[r]; j < row_ptr[r + 1]; ++j) sum += val[j] * x[col[j]];
        y[r] = sum;
    }
}

/* Algorithm 2 (s = 1) and the head+tail1 / head+tail1+tail2 operators:
 * split column and slot, read the value with s segments, multiply and
 * accumulate in FP64 in row order. */
void or_gse_spmv(int32_t n_rows, const int32_t* row_ptr, const uint32_t* col_idx,
                 const uint16_t* head, const uint16_t* tail1, const uint32_t* tail2,
                 const int16_t* sem, int idx_bits, int layout, int s, const double* x,
                 double* y) {
    for (int32_t r = 0; r < n_rows; ++r) {
        double sum = 0.0;
        for (int32_t j = row_ptr[r]; j < row_ptr[r + 1]; ++j) {
            double v = or_decode_one(col_idx[j], head[j], tail1[j], tail2[j], sem, idx_bits,
                                     layout, s);
            sum += v * x[column_of(col_idx[j], idx_bits, layout)];
        }
        y[r] = sum;
    }
}

void or_gse_spmv_rows(const int32_t* rows, int32_t n_sel, const int32_t* row_ptr,
                      const uint32_t* col_idx, const uint16_t* head,
                      const uint16_t* tail1, const uint32_t* tail2,
                      const int16_t* sem, int idx_bits, int layout, int s, const double* x,
                      double* y_sel) {
    for (int32_t q = 0; q < n_sel; ++q) {
        int32_t r = rows[q];
        double sum = 0.0;
        for (int32_t j = row_ptr[r]; j < row_ptr[r + 1]; ++j) {
            double v = or_decode_one(col_idx[j], head[j], tail1[j], tail2[j], sem, idx_bits,
                                     layout, s);
            sum += v * x[column_of(col_idx[j], idx_bits, layout)];
        }
        y_sel[q] = sum;
    }
}

/* ------------------------------------------------------------------------ */
/* Section III-D.  Metrics over the residual history at iteration j:
 *   RSD   (Eq. 3): population standard deviation of resid[j-t..j-1] over
 *                  their mean;
 *   nDec  (Eqs. 4-5): number of i in [j-t, j-1] with resid[i] > resid[i+1];
 *   relDec (Eq. 6): (resid[j-t] - resid[j-1]) / resid[j-t].              */
void or_window_metrics(const double* resid, int32_t j, int32_t t,
                       double* rsd, int32_t* ndec, double* reldec) {
    double avg = 0.0;
    for (int32_t i = j - t; i <= j - 1; ++i) avg += resid[i];
    avg /= (double)t;
    double var = 0.0;
    for (int32_t i = j - t; i <= j - 1; ++i) var += (resid[i] - avg) * (resid[i] - avg);
    var /= (double)t;
    *rsd = sqrt(var) / avg;
    int32_t n = 0;
    for (int32_t i = j - t; i <= j - 1; ++i) n += (resid[i] > resid[i + 1]) ? 1 : 0;
    *ndec = n;
    *reldec = (resid[j - t] - resid[j - 1]) / resid[j - t];
}

/* Conditions 1-3, evaluated only at j = l + q*m (q >= 0) once t residuals
 * exist.  Returns the first condition that holds (1, 2 or 3) or 0.        */
int or_precision_trigger(const double* resid, int32_t j, const or_params* p) {
    if (j < p->l || j < p->t || p->m <= 0 || ((j - p->l) % p->m) != 0) return OR_TRIG_NONE;
    double rsd, reldec;
    int32_t ndec;
    or_window_metrics(resid, j, p->t, &rsd, &ndec, &reldec);
    int below, at_or_above;
    if (p->ndec_rule == 1) { below = 2 * ndec < p->t; at_or_above = !below; }
    else { below = ndec < p->ndec_limit; at_or_above = !below; }
    if (rsd > p->rsd_limit && below) return OR_TRIG_C1;
    if (at_or_above && reldec < p->reldec_limit) return OR_TRIG_C2;
    if (ndec == 0) return OR_TRIG_C3;
    return OR_TRIG_NONE;
}

/* ------------------------------------------------------------------------ */
static void apply_op(const or_matrix* A, int s, const double* x, double* y) {
    if (s == OR_S_LP) or_lp_spmv(A->n_rows, A->row_ptr, A->col, A->lp_val, A->lp_fmt, x, y);
    else if (s <= 0) or_csr_spmv(A->n_rows, A->row_ptr, A->col, A->val, x, y);
    else if (A->block_rows > 0)
        or_gse_spmv_blocks(A->n_rows, A->row_ptr, A->col_idx, A->head, A->tail1, A->tail2,
                           A->block_sem, A->block_rows, A->idx_bits, A->layout, s, x, y);
    else or_gse_spmv(A->n_rows, A->row_ptr, A->col_idx, A->head, A->tail1, A->tail2,
                     A->sem64, A->idx_bits, A->layout, s, x, y);
}

static double dot(int32_t n, const double* a, const double* b) {
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* r = b - A_s x ; returns r.r */
static double residual(const or_matrix* A, int s, const double* b, const double* x,
                       double* r) {
    apply_op(A, s, x, r);
    for (int32_t i = 0; i < A->n_rows; ++i) r[i] = b[i] - r[i];
    return dot(A->n_rows, r, r);
}

static int final_segments(const or_params* p) {
    if (p->fixed_segments == OR_S_LP) return OR_S_LP;  /* the 16-bit operator judges itself */
    return p->fixed_segments < 0 ? 0 : 3;  /* 0: FP64 CSR operator */
}

/* Is the current operator the one convergence is judged on? */
static int operator_is_final(const or_matrix* A, const or_params* p, int s) {
    if (p->fixed_segments != 0) return 1;
    if (s >= 3) return 1;
    return A->eta3 && A->eta3[s - 1] == 0.0;
}

static void init_report(or_report* rep) {
    memset(rep, 0, sizeof *rep);
    rep->switch_iter[0] = rep->switch_iter[1] = -1;
}

/* CG (Hestenes-Stiefel form) with FP64 vectors; only the operator A_s uses
 * the reduced segments.  The stepped scheme (Algorithm 3 with Conditions
 * 1-3) raises s by one when a condition holds on the check grid.  Readings
 * beyond the paper: a floor trigger (relres <= floor_c*eta_s), escalation
 * when the tolerance is met with an inexact operator, escalation instead of
 * failure on breakdown below s = 3, and at every switch the residual is
 * recomputed with the new operator (r = b - A_{s+1} x) and, in restart mode,
 * p = r.  Convergence is accepted only after the explicit residual with the
 * final operator meets the tolerance. */
int or_cg(const or_matrix* A, const double* b, double* x, const or_params* p,
          or_report* rep, double* hist, int32_t* seg_hist) {
    int32_t n = A->n_rows;
    init_report(rep);
    double* r = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* pv = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* q = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!r || !pv || !q) { free(r); free(pv); free(q); return OR_ERR_ARG; }
    int stepped = (p->fixed_segments == 0);
    int s = stepped ? p->start_segments
                    : (p->fixed_segments > 0 ? p->fixed_segments
                                             : (p->fixed_segments == OR_S_LP ? OR_S_LP : 0));
    int fin = final_segments(p);
    double nb = sqrt(dot(n, b, b));
    if (nb == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        rep->status = OR_OK;
        if (hist) hist[0] = 0.0;
        free(r); free(pv); free(q);
        return OR_OK;
    }
    double rho = residual(A, s, b, x, r);
    memcpy(pv, r, sizeof(double) * (size_t)n);
    double relres = sqrt(rho) / nb;
    if (hist) hist[0] = relres;
    if (seg_hist) seg_hist[0] = s;
    int32_t it = 0;
    int nsw = 0;
    int status = OR_NOT_CONVERGED;
    for (;;) {
        int trig = OR_TRIG_NONE;
        if (relres <= p->tol) {
            if (operator_is_final(A, p, s)) {
                double rt = sqrt(residual(A, fin, b, x, q)) / nb;
                if (rt <= p->tol) { status = OR_OK; break; }
                rho = residual(A, s, b, x, r);  /* replace the drifted residual */
                memcpy(pv, r, sizeof(double) * (size_t)n);
                relres = sqrt(rho) / nb;
                if (relres <= p->tol) { status = OR_NOT_CONVERGED; break; }
            } else {
                trig = OR_TRIG_TOL;
            }
        }
        if (trig == OR_TRIG_NONE) {
            if (it >= p->max_iter) break;
            apply_op(A, s, pv, q);
            double pq = dot(n, pv, q);
            if (!(pq > 0.0) || !isfinite(pq)) {
                if (stepped && s < 3) trig = OR_TRIG_BREAKDOWN;
                else { status = OR_ERR_BREAKDOWN; break; }
            } else {
                double alpha = rho / pq;
                for (int32_t i = 0; i < n; ++i) x[i] += alpha * pv[i];
                for (int32_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
                double rho_new = dot(n, r, r);
                it += 1;
                rep->iters_per_seg[(s > 0 ? s : 3) - 1] += 1;
                relres = sqrt(rho_new) / nb;
                if (hist) hist[it] = relres;
                if (seg_hist) seg_hist[it] = s;
                double beta = rho_new / rho;
                rho = rho_new;
                for (int32_t i = 0; i < n; ++i) pv[i] = r[i] + beta * pv[i];
                if (stepped && s < 3 && relres > p->tol) {
                    double eta = A->eta3 ? A->eta3[s - 1] : 0.0;
                    if (p->floor_c > 0.0 && eta > 0.0 && relres <= p->floor_c * eta)
                        trig = OR_TRIG_FLOOR;
                    else if (hist)
                        trig = or_precision_trigger(hist, it, p);
                }
            }
        }
        if (trig != OR_TRIG_NONE) {
            if (nsw < 2) { rep->switch_iter[nsw] = it; rep->switch_trigger[nsw] = trig; }
            nsw += 1;
            s += 1;
            double rho_old = rho;
            rho = residual(A, s, b, x, r);
            /* the direction is kept (switch_mode 1), restarted as p = r
             * (switch_mode 0), or -- switch_mode 2 -- kept only while the
             * replacement leaves the residual norm within a factor of two */
            int reset_p = p->switch_mode == 0 ||
                          (p->switch_mode == 2 && (rho > 4.0 * rho_old || 4.0 * rho < rho_old));
            if (reset_p) memcpy(pv, r, sizeof(double) * (size_t)n);
            relres = sqrt(rho) / nb;
        }
    }
    rep->status = status;
    rep->iters = it;
    rep->relres_recursive = relres;
    rep->relres_true = sqrt(residual(A, fin, b, x, q)) / nb;
    free(r); free(pv); free(q);
    return status;
}

/* Givens rotation zeroing b against a, with r = sqrt(a^2 + b^2). */
static void givens(double a, double b, double* c, double* s) {
    double r = sqrt(a * a + b * b);
    if (r == 0.0) { *c = 1.0; *s = 0.0; return; }
    *c = a / r;
    *s = b / r;
}

/* Restarted GMRES(m) with FP64 Arnoldi vectors, Givens rotations and the
 * same stepped operator schedule as CG.  The monitored residual is the
 * least-squares estimate |g_{j+1}|/||b||.  A switch ends the cycle; the next
 * cycle starts from the explicit residual of the new operator. */
/* One GMRES cycle with Gram-Schmidt applied twice, the second pass delayed
 * by one step so that each step needs one reduction (delayed classical
 * Gram-Schmidt, DCGS2: Swirydowicz, Langou, Ananthan, Yang and Thomas,
 * "Low synchronization Gram-Schmidt and GMRES algorithms", 2020; Bielich et
 * al., "Low-synch Gram-Schmidt with delayed reorthogonalization for Krylov
 * solvers", 2022).  Not part of the paper's method: a variant of its GMRES
 * that reaches the same Krylov iterates with fewer passes over the basis.
 *
 * V[0] holds u_0 = r (not normalised).  Step j (0 <= j <= m) starts with
 * the final basis q_0..q_{j-1} in V[0..j-1] and u_j in V[j], the new
 * direction after its first projection only.  With z = A_s u_j (not for
 * j = m) one reduction gives a = Q^T u_j, omega = u_j.u_j, c = Q^T z and
 * gamma = u_j.z.  Then
 *   beta = sqrt(omega - |a|^2)   (the norm of u_j after its second projection)
 *   q_j = (u_j - Q a) / beta
 * closes Arnoldi column j - 1: H[0..j-1][j-1] = h1 + a, H[j][j-1] = beta,
 * the rotations and the residual estimate as in the other variants.  With
 * t = q_j.z = (gamma - a.c) / beta, A q_j = (z - A Q a) / beta and
 * A Q = Q_j Hbar (the Arnoldi relation of the columns closed so far), the
 * next direction and its first projection coefficients are
 *   u_{j+1} = (z - Q c - t q_j) / beta,
 *   h1 = ([c; t] - Hbar a) / beta       (provisional column j),
 * so the step reads the basis twice: once for the dots, once for q_j and
 * u_{j+1}.  The residual estimate of column j - 1 is known only after the
 * product with u_j, so a cycle that stops at column j - 1 has computed one
 * product more than the other variants.  beta^2 at or below 1e-28 omega is
 * taken as 0 (u_j lies in the span of Q: exact in this space).
 * Returns the number of closed columns; *trig the controller's switch. */
static int dcgs2_cycle(const or_matrix* A, const or_params* p, int s, int stepped, int m,
                       int32_t n, size_t nn, double nb, double* V, double* z, double* H,
                       double* Hu, double* h1, double* av, double* bv, double* cs, double* sn,
                       double* g, int32_t* it, double* relres, int* trig, or_report* rep,
                       double* hist, int32_t* seg_hist) {
#define HH(i, j) H[(size_t)(i) * (size_t)m + (size_t)(j)]
#define HU(i, j) Hu[(size_t)(i) * (size_t)m + (size_t)(j)]
    int k_used = 0;
    for (int j = 0; j <= m; ++j) {
        double* uj = V + (size_t)j * nn;
        const int have_z = j < m;
        if (have_z) apply_op(A, s, uj, z);
        for (int i = 0; i < j; ++i) av[i] = dot(n, V + (size_t)i * nn, uj);
        double om = dot(n, uj, uj);
        double ga = 0.0;
        if (have_z) {
            for (int i = 0; i < j; ++i) bv[i] = dot(n, V + (size_t)i * nn, z);
            ga = dot(n, uj, z);
        }
        double aa = 0.0;
        for (int i = 0; i < j; ++i) aa += av[i] * av[i];
        double b2 = om - aa;
        double bet = b2 > 1e-28 * om ? sqrt(b2) : 0.0;
        if (j == 0) {
            g[0] = bet;
        } else {
            /* Arnoldi column j - 1 is closed */
            for (int i = 0; i < j; ++i) HU(i, j - 1) = h1[i] + av[i];
            HU(j, j - 1) = bet;
            for (int i = 0; i <= j; ++i) HH(i, j - 1) = HU(i, j - 1);
            for (int i = 0; i < j - 1; ++i) {
                double t0 = cs[i] * HH(i, j - 1) + sn[i] * HH(i + 1, j - 1);
                HH(i + 1, j - 1) = -sn[i] * HH(i, j - 1) + cs[i] * HH(i + 1, j - 1);
                HH(i, j - 1) = t0;
            }
            givens(HH(j - 1, j - 1), HH(j, j - 1), &cs[j - 1], &sn[j - 1]);
            HH(j - 1, j - 1) = cs[j - 1] * HH(j - 1, j - 1) + sn[j - 1] * HH(j, j - 1);
            HH(j, j - 1) = 0.0;
            g[j] = -sn[j - 1] * g[j - 1];
            g[j - 1] = cs[j - 1] * g[j - 1];
            *it += 1;
            rep->iters_per_seg[(s > 0 ? s : 3) - 1] += 1;
            k_used = j;
            *relres = fabs(g[j]) / nb;
            if (hist) hist[*it] = *relres;
            if (seg_hist) seg_hist[*it] = s;
            if (bet == 0.0) break;  /* happy breakdown: exact in this space */
            if (*relres <= p->tol) break;
            if (stepped && s < 3) {
                double eta = A->eta3 ? A->eta3[s - 1] : 0.0;
                if (p->floor_c > 0.0 && eta > 0.0 && *relres <= p->floor_c * eta)
                    *trig = OR_TRIG_FLOOR;
                else if (hist)
                    *trig = or_precision_trigger(hist, *it, p);
                if (*trig != OR_TRIG_NONE) break;
            }
            if (j == m || *it >= p->max_iter) break;
        }
        if (bet == 0.0) break;  /* r = 0 at the start of the cycle */
        /* first projection of A q_j, q_j and u_{j+1} */
        double t = ga;
        for (int i = 0; i < j; ++i) t -= av[i] * bv[i];
        t /= bet;
        for (int i = 0; i <= j; ++i) {
            double c = i < j ? bv[i] : t;
            for (int k = 0; k < j; ++k) c -= HU(i, k) * av[k];
            h1[i] = c / bet;
        }
        double* un = V + (size_t)(j + 1) * nn;
        for (int32_t e = 0; e < n; ++e) {
            double q = uj[e];
            for (int i = 0; i < j; ++i) q -= av[i] * V[(size_t)i * nn + e];
            q /= bet;
            double u = z[e];
            for (int i = 0; i < j; ++i) u -= bv[i] * V[(size_t)i * nn + e];
            u -= t * q;
            uj[e] = q;
            un[e] = u / bet;
        }
    }
#undef HH
#undef HU
    return k_used;
}

int or_gmres(const or_matrix* A, const double* b, double* x, const or_params* p,
             or_report* rep, double* hist, int32_t* seg_hist) {
    int32_t n = A->n_rows;
    int m = p->restart;
    init_report(rep);
    if (m < 1) return OR_ERR_ARG;
    size_t nn = (size_t)(n > 0 ? n : 1);
    double* V = (double*)malloc(sizeof(double) * nn * (size_t)(m + 1));
    double* H = (double*)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));
    double* cs = (double*)malloc(sizeof(double) * (size_t)m);
    double* sn = (double*)malloc(sizeof(double) * (size_t)m);
    double* g = (double*)malloc(sizeof(double) * (size_t)(m + 1));
    double* y = (double*)malloc(sizeof(double) * (size_t)m);
    double* h2 = (double*)malloc(sizeof(double) * (size_t)(m + 1));
    double* w = (double*)malloc(sizeof(double) * nn);
    /* delayed CGS2 only: the Hessenberg matrix before the rotations, the
     * provisional column, and the dots of one step */
    double* Hu = (double*)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));
    double* h1 = (double*)malloc(sizeof(double) * (size_t)(m + 1));
    double* av = (double*)malloc(sizeof(double) * (size_t)(m + 1));
    double* bv = (double*)malloc(sizeof(double) * (size_t)(m + 1));
    if (!V || !H || !cs || !sn || !g || !y || !h2 || !w || !Hu || !h1 || !av || !bv) {
        free(V); free(H); free(cs); free(sn); free(g); free(y); free(h2); free(w);
        free(Hu); free(h1); free(av); free(bv);
        return OR_ERR_ARG;
    }
#define HH(i, j) H[(size_t)(i) * (size_t)m + (size_t)(j)]
#define HU(i, j) Hu[(size_t)(i) * (size_t)m + (size_t)(j)]
    int stepped = (p->fixed_segments == 0);
    int s = stepped ? p->start_segments
                    : (p->fixed_segments > 0 ? p->fixed_segments
                                             : (p->fixed_segments == OR_S_LP ? OR_S_LP : 0));
    int fin = final_segments(p);
    double nb = sqrt(dot(n, b, b));
    int32_t it = 0;
    int nsw = 0;
    int status = OR_NOT_CONVERGED;
    double relres = 0.0;
    if (nb == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        rep->status = OR_OK;
        if (hist) hist[0] = 0.0;
        goto done;
    }
    for (;;) {
        double beta = sqrt(residual(A, s, b, x, V));
        relres = beta / nb;
        if (it == 0) { if (hist) hist[0] = relres; if (seg_hist) seg_hist[0] = s; }
        int trig = OR_TRIG_NONE;
        if (relres <= p->tol) {
            /* the residual just formed is the final operator's: done */
            if (s == fin || s == 3) { status = OR_OK; break; }
            /* otherwise convergence is judged on the final operator's residual;
             * a fixed segment count cannot escalate and ends here either way */
            if (operator_is_final(A, p, s)) {
                double rt = sqrt(residual(A, fin, b, x, w)) / nb;
                if (rt <= p->tol) { status = OR_OK; break; }
                if (p->fixed_segments != 0) break;
            }
            trig = OR_TRIG_TOL;
        }
        if (trig != OR_TRIG_NONE) {
            if (s >= 3) break;
            if (nsw < 2) { rep->switch_iter[nsw] = it; rep->switch_trigger[nsw] = trig; }
            nsw += 1;
            s += 1;
            continue;
        }
        if (it >= p->max_iter) break;
        for (int k = 0; k <= m; ++k) g[k] = 0.0;
        int k_used = 0;
        if (p->orth == 2) {
            k_used = dcgs2_cycle(A, p, s, stepped, m, n, nn, nb, V, w, H, Hu, h1, av, bv, cs, sn,
                                 g, &it, &relres, &trig, rep, hist, seg_hist);
            goto cycle_end;
        }
        for (int32_t i = 0; i < n; ++i) V[i] /= beta;
        g[0] = beta;
        for (int j = 0; j < m && it < p->max_iter; ++j) {
            double* vj = V + (size_t)j * nn;
            apply_op(A, s, vj, w);
            if (p->orth == 1) {  /* classical Gram-Schmidt, applied twice */
                for (int i = 0; i <= j; ++i) HH(i, j) = dot(n, V + (size_t)i * nn, w);
                for (int i = 0; i <= j; ++i) {
                    const double* vi = V + (size_t)i * nn;
                    for (int32_t e = 0; e < n; ++e) w[e] -= HH(i, j) * vi[e];
                }
                for (int i = 0; i <= j; ++i) h2[i] = dot(n, V + (size_t)i * nn, w);
                for (int i = 0; i <= j; ++i) {
                    const double* vi = V + (size_t)i * nn;
                    for (int32_t e = 0; e < n; ++e) w[e] -= h2[i] * vi[e];
                    HH(i, j) += h2[i];
                }
            } else {  /* modified Gram-Schmidt */
                for (int i = 0; i <= j; ++i) {
                    const double* vi = V + (size_t)i * nn;
                    double h = dot(n, vi, w);
                    HH(i, j) = h;
                    for (int32_t e = 0; e < n; ++e) w[e] -= h * vi[e];
                }
            }
            double hn = sqrt(dot(n, w, w));
            HH(j + 1, j) = hn;
            for (int i = 0; i < j; ++i) {
                double t0 = cs[i] * HH(i, j) + sn[i] * HH(i + 1, j);
                HH(i + 1, j) = -sn[i] * HH(i, j) + cs[i] * HH(i + 1, j);
                HH(i, j) = t0;
            }
            givens(HH(j, j), HH(j + 1, j), &cs[j], &sn[j]);
            HH(j, j) = cs[j] * HH(j, j) + sn[j] * HH(j + 1, j);
            HH(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            it += 1;
            rep->iters_per_seg[(s > 0 ? s : 3) - 1] += 1;
            k_used = j + 1;
            relres = fabs(g[j + 1]) / nb;
            if (hist) hist[it] = relres;
            if (seg_hist) seg_hist[it] = s;
            if (hn == 0.0) break;  /* happy breakdown: exact in this space */
            double* vn = V + (size_t)(j + 1) * nn;
            for (int32_t e = 0; e < n; ++e) vn[e] = w[e] / hn;
            if (relres <= p->tol) break;
            if (stepped && s < 3) {
                double eta = A->eta3 ? A->eta3[s - 1] : 0.0;
                if (p->floor_c > 0.0 && eta > 0.0 && relres <= p->floor_c * eta)
                    trig = OR_TRIG_FLOOR;
                else if (hist)
                    trig = or_precision_trigger(hist, it, p);
                if (trig != OR_TRIG_NONE) break;
            }
        }
    cycle_end:
        for (int i = k_used - 1; i >= 0; --i) {
            double acc = g[i];
            for (int k = i + 1; k < k_used; ++k) acc -= HH(i, k) * y[k];
            y[i] = acc / HH(i, i);
        }
        for (int k = 0; k < k_used; ++k) {
            const double* vk = V + (size_t)k * nn;
            for (int32_t e = 0; e < n; ++e) x[e] += y[k] * vk[e];
        }
        if (trig != OR_TRIG_NONE) {
            if (nsw < 2) { rep->switch_iter[nsw] = it; rep->switch_trigger[nsw] = trig; }
            nsw += 1;
            s += 1;
        }
    }
done:
    rep->status = status;
    rep->iters = it;
    rep->relres_recursive = relres;
    rep->relres_true = nb == 0.0 ? 0.0 : sqrt(residual(A, fin, b, x, w)) / nb;
#undef HH
#undef HU
    free(V); free(H); free(cs); free(sn); free(g); free(y); free(h2); free(w);
    free(Hu); free(h1); free(av); free(bv);
    return status;
}
