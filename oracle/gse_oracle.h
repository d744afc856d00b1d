/*
 * gse_oracle.h -- sequential CPU oracle for the group-shared-exponent (GSE)
 * format with segmented mantissa storage (SEM), and for the CG / GMRES
 * solvers built on it.
 *
 * TEST INFRASTRUCTURE.  This library is the reference the GPU library is
 * checked against.  It is plain C99, single threaded, FP64, written for
 * readability rather than speed, and shares no code, header or table with the
 * GPU library.  Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.
 *
 * Format (Section III-B, Algorithms 1 and 2, Section III-C.1):
 *   - a table of up to 64 shared exponents, each stored as (biased
 *     exponent+1);
 *   - per non-zero: a slot index of b = ceil(log2 k) bits for a table of k
 *     shared exponents (the number of shared exponents sets the index width,
 *     Section III-B.1), kept in the top b bits of the 32-bit column index
 *     (Section III-C.1), and a 64-bit word  sign<<63 | F63  where F63 is |v|
 *     on the fixed-point grid 2^(SEM-1023-63) of its slot, truncated toward
 *     zero; or, when the column field is too narrow, the index in the value
 *     word (Algorithm 1's EI_bit): sign | index | F on a 63-b bit field;
 *   - the word is split into three planes: head (bits 63..48), tail1
 *     (bits 47..32) and tail2 (bits 31..0).  Reading s planes gives a
 *     W_s = 15, 31 or 63 bit magnitude.
 */
#ifndef GSE_ORACLE_H
#define GSE_ORACLE_H
#include <stdint.h>

#define OR_MAX_EXP 64

enum { OR_OK = 0, OR_NOT_CONVERGED = 2, OR_ERR_ARG = -1, OR_ERR_NONFINITE = -2,
       OR_ERR_RANGE = -3, OR_ERR_BREAKDOWN = -5 };

/* switch triggers recorded in reports */
enum { OR_TRIG_NONE = 0, OR_TRIG_C1 = 1, OR_TRIG_C2 = 2, OR_TRIG_C3 = 3,
       OR_TRIG_FLOOR = 4, OR_TRIG_TOL = 5, OR_TRIG_BREAKDOWN = 6 };

typedef struct {
    double tol;          /* relative residual target ||r||/||b|| */
    int32_t max_iter;    /* CG iteration cap; GMRES: restart*max_restarts */
    int32_t restart;     /* GMRES cycle length */
    int32_t max_restarts;
    int32_t start_segments;  /* 1..3 */
    int32_t fixed_segments;  /* 0: stepped, 1..3: fixed; -1: plain FP64 CSR;
                                -2: the FP16 / BF16 operator of the matrix (lp_val) */
    int32_t l, t, m;         /* controller schedule (Section III-D) */
    double rsd_limit;
    int32_t ndec_limit;
    double reldec_limit;
    int32_t ndec_rule;       /* 0: compare nDec with ndec_limit, 1: with t/2 */
    double floor_c;          /* switch once relres <= floor_c*eta_s (0: off) */
    int32_t switch_mode;     /* CG after a switch: 0 restart p = r, 1 keep p, 2 keep p while
                                the residual replacement keeps ||r|| within a factor 2 */
    int32_t orth;            /* GMRES: 0 MGS, 1 CGS2, 2 CGS2 with the second pass delayed one step
                                (one reduction per step) */
} or_params;

typedef struct {
    int32_t status;
    int32_t iters;
    int32_t iters_per_seg[3];
    int32_t switch_iter[2];
    int32_t switch_trigger[2];
    double relres_recursive;
    double relres_true;
} or_report;

/* ---- format ----
 * Tables (sem64) always hold OR_MAX_EXP entries, unused ones 0.  idx_bits is
 * the slot-index width b of the column word: column = word & (2^(32-b) - 1),
 * slot = word >> (32 - b) (slot 0 when b = 0). */
int or_index_bits(int num_exp);
int64_t or_exponent_histogram(const double* val, int64_t nnz, uint32_t* hist2048);
int or_select_shared_exponents(const uint32_t* hist2048, int num_exp, int16_t* sem64);
int or_encode_values(const double* val, const int32_t* col, int64_t nnz,
                     const int16_t* sem64, int idx_bits, int layout, uint32_t* col_idx,
                     uint16_t* head, uint16_t* tail1, uint32_t* tail2);
/* layout: 0 index in the column word, 1 in the value (Algorithm 1's EI_bit:
 * sign | index | 63 - idx_bits magnitude bits), -1 the column word unless the
 * column field is too narrow for n_cols; *layout_out receives the choice. */
int or_encode(const int32_t* row_ptr, const int32_t* col, const double* val,
              int32_t n_rows, int32_t n_cols, int64_t nnz, int num_exp, int layout,
              const int16_t* sem_in, int16_t* sem_out64, uint32_t* col_idx,
              uint16_t* head, uint16_t* tail1, uint32_t* tail2, double* eta3,
              double* exact_frac, int* layout_out);
double or_decode_one(uint32_t col_word, uint16_t head, uint16_t tail1,
                     uint32_t tail2, const int16_t* sem64, int idx_bits, int layout, int s);
void or_decode(const uint32_t* col_idx, const uint16_t* head, const uint16_t* tail1,
               const uint32_t* tail2, int64_t nnz, const int16_t* sem64, int idx_bits,
               int layout, int s, double* out);

/* Per-row-block tables (Section III-B.1, sampling): block b covers rows
 * [b*block_rows, (b+1)*block_rows) and has the table block_sem[b*64 .. b*64+63].
 * sample_rows: one row of each block whose exponents choose its table, or
 * NULL to choose from all of the block's values.  Errors as or_encode, and
 * OR_ERR_ARG for a sample row outside its block. */
int or_encode_blocks(const int32_t* row_ptr, const int32_t* col, const double* val,
                     int32_t n_rows, int32_t n_cols, int64_t nnz, int num_exp, int layout,
                     int32_t block_rows, const int32_t* sample_rows, int16_t* block_sem,
                     uint32_t* col_idx, uint16_t* head, uint16_t* tail1, uint32_t* tail2,
                     double* eta3, double* exact_frac, int* layout_out);
/* One table for the matrix from the pooled exponent counts of one drawn row
 * per block (sample_rows, required), the matrix's largest exponent added if
 * missed; sem_out as for or_encode. */
int or_encode_sampled(const int32_t* row_ptr, const int32_t* col, const double* val,
                      int32_t n_rows, int32_t n_cols, int64_t nnz, int num_exp, int layout,
                      int32_t block_rows, const int32_t* sample_rows, int16_t* sem_out64,
                      uint32_t* col_idx, uint16_t* head, uint16_t* tail1, uint32_t* tail2,
                      double* eta3, double* exact_frac, int* layout_out);
void or_gse_spmv_blocks(int32_t n_rows, const int32_t* row_ptr, const uint32_t* col_idx,
                        const uint16_t* head, const uint16_t* tail1, const uint32_t* tail2,
                        const int16_t* block_sem, int32_t block_rows, int idx_bits, int layout,
                        int s, const double* x, double* y);

/* ---- FP16 / BF16 comparators (Section IV-C) ----
 * fmt: OR_LP_FP16 (IEEE binary16) or OR_LP_BF16 (bfloat16).  Values are
 * rounded once, to nearest with ties to even; overflow gives an infinity and
 * is counted (or_lp_convert returns the number of overflows). */
#define OR_LP_FP16 1
#define OR_LP_BF16 2
uint16_t or_lp_round(double v, int fmt, int* overflow);
double or_lp_widen(uint16_t h, int fmt);
int64_t or_lp_convert(const double* val, int64_t nnz, int fmt, uint16_t* out);
void or_lp_spmv(int32_t n_rows, const int32_t* row_ptr, const int32_t* col,
                const uint16_t* val16, int fmt, const double* x, double* y);

/* ---- SpMV ---- */
void or_csr_spmv(int32_t n_rows, const int32_t* row_ptr, const int32_t* col,
                 const double* val, const double* x, double* y);
void or_gse_spmv(int32_t n_rows, const int32_t* row_ptr, const uint32_t* col_idx,
                 const uint16_t* head, const uint16_t* tail1, const uint32_t* tail2,
                 const int16_t* sem64, int idx_bits, int layout, int s, const double* x,
                 double* y);
void or_gse_spmv_rows(const int32_t* rows, int32_t n_sel, const int32_t* row_ptr,
                      const uint32_t* col_idx, const uint16_t* head,
                      const uint16_t* tail1, const uint32_t* tail2,
                      const int16_t* sem64, int idx_bits, int layout, int s, const double* x,
                      double* y_sel);

/* ---- controller (Section III-D, Eqs. 3-6, Conditions 1-3) ---- */
void or_window_metrics(const double* resid, int32_t j, int32_t t,
                       double* rsd, int32_t* ndec, double* reldec);
int or_precision_trigger(const double* resid, int32_t j, const or_params* p);

/* ---- solvers ----
 * The matrix is either plain FP64 CSR (fixed_segments == -1: col/val used) or
 * GSE planes (col_idx/head/tail1/tail2/sem64/idx_bits used).  x holds x0 on entry.
 * hist (optional, may be NULL) receives relres per iteration, [max_iter+1];
 * seg_hist (optional) the segment count used by each iteration.           */
typedef struct {
    int32_t n_rows;
    const int32_t* row_ptr;
    const int32_t* col;
    const double* val;
    const uint32_t* col_idx;
    const uint16_t* head;
    const uint16_t* tail1;
    const uint32_t* tail2;
    const int16_t* sem64;
    const double* eta3;
    int32_t idx_bits;
    int32_t layout;          /* 0: slot in the column word, 1: in the value */
    const uint16_t* lp_val;  /* FP16 / BF16 values (fixed_segments == -2) */
    int32_t lp_fmt;
    const int16_t* block_sem;  /* per-row-block tables (or_encode_blocks) when block_rows > 0 */
    int32_t block_rows;
} or_matrix;

#define OR_S_LP (-2)

int or_cg(const or_matrix* A, const double* b, double* x, const or_params* p,
          or_report* rep, double* hist, int32_t* seg_hist);
int or_gmres(const or_matrix* A, const double* b, double* x, const or_params* p,
             or_report* rep, double* hist, int32_t* seg_hist);

#endif
