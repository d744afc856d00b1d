/*
 * gse.h -- C ABI of libgse: sparse matrices in the group-shared-exponent,
 * segmented-mantissa format (GSE-SEM) on AMD Instinct MI355X (gfx950), and
 * the stepped mixed-precision CG / GMRES solvers built on them.
 *
 * The paper: "Precision-Aware Iterative Algorithms Based on Group-Shared
 * Exponents of Floating-Point Numbers" (arXiv 2411.04686).
 *
 * Conventions shared by every entry point
 *   - Every call returns a gse_status; nothing throws, exits or prints.  On an
 *     error, gse_last_error() returns a thread-local message.
 *   - All arguments are validated on the host before anything is launched.
 *     A failing HIP call maps to GSE_ERR_HIP (its text in gse_last_error()).
 *   - Device pointers are plain device addresses (hipMalloc or a framework
 *     allocator); the library does not take ownership of any of them and
 *     never allocates device memory: scratch comes from a caller workspace
 *     (gse_encode_static: a fixed static device array instead).
 *   - `stream` is a hipStream_t passed as void* (NULL: the null stream).
 *     gse_spmv is asynchronous on it; gse_encode, gse_plan, gse_cg and
 *     gse_gmres synchronize it before returning.
 *   - Matrices are CSR with int32 row pointers (ascending, row_ptr[0] == 0),
 *     int32 column indices and FP64 values; the number of non-zeros must be
 *     below 2^31 - 2^16.  With k shared exponents the top b = ceil(log2 k)
 *     bits of each column word hold the slot index, so up to 2^(32 - b)
 *     columns (2^29 for the default k = 8, 2^26 for k = 64); wider matrices
 *     keep the index in the value word instead (GSE_IDX_VALUE).
 *   - "Planes" are per-non-zero arrays.  They must hold gse_pad(nnz) entries
 *     (nnz rounded up to a multiple of 16) and start on a 16-byte boundary;
 *     entries past nnz are never interpreted (the kernels load them as part of
 *     aligned vectors and mask them).
 */
#ifndef GSE_H
#define GSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gse_status;
#define GSE_OK 0
#define GSE_PENDING 1           /* serving: ticket not finished yet */
#define GSE_NOT_CONVERGED 2     /* solve stopped at its cap; report filled */
#define GSE_ERR_ARG (-1)        /* invalid argument (NULL, size, alignment) */
#define GSE_ERR_NONFINITE (-2)  /* Inf/NaN among the matrix values */
#define GSE_ERR_RANGE (-3)      /* size limits, or a value the table cannot hold */
#define GSE_ERR_NOMEM (-4)      /* workspace / arena too small */
#define GSE_ERR_BREAKDOWN (-5)  /* CG p.Ap <= 0 or non-finite with all segments */
#define GSE_ERR_HIP (-6)        /* a HIP runtime call failed */
#define GSE_ERR_TICKET (-7)     /* serving: unknown ticket */

#define GSE_MAX_EXP 64          /* shared exponents per matrix (up to a 6-bit index) */

/* Smallest block of rows with a table of its own (gse_encode_blocks). */
#define GSE_MIN_BLOCK_ROWS 128

/* Where the slot index lives (gse_matrix.idx_layout). */
#define GSE_IDX_AUTO 0          /* input: the column word unless n_cols needs its top bits */
#define GSE_IDX_COLUMN 1        /* top bits of the column word */
#define GSE_IDX_VALUE 2         /* top bits of the value word, below the sign */

/* Number of entries a plane must hold for `nnz` non-zeros. */
int64_t gse_pad(int64_t nnz);

/* ------------------------------------------------------------------------
 * Encoded matrix.  Section III-B (format), Section III-B.3 and Fig. 3
 * (segmented storage), Section III-C.1 (slot index in the column word).
 *
 * Each non-zero v is stored as a 64-bit word  sign<<63 | F  where
 * F = floor(|v| * 2^(1086 - SEM[slot])) is its magnitude on the fixed-point
 * grid of its slot (the hidden one explicit, truncation toward zero), and
 * SEM[slot] = e_slot + 1 is the shared exponent stored incremented.  The
 * word is split into three planes:
 *   head  = bits 63..48 (sign and 15 magnitude bits),
 *   tail1 = bits 47..32,
 *   tail2 = bits 31..0,
 * and the column word is  col | slot << (32 - b), where b = ceil(log2 k) is
 * the slot-index width for k shared exponents (Section III-B.1: the number
 * of shared exponents sets the index width; b = 0 stores the bare column).
 * When the column field is too narrow for n_cols (or on request), the slot
 * goes into the value instead (Section III-C.1, Algorithm 1's EI_bit): the
 * word is  sign<<63 | slot<<(63-b) | F  with F = floor(|v| 2^(1086-b-SEM))
 * on a 63 - b bit field, the head keeps 15 - b magnitude bits, the column
 * word is the bare column, and W_s = 15 - b, 31 - b, 63 - b.
 * Reading s planes gives the value
 * +-(F >> (63 - W_s)) * 2^(SEM - 1023 - W_s), W_s = 15, 31, 63.
 *
 * Caller-owned device buffers (set the pointers before gse_encode):
 *   col_idx, head, tail1, tail2 : gse_pad(nnz) entries each, 16-byte aligned;
 *   tile_row                    : tile_cap int32 entries, at least
 *                                 gse_tile_entries(nnz) (the SpMV schedule).
 * row_ptr is recorded by gse_encode and must stay valid while A is used.
 * Host fields (sem, eta, exact_frac, tile_*) are written by the library.
 */
typedef struct gse_matrix {
    int32_t n_rows;
    int32_t n_cols;
    int64_t nnz;
    int32_t num_exp;           /* k, 1..64 (Section IV-B sweeps 2..64 and picks 8) */
    int32_t num_used;          /* slots actually populated */
    int32_t idx_bits;          /* slot-index width b = ceil(log2 num_exp) (written by encode) */
    int32_t idx_layout;        /* in: GSE_IDX_AUTO / COLUMN / VALUE; out: COLUMN or VALUE */
    int16_t sem[GSE_MAX_EXP];  /* shared exponents, biased + 1; 0 = unused */
    const int32_t* row_ptr;    /* device [n_rows + 1] */
    uint32_t* col_idx;         /* device plane */
    uint16_t* head;            /* device plane */
    uint16_t* tail1;           /* device plane */
    uint32_t* tail2;           /* device plane */
    int32_t* tile_row;         /* device [tile_cap] */
    int32_t tile_cap;
    int32_t tile_nnz;          /* non-zeros per SpMV tile (set by gse_plan) */
    int32_t n_tiles;
    int32_t rv_lanes;          /* > 0: row-vector SpMV schedule, lanes per row; 0: tiles */
    int32_t max_row_nnz;       /* longest row (set by gse_encode / gse_plan) */
    double eta[3];             /* ||A - A_s||_inf / ||A||_inf, s = 1, 2, 3 */
    double exact_frac;         /* share of non-zeros whose exponent is shared */
    int32_t block_rows;        /* 0: the one table sem[]; > 0: rows per block, each block
                                  with its own table in block_sem (gse_encode_blocks) */
    int32_t block_stride;      /* entries per block in block_sem: 2^idx_bits */
    int16_t* block_sem;        /* device [ceil(n_rows / block_rows) * block_stride] */
} gse_matrix;

/* Plain FP64 CSR operand for the baseline operators on the same schedule.
 * col and val must hold gse_pad(nnz) entries and be 16-byte aligned. */
typedef struct gse_csr {
    int32_t n_rows;
    int32_t n_cols;
    int64_t nnz;
    const int32_t* row_ptr;    /* device [n_rows + 1] */
    const int32_t* col;        /* device [gse_pad(nnz)] */
    const double* val;         /* device [gse_pad(nnz)] */
    int32_t* tile_row;         /* device [tile_cap] */
    int32_t tile_cap;
    int32_t tile_nnz;
    int32_t n_tiles;
    int32_t rv_lanes;
    int32_t max_row_nnz;
} gse_csr;

/* Entries tile_row needs for any tile size the library may choose. */
int32_t gse_tile_entries(int64_t nnz);

/* Device workspace gse_encode needs (bytes).  n_rows and nnz as in CSR. */
gse_status gse_encode_workspace(int64_t nnz, int32_t n_rows, size_t* ws_bytes);

/* Convert a device FP64 CSR matrix into GSE-SEM planes.
 * Section III-B.1 (shared-exponent extraction: exponent histogram, the k
 * most frequent), Section III-B.2 (table stored +1; the maximum exponent is
 * forced into the last slot if the k most frequent miss it), Algorithm 1
 * (per-value slot search, denormalised mantissa) in its 64-bit form.
 *   row_ptr, col, val : device CSR (col/val: nnz entries, no padding needed).
 *   num_exp           : k in 1..64; the slot index takes ceil(log2 k) bits.
 *   sem_in            : host array of num_exp shared exponents (biased + 1)
 *                       to reuse a table (Section III-B.1); NULL computes it.
 *                       A reused table that leaves a value without a larger
 *                       shared exponent gives GSE_ERR_RANGE.
 *   A                 : in: plane pointers, tile_row/tile_cap and idx_layout
 *                       (GSE_IDX_AUTO unless a layout is wanted); out: every
 *                       other field; the SpMV schedule is chosen as by
 *                       gse_plan(A, 1024, -1).
 *   ws, ws_bytes      : device workspace of gse_encode_workspace() bytes.
 * Errors: GSE_ERR_NONFINITE (Inf/NaN value), GSE_ERR_RANGE (sizes, a shared
 * exponent below 63 whose grid would leave the normal range, uncovered
 * value), GSE_ERR_ARG, GSE_ERR_NOMEM, GSE_ERR_HIP.  On error the planes are
 * unspecified.  Synchronizes `stream`. */
gse_status gse_encode(const int32_t* row_ptr, const int32_t* col, const double* val,
                      int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t num_exp,
                      const int16_t* sem_in, gse_matrix* A, void* ws, size_t ws_bytes,
                      void* stream);

/* Per-row-block shared-exponent tables (Section III-B.1: for a low
 * preprocessing cost the matrix is cut into row blocks and one random row of
 * each block stands for the exponent distribution of that block).  Rows
 * [b*block_rows, (b+1)*block_rows) form block b (the last may be shorter);
 * each block gets a table of num_exp shared exponents, chosen as gse_encode
 * chooses the global one (count descending, ties to the larger exponent, the
 * maximum forced in), from the exponents of sample_rows[b] -- or, with
 * sample_rows NULL, of all the block's values -- and then, if the table
 * misses the block's own largest exponent, that exponent in the next free
 * slot or in place of the last one (every value needs a shared exponent
 * above its own, Section III-B.2).  Each non-zero is encoded (Algorithm 1)
 * against its block's table; the planes, slot index and layouts are those
 * of gse_encode.
 *   block_rows  : >= GSE_MIN_BLOCK_ROWS.
 *   sample_rows : device int32 [ceil(n_rows / block_rows)], one row of each
 *                 block (drawn by the caller), or NULL.
 *   A           : as for gse_encode, plus block_sem: device int16 buffer of
 *                 gse_block_table_entries() entries, written here (block b's
 *                 table at b * block_stride, block_stride = 2^idx_bits,
 *                 unused slots 0).  Out: block_rows, block_stride, eta,
 *                 exact_frac (measured against each block's own exponents),
 *                 num_used (the most slots any block uses); sem[] is zero.
 * The SpMV of such a matrix stages each row's table in LDS and runs the
 * row-tile schedule (rv_lanes 0 with 1024-non-zero tiles, rows of at most
 * eight non-zeros) or the row-vector one (rv_lanes > 0; with rv_lanes 0 on
 * longer rows, lanes from the mean row length).  The encoder and
 * gse_plan(A, 1024, -1) choose between them by the longest row;
 * gse_autotune times both.  gse_spmv, gse_cg and gse_gmres take such a
 * matrix; the batched solver and the server do not (GSE_ERR_ARG).
 * Errors: those of gse_encode; GSE_ERR_ARG for block_rows below the minimum,
 * a NULL block_sem, or a sample row outside its block.  Synchronizes `stream`. */
gse_status gse_encode_blocks(const int32_t* row_ptr, const int32_t* col, const double* val,
                             int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t num_exp,
                             int32_t block_rows, const int32_t* sample_rows, gse_matrix* A,
                             void* ws, size_t ws_bytes, void* stream);
/* Entries block_sem needs (0 for invalid arguments). */
int64_t gse_block_table_entries(int32_t n_rows, int32_t block_rows, int32_t num_exp);

/* One shared-exponent table for the whole matrix, chosen from a sample
 * (Section III-B.1: one random row of each row block stands for that
 * block's exponents): the exponent counts of the drawn rows sample_rows[b],
 * one in each block of block_rows rows, are pooled and the table is chosen
 * from them as gse_encode chooses it from the full histogram (count
 * descending, ties to the larger exponent, the pool's maximum forced in);
 * then, if the table misses the matrix's own largest exponent, that exponent
 * goes into the next free slot or in place of the last one (every value needs
 * a shared exponent above its own, Section III-B.2).  The planes, index
 * layouts, eta, exact_frac and default plan are those of gse_encode with that
 * table; the result is an ordinary one-table matrix (block_rows 0) that every
 * operator, solver, the batched solver and the server take.
 *   block_rows  : >= 1 (rows per sampled block; the last may be shorter).
 *   sample_rows : device int32 [ceil(n_rows / block_rows)], one row of each
 *                 block, drawn by the caller; required.
 * Errors: those of gse_encode; GSE_ERR_ARG for block_rows < 1, a NULL
 * sample_rows or a sample row outside its block.  Workspace as gse_encode.
 * Synchronizes `stream`. */
gse_status gse_encode_sampled(const int32_t* row_ptr, const int32_t* col, const double* val,
                              int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t num_exp,
                              int32_t block_rows, const int32_t* sample_rows, gse_matrix* A,
                              void* ws, size_t ws_bytes, void* stream);

/* gse_encode for callers that cannot allocate device memory (tight serving
 * loops, harnesses that forbid hipMalloc; not for use under graph capture,
 * as it reads the table back and synchronizes like gse_encode):
 * the same encoder, planes, table, eta and default plan, bit for bit, but its
 * scratch record lives in a static device array of
 * gse_encode_static_scratch_bytes() bytes (16 KiB) that each GPU the library
 * runs on holds until the process ends.  The record's size does not depend on
 * the matrix; a build whose record outgrew the array would return
 * GSE_ERR_NOMEM.  The caller still passes the CSR input, the planes and
 * tile_row in A as for gse_encode.  No hipMalloc, hipFree or allocating
 * library call is made; the scratch is cleared by a kernel at the start of
 * every call.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (concurrent host threads, or streams running at once)
 * race and must be serialized by the caller.  Errors as gse_encode.
 * Synchronizes `stream`. */
gse_status gse_encode_static(const int32_t* row_ptr, const int32_t* col, const double* val,
                             int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t num_exp,
                             const int16_t* sem_in, gse_matrix* A, void* stream);
size_t gse_encode_static_scratch_bytes(void);

/* (Re)build the SpMV schedule.  Two schedules exist:
 *   tiles       (rv_lanes == 0): fixed runs of tile_nnz non-zeros (1024, 2048
 *               or 4096) per workgroup step, rows of any length; with 1024
 *               and no row longer than eight non-zeros, runs of 192 rows
 *               instead (the tile table is then not read);
 *   row-vector  (rv_lanes = 1, 2, 4, ..., 64): that many lanes per row,
 *               for matrices whose rows are short and of similar length.
 * rv_lanes == -1 picks the default (tiles).  The tile table is always
 * built.  Synchronizes `stream`. */
gse_status gse_plan(gse_matrix* A, int32_t tile_nnz, int32_t rv_lanes, void* stream);
gse_status gse_csr_plan(gse_csr* M, int32_t tile_nnz, int32_t rv_lanes, void* stream);

/* y = A_s x with s = k_segments in {1, 2, 3}: the head-only operator of
 * Algorithm 2 and its head+tail1 and head+tail1+tail2 variants
 * (Section III-C.2).  Values are read with s planes and multiplied and
 * accumulated in FP64 (Section III-C.2).  x: device [n_cols], y: device
 * [n_rows]; x and y must not overlap (GSE_ERR_ARG).  Asynchronous on `stream`. */
gse_status gse_spmv(const gse_matrix* A, int32_t k_segments, const double* x, double* y,
                    void* stream);

/* Choose the SpMV schedule of A for k_segments by timing the candidates
 * (tiles of 1024 / 2048 / 4096 non-zeros; 1 ... 64 lanes per row, from an
 * eighth of the longest row up, when no row is longer than 64; for
 * per-row-block tables the row-tile ring and 1 ... 64 lanes) with `reps`
 * launches each on the caller's x
 * (device [n_cols]) and y (device [n_rows], overwritten), back to back on
 * the same operand as the solvers call it, then plan the fastest.  Results
 * are cached per process by format, segment count, size, longest row and
 * the share of rows in each power-of-two length class (the row pointers are
 * read to the host once per call) and, if the environment variable
 * GSE_AUTOTUNE_CACHE names a file, in that file.  Synchronizes `stream`. */
gse_status gse_autotune(gse_matrix* A, int32_t k_segments, const double* x, double* y,
                        int32_t reps, void* stream);
gse_status gse_csr_autotune(gse_csr* M, const double* x, double* y, int32_t reps, void* stream);

/* Baseline: y = A x with plain FP64 CSR values on the same tile schedule
 * (the FP64-SpMV the paper compares against, Section IV-A). */
gse_status gse_csr_spmv(const gse_csr* M, const double* x, double* y, void* stream);

/* ------------------------------------------------------------------------
 * The FP16 / BF16 comparators (Section IV-C): every value stored as one
 * IEEE binary16 (GSE_LP_FP16) or bfloat16 (GSE_LP_BF16) word -- the same
 * width as the GSE-SEM head -- next to its plain int32 column, widened to
 * FP64 in the SpMV and multiplied and accumulated in FP64. */
#define GSE_LP_FP16 1
#define GSE_LP_BF16 2

typedef struct gse_lp_matrix {
    int32_t n_rows;
    int32_t n_cols;
    int64_t nnz;
    int32_t fmt;               /* GSE_LP_FP16 or GSE_LP_BF16 */
    int32_t pad;
    const int32_t* row_ptr;    /* device [n_rows + 1], recorded by gse_lp_convert */
    int32_t* col;              /* device plane [gse_pad(nnz)], 16-byte aligned */
    uint16_t* val;             /* device plane [gse_pad(nnz)], 16-byte aligned */
    int32_t* tile_row;         /* device [tile_cap] */
    int32_t tile_cap;
    int32_t tile_nnz;
    int32_t n_tiles;
    int32_t rv_lanes;
    int32_t max_row_nnz;
    int32_t pad2;
    int64_t overflow;          /* values that rounded past the largest finite one (to +-inf) */
    double eta;                /* ||A - A_h||_inf / ||A||_inf (inf after an overflow) */
} gse_lp_matrix;

/* Device workspace gse_lp_convert needs (bytes). */
gse_status gse_lp_workspace(size_t* ws_bytes);

/* Round a device FP64 CSR matrix to FP16 or BF16: each value rounded once,
 * to nearest with ties to even (a magnitude past the largest finite value
 * becomes an infinity and is counted in M->overflow -- the overflow the
 * paper reports for FP16, Section IV-D.2); columns copied.  M: in: col, val,
 * tile_row, tile_cap; out: every other field, the schedule as by
 * gse_lp_plan(M, 1024, -1).  ws: device, 256-byte aligned, of
 * gse_lp_workspace() bytes.  Synchronizes `stream`. */
gse_status gse_lp_convert(const int32_t* row_ptr, const int32_t* col, const double* val,
                          int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t fmt,
                          gse_lp_matrix* M, void* ws, size_t ws_bytes, void* stream);
gse_status gse_lp_plan(gse_lp_matrix* M, int32_t tile_nnz, int32_t rv_lanes, void* stream);

/* y = A_h x with the 16-bit values widened to FP64 (FP16-SpMV / BF16-SpMV of
 * Section IV-C), on the same schedules as gse_spmv.  Asynchronous. */
gse_status gse_lp_spmv(const gse_lp_matrix* M, const double* x, double* y, void* stream);

/* ------------------------------------------------------------------------
 * Solvers for A x = b (Section I), stepped mixed precision per Section III-D
 * (Algorithm 3, Eqs. 3-6, Conditions 1-3).  Only the operator reads reduced
 * segments; dot products, residuals and the x / r / p updates are FP64
 * (Section IV-D.3). */
#define GSE_CG 0
#define GSE_GMRES 1

#define GSE_TRIG_NONE 0
#define GSE_TRIG_C1 1         /* Condition 1 */
#define GSE_TRIG_C2 2         /* Condition 2 */
#define GSE_TRIG_C3 3         /* Condition 3 */
#define GSE_TRIG_FLOOR 4      /* relres <= floor_c * eta_s (addition) */
#define GSE_TRIG_TOL 5        /* tolerance met with an inexact operator */
#define GSE_TRIG_BREAKDOWN 6  /* CG breakdown below three segments */

typedef struct gse_params {
    double tol;               /* relative residual ||b - A x|| / ||b|| */
    int32_t max_iter;         /* iteration cap (CG 5000, GMRES 30*500 in IV-A) */
    int32_t restart;          /* GMRES cycle length (30 in IV-A) */
    int32_t start_segments;   /* first s (1 per Algorithm 3) */
    int32_t fixed_segments;   /* 0: stepped; 1..3: fixed s */
    int32_t l, t, m;          /* controller schedule (Section III-D) */
    double rsd_limit;         /* Condition 1 threshold */
    int32_t ndec_limit;       /* nDec threshold for Conditions 1-2 */
    double reldec_limit;      /* Condition 2 threshold */
    int32_t ndec_rule;        /* 0: compare nDec with ndec_limit; 1: with t/2 */
    double floor_c;           /* floor trigger factor, 0 disables */
    int32_t switch_mode;      /* CG after a switch: 0 p = r, 1 keep p, 2 (default) keep p
                                 unless the residual replacement changes ||r|| by more
                                 than a factor of 2, then p = r */
    int32_t record_history;   /* kept for callers; the history is always recorded */
    int32_t launch_mode;      /* 0: iterations replayed from HIP graphs, 1: direct launches
                                 (CG on systems of at most 4096 rows whose rows hold at most 8
                                 non-zeros runs every iteration of a segment count in one
                                 launch of one workgroup, in either mode) */
    int32_t orth;             /* GMRES Gram-Schmidt: 1 classical applied twice (CGS2: two
                                 reductions and three passes over the basis per step); 2 the
                                 same with the second pass delayed one step (DCGS2: one
                                 reduction, two passes; restart <= 32); 0 (default) DCGS2
                                 when restart <= 32, else CGS2.  Both reach the Krylov
                                 iterates of Section IV-A's GMRES(30) to rounding; DCGS2
                                 learns each residual estimate one product later, so a
                                 cycle that stops computes one product more. */
} gse_params;

typedef struct gse_report {
    gse_status status;
    int32_t iters;
    int32_t iters_per_seg[3];
    int32_t switch_iter[2];       /* -1: no switch */
    int32_t switch_trigger[2];    /* GSE_TRIG_* */
    double relres_recursive;      /* the solver's own residual estimate */
    double relres_true;           /* ||b - A_3 x|| / ||b|| recomputed at the end */
    double time_ms;               /* wall time of the call */
} gse_report;

/* Fill `p` with the paper's CG (method GSE_CG) or GMRES presets
 * (Section IV-D.1) and tol = 1e-10, floor_c = 10, restart 30. */
gse_status gse_default_params(int32_t method, gse_params* p);

/* Workspace bytes for a solve of an n_rows x n_rows system with up to
 * n_tiles SpMV tiles (gse_tile_entries(nnz)). */
gse_status gse_solver_workspace(int32_t method, int32_t n_rows, int64_t nnz, int32_t restart,
                                int32_t max_iter, size_t* ws_bytes);

/* Stepped (or fixed-segment) CG.  b: device [n], x: device [n], x0 on
 * entry, solution on return.  Blocks until the solve ends.  Returns
 * GSE_OK, GSE_NOT_CONVERGED, GSE_ERR_BREAKDOWN or an error.  Results are
 * bit-reproducible for a given operator, format and parameter set. */
gse_status gse_cg(const gse_matrix* A, const double* b, double* x, const gse_params* p,
                  gse_report* rep, void* ws, size_t ws_bytes, void* stream);

/* Stepped (or fixed-segment) restarted GMRES(p->restart), classical
 * Gram-Schmidt applied twice, Givens rotations on the device. */
gse_status gse_gmres(const gse_matrix* A, const double* b, double* x, const gse_params* p,
                     gse_report* rep, void* ws, size_t ws_bytes, void* stream);

/* The FP16 / BF16 comparator solvers of Section IV-D.3: the same CG and
 * GMRES with the fixed 16-bit operator A_h (p->fixed_segments and the
 * controller are ignored).  Convergence is judged on A_h's own residual
 * (relres_true is ||b - A_h x|| / ||b||); the distance to the FP64 matrix's
 * solution is the caller's to measure.  A non-finite value (an overflowed
 * FP16 entry) ends the solve with GSE_ERR_BREAKDOWN or GSE_NOT_CONVERGED. */
gse_status gse_lp_cg(const gse_lp_matrix* M, const double* b, double* x, const gse_params* p,
                     gse_report* rep, void* ws, size_t ws_bytes, void* stream);
gse_status gse_lp_gmres(const gse_lp_matrix* M, const double* b, double* x, const gse_params* p,
                        gse_report* rep, void* ws, size_t ws_bytes, void* stream);

/* Baselines: the same solvers with plain FP64 CSR values. */
gse_status gse_csr_cg(const gse_csr* M, const double* b, double* x, const gse_params* p,
                      gse_report* rep, void* ws, size_t ws_bytes, void* stream);
gse_status gse_csr_gmres(const gse_csr* M, const double* b, double* x, const gse_params* p,
                         gse_report* rep, void* ws, size_t ws_bytes, void* stream);

/* Copy the residual history of the last solve that ran with record_history
 * on `ws`: relres[i] and the segment count of iteration i, i = 0..iters.
 * hist / seg: host arrays of at least cap entries.  Synchronizes. */
gse_status gse_solve_history(const void* ws, int32_t cap, double* hist, int32_t* seg,
                             void* stream);

/* ------------------------------------------------------------------------
 * Batched stepped CG: n_sys independent SPD systems of any sizes solved
 * together, each with its own operator, segment count and stepped controller
 * (Section III-D per system), all advanced by one set of kernel launches per
 * iteration (16-iteration epochs replayed from a HIP graph when
 * p->launch_mode == 0).  A system's iterates and result are bit-identical
 * whether it is solved alone or in any batch.  The SpMV stages tiles of up to
 * 2048 non-zeros in LDS, so operators planned with tile_nnz 1024 (the
 * default) run fastest; any valid plan is accepted.  A system of at least
 * 2^16 rows planned on the row-tile ring (rows of at most 8 non-zeros,
 * tile_nnz 1024) takes its product from that single-system kernel: such
 * systems share one grouped launch per ring instance and iteration, each on
 * workgroups of its own; epochs holding them are launched directly. */
typedef struct gse_system {
    const gse_matrix* A;   /* stepped GSE-SEM operator, or NULL */
    const gse_csr* M;      /* FP64 CSR operator, used when A is NULL */
    const double* b;       /* device [n_rows] */
    double* x;             /* device [n_rows], 16-byte aligned: x0 in, solution out */
} gse_system;

/* Workspace bytes for gse_batch_cg on these systems with p->max_iter. */
gse_status gse_batch_workspace(int32_t n_sys, const gse_system* sys, const gse_params* p,
                               size_t* ws_bytes);

/* Solve all systems with the same parameters `p` (CG presets).  rep: host
 * array of n_sys reports.  ws: device, 256-byte aligned, at least
 * gse_batch_workspace bytes; it holds the per-system vectors, histories and
 * the work lists.  Blocks until every system has stopped.  Returns GSE_OK
 * when all converged, else the first non-OK status in system order (each
 * report carries its own). */
gse_status gse_batch_cg(int32_t n_sys, const gse_system* sys, const gse_params* p,
                        gse_report* rep, void* ws, size_t ws_bytes, void* stream);

/* Residual and segment history of system `index` of the last gse_batch_cg
 * on `ws` (as gse_solve_history).  Synchronizes. */
gse_status gse_batch_history(const void* ws, int32_t index, int32_t cap, double* hist,
                             int32_t* seg, void* stream);

/* ------------------------------------------------------------------------
 * Solver server: requests (host CSR + b) arrive at any time and join the
 * running batch of stepped CG solves above.  The caller hands over one
 * device arena at creation; the server sub-allocates every device buffer of
 * a request from it (operator planes, vectors, history, plus a transient
 * FP64 copy and encode workspace released right after the encode) and never
 * calls hipMalloc.  Admission is first come, first served: the oldest
 * waiting request starts as soon as a batch slot is free and its blocks fit
 * in the arena.  One worker thread per server does the device work on its
 * own stream; submit / poll / stats are thread-safe. */
#define GSE_FMT_GSE 0      /* stepped GSE-SEM operator (encoded on arrival) */
#define GSE_FMT_CSR64 1    /* FP64 CSR operator (the baseline) */

typedef struct gse_request {
    int32_t n_rows;          /* square system, n_rows >= 1 */
    int64_t nnz;
    const int32_t* row_ptr;  /* host CSR [n_rows+1], [nnz], [nnz]; with b and x these */
    const int32_t* col;      /* host arrays must stay valid until the ticket completes */
    const double* val;
    const double* b;         /* host [n_rows] */
    double* x;               /* host [n_rows]: x0 when x0_given, the solution on completion */
    int32_t format;          /* GSE_FMT_GSE or GSE_FMT_CSR64 */
    int32_t num_exp;         /* shared exponents for GSE_FMT_GSE (1..64) */
    int32_t x0_given;        /* 1: start from x, 0: from zero */
    gse_params params;       /* CG parameters (gse_default_params(GSE_CG, ...)) */
} gse_request;

typedef struct gse_solver gse_solver;

typedef struct gse_server_stats {
    int64_t queued;               /* submitted, waiting for admission */
    int64_t running;              /* admitted, not finished */
    int64_t admitted, completed;  /* totals since creation */
    int64_t arena_bytes;          /* bytes the requests may use */
    int64_t arena_used, arena_peak, arena_largest_free;
} gse_server_stats;

/* arena: device, 256-byte aligned, owned by the caller and untouched by it
 * until gse_solver_destroy returns; a fixed part holds the batch tables for
 * max_slots systems.  stream: the caller's stream, synchronized once so the
 * arena is ready.  The device current at the call is the server's. */
gse_status gse_solver_create(void* arena, size_t arena_bytes, int32_t max_slots, void* stream,
                             gse_solver** out);
/* Bytes a request occupies while it runs (resident) and during its encode
 * (transient, GSE only). */
gse_status gse_solver_footprint(const gse_request* rq, size_t* resident, size_t* transient);
/* Queue a request (validated on the host, CSR structure included); returns a
 * ticket.  GSE_ERR_NOMEM if it can never fit in the arena. */
gse_status gse_solver_submit(gse_solver* s, const gse_request* rq, uint64_t* ticket);
/* GSE_PENDING while the ticket runs or waits; GSE_OK once it has finished,
 * with rep filled (rep->status: the solve's status; rep->time_ms: submit to
 * completion) and the ticket retired; GSE_ERR_TICKET for an unknown one. */
gse_status gse_solver_poll(gse_solver* s, uint64_t ticket, gse_report* rep);
gse_status gse_solver_stats(gse_solver* s, gse_server_stats* out);
/* Stop the worker after its current step; unfinished tickets are dropped. */
gse_status gse_solver_destroy(gse_solver* s);

/* ------------------------------------------------------------------------ */
/* Diagnostic: dst = src, `bytes` a multiple of 16, both 16-byte aligned;
 * the reference streaming kernel for HBM bandwidth and counter scaling. */
gse_status gse_stream_copy(const void* src, void* dst, size_t bytes, void* stream);
/* Diagnostic: dst[i] = src[8i] + ... + src[8i+7] for i < n_out (FP64, src
 * [8 n_out], dst [n_out], 16-byte aligned): a streaming kernel that reads
 * eight bytes for each one it writes (89 % reads), the read-dominated mix of
 * the SpMV, as its bandwidth ceiling (coalesced non-temporal 16-byte loads,
 * eight workgroups per CU).  Asynchronous. */
gse_status gse_stream_reduce8(const double* src, double* dst, size_t n_out, void* stream);

const char* gse_status_str(gse_status s);
const char* gse_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GSE_H */
