/*
 * qbsm -- block-sparse quadtree matrix multiply on AMD MI355X (gfx950).
 *
 * C ABI of libqbsm.so.  Plain pointers and sizes only.
 *
 * Method (Rubensson, Rudberg, Kruchinina, Artemov, "The Chunks and Tasks
 * Matrix Library 2.0"):
 *   - Sec. 2: a matrix is a sparse quadtree -- identically zero, a small leaf
 *     matrix, or four quadrants that are themselves sparse quadtrees; matrix
 *     operations are recursive algorithms over the nonzero branches.
 *   - Sec. 2.1: a non-leaf node refers to its four children; a nil child is an
 *     identically zero quadrant.  Each task handles one quadtree level and a
 *     task with a nil input does no work (this is how sparsity is exploited).
 *     The dense leaf type stores elements column-wise.
 *   - Sec. 2.2: construction from index/value vectors, extraction, regular
 *     matrix-matrix multiplication, truncation of small parts.
 *
 * Conventions for every call
 *   - All array arguments are DEVICE pointers unless stated otherwise; scalar
 *     results are written through HOST pointers.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every launch of a call goes to that stream.  Calls that report sizes
 *     (set_blocks, multiply_symbolic) synchronise the stream before returning.
 *   - A leaf block is bs x bs, column-major (element (r,c) at r + c*bs).
 *     Edge blocks of a matrix whose size is not a multiple of bs are padded;
 *     the library zeroes the padding of every block it stores or writes.
 *   - Block coordinates (I,J) are 0-based.  Matrices may be rectangular; the
 *     block grid side is limited to 65536 (quadtree depth <= 16).
 *   - Every call returns a qbsm_status; nothing is thrown or aborted across
 *     the ABI.  qbsm_last_error() gives a per-thread text for the last
 *     failure.  NaN/Inf values propagate per IEEE 754.
 *   - Handles are not thread safe: do not use one handle from two threads at
 *     once, and keep a plan's matrices alive (and their patterns unchanged)
 *     for the plan's lifetime.
 *   - Device memory comes from the allocator set by qbsm_set_allocator
 *     (default: hipMallocAsync / hipFreeAsync on the call's stream, from the
 *     device's default memory pool; the library raises that pool's release
 *     threshold so that memory freed by one call is reused by the next
 *     instead of returning to the driver at each synchronisation).
 */
#ifndef QBSM_H
#define QBSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* C++ sees the enumerations with a fixed 32-bit underlying type, so that any
 * int32 value a C caller passes is a valid value on the library's side (the
 * library rejects unknown ones); C sees plain int-sized enumerations. */
#ifdef __cplusplus
#define QBSM_ENUM(name) enum name : int32_t
#else
#define QBSM_ENUM(name) enum name
#endif

typedef QBSM_ENUM(qbsm_status_e) {
    QBSM_OK = 0,
    QBSM_ERR_ARG = 1,         /* null pointer, negative size, bad enum value        */
    QBSM_ERR_SHAPE = 2,       /* inner dimensions / leaf sizes do not agree         */
    QBSM_ERR_PATTERN = 3,     /* duplicate or out-of-range block coordinates        */
    QBSM_ERR_OOM = 4,         /* the allocator returned NULL                        */
    QBSM_ERR_HIP = 5,         /* a HIP runtime call failed                          */
    QBSM_ERR_UNSUPPORTED = 6, /* size or option outside what the library handles    */
    QBSM_ERR_STATE = 7        /* handle not ready (e.g. matrix without blocks)      */
} qbsm_status;

/* Arithmetic of the leaf products.  Operands are stored by the library in
 * the mode's format, products accumulate on the GPU's matrix cores (MFMA):
 *   QBSM_F64    FP64 operands, FP64 accumulation, FP64 result.
 *   QBSM_F32    operands rounded to binary32 (RNE), FP32 accumulation, FP32 result.
 *   QBSM_BF16   operands rounded to bfloat16 (RNE, straight from FP64), FP32
 *               accumulation, FP32 result.
 *   QBSM_BF16X3 split precision: x = hi + lo with hi = bf16(x), lo = bf16(x - hi)
 *               (lo = 0 where hi is not finite); a*b ~ hi_a*hi_b + hi_a*lo_b +
 *               lo_a*hi_b, FP32 accumulation, FP32 result.  An infinite input
 *               gives a non-finite result (Inf, or NaN where the split terms of
 *               its partner differ in sign) in exactly the elements it reaches.
 *   QBSM_OZAKI_I8 Ozaki splitting (Ozaki, Ogita, Oishi and Rump 2012) on
 *               8-bit integer MFMA: each line of a leaf (a row of the left
 *               operand, a column of the right one) gets the exponent e of its
 *               largest magnitude m (m < 2^e; one more when m lies within 0.4 %
 *               below 2^e), each element x is truncated to the integer
 *               M = sign(x) floor(|x| 2^(47 - e)) and M is written as 6
 *               balanced base-256 digits in [-128, 127] on the grids
 *               2^(e + 1 - 8t), t = 1..6.  The 21 digit pairs with
 *               t + u <= 7 are multiplied; the products of one pair group
 *               (t + u fixed) over one leaf sum exactly in 32-bit integers, are
 *               combined in FP64, scaled by 2^(e_row + e_col) (so the whole FP64
 *               exponent range is covered) and accumulated in FP64; FP64 result.
 *               Needs 64 x 64 leaves and a plan with unit 64 or 128 (see
 *               qbsm_plan_opts).  A line holding an Inf or NaN makes every
 *               element its leaf products reach NaN.
 * In every mode a product exists only where both leaf blocks are stored: an
 * Inf or NaN never meets the implicit zeros of a nil block. */
typedef QBSM_ENUM(qbsm_mode_e) {
    QBSM_F64 = 0,
    QBSM_F32 = 1,
    QBSM_BF16 = 2,
    QBSM_BF16X3 = 3,
    QBSM_OZAKI_I8 = 4
} qbsm_mode;

typedef struct qbsm_matrix_ *qbsm_matrix;
typedef struct qbsm_plan_ *qbsm_plan;
typedef struct qbsm_batch_ *qbsm_batch;

/* Device allocator hooks.  alloc(bytes, stream, ctx) returns device memory
 * usable on `stream` or NULL; release(ptr, stream, ctx) returns it.  Passing
 * two NULL functions restores the default.  Not thread safe w.r.t. calls in
 * flight. */
typedef void *(*qbsm_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*qbsm_release_fn)(void *ptr, void *stream, void *ctx);
qbsm_status qbsm_set_allocator(qbsm_alloc_fn alloc, qbsm_release_fn release, void *ctx);

const char *qbsm_status_string(qbsm_status st);
const char *qbsm_last_error(void);
/* Library version as 10000*major + 100*minor + patch. */
int32_t qbsm_version(void);

/* ---------------------------------------------------------------- matrices */

/* An empty (identically zero) nrows x ncols matrix with leaf size bs
 * (Sec. 2: the zero quadtree).  bs must be 32, 64 or 128.  The handle owns
 * all memory it later allocates. */
qbsm_status qbsm_matrix_create(int64_t nrows, int64_t ncols, int32_t bs, qbsm_matrix *out);
qbsm_status qbsm_matrix_destroy(qbsm_matrix m);

/* Construction from leaf blocks (Sec. 2.2, assignment from index and value
 * vectors, at leaf-block granularity) followed by block truncation.
 *   brow, bcol : int32[nblk] block coordinates (device), any order.
 *   vals       : double[nblk * bs * bs] (device), block t at t*bs*bs, column-major.
 *   drop_tol   : 0 keeps every block; otherwise block t is dropped iff its
 *                FP64 Frobenius norm is < drop_tol (equality and NaN keep) --
 *                the truncation operation of Sec. 2.2 at block granularity.
 *   nkept      : host out, number of stored blocks after truncation.
 * The values are copied (the caller keeps ownership of its buffers); padding
 * beyond the logical size is stored as zero.  Replaces any previous content.
 * Errors: QBSM_ERR_PATTERN for a coordinate outside the block grid or a
 * repeated (I,J) (checked on the device before anything is stored; the
 * matrix is left unchanged). */
qbsm_status qbsm_matrix_set_blocks(qbsm_matrix m, int64_t nblk, const int32_t *brow,
                                   const int32_t *bcol, const double *vals, double drop_tol,
                                   void *stream, int64_t *nkept);

/* Rounds the stored values to binary32 (round to nearest even) and frees
 * the FP64 copy, halving the matrix's memory when it only feeds FP32 or
 * BF16 modes.  A later QBSM_F64 multiply of this matrix uses the rounded
 * values; readback widens them exactly.  No effect on an FP32-stored matrix. */
qbsm_status qbsm_matrix_store_f32(qbsm_matrix m, void *stream);

/* Packs the matrix's current values for the numeric phase of `mode` ahead of
 * use, so that the packing runs while the symbolic phase is still being
 * worked out (Sec. 2.1: the task templates leave scheduling to the runtime,
 * and the operand preparation of a multiply does not depend on its symbolic
 * phase).
 *   roles : 1 = as a left operand (row lines), 2 = as a right operand
 *           (column lines), 3 = both (A * A).  A transposed use swaps them.
 * The packing kernels run on a library-owned stream (one per device, default
 * priority) that first waits for everything already queued on `stream`; the
 * pack memory is taken on `stream`.  Nothing is synchronised.  Every later
 * use of the packs (numeric phase, batch creation and runs, on any stream)
 * waits for them, and replacing or freeing the matrix's values
 * (set_blocks, store_f32, destroy, use as a numeric output) first orders the
 * affected streams after them.  Packs that are already current are left
 * alone.  Errors: QBSM_ERR_STATE without blocks, QBSM_ERR_ARG for bad roles. */
qbsm_status qbsm_matrix_prepack(qbsm_matrix m, qbsm_mode mode, int32_t roles, void *stream);

/* Shape and stored-block count (host outs; any may be NULL). */
qbsm_status qbsm_matrix_info(qbsm_matrix m, int64_t *nrows, int64_t *ncols, int32_t *bs,
                             int64_t *nblk);

/* Extraction (Sec. 2.2), at leaf-block granularity: the stored pattern in
 * canonical row-major (I, J) order into device int32[nblk] arrays. */
qbsm_status qbsm_matrix_get_pattern(qbsm_matrix m, int32_t *brow, int32_t *bcol, void *stream);

/* Extraction (Sec. 2.2; leaf matrices are stored column-wise, Sec. 2.1):
 * the values of the stored blocks, in the canonical order of
 * qbsm_matrix_get_pattern, as FP64 column-major blocks into device
 * double[nblk * bs * bs] (caller-owned).  Results of an FP32 mode are
 * widened exactly; padding beyond the logical size reads as zero.
 * Errors: QBSM_ERR_ARG for a null array when blocks are stored.  Does not
 * synchronise. */
qbsm_status qbsm_matrix_get_values(qbsm_matrix m, double *vals, void *stream);

/* Construction from elements (Sec. 2.2, assignment from vectors of row
 * indices, column indices and values):
 *   row, col : int64[n] element coordinates (device), any order.
 *   val      : double[n] values (device).
 *   nblk     : host out, number of stored leaves.
 * The leaves are the blocks holding at least one given element (in storage
 * order); their other elements, and the padding, are zero.  Replaces any
 * previous content.  Errors: QBSM_ERR_PATTERN for a coordinate outside the
 * matrix or a repeated (row, col) (checked on the device; the matrix is left
 * unchanged).  Synchronises the stream. */
qbsm_status qbsm_matrix_set_elements(qbsm_matrix m, int64_t n, const int64_t *row, const int64_t *col,
                                     const double *val, void *stream, int64_t *nblk);

/* Extraction of elements (Sec. 2.2, extraction of the elements given by
 * vectors of row and column indices): val[q] = A(row[q], col[q]) as FP64
 * (device arrays), zero where no leaf is stored.  Errors: QBSM_ERR_ARG for a
 * coordinate outside the matrix (checked on the device; synchronises). */
qbsm_status qbsm_matrix_get_elements(qbsm_matrix m, int64_t n, const int64_t *row, const int64_t *col,
                                     double *val, void *stream);

/* Truncation with error control (Sec. 2.2, removal of small matrix elements
 * with control of the error), at leaf granularity in the Frobenius norm:
 * with the leaves ordered by FP64 Frobenius norm ascending (ties in storage
 * order), the longest leading run whose squared norms sum to at most eps^2
 * is removed, so that ||A_before - A_after||_F <= eps.  Leaves with a NaN
 * norm stay, and so does every leaf from the first at which the running sum
 * of squared norms is no longer finite (an infinite norm is never within
 * eps, however large).  eps = 0 removes the identically zero leaves only.
 *   nkept : host out, leaves left.  Synchronises the stream.
 * Errors: QBSM_ERR_ARG for eps < 0 or NaN; QBSM_ERR_STATE without blocks. */
qbsm_status qbsm_matrix_truncate(qbsm_matrix m, double eps, void *stream, int64_t *nkept);

/* Matrix addition (Sec. 2.2, regular addition): C = alpha*A + beta*B on the
 * union of the two leaf patterns (no leaf is dropped; a missing block counts
 * as zero).  Each element is rounded as alpha*a, beta*b and their sum, in
 * FP64; the result is stored in FP64.  C must have A's shape and leaf size
 * and must not be A or B; its previous content is replaced.  Errors:
 * QBSM_ERR_SHAPE for differing shapes, QBSM_ERR_ARG for aliasing or a
 * non-finite coefficient, QBSM_ERR_STATE without blocks.  Synchronises. */
qbsm_status qbsm_matrix_add(double alpha, qbsm_matrix A, double beta, qbsm_matrix B, qbsm_matrix C,
                            void *stream);

/* Addition of a scaled identity (Sec. 2.2), in place: A += sigma*I, sigma
 * added to the elements (r, r), r < min(nrows, ncols); missing diagonal
 * leaves are created.  The result is stored in FP64.  Errors: QBSM_ERR_ARG
 * for a non-finite sigma, QBSM_ERR_STATE without blocks.  Synchronises. */
qbsm_status qbsm_matrix_add_identity(qbsm_matrix A, double sigma, void *stream);

/* Extraction of selected blocks (Sec. 2.2, extraction of the elements given
 * by index vectors, at leaf-block granularity): for q in [0, n), block
 * (brow[q], bcol[q]) is written as an FP64 column-major bs x bs block to
 * vals + q*bs*bs (device), zero when the block is not stored.  Errors:
 * QBSM_ERR_PATTERN if a coordinate lies outside the block grid (checked on
 * the device; synchronises the stream). */
qbsm_status qbsm_matrix_extract_blocks(qbsm_matrix m, int64_t n, const int32_t *brow,
                                       const int32_t *bcol, double *vals, void *stream);

/* ---------------------------------------------------------------- multiply */

/* Options of the symbolic phase.  unit: side, in elements, of the C quadtree
 * node that one GPU workgroup owns (the depth where the recursion hands over
 * to a dense kernel); 0 picks the default (128).  Must be bs * 2^s with s in
 * 0..2 and a value in {64, 128, 256}.  A plan with unit 256 serves the
 * 4-byte-accumulator modes (F32, BF16, BF16X3); its FP64 numeric phase
 * returns QBSM_ERR_UNSUPPORTED (a 256 x 256 FP64 accumulator exceeds the
 * register file of one compute unit).  QBSM_OZAKI_I8 runs on plans with
 * unit 64 or 128 and 64 x 64 leaves (its six slices per operand leave no
 * LDS for a 256-wide unit) and returns QBSM_ERR_UNSUPPORTED otherwise. */
typedef struct {
    int32_t unit;
    /* 1: only the output blocks with I <= J are formed (the symmetric square
     * of Sec. 2.2: for a symmetric A, A * A is symmetric and its upper
     * triangle holds it all; with a transposed right operand, A * A^T is the
     * symmetric rank-k construction of the same section; about half the leaf
     * products).  Needs a square product and no mask; the output's pattern is
     * the upper triangle of the product's pattern.  0: every block. */
    int32_t upper;
    /* Sparse approximate multiply (Sec. 1 and 2.2 name it for matrices with
     * decay): > 0 leaves out every leaf product A_IK * B_KJ whose FP64
     * Frobenius norms satisfy ||A_IK|| * ||B_KJ|| < spamm_tol (the strict test
     * of truncation), so C holds the blocks with at least one remaining
     * product and its error is at most the sum of the left-out norm products.
     * The norms are taken from the values current at the symbolic phase.
     * 0 = the regular multiply.  Ignored by qbsm_multiply_backward. */
    double spamm_tol;
    /* Schedule of the numeric phase (how workgroups take the plan's units;
     * results are the same bit for bit).  0 = automatic: one workgroup per
     * unit, on a single-LDS-stage kernel that fits more workgroups per
     * compute unit for QBSM_F64 plans at unit 128 without transposed
     * operands and for QBSM_BF16 and
     * QBSM_BF16X3 plans at unit 128 with at most 1.25 unit-level pairs per
     * unit (about one leaf product per unit, where the multiply is bound by
     * memory), else on the double-buffered kernel.  1 = one workgroup per
     * unit, double-buffered kernel.
     * 2 = streamed where the mode and unit
     * allow it: resident workgroups each run every G-th unit, reading the
     * next unit's metadata and issuing its first operand copies before
     * storing the current unit's output (units 64 and 128, all modes but
     * QBSM_OZAKI_I8; elsewhere one workgroup per unit).  Used by
     * qbsm_multiply_numeric, qbsm_multiply_backward and (from the forward
     * plan) qbsm_multiply_backward_plan; the batched and no-allocation entry
     * points keep their own schedules.  QBSM_ERR_ARG for another value. */
    int32_t schedule;
    int32_t reserved[3];
} qbsm_plan_opts;

/* Symbolic phase of C = A * B (Sec. 2 and 2.1: the recursive multiply over
 * nonzero quadtree branches; a pair with a nil operand is pruned).
 * Walks the two quadtrees level by level from the root, keeping only node
 * pairs whose both operands are non-nil, and records the nonzero leaf-pair
 * products and the block pattern of C.  Integer work, deterministic.
 *   A : m x k, B : k x n, equal leaf sizes.  A and B may be the same handle.
 *   opts may be NULL.  Host outs nblk_C (blocks of C) and nprod (nonzero
 *   leaf products) may be NULL.
 * Errors: QBSM_ERR_SHAPE for k mismatch or different bs; QBSM_ERR_STATE if
 * a matrix has never been given blocks (an empty set_blocks is fine). */
qbsm_status qbsm_multiply_symbolic(qbsm_matrix A, qbsm_matrix B, const qbsm_plan_opts *opts,
                                   void *stream, qbsm_plan *plan, int64_t *nblk_C,
                                   int64_t *nprod);

/* Generalised symbolic phase: out = op(L) * op(R) restricted to the block
 * pattern of `mask` (mask may be NULL for no restriction); op transposes
 * when the flag is nonzero.  With a mask, the output has exactly the mask's
 * pattern and blocks without any product are zero.  Used for the masked
 * adjoints of the multiply; same errors as qbsm_multiply_symbolic. */
qbsm_status qbsm_multiply_symbolic_ex(qbsm_matrix L, int32_t trans_l, qbsm_matrix R,
                                      int32_t trans_r, qbsm_matrix mask,
                                      const qbsm_plan_opts *opts, void *stream, qbsm_plan *plan,
                                      int64_t *nblk_out, int64_t *nprod);

/* Plan facts (host outs, any may be NULL): output blocks, nonzero leaf
 * products, block-level flops 2*sum(m_I k_K n_J) over the products with
 * logical sizes, the work unit side, the number of work units (C quadtree
 * nodes at the unit level) and of node pairs at that level. */
qbsm_status qbsm_plan_info(qbsm_plan p, int64_t *nblk_out, int64_t *nprod, int64_t *flops,
                           int32_t *unit, int64_t *nunits, int64_t *npairs);

/* The nonzero leaf products in canonical (I, J, K) order (row-major output
 * block, then contraction index ascending), as device int32[nprod] arrays.
 * Coordinates are those of op(L) (I,K) and op(R) (K,J). */
qbsm_status qbsm_plan_get_products(qbsm_plan p, int32_t *I, int32_t *K, int32_t *J,
                                   void *stream);

qbsm_status qbsm_plan_destroy(qbsm_plan p);

/* Numeric phase of the regular multiply (Sec. 2.2), the part the paper
 * leaves to its leaf library (Sec. 2.1: a leaf is a small dense matrix whose
 * product is one dense kernel call; Sec. 3 runs that call on 64 x 64 blocks
 * inside larger leaves): every nonzero leaf-block product of the plan on
 * the matrix cores, with a segmented, atomic-free accumulation -- every
 * output block is owned by one workgroup, which sums its products with the
 * contraction index ascending and writes the block once, so C_IJ is the sum
 * over K of L_IK R_KJ with exactly the plan's products.
 *   p    : plan from the symbolic phase; its operands must still have the
 *          patterns they had then (QBSM_ERR_STATE otherwise).
 *   mode : arithmetic of the leaf products (qbsm_mode).
 *   out  : receives the plan's output pattern and values, stored FP64 for
 *          QBSM_F64 and QBSM_OZAKI_I8, FP32 otherwise; its shape must be
 *          rows(op(L)) x cols(op(R)) with the same bs (QBSM_ERR_SHAPE) and it
 *          must not be an operand (QBSM_ERR_ARG).  Its memory is taken from
 *          the allocator unless it already holds this plan's result layout.
 * The operands' current values are used (they may change between calls as
 * long as their patterns do not); operand packs are made or refreshed as
 * needed.  QBSM_ERR_UNSUPPORTED for a unit side the mode does not run at.
 * Does not synchronise. */
qbsm_status qbsm_multiply_numeric(qbsm_plan p, qbsm_mode mode, qbsm_matrix out, void *stream);

/* Bytes of the library's per-device scratch array used by
 * qbsm_multiply_numeric_noalloc (64 MiB). */
#define QBSM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  The
 * numeric phase of qbsm_multiply_numeric (same kernels, same results bit for
 * bit) with two differences:
 *   - the operand packs (with their non-finite flags and, in the Ozaki mode,
 *     the line exponents) go to a file-scope device array of
 *     QBSM_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until
 *     the process ends, instead of allocator memory;
 *   - the result goes to the caller's array out_vals instead of a matrix
 *     handle: device memory of nblk_out * bs * bs elements, double for
 *     QBSM_F64 and QBSM_OZAKI_I8 and float otherwise.  Block t of the
 *     plan's output pattern is written column-major at t * bs * bs, the blocks
 *     taken in ascending Morton (Z) order of (I, J) -- the bits of I and J
 *     interleaved, I's bit above J's at every level -- which is the storage
 *     order of the matrix qbsm_multiply_numeric fills.  Padding beyond the
 *     logical size is written as zero; with a masked plan the mask's blocks
 *     without products are written as zero.
 * Nothing is allocated (no hipMalloc, no allocator hook) and nothing is
 * synchronised: launches only.  The plan's quadtree tables must be the ones
 * its symbolic phase made (QBSM_ERR_STATE otherwise).
 * The scratch array is shared by every call on one GPU and keeps the last
 * call's contents; each call writes what it reads first.  Calls that overlap
 * on one GPU (different streams or host threads) race on it: order them.
 * Errors: as qbsm_multiply_numeric; QBSM_ERR_UNSUPPORTED, before any launch,
 * when the two operand packs need more than QBSM_NOALLOC_SCRATCH_BYTES (bytes
 * per stored leaf and operand: bs*bs times 8 for F64, 4 for F32 and BF16X3,
 * 2 for BF16, 7 for the Ozaki mode plus 4*bs for its line exponents; each
 * operand's total rounded up to 256). */
qbsm_status qbsm_multiply_numeric_noalloc(qbsm_plan p, qbsm_mode mode, void *out_vals, void *stream);

/* Masked backward of C = A * B for an upstream gradient dC given on C's
 * pattern (dC may hold any subset of C's blocks):
 *   dA = (dC * B^T) restricted to A's pattern,
 *   dB = (A^T * dC) restricted to B's pattern.
 * dA / dB receive A's / B's pattern (either may be NULL to skip it); blocks
 * of the pattern without a product are zero.  Every term is one forward leaf
 * product (Sec. 2: the product list of the recursive multiply) whose dC
 * block exists, so the forward product list is regrouped -- by A block for
 * dA, by B block for dB -- instead of walking the quadtrees again: one
 * symbolic walk (the forward one, unit side from opts, spamm_tol and upper
 * ignored) and two numeric phases on `stream`.  Errors: QBSM_ERR_SHAPE when
 * dC is not shaped like A*B; QBSM_ERR_ARG when an output is dC or both
 * outputs are the same handle. */
qbsm_status qbsm_multiply_backward(qbsm_matrix A, qbsm_matrix B, qbsm_matrix dC, qbsm_mode mode,
                                   const qbsm_plan_opts *opts, qbsm_matrix dA, qbsm_matrix dB,
                                   void *stream);

/* The same backward from the plan of the forward product (a regular plan of
 * qbsm_multiply_symbolic: no transposes, mask, spamm_tol or upper option,
 * QBSM_ERR_UNSUPPORTED otherwise; its operands' patterns unchanged,
 * QBSM_ERR_STATE otherwise): no symbolic walk at all, only the regrouping of
 * its product list (a stable sort on device) and the two numeric phases.
 * The forward plan keeps its unit side. */
qbsm_status qbsm_multiply_backward_plan(qbsm_plan forward, qbsm_matrix dC, qbsm_mode mode, qbsm_matrix dA,
                                        qbsm_matrix dB, void *stream);

/* ----------------------------------------------------------------- batched */

/* Batched numeric phase over n independent plans: one persistent kernel
 * launch serves every output work unit of every member, units ordered
 * longest-processing-time first and pulled from a device work counter.
 * qbsm_batch_create validates, allocates the outputs and operand packs and
 * builds the work list (synchronises).  All plans must use the same work
 * unit side.  outs[i] receives plans[i]'s result. */
qbsm_status qbsm_batch_create(int32_t n, const qbsm_plan *plans, qbsm_mode mode,
                              qbsm_matrix *outs, void *stream, qbsm_batch *batch);
/* Launch-only part (operand packing + the persistent kernel); no allocation
 * and no synchronisation, so it may be captured into a HIP graph.  Before any
 * launch it checks that the batch still matches its matrices: errors
 * QBSM_ERR_STATE if a member plan is stale (an operand's pattern changed), an
 * operand's values were stored again (new pack buffers) or an output was
 * filled by another plan since qbsm_batch_create; create the batch again.
 * The batch's outputs and operands must outlive it. */
qbsm_status qbsm_batch_run(qbsm_batch batch, void *stream);
/* Captures qbsm_batch_run into a HIP graph on first use, then replays it. */
qbsm_status qbsm_batch_run_graph(qbsm_batch batch, void *stream);
/* Persistent workgroups per compute unit (default 0 = chosen by the library). */
qbsm_status qbsm_batch_set_occupancy(qbsm_batch batch, int32_t wg_per_cu);
qbsm_status qbsm_batch_destroy(qbsm_batch batch);

/* ----------------------------------------------------------------- tuning */

/* Result of qbsm_batch_autotune. */
typedef struct {
    int32_t unit;           /* fastest work-unit side */
    int32_t wg_per_cu;      /* fastest persistent occupancy, workgroups per compute unit */
    double ms;              /* its time per batched run (operand packing + persistent kernel) */
    double times_ms[3][4];  /* [unit 64, 128, 256][occupancy 1..4], < 0 where not applicable */
} qbsm_batch_tuning;

/* Autotuner of the batched form's tile schedule (the batch of Sec. 2.2
 * multiplies that qbsm_batch_create runs in one launch): for every work-unit
 * side that all members can run at -- which fixes the leaf-product kernel's
 * wave tile, its LDS stage and how many leaves one workgroup owns -- and
 * every persistent occupancy the kernel allows (at most 4 workgroups per
 * compute unit), builds the plans of L[i] * R[i] and a batch over them, runs
 * it once and then times `reps` runs with HIP events; reports the fastest
 * setting and the whole table.  Pass a representative subset of a large
 * batch: the trial batches allocate their own outputs and packs, which are
 * freed before returning.  Synchronises.  Errors: QBSM_ERR_UNSUPPORTED when
 * no unit side serves every member in this mode. */
qbsm_status qbsm_batch_autotune(int32_t n, const qbsm_matrix *L, const qbsm_matrix *R, qbsm_mode mode,
                                int32_t reps, void *stream, qbsm_batch_tuning *out);

/* Times the numeric phase of C = A * B for every valid unit side (symbolic
 * + numeric, `reps` timed repetitions after one warm-up) and reports the
 * fastest.  times_ms (host, may be NULL) receives 3 entries in the order
 * unit = 64, 128, 256 (negative when not applicable to the leaf size or the
 * mode; QBSM_OZAKI_I8 has units 64 and 128). */
qbsm_status qbsm_autotune_unit(qbsm_matrix A, qbsm_matrix B, qbsm_mode mode, int32_t reps,
                               void *stream, int32_t *best_unit, double *times_ms);

/* --------------------------------------------------------------- profiling */

/* Kernel timing: when enabled, HIP events are recorded on the launch stream
 * around every launch of the given kernel class (0 = numeric leaf-product
 * kernel, 1 = operand packing).  qbsm_profile_read synchronises the
 * recorded events and returns the launch count and summed GPU time in ms
 * since the last reset.  Not thread safe; off by default. */
qbsm_status qbsm_profile_enable(int32_t on);
qbsm_status qbsm_profile_reset(void);
qbsm_status qbsm_profile_read(int32_t kernel_class, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* QBSM_H */
