/*
 * CPU oracle for the block-sparse multiply -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct FP64 code.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load this library; the GPU
 * library never does, and the two share no code.
 *
 * What it computes (the plain definition the quadtree multiply reaches,
 * paper Sec. 2: a product with a nil (zero) operand is nil, sums over the
 * non-nil terms):
 *
 *   C_IJ = sum over K ascending with (I,K) in P_A and (K,J) in P_B of A_IK * B_KJ
 *
 * Leaf blocks are bs x bs, column-major (paper Sec. 2.1, basic dense leaf
 * type).  Every leaf product is  c_ij += a_il * b_lj  with l ascending, after
 * the previous leaf products of the same C block; no fused multiply-add
 * (build with -ffp-contract=off), so the result is fully determined.  OpenMP
 * parallelism is over output blocks only and never changes a summation order.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* OpenMP threads of the calls that follow (n >= 1); returns the count used
 * before.  Lets a caller time the same oracle on all threads and on one. */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    const int before = omp_get_max_threads();
    if (n >= 1) omp_set_num_threads(n);
    return before;
#else
    (void)n;
    return 1;
#endif
}

/* Frobenius norm of each block: sqrt of the sum of squares, summed in
 * column-major element order, FP64 (the truncation rule of paper Sec. 2.2
 * applied at block granularity). */
void oracle_block_fnorm(int64_t nblk, int32_t bs, const double *vals, double *out)
{
    const int64_t n2 = (int64_t)bs * bs;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nblk; ++b) {
        const double *x = vals + b * n2;
        double s = 0.0;
        for (int64_t e = 0; e < n2; ++e) s += x[e] * x[e];
        out[b] = sqrt(s);
    }
}

/* Element (r, l) of a leaf operand, optionally transposed. */
static inline double leaf_at(const double *x, int32_t bs, int trans, int32_t r, int32_t l)
{
    return trans ? x[l + (int64_t)r * bs] : x[r + (int64_t)l * bs];
}

/*
 * Segmented block products.
 *   out block o (o in [0, nout)) = sum over t in [seg[o], seg[o+1]) of
 *       op(L[lidx[t]]) * op(R[ridx[t]])
 * in the order t ascending (the caller lists each segment with the
 * contraction block index ascending).  op() transposes when the flag is set.
 * The output blocks are overwritten (zero-initialised first).
 */
void oracle_segmented_products(int32_t bs, int64_t nout, const int64_t *seg,
                               const int64_t *lidx, const int64_t *ridx,
                               const double *L, const double *R,
                               int transL, int transR, double *out)
{
    const int64_t n2 = (int64_t)bs * bs;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t o = 0; o < nout; ++o) {
        double *c = out + o * n2;
        memset(c, 0, sizeof(double) * (size_t)n2);
        for (int64_t t = seg[o]; t < seg[o + 1]; ++t) {
            const double *a = L + lidx[t] * n2;
            const double *b = R + ridx[t] * n2;
            if (!transL) {
                /* column j of c, then l ascending, rows innermost: each c_ij
                 * still receives its terms with l ascending. */
                for (int32_t j = 0; j < bs; ++j)
                    for (int32_t l = 0; l < bs; ++l) {
                        const double blj = leaf_at(b, bs, transR, l, j);
                        const double *acol = a + (int64_t)l * bs;
                        double *ccol = c + (int64_t)j * bs;
                        for (int32_t i = 0; i < bs; ++i) ccol[i] += acol[i] * blj;
                    }
            } else {
                for (int32_t j = 0; j < bs; ++j)
                    for (int32_t l = 0; l < bs; ++l) {
                        const double blj = leaf_at(b, bs, transR, l, j);
                        double *ccol = c + (int64_t)j * bs;
                        for (int32_t i = 0; i < bs; ++i)
                            ccol[i] += leaf_at(a, bs, 1, i, l) * blj;
                    }
            }
        }
    }
}
