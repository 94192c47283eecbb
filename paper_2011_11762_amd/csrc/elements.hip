// Element-level assignment and extraction, truncation with error control and
// matrix addition (the construction, extraction, truncation and addition task
// types of Sec. 2.2), on the block-sparse storage: Morton-ordered leaves,
// column-major inside.
#include <cmath>

#include <hipcub/hipcub.hpp>

#include "common.h"

namespace qbsm {

namespace {

struct ElemStatus {
    int32_t range_err;
    int32_t dup;
    int64_t nblk;
};

// Morton key of block (i, j): bits of i above those of j.
__device__ __forceinline__ uint32_t block_key(uint32_t i, uint32_t j) {
    uint32_t k = 0;
    for (int b = 0; b < 16; ++b) k |= (((i >> b) & 1u) << (2 * b + 1)) | (((j >> b) & 1u) << (2 * b));
    return k;
}

__global__ void k_elem_keys(const int64_t *row, const int64_t *col, int64_t n, int64_t nrows, int64_t ncols,
                            int32_t bs, uint32_t *keys, int32_t *off, ElemStatus *st) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t r = row[t], c = col[t];
    const bool ok = r >= 0 && c >= 0 && r < nrows && c < ncols;
    if (!ok) st->range_err = 1;
    keys[t] = ok ? block_key((uint32_t)(r / bs), (uint32_t)(c / bs)) : 0u;
    off[t] = ok ? (int32_t)((r % bs) + (c % bs) * bs) : 0;
}

// Element t lands at leaf rank[t], offset off[t]; a second element at the
// same place marks the input as repeated.
__global__ void k_elem_scatter(const double *val, const uint32_t *keys, const int32_t *off, const int32_t *rank,
                               int64_t n, int64_t n2, double *pool, int32_t *hits, uint32_t *okeys,
                               ElemStatus *st) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t pos = (int64_t)rank[t] * n2 + off[t];
    if (atomicAdd(hits + pos, 1) != 0) st->dup = 1;
    pool[pos] = val[t];
    okeys[rank[t]] = keys[t];  // every element of a leaf writes the same key
}

template <class T>
__global__ void k_elem_get(const uint32_t *keys, int64_t nblk, const T *vals, int32_t bs, const int64_t *row,
                           const int64_t *col, int64_t n, int64_t nrows, int64_t ncols, double *out,
                           ElemStatus *st) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t r = row[t], c = col[t];
    if (r < 0 || c < 0 || r >= nrows || c >= ncols) {
        st->range_err = 1;
        out[t] = 0.0;
        return;
    }
    const uint32_t k = block_key((uint32_t)(r / bs), (uint32_t)(c / bs));
    int64_t lo = 0, hi = nblk;  // first stored key >= k
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    out[t] = (lo < nblk && keys[lo] == k) ? (double)vals[lo * (int64_t)bs * bs + (r % bs) + (c % bs) * bs] : 0.0;
}

// Squared leaf norms as sort keys; a NaN becomes the canonical positive NaN,
// which sorts after every number and keeps its leaf.
__global__ void k_sq_norms(const double *norms, int64_t n, double *sq, int32_t *idx) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double v = norms[t] * norms[t];
    sq[t] = isnan(v) ? __longlong_as_double(0x7FF8000000000000ll) : v;
    idx[t] = (int32_t)t;
}

// Number of leading partial sums that are finite and <= lim (the sums do
// not decrease, and stay infinite or NaN once they are): an infinite norm is
// never within the bound, also where lim itself overflows.
__global__ void k_cut(const double *csum, int64_t n, double lim, int64_t *k) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (csum[mid] <= lim && isfinite(csum[mid])) lo = mid + 1;
        else hi = mid;
    }
    *k = lo;
}

__global__ void k_drop_flags(const int32_t *idx_sorted, const int64_t *k, int64_t n, int32_t *keep) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    keep[idx_sorted[t]] = t < *k ? 0 : 1;
}

template <class T>
__global__ void __launch_bounds__(256) k_gather_kept(const int32_t *keep, const int32_t *pos, int64_t n,
                                                     const uint32_t *keys, const T *vals, int64_t n2,
                                                     uint32_t *okeys, T *ovals) {
    const int64_t b = blockIdx.x;
    if (b >= n || !keep[b]) return;
    const int64_t o = pos[b];
    if (threadIdx.x == 0) okeys[o] = keys[b];
    for (int64_t e = threadIdx.x; e < n2; e += 256) ovals[o * n2 + e] = vals[b * n2 + e];
}

void commit_new_pattern(Matrix &m, hipStream_t s) {
    m.has_blocks = true;
    m.version++;
    m.pattern_id++;
    m.filled_by = 0;
    m.trees.clear();
    m.packs.clear();
    m.stream = s;
}

}  // namespace

int64_t matrix_set_elements(Matrix &m, int64_t n, const int64_t *row, const int64_t *col, const double *val,
                            hipStream_t s) {
    QB_CHECK(n >= 0, QBSM_ERR_ARG, "n must be >= 0");
    QB_CHECK(n == 0 || (row && col && val), QBSM_ERR_ARG, "null element arrays");
    QB_CHECK(n <= (int64_t)INT32_MAX, QBSM_ERR_UNSUPPORTED, "too many elements");
    matrix_settle(m, s);
    const int64_t n2 = (int64_t)m.bs * m.bs;
    DArr<ElemStatus> st(1, s);
    fill_bytes_zero(st.p, sizeof(ElemStatus), s);
    DArr<uint32_t> keys(n ? n : 1, s);
    DArr<int32_t> off(n ? n : 1, s), rank(n ? n : 1, s), dummy(1, s);
    const uint64_t range = (uint64_t)1 << (2 * ceil_log2(m.nbr > m.nbc ? m.nbr : m.nbc));
    if (n) {
        k_elem_keys<<<grid_for(n, 256), 256, 0, s>>>(row, col, n, m.nrows, m.ncols, m.bs, keys.p, off.p, st.p);
        QB_LAUNCH_CHECK();
    }
    // leaf rank of every element: its block among the distinct blocks (Morton order)
    bitmap_rank(keys.p, nullptr, n, range, rank.p, dummy.p, &st.p->nblk, s);
    ElemStatus h = read_back(st.p, s);
    QB_CHECK(!h.range_err, QBSM_ERR_PATTERN, "element index outside the matrix");
    const int64_t nb = n ? h.nblk : 0;
    DArr<double> pool(nb ? nb * n2 : 1, s);
    DArr<int32_t> hits(nb ? nb * n2 : 1, s);
    DArr<uint32_t> okeys(nb ? nb : 1, s);
    if (nb) {
        fill_bytes_zero(pool.p, nb * n2 * sizeof(double), s);
        fill_bytes_zero(hits.p, nb * n2 * sizeof(int32_t), s);
        k_elem_scatter<<<grid_for(n, 256), 256, 0, s>>>(val, keys.p, off.p, rank.p, n, n2, pool.p, hits.p,
                                                       okeys.p, st.p);
        QB_LAUNCH_CHECK();
    }
    h = read_back(st.p, s);
    QB_CHECK(!h.dup, QBSM_ERR_PATTERN, "repeated element");
    m.v64 = std::move(pool);
    m.v32.reset();
    ++m.storage_id;
    m.keys = std::move(okeys);
    m.nblk = nb;
    m.storage = ST_F64;
    commit_new_pattern(m, s);
    return nb;
}

void matrix_get_elements(Matrix &m, int64_t n, const int64_t *row, const int64_t *col, double *val,
                         hipStream_t s) {
    QB_CHECK(m.has_blocks, QBSM_ERR_STATE, "matrix has no blocks yet");
    QB_CHECK(n >= 0, QBSM_ERR_ARG, "n must be >= 0");
    if (!n) return;
    QB_CHECK(row && col && val, QBSM_ERR_ARG, "null element arrays");
    DArr<ElemStatus> st(1, s);
    fill_bytes_zero(st.p, sizeof(ElemStatus), s);
    if (m.storage == ST_F32)
        k_elem_get<float><<<grid_for(n, 256), 256, 0, s>>>(m.keys.p, m.nblk, m.v32.p, m.bs, row, col, n, m.nrows,
                                                          m.ncols, val, st.p);
    else
        k_elem_get<double><<<grid_for(n, 256), 256, 0, s>>>(m.keys.p, m.nblk, m.v64.p, m.bs, row, col, n, m.nrows,
                                                           m.ncols, val, st.p);
    QB_LAUNCH_CHECK();
    QB_CHECK(!read_back(st.p, s).range_err, QBSM_ERR_ARG, "element index outside the matrix");
}

int64_t matrix_truncate(Matrix &m, double eps, hipStream_t s) {
    QB_CHECK(m.has_blocks, QBSM_ERR_STATE, "matrix has no blocks yet");
    QB_CHECK(eps >= 0.0 && !std::isnan(eps), QBSM_ERR_ARG, "eps must be >= 0");
    const int64_t n = m.nblk;
    if (!n) return 0;
    QB_CHECK(n <= (int64_t)INT32_MAX, QBSM_ERR_UNSUPPORTED, "too many blocks");
    matrix_settle(m, s);
    const double *norms = matrix_norms(m, s);
    DArr<double> sq(n, s), sq_sorted(n, s), csum(n, s);
    DArr<int32_t> idx(n, s), idx_sorted(n, s), keep(n, s), pos(n + 1, s);
    DArr<int64_t> k(1, s), nkept(1, s);
    k_sq_norms<<<grid_for(n, 256), 256, 0, s>>>(norms, n, sq.p, idx.p);
    QB_LAUNCH_CHECK();
    // ascending squared norms, ties in storage order (the radix sort is stable)
    size_t tmp_sort = 0, tmp_scan = 0;
    QB_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_sort, sq.p, sq_sorted.p, idx.p, idx_sorted.p, (int)n,
                                              0, 64, s));
    QB_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, tmp_scan, sq_sorted.p, csum.p, (int)n, s));
    DArr<uint8_t> tmp(tmp_sort > tmp_scan ? tmp_sort : tmp_scan, s);
    QB_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tmp_sort, sq.p, sq_sorted.p, idx.p, idx_sorted.p, (int)n,
                                              0, 64, s));
    QB_HIP(hipcub::DeviceScan::InclusiveSum(tmp.p, tmp_scan, sq_sorted.p, csum.p, (int)n, s));
    k_cut<<<1, 1, 0, s>>>(csum.p, n, eps * eps, k.p);
    QB_LAUNCH_CHECK();
    k_drop_flags<<<grid_for(n, 256), 256, 0, s>>>(idx_sorted.p, k.p, n, keep.p);
    QB_LAUNCH_CHECK();
    exclusive_scan_i32(keep.p, pos.p, n, nkept.p, s);
    const int64_t nk = read_back(nkept.p, s);
    if (nk == n) return n;
    const int64_t n2 = (int64_t)m.bs * m.bs;
    DArr<uint32_t> okeys(nk ? nk : 1, s);
    if (m.storage == ST_F32) {
        DArr<float> ov(nk ? nk * n2 : 1, s);
        k_gather_kept<float><<<(unsigned)n, 256, 0, s>>>(keep.p, pos.p, n, m.keys.p, m.v32.p, n2, okeys.p, ov.p);
        QB_LAUNCH_CHECK();
        m.v32 = std::move(ov);
        ++m.storage_id;
    } else {
        DArr<double> ov(nk ? nk * n2 : 1, s);
        k_gather_kept<double><<<(unsigned)n, 256, 0, s>>>(keep.p, pos.p, n, m.keys.p, m.v64.p, n2, okeys.p, ov.p);
        QB_LAUNCH_CHECK();
        m.v64 = std::move(ov);
        ++m.storage_id;
    }
    m.keys = std::move(okeys);
    m.nblk = nk;
    commit_new_pattern(m, s);
    return nk;
}

}  // namespace qbsm

// ------------------------------------------------------------------ addition
namespace qbsm {

namespace {

// Diagonal block keys 0 .. nbd-1 appended after the first operand's keys.
__global__ void k_diag_keys(int64_t nbd, uint32_t *keys) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nbd) keys[t] = block_key((uint32_t)t, (uint32_t)t);
}

__global__ void k_union_keys(const uint32_t *keys, const int32_t *rank, int64_t n, uint32_t *okeys) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) okeys[rank[t]] = keys[t];  // equal keys write equal values
}

// out[rank[t]] += coef * src[t], block by block; one workgroup per block.
// Products and sums are rounded separately (contraction off), so that
// alpha*a + beta*b is rounded as two products and one sum.
template <class T>
__global__ void __launch_bounds__(256) k_add_scaled(const T *src, const int32_t *rank, int64_t n, int64_t n2,
                                                    double coef, double *out) {
    const int64_t t = blockIdx.x;
    if (t >= n) return;
    double *o = out + (int64_t)rank[t] * n2;
    const T *x = src + t * n2;
    for (int64_t e = threadIdx.x; e < n2; e += 256) {
#pragma clang fp contract(off)
        const double p = coef * (double)x[e];
        o[e] = o[e] + p;
    }
}

// sigma on the diagonal elements (r, r), r < nd, of the diagonal blocks.
__global__ void k_add_diag(const int32_t *rank, int64_t nbd, int32_t bs, int64_t nd, double sigma, double *out) {
    const int64_t t = blockIdx.x;
    if (t >= nbd) return;
    const int64_t n2 = (int64_t)bs * bs;
    for (int r = threadIdx.x; r < bs; r += blockDim.x) {
        if (t * bs + r >= nd) continue;
        double *o = out + (int64_t)rank[t] * n2 + r + (int64_t)r * bs;
        *o = *o + sigma;
    }
}

void add_operand(const Matrix &m, const int32_t *rank, double coef, double *pool, hipStream_t s) {
    const int64_t n2 = (int64_t)m.bs * m.bs;
    if (!m.nblk) return;
    if (m.storage == ST_F32)
        k_add_scaled<float><<<(unsigned)m.nblk, 256, 0, s>>>(m.v32.p, rank, m.nblk, n2, coef, pool);
    else
        k_add_scaled<double><<<(unsigned)m.nblk, 256, 0, s>>>(m.v64.p, rank, m.nblk, n2, coef, pool);
    QB_LAUNCH_CHECK();
}

// Union of the stored keys of a (and of b, or of the diagonal blocks), ranked
// in Morton order; returns the number of distinct leaves (host read).
int64_t union_rank(const Matrix &a, const Matrix *b, int64_t nbd, DArr<uint32_t> &keys, DArr<int32_t> &rank,
                   DArr<uint32_t> &okeys, hipStream_t s) {
    const int64_t na = a.nblk, nb = b ? b->nblk : nbd;
    const int64_t n = na + nb;
    keys.alloc(n ? n : 1, s);
    rank.alloc(n ? n : 1, s);
    if (na) QB_HIP(hipMemcpyAsync(keys.p, a.keys.p, na * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    if (b && nb) QB_HIP(hipMemcpyAsync(keys.p + na, b->keys.p, nb * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    if (!b && nb) {
        k_diag_keys<<<grid_for(nb, 256), 256, 0, s>>>(nb, keys.p + na);
        QB_LAUNCH_CHECK();
    }
    const uint64_t range = (uint64_t)1 << (2 * ceil_log2(a.nbr > a.nbc ? a.nbr : a.nbc));
    DArr<int32_t> dummy(1, s);
    DArr<int64_t> cnt(1, s);
    bitmap_rank(keys.p, nullptr, n, range, rank.p, dummy.p, cnt.p, s);
    const int64_t nu = n ? read_back(cnt.p, s) : 0;
    okeys.alloc(nu ? nu : 1, s);
    if (n) {
        k_union_keys<<<grid_for(n, 256), 256, 0, s>>>(keys.p, rank.p, n, okeys.p);
        QB_LAUNCH_CHECK();
    }
    return nu;
}

void commit_values(Matrix &m, DArr<uint32_t> &okeys, DArr<double> &pool, int64_t nblk, hipStream_t s) {
    m.keys = std::move(okeys);
    m.v64 = std::move(pool);
    m.v32.reset();
    ++m.storage_id;
    m.nblk = nblk;
    m.storage = ST_F64;
    commit_new_pattern(m, s);
}

}  // namespace

void matrix_add(double alpha, Matrix &A, double beta, Matrix &B, Matrix &C, hipStream_t s) {
    QB_CHECK(A.has_blocks && B.has_blocks, QBSM_ERR_STATE, "matrix has no blocks yet");
    QB_CHECK(A.nrows == B.nrows && A.ncols == B.ncols && A.bs == B.bs, QBSM_ERR_SHAPE, "operands differ in shape");
    QB_CHECK(C.nrows == A.nrows && C.ncols == A.ncols && C.bs == A.bs, QBSM_ERR_SHAPE, "output shape differs");
    QB_CHECK(&C != &A && &C != &B, QBSM_ERR_ARG, "output aliases an operand");
    QB_CHECK(std::isfinite(alpha) && std::isfinite(beta), QBSM_ERR_ARG, "alpha and beta must be finite");
    matrix_settle(A, s);
    matrix_settle(B, s);
    matrix_settle(C, s);
    DArr<uint32_t> keys, okeys;
    DArr<int32_t> rank;
    const int64_t nu = union_rank(A, &B, 0, keys, rank, okeys, s);
    const int64_t n2 = (int64_t)A.bs * A.bs;
    DArr<double> pool(nu ? nu * n2 : 1, s);
    if (nu) fill_bytes_zero(pool.p, nu * n2 * sizeof(double), s);
    add_operand(A, rank.p, alpha, pool.p, s);
    add_operand(B, rank.p + A.nblk, beta, pool.p, s);
    commit_values(C, okeys, pool, nu, s);
}

void matrix_add_identity(Matrix &A, double sigma, hipStream_t s) {
    QB_CHECK(A.has_blocks, QBSM_ERR_STATE, "matrix has no blocks yet");
    QB_CHECK(std::isfinite(sigma), QBSM_ERR_ARG, "sigma must be finite");
    matrix_settle(A, s);
    const int64_t nd = A.nrows < A.ncols ? A.nrows : A.ncols;
    const int64_t nbd = (nd + A.bs - 1) / A.bs;
    DArr<uint32_t> keys, okeys;
    DArr<int32_t> rank;
    const int64_t nu = union_rank(A, nullptr, nbd, keys, rank, okeys, s);
    const int64_t n2 = (int64_t)A.bs * A.bs;
    DArr<double> pool(nu ? nu * n2 : 1, s);
    if (nu) fill_bytes_zero(pool.p, nu * n2 * sizeof(double), s);
    add_operand(A, rank.p, 1.0, pool.p, s);
    if (nbd) {
        k_add_diag<<<(unsigned)nbd, 64, 0, s>>>(rank.p + A.nblk, nbd, A.bs, nd, sigma, pool.p);
        QB_LAUNCH_CHECK();
    }
    commit_values(A, okeys, pool, nu, s);
}

}  // namespace qbsm
