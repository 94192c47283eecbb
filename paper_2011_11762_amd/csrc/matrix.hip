// Matrix handles: construction from leaf blocks, block truncation, the
// sparse quadtree (Morton-ordered node tables), readback and operand packing.
#include <cmath>

#include "common.h"
#include "device_math.h"

namespace qbsm {

namespace {

// Morton key of block (I, J): bits of I and J interleaved, I's bit above J's
// at every level, so the two low bits of a key are the child slot
// q = 2*rowbit + colbit (quadrant order 00, 01, 10, 11).
__device__ __forceinline__ uint32_t morton2(uint32_t i, uint32_t j) {
    uint32_t k = 0;
#pragma unroll
    for (int b = 0; b < 16; ++b) {
        k |= ((i >> b) & 1u) << (2 * b + 1);
        k |= ((j >> b) & 1u) << (2 * b);
    }
    return k;
}

__device__ __forceinline__ void demorton2(uint32_t k, uint32_t &i, uint32_t &j) {
    i = 0;
    j = 0;
#pragma unroll
    for (int b = 0; b < 16; ++b) {
        i |= ((k >> (2 * b + 1)) & 1u) << b;
        j |= ((k >> (2 * b)) & 1u) << b;
    }
}

struct SetStatus {
    int32_t range_err;
    int32_t dup;
    int64_t nkept;
    int64_t ndistinct;
};

// Keys + range check for every input block.
__global__ void k_keys(const int32_t *brow, const int32_t *bcol, int64_t n, int64_t nbr, int64_t nbc,
                       uint32_t *keys, uint8_t *valid, SetStatus *st) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int32_t i = brow[t], j = bcol[t];
    bool ok = i >= 0 && j >= 0 && i < nbr && j < nbc;
    valid[t] = ok ? 1 : 0;
    keys[t] = ok ? morton2((uint32_t)i, (uint32_t)j) : 0u;
    if (!ok) st->range_err = 1;
}

// FP64 Frobenius norm of the logical part of each block; keep iff not (norm < tol).
__global__ void __launch_bounds__(256) k_norm_keep(const double *vals, const int32_t *brow,
                                                   const int32_t *bcol, const uint8_t *valid,
                                                   int64_t n, int32_t bs, int64_t nrows,
                                                   int64_t ncols, double tol, uint8_t *keep) {
    int64_t t = blockIdx.x;
    if (t >= n) return;
    __shared__ double red[256];
    double s = 0.0;
    if (valid[t]) {
        const int64_t mr = min((int64_t)bs, nrows - (int64_t)brow[t] * bs);
        const int64_t nc = min((int64_t)bs, ncols - (int64_t)bcol[t] * bs);
        const double *x = vals + t * (int64_t)bs * bs;
        const int r = threadIdx.x % bs;  // bs <= 128 divides 256
        for (int c = threadIdx.x / bs; c < bs; c += 256 / bs) {
            if (r < mr && c < nc) {
                double v = x[r + (int64_t)c * bs];
                s += v * v;
            }
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double nrm = sqrt(red[0]);
        keep[t] = (valid[t] && !(nrm < tol)) ? 1 : 0;
    }
}

__global__ void k_copy_flags(const uint8_t *valid, int64_t n, uint8_t *keep) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) keep[t] = valid[t];
}

// Scatter kept blocks into Morton order, zeroing the padding.
__global__ void __launch_bounds__(256) k_store_blocks(const double *vals, const int32_t *brow,
                                                      const int32_t *bcol, const uint32_t *keys,
                                                      const int32_t *rank, int64_t n, int32_t bs,
                                                      int64_t nrows, int64_t ncols, double *pool,
                                                      uint32_t *okeys) {
    int64_t t = blockIdx.x;
    if (t >= n) return;
    int32_t r = rank[t];
    if (r < 0) return;
    const int64_t mr = min((int64_t)bs, nrows - (int64_t)brow[t] * bs);
    const int64_t nc = min((int64_t)bs, ncols - (int64_t)bcol[t] * bs);
    const int64_t n2 = (int64_t)bs * bs;
    const double *x = vals + t * n2;
    double *y = pool + (int64_t)r * n2;
    if (mr == bs && nc == bs) {
        for (int64_t e = threadIdx.x; e < n2 / 2; e += 256)
            reinterpret_cast<double2 *>(y)[e] = reinterpret_cast<const double2 *>(x)[e];
    } else {
        const int rr = threadIdx.x % bs;
        for (int cc = threadIdx.x / bs; cc < bs; cc += 256 / bs) {
            int64_t e = rr + (int64_t)cc * bs;
            y[e] = (rr < mr && cc < nc) ? x[e] : 0.0;
        }
    }
    if (threadIdx.x == 0) okeys[r] = keys[t];
}

__global__ void k_narrow(const double *x, float *y, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) y[i] = (float)x[i];
}

// ---- quadtree build: one level from its children level
__global__ void k_tree_flags(const uint32_t *ckeys, const int64_t *ncount, int64_t cap, int32_t *flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    int64_t n = *ncount;
    int32_t f = 0;
    if (i < n) f = (i == 0 || (ckeys[i] >> 2) != (ckeys[i - 1] >> 2)) ? 1 : 0;
    flags[i] = f;
}

__global__ void k_tree_link(const uint32_t *ckeys, const int64_t *ncount, int64_t cap,
                            const int32_t *scan, uint32_t *pkeys, int32_t *child) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    int64_t n = *ncount;
    if (i >= n) return;
    // parent index = number of parent starts at or before i, minus one
    bool start = (i == 0 || (ckeys[i] >> 2) != (ckeys[i - 1] >> 2));
    int32_t p = scan[i] + (start ? 1 : 0) - 1;
    if (start) pkeys[p] = ckeys[i] >> 2;
    child[(int64_t)p * 4 + (ckeys[i] & 3u)] = (int32_t)i;
}

__global__ void k_desc2(const int32_t *child_hi, const int32_t *child_lo, int64_t n, int32_t *desc) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * 16) return;
    int64_t node = t >> 4;
    int q = (int)(t & 15);
    int qh = q >> 2, ql = q & 3;
    int32_t c = child_hi[node * 4 + qh];
    desc[t] = c < 0 ? -1 : child_lo[(int64_t)c * 4 + ql];
}

// ---- readback
__global__ void k_rm_keys(const uint32_t *keys, int64_t n, int64_t nbc, uint32_t *rmk, int32_t *bi,
                          int32_t *bj) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    uint32_t i, j;
    demorton2(keys[t], i, j);
    rmk[t] = (uint32_t)((uint64_t)i * (uint64_t)nbc + j);
    if (bi) { bi[t] = (int32_t)i; bj[t] = (int32_t)j; }
}

__global__ void k_scatter_pattern(const int32_t *bi, const int32_t *bj, const int32_t *rank, int64_t n,
                                  int32_t *brow, int32_t *bcol) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    brow[rank[t]] = bi[t];
    bcol[rank[t]] = bj[t];
}

template <class T>
__global__ void __launch_bounds__(256) k_scatter_values(const T *pool, const int32_t *rank, int64_t n,
                                                        int32_t bs, double *out) {
    int64_t t = blockIdx.x;
    if (t >= n) return;
    const int64_t n2 = (int64_t)bs * bs;
    const T *x = pool + t * n2;
    double *y = out + (int64_t)rank[t] * n2;
    for (int64_t e = threadIdx.x; e < n2; e += 256) y[e] = (double)x[e];
}

// One workgroup per requested block: binary search of its Morton key among
// the stored (sorted) keys, then a copy or a zero block.
template <class T>
__global__ void __launch_bounds__(256) k_extract(const uint32_t *keys, int64_t nblk, const T *pool, int32_t bs,
                                                 int64_t nbr, int64_t nbc, const int32_t *qi, const int32_t *qj,
                                                 int64_t nq, double *out, int32_t *bad) {
    const int64_t q = blockIdx.x;
    if (q >= nq) return;
    __shared__ int64_t s_idx;
    const int32_t i = qi[q], j = qj[q];
    const bool ok = i >= 0 && j >= 0 && i < nbr && j < nbc;
    if (threadIdx.x == 0) {
        int64_t idx = -1;
        if (ok) {
            const uint32_t k = morton2((uint32_t)i, (uint32_t)j);
            int64_t lo = 0, hi = nblk;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (keys[mid] < k) lo = mid + 1; else hi = mid;
            }
            if (lo < nblk && keys[lo] == k) idx = lo;
        } else {
            *bad = 1;
        }
        s_idx = idx;
    }
    __syncthreads();
    const int64_t n2 = (int64_t)bs * bs;
    const int64_t idx = s_idx;
    double *y = out + q * n2;
    for (int64_t e = threadIdx.x; e < n2; e += 256) y[e] = idx >= 0 ? (double)pool[idx * n2 + e] : 0.0;
}

// ---- operand packing
// Packed leaf layout: [part][chunk][line][LB bytes], lines = rows (ROLE_ROW)
// or columns (ROLE_COL) with the contraction index running along a line;
// the 16-byte pieces of a line are stored at slot piece ^ piece_swizzle(line).
// One thread converts and writes one 16-byte piece.  Column lines read
// contiguous source runs (piece-fastest thread order); row lines read
// across the column-major source (line-fastest thread order).
// Converts one 16-byte piece (EPP source values) to the mode and stores it
// (both parts for the split mode, the lo part n2 * EB bytes after the hi
// part); returns whether a packed value is Inf or NaN.
template <int MODE>
__device__ __forceinline__ bool store_piece(const double *v, uint8_t *o, int64_t n2) {
    constexpr int EB = MODE == QBSM_F64 ? 8 : MODE == QBSM_F32 ? 4 : 2;
    constexpr int PARTS = MODE == QBSM_BF16X3 ? 2 : 1;
    bool bad = false;  // a packed value (after the conversion to the mode) is Inf or NaN
    if (MODE == QBSM_F64) {
        bad = !isfinite(v[0]) || !isfinite(v[1]);
        *reinterpret_cast<double2 *>(o) = make_double2(v[0], v[1]);
    } else if (MODE == QBSM_F32) {
        const float4 f = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
        bad = !isfinite(f.x) || !isfinite(f.y) || !isfinite(f.z) || !isfinite(f.w);
        *reinterpret_cast<float4 *>(o) = f;
    } else {
        uint16_t h[8], lo[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            h[e] = bf16_rne_bits(v[e]);
            const bool hinf = (h[e] & 0x7F80u) == 0x7F80u;  // hi part Inf or NaN
            // the residual of an infinite (or overflowing) value is not
            // defined: its lo part is zero, so Inf stays Inf in the product
            lo[e] = hinf ? (uint16_t)0 : bf16_rne_bits(v[e] - bf16_bits_to_double(h[e]));
            bad |= hinf;
        }
        uint4 hv, lv;
        hv.x = h[0] | ((uint32_t)h[1] << 16); hv.y = h[2] | ((uint32_t)h[3] << 16);
        hv.z = h[4] | ((uint32_t)h[5] << 16); hv.w = h[6] | ((uint32_t)h[7] << 16);
        *reinterpret_cast<uint4 *>(o) = hv;
        if (PARTS == 2) {
            lv.x = lo[0] | ((uint32_t)lo[1] << 16); lv.y = lo[2] | ((uint32_t)lo[3] << 16);
            lv.z = lo[4] | ((uint32_t)lo[5] << 16); lv.w = lo[6] | ((uint32_t)lo[7] << 16);
            *reinterpret_cast<uint4 *>(o + n2 * EB) = lv;
        }
    }
    return bad;
}

// Packed layout per leaf: [part][chunk c][line l][LB bytes], LB = bk * EB;
// the 16-byte pieces of a line are stored at slot piece ^ piece_swizzle(line).
// One thread converts and writes one 16-byte piece.  Column lines read
// contiguous source runs (piece-fastest thread order); row lines read
// across the column-major source (line-fastest thread order).
template <class Src, int MODE>
__global__ void __launch_bounds__(256) k_pack(const Src *src, int64_t nblk, int32_t bs, int32_t bk, int role,
                                              uint8_t *dst, int32_t *nonfinite) {
    constexpr int EB = MODE == QBSM_F64 ? 8 : MODE == QBSM_F32 ? 4 : 2;  // bytes per element
    constexpr int EPP = 16 / EB;                                          // elements per piece
    constexpr int PARTS = MODE == QBSM_BF16X3 ? 2 : 1;
    const int LB = bk * EB;
    const int ppl = LB / 16;
    const int64_t nc = bs / bk;
    const int64_t per_leaf = nc * bs * ppl;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nblk * per_leaf) return;
    const int64_t leaf = t / per_leaf;
    const int64_t rem = t - leaf * per_leaf;
    int64_t c, l, piece;
    if (role == ROLE_COL) {
        piece = rem % ppl;
        l = (rem / ppl) % bs;
        c = rem / (ppl * (int64_t)bs);
    } else {
        l = rem % bs;
        piece = (rem / bs) % ppl;
        c = rem / ((int64_t)bs * ppl);
    }
    const int64_t n2 = (int64_t)bs * bs;
    const Src *x = src + leaf * n2;
    const int64_t k0 = c * bk + piece * EPP;
    double v[EPP];
#pragma unroll
    for (int e = 0; e < EPP; ++e)
        v[e] = role == ROLE_COL ? (double)x[(k0 + e) + l * bs] : (double)x[l + (k0 + e) * bs];
    uint8_t *o = dst + leaf * (PARTS * n2 * EB) + c * (int64_t)bs * LB + l * LB +
                 ((piece ^ piece_swizzle((int)l, LB)) << 4);
    if (store_piece<MODE>(v, o, n2)) *nonfinite = 1;
}

// Both roles of one matrix in one pass (the left and the right operand of
// A * A): one workgroup per leaf reads the leaf once into LDS and writes the
// row-line and the column-line packs from there.  Leaves of 32 and 64.

template <class Src, int MODE, int BS>
__global__ void __launch_bounds__(256) k_pack2(const Src *src, int32_t bk, uint8_t *dst_row, uint8_t *dst_col,
                                               int32_t *nf_row, int32_t *nf_col) {
    constexpr int EB = MODE == QBSM_F64 ? 8 : MODE == QBSM_F32 ? 4 : 2;
    constexpr int EPP = 16 / EB;
    constexpr int PARTS = MODE == QBSM_BF16X3 ? 2 : 1;
    constexpr int bs = BS;
    constexpr int64_t n2 = (int64_t)BS * BS;
    static_assert(n2 % 256 == 0, "whole leaf rounds");
    // the leaf in LDS with a column stride of bs + 1 doubles: the row-line
    // reads (consecutive rows) and the column-line reads (consecutive pieces
    // and columns) then fall on distinct banks
    constexpr int ld = BS + 1;
    __shared__ double x[ld * BS];
    const int64_t leaf = blockIdx.x;
    const Src *g = src + leaf * n2;
    Src t[n2 / 256];
#pragma unroll
    for (int q = 0; q < n2 / 256; ++q) t[q] = g[threadIdx.x + 256 * q];  // all loads in flight at once
#pragma unroll
    for (int q = 0; q < n2 / 256; ++q) {
        const int i = threadIdx.x + 256 * q;
        x[(i % BS) + (i / BS) * ld] = (double)t[q];
    }
    __syncthreads();
    const int LB = bk * EB;
    const int ppl = LB / 16;
    const int per_role = (bs / bk) * bs * ppl;
    bool bad_row = false, bad_col = false;
    for (int r = threadIdx.x; r < 2 * per_role; r += 256) {
        const bool col = r >= per_role;
        const int rem = col ? r - per_role : r;
        int c, l, piece;
        if (col) {
            piece = rem % ppl;
            l = (rem / ppl) % bs;
            c = rem / (ppl * bs);
        } else {
            l = rem % bs;
            piece = (rem / bs) % ppl;
            c = rem / (bs * ppl);
        }
        const int k0 = c * bk + piece * EPP;
        double v[EPP];
#pragma unroll
        for (int e = 0; e < EPP; ++e) v[e] = col ? x[(k0 + e) + l * ld] : x[l + (k0 + e) * ld];
        uint8_t *o = (col ? dst_col : dst_row) + leaf * (PARTS * n2 * EB) + (int64_t)c * bs * LB + l * LB +
                     ((piece ^ piece_swizzle(l, LB)) << 4);
        const bool bad = store_piece<MODE>(v, o, n2);
        if (col) bad_col |= bad; else bad_row |= bad;
    }
    if (bad_row) *nf_row = 1;
    if (bad_col) *nf_col = 1;
}

// Ozaki splitting: 6 slices of 8-bit digits per element (each exact in
// bfloat16) on the exponent grid of the element's packed line.
constexpr int OZ_SLICES = 6, OZ_BITS = 8;

// Exponent e of every packed line (a row of a leaf for the left operand, a
// column for the right one): the largest finite magnitude m of the line
// satisfies m < 2^e (e = 0 for an all-zero line).
template <class Src>
__global__ void __launch_bounds__(256) k_oz_exp(const Src *src, int64_t nblk, int32_t bs, int role, int32_t *ex) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nblk * bs) return;
    const int64_t leaf = t / bs;
    const int l = (int)(t - leaf * bs);
    const Src *x = src + leaf * (int64_t)bs * bs;
    double m = 0.0;
    for (int k = 0; k < bs; ++k) {
        const double v = fabs((double)(role == ROLE_COL ? x[k + (int64_t)l * bs] : x[l + (int64_t)k * bs]));
        if (isfinite(v) && v > m) m = v;
    }
    int e = 0;
    if (m > 0.0) (void)frexp(m, &e);
    ex[t] = e;
}

// One 16-byte piece (8 elements) of one packed line, all 6 slices: element x
// with line exponent e is cut into N = floor(|x| 2^(48 - e)) < 2^48 and slice
// t holds sign(x) * digit_t(N) * 2^(e - 8t), digit t being bits
// [48 - 8t, 56 - 8t) of N.  An Inf or NaN element is its own first slice.
template <class Src>
__global__ void __launch_bounds__(256) k_pack_oz(const Src *src, int64_t nblk, int32_t bs, int32_t bk, int role,
                                                 const int32_t *ex, uint8_t *dst, int32_t *nonfinite) {
    constexpr int EB = 2, EPP = 8;
    const int LB = bk * EB;
    const int ppl = LB / 16;
    const int64_t nc = bs / bk;
    const int64_t per_leaf = nc * bs * ppl;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nblk * per_leaf) return;
    const int64_t leaf = t / per_leaf;
    const int64_t rem = t - leaf * per_leaf;
    int64_t c, l, piece;
    if (role == ROLE_COL) {
        piece = rem % ppl;
        l = (rem / ppl) % bs;
        c = rem / (ppl * (int64_t)bs);
    } else {
        l = rem % bs;
        piece = (rem / bs) % ppl;
        c = rem / ((int64_t)bs * ppl);
    }
    const int64_t n2 = (int64_t)bs * bs;
    const Src *x = src + leaf * n2;
    const int64_t k0 = c * bk + piece * EPP;
    const int e = ex[leaf * bs + l];
    uint16_t d[OZ_SLICES][EPP];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < EPP; ++k) {
        const double v = role == ROLE_COL ? (double)x[(k0 + k) + l * bs] : (double)x[l + (k0 + k) * bs];
        if (!isfinite(v)) {
            bad = true;
            d[0][k] = bf16_rne_bits(v);
#pragma unroll
            for (int q = 1; q < OZ_SLICES; ++q) d[q][k] = 0;
            continue;
        }
        const uint64_t n = (uint64_t)floor(ldexp(fabs(v), OZ_SLICES * OZ_BITS - e));
        const double sg = v < 0.0 ? -1.0 : 1.0;
#pragma unroll
        for (int q = 0; q < OZ_SLICES; ++q) {
            const int sh = OZ_BITS * (OZ_SLICES - 1 - q);
            const double digit = (double)((n >> sh) & 0xFFu);
            d[q][k] = bf16_rne_bits(sg * ldexp(digit, e - OZ_BITS * (q + 1)));  // exact: 8 significant bits
        }
    }
    uint8_t *o = dst + leaf * (OZ_SLICES * n2 * EB) + c * (int64_t)bs * LB + l * LB +
                 ((piece ^ piece_swizzle((int)l, LB)) << 4);
#pragma unroll
    for (int q = 0; q < OZ_SLICES; ++q) {
        uint4 w;
        w.x = d[q][0] | ((uint32_t)d[q][1] << 16); w.y = d[q][2] | ((uint32_t)d[q][3] << 16);
        w.z = d[q][4] | ((uint32_t)d[q][5] << 16); w.w = d[q][6] | ((uint32_t)d[q][7] << 16);
        *reinterpret_cast<uint4 *>(o + q * n2 * EB) = w;
    }
    if (bad) *nonfinite = 1;
}

size_t mode_elem_bytes(qbsm_mode mode) {
    switch (mode) {
        case QBSM_F64: return 8;
        case QBSM_F32: return 4;
        default: return 2;
    }
}
int mode_parts(qbsm_mode mode) { return mode == QBSM_BF16X3 ? 2 : mode == QBSM_OZAKI_BF16 ? OZ_SLICES : 1; }

}  // namespace

int mode_bk(qbsm_mode mode, int bs) {
    // K chunk per packed line: 128-byte lines, except the two-part split mode
    // (64-byte lines) so that two LDS stages of both parts fit in 64 KB
    int bk = (mode == QBSM_BF16X3 || mode == QBSM_OZAKI_BF16 ? 64 : 128) / (int)mode_elem_bytes(mode);
    return bk < bs ? bk : bs;
}

int64_t matrix_set_blocks(Matrix &m, int64_t n, const int32_t *brow, const int32_t *bcol,
                          const double *vals, double drop_tol, hipStream_t s) {
    QB_CHECK(n >= 0, QBSM_ERR_ARG, "nblk must be >= 0");
    QB_CHECK(n == 0 || (brow && bcol && vals), QBSM_ERR_ARG, "null block arrays");
    QB_CHECK(!(drop_tol < 0.0) && !std::isnan(drop_tol), QBSM_ERR_ARG, "drop_tol must be >= 0");
    QB_CHECK(n <= (int64_t)INT32_MAX, QBSM_ERR_UNSUPPORTED, "too many blocks");
    DArr<SetStatus> st(1, s);
    QB_HIP(hipMemsetAsync(st.p, 0, sizeof(SetStatus), s));
    DArr<uint32_t> keys(n ? n : 1, s);
    DArr<uint8_t> valid(n ? n : 1, s), keep(n ? n : 1, s);
    DArr<int32_t> rank(n ? n : 1, s), rank2(n ? n : 1, s);
    const uint64_t range = (uint64_t)1 << (2 * ceil_log2(m.nbr > m.nbc ? m.nbr : m.nbc));
    if (n) {
        k_keys<<<grid_for(n, 256), 256, 0, s>>>(brow, bcol, n, m.nbr, m.nbc, keys.p, valid.p, st.p);
        QB_LAUNCH_CHECK();
    }
    // duplicates among all in-range input blocks
    bitmap_rank(keys.p, valid.p, n, range, rank2.p, &st.p->dup, &st.p->ndistinct, s);
    if (n) {
        if (drop_tol > 0.0) {
            k_norm_keep<<<(unsigned)n, 256, 0, s>>>(vals, brow, bcol, valid.p, n, m.bs, m.nrows, m.ncols,
                                                    drop_tol, keep.p);
        } else {
            k_copy_flags<<<grid_for(n, 256), 256, 0, s>>>(valid.p, n, keep.p);
        }
        QB_LAUNCH_CHECK();
    }
    DArr<int32_t> dummy(1, s);
    bitmap_rank(keys.p, keep.p, n, range, rank.p, dummy.p, &st.p->nkept, s);
    SetStatus h = read_back(st.p, s);
    QB_CHECK(!h.range_err, QBSM_ERR_PATTERN, "block coordinate outside the block grid");
    QB_CHECK(!h.dup, QBSM_ERR_PATTERN, "repeated block coordinate");
    const int64_t nk = h.nkept;
    DArr<double> pool(nk * (int64_t)m.bs * m.bs, s);
    DArr<uint32_t> okeys(nk, s);
    if (n && nk) {
        k_store_blocks<<<(unsigned)n, 256, 0, s>>>(vals, brow, bcol, keys.p, rank.p, n, m.bs, m.nrows,
                                                   m.ncols, pool.p, okeys.p);
        QB_LAUNCH_CHECK();
    }
    m.v64 = std::move(pool);
    m.v32.reset();
    m.keys = std::move(okeys);
    m.nblk = nk;
    m.storage = ST_F64;
    m.has_blocks = true;
    m.version++;
    m.pattern_id++;
    m.filled_by = 0;
    m.trees.clear();
    m.packs.clear();
    m.stream = s;
    return nk;
}

void matrix_store_f32(Matrix &m, hipStream_t s) {
    if (m.storage != ST_F64) return;
    const int64_t n = m.nblk * (int64_t)m.bs * m.bs;
    DArr<float> v(n ? n : 1, s);
    if (n) {
        const unsigned g = grid_for(n, 256) > 65536 ? 65536 : grid_for(n, 256);
        k_narrow<<<g, 256, 0, s>>>(m.v64.p, v.p, n);
        QB_LAUNCH_CHECK();
    }
    m.v32 = std::move(v);
    m.v64.reset();
    m.storage = ST_F32;
    m.version++;
    m.packs.clear();
}

Tree &matrix_tree(Matrix &m, int D, hipStream_t s) {
    auto it = m.trees.find(D);
    if (it != m.trees.end()) return *it->second;
    auto t = std::make_unique<Tree>();
    t->D = D;
    t->n.assign(D + 1, 0);
    t->child.resize(D);
    t->key.resize(D + 1);
    const int64_t cap = m.nblk;
    DArr<int64_t> counts(D + 1, s);
    // level D: the leaves themselves (storage order is Morton order)
    t->key[D].alloc(cap ? cap : 1, s);
    if (cap)
        QB_HIP(hipMemcpyAsync(t->key[D].p, m.keys.p, cap * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    int64_t nleaf = cap;
    QB_HIP(hipMemcpyAsync(counts.p + D, &nleaf, sizeof(int64_t), hipMemcpyHostToDevice, s));
    DArr<int32_t> flags(cap ? cap : 1, s), scan((cap ? cap : 1) + 1, s);
    for (int l = D - 1; l >= 0; --l) {
        t->key[l].alloc(cap ? cap : 1, s);
        t->child[l].alloc((cap ? cap : 1) * 4, s);
        fill_i32(t->child[l].p, -1, (cap ? cap : 1) * 4, s);
        if (cap) {
            k_tree_flags<<<grid_for(cap, 256), 256, 0, s>>>(t->key[l + 1].p, counts.p + l + 1, cap, flags.p);
            QB_LAUNCH_CHECK();
            exclusive_scan_i32(flags.p, scan.p, cap, counts.p + l, s);
            k_tree_link<<<grid_for(cap, 256), 256, 0, s>>>(t->key[l + 1].p, counts.p + l + 1, cap, scan.p,
                                                           t->key[l].p, t->child[l].p);
            QB_LAUNCH_CHECK();
        } else {
            int64_t zero = 0;
            QB_HIP(hipMemcpyAsync(counts.p + l, &zero, sizeof(int64_t), hipMemcpyHostToDevice, s));
        }
    }
    QB_HIP(hipMemcpyAsync(t->n.data(), counts.p, (D + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    QB_HIP(hipStreamSynchronize(s));
    Tree &ref = *t;
    m.trees[D] = std::move(t);
    return ref;
}

const int32_t *tree_desc(Matrix &m, Tree &t, int s_lvl, hipStream_t st) {
    (void)m;
    if (s_lvl == 0) return nullptr;
    if (s_lvl == 1) return t.D >= 1 ? t.child[t.D - 1].p : nullptr;
    auto it = t.desc.find(s_lvl);
    if (it != t.desc.end()) return it->second.p;
    QB_CHECK(s_lvl == 2 && t.D >= 2, QBSM_ERR_UNSUPPORTED, "unit level too far above the leaves");
    const int64_t n = t.n[t.D - 2];
    DArr<int32_t> d((n ? n : 1) * 16, st);
    if (n) {
        k_desc2<<<grid_for(n * 16, 256), 256, 0, st>>>(t.child[t.D - 2].p, t.child[t.D - 1].p, n, d.p);
        QB_LAUNCH_CHECK();
    }
    const int32_t *p = d.p;
    t.desc[s_lvl] = std::move(d);
    return p;
}

void matrix_morton_to_rowmajor_rank(Matrix &m, int32_t *rank, hipStream_t s) {
    const int64_t n = m.nblk;
    if (!n) return;
    DArr<uint32_t> rmk(n, s);
    k_rm_keys<<<grid_for(n, 256), 256, 0, s>>>(m.keys.p, n, m.nbc, rmk.p, nullptr, nullptr);
    QB_LAUNCH_CHECK();
    DArr<int32_t> dup(1, s);
    DArr<int64_t> cnt(1, s);
    bitmap_rank(rmk.p, nullptr, n, (uint64_t)m.nbr * (uint64_t)m.nbc, rank, dup.p, cnt.p, s);
}

void matrix_get_pattern(Matrix &m, int32_t *brow, int32_t *bcol, hipStream_t s) {
    const int64_t n = m.nblk;
    if (!n) return;
    DArr<uint32_t> rmk(n, s);
    DArr<int32_t> bi(n, s), bj(n, s), rank(n, s);
    k_rm_keys<<<grid_for(n, 256), 256, 0, s>>>(m.keys.p, n, m.nbc, rmk.p, bi.p, bj.p);
    QB_LAUNCH_CHECK();
    DArr<int32_t> dup(1, s);
    DArr<int64_t> cnt(1, s);
    bitmap_rank(rmk.p, nullptr, n, (uint64_t)m.nbr * (uint64_t)m.nbc, rank.p, dup.p, cnt.p, s);
    k_scatter_pattern<<<grid_for(n, 256), 256, 0, s>>>(bi.p, bj.p, rank.p, n, brow, bcol);
    QB_LAUNCH_CHECK();
}

void matrix_get_values(Matrix &m, double *vals, hipStream_t s) {
    const int64_t n = m.nblk;
    if (!n) return;
    DArr<int32_t> rank(n, s);
    matrix_morton_to_rowmajor_rank(m, rank.p, s);
    if (m.storage == ST_F64)
        k_scatter_values<double><<<(unsigned)n, 256, 0, s>>>(m.v64.p, rank.p, n, m.bs, vals);
    else
        k_scatter_values<float><<<(unsigned)n, 256, 0, s>>>(m.v32.p, rank.p, n, m.bs, vals);
    QB_LAUNCH_CHECK();
}

void matrix_extract_blocks(Matrix &m, int64_t n, const int32_t *brow, const int32_t *bcol, double *vals,
                           hipStream_t s) {
    QB_CHECK(n >= 0, QBSM_ERR_ARG, "negative count");
    if (!n) return;
    QB_CHECK(brow && bcol && vals, QBSM_ERR_ARG, "null arrays");
    QB_CHECK(n <= (int64_t)INT32_MAX, QBSM_ERR_UNSUPPORTED, "too many blocks requested");
    DArr<int32_t> bad(1, s);
    fill_i32(bad.p, 0, 1, s);
    if (m.storage == ST_F32)
        k_extract<float><<<(unsigned)n, 256, 0, s>>>(m.keys.p, m.nblk, m.v32.p, m.bs, m.nbr, m.nbc, brow, bcol, n,
                                                      vals, bad.p);
    else
        k_extract<double><<<(unsigned)n, 256, 0, s>>>(m.keys.p, m.nblk, m.v64.p, m.bs, m.nbr, m.nbc, brow, bcol, n,
                                                       vals, bad.p);
    QB_LAUNCH_CHECK();
    QB_CHECK(read_back(bad.p, s) == 0, QBSM_ERR_PATTERN, "block coordinate outside the block grid");
}

void pack_launch(Matrix &m, qbsm_mode mode, Role role, Pack &pk, hipStream_t s) {
    const int bk = mode_bk(mode, m.bs);
    const int ppl = bk * (int)mode_elem_bytes(mode) / 16;
    const int64_t work = m.nblk * (m.bs / bk) * (int64_t)m.bs * ppl;
    if (!work) {
        fill_i32(pk.nonfinite.p, 0, 1, s);
        return;
    }
    const unsigned g = grid_for(work, 256);
    uint8_t *dst = pk.buf.p;
    ProfScope prof(PROF_PACK, s);
    fill_i32(pk.nonfinite.p, 0, 1, s);
    if (mode == QBSM_OZAKI_BF16) {
        const unsigned ge = grid_for(m.nblk * m.bs, 256);
        if (m.storage == ST_F64) {
            k_oz_exp<double><<<ge, 256, 0, s>>>(m.v64.p, m.nblk, m.bs, (int)role, pk.aux.p);
            k_pack_oz<double><<<g, 256, 0, s>>>(m.v64.p, m.nblk, m.bs, bk, (int)role, pk.aux.p, dst, pk.nonfinite.p);
        } else {
            k_oz_exp<float><<<ge, 256, 0, s>>>(m.v32.p, m.nblk, m.bs, (int)role, pk.aux.p);
            k_pack_oz<float><<<g, 256, 0, s>>>(m.v32.p, m.nblk, m.bs, bk, (int)role, pk.aux.p, dst, pk.nonfinite.p);
        }
        QB_LAUNCH_CHECK();
        return;
    }
#define QB_PACK(SRC, PTR, MODE) \
    k_pack<SRC, MODE><<<g, 256, 0, s>>>(PTR, m.nblk, m.bs, bk, (int)role, dst, pk.nonfinite.p)
    if (m.storage == ST_F64) {
        switch (mode) {
            case QBSM_F64: QB_PACK(double, m.v64.p, QBSM_F64); break;
            case QBSM_F32: QB_PACK(double, m.v64.p, QBSM_F32); break;
            case QBSM_BF16: QB_PACK(double, m.v64.p, QBSM_BF16); break;
            case QBSM_BF16X3: QB_PACK(double, m.v64.p, QBSM_BF16X3); break;
            default: break;  // Ozaki: packed above
        }
    } else {
        switch (mode) {
            case QBSM_F64: QB_PACK(float, m.v32.p, QBSM_F64); break;
            case QBSM_F32: QB_PACK(float, m.v32.p, QBSM_F32); break;
            case QBSM_BF16: QB_PACK(float, m.v32.p, QBSM_BF16); break;
            case QBSM_BF16X3: QB_PACK(float, m.v32.p, QBSM_BF16X3); break;
            default: break;  // Ozaki: packed above
        }
    }
#undef QB_PACK
    QB_LAUNCH_CHECK();
}

void matrix_pack_pair(Matrix &m, qbsm_mode mode, hipStream_t s) {
    const int bs = m.bs;
    const int64_t n2 = (int64_t)bs * bs;
    const size_t bytes = (size_t)m.nblk * n2 * mode_elem_bytes(mode) * mode_parts(mode);
    Pack &pr = m.packs[std::make_pair((int)mode, (int)ROLE_ROW)];
    Pack &pc = m.packs[std::make_pair((int)mode, (int)ROLE_COL)];
    const bool stale_r = pr.buf.n != bytes || pr.version != m.version || !pr.buf.p;
    const bool stale_c = pc.buf.n != bytes || pc.version != m.version || !pc.buf.p;
    if (!stale_r || !stale_c || (bs != 32 && bs != 64) || m.nblk == 0 || mode == QBSM_OZAKI_BF16)
        return;  // per-role packs do the rest
    if (pr.buf.n != bytes) pr.buf.alloc(bytes, s);
    if (pc.buf.n != bytes) pc.buf.alloc(bytes, s);
    if (!pr.nonfinite.p) pr.nonfinite.alloc(1, s);
    if (!pc.nonfinite.p) pc.nonfinite.alloc(1, s);
    const int bk = mode_bk(mode, bs);
    ProfScope prof(PROF_PACK, s);
    fill_i32(pr.nonfinite.p, 0, 1, s);
    fill_i32(pc.nonfinite.p, 0, 1, s);
    const unsigned g = (unsigned)m.nblk;
#define QB_PACK2(SRC, PTR, MODE)                                                                          \
    if (bs == 32)                                                                                         \
        k_pack2<SRC, MODE, 32><<<g, 256, 0, s>>>(PTR, bk, pr.buf.p, pc.buf.p, pr.nonfinite.p, pc.nonfinite.p); \
    else                                                                                                  \
        k_pack2<SRC, MODE, 64><<<g, 256, 0, s>>>(PTR, bk, pr.buf.p, pc.buf.p, pr.nonfinite.p, pc.nonfinite.p)
    if (m.storage == ST_F64) {
        switch (mode) {
            case QBSM_F64: QB_PACK2(double, m.v64.p, QBSM_F64); break;
            case QBSM_F32: QB_PACK2(double, m.v64.p, QBSM_F32); break;
            case QBSM_BF16: QB_PACK2(double, m.v64.p, QBSM_BF16); break;
            case QBSM_BF16X3: QB_PACK2(double, m.v64.p, QBSM_BF16X3); break;
            default: break;  // Ozaki: one pack per role
        }
    } else {
        switch (mode) {
            case QBSM_F64: QB_PACK2(float, m.v32.p, QBSM_F64); break;
            case QBSM_F32: QB_PACK2(float, m.v32.p, QBSM_F32); break;
            case QBSM_BF16: QB_PACK2(float, m.v32.p, QBSM_BF16); break;
            case QBSM_BF16X3: QB_PACK2(float, m.v32.p, QBSM_BF16X3); break;
            default: break;  // Ozaki: one pack per role
        }
    }
#undef QB_PACK2
    QB_LAUNCH_CHECK();
    pr.version = m.version;
    pc.version = m.version;
}

PackView matrix_pack(Matrix &m, qbsm_mode mode, Role role, hipStream_t s) {
    const int bs = m.bs;
    const int bk = mode_bk(mode, bs);
    const int64_t n2 = (int64_t)bs * bs;
    PackView v;
    auto key = std::make_pair((int)mode, (int)role);
    Pack &pk = m.packs[key];
    const size_t bytes = (size_t)m.nblk * n2 * mode_elem_bytes(mode) * mode_parts(mode);
    if (pk.buf.n != bytes || pk.version != m.version || !pk.buf.p) {
        if (pk.buf.n != bytes) pk.buf.alloc(bytes, s);
        if (!pk.nonfinite.p) pk.nonfinite.alloc(1, s);
        if (mode == QBSM_OZAKI_BF16 && pk.aux.n != (size_t)(m.nblk * bs)) pk.aux.alloc(m.nblk * bs ? m.nblk * bs : 1, s);
        pack_launch(m, mode, role, pk, s);
        pk.version = m.version;
    }
    v.ptr = pk.buf.p;
    v.leaf_stride = n2 * mode_parts(mode);
    v.part_stride = n2;
    v.line_stride = bk;
    v.chunk_stride = (int32_t)((int64_t)bs * bk);
    v.nonfinite = pk.nonfinite.p;
    return v;
}

}  // namespace qbsm
