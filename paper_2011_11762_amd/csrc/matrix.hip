// Matrix handles: construction from leaf blocks, block truncation, the
// sparse quadtree (Morton-ordered node tables), readback and operand packing.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <type_traits>

#include "common.h"
#include "device_math.h"
#include "trees.h"

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

// Key of the level-`sh / 2`-up ancestor: the key shifted right by sh bits
// (sh = 32 at the root of a depth-16 tree, where a plain shift of a 32-bit
// value is undefined).
__device__ __forceinline__ uint32_t key_above(uint32_t k, int sh) { return sh < 32 ? k >> sh : 0u; }

struct SetStatus {
    int32_t range_err;
    int32_t dup;
    int64_t nkept;
    int64_t ndistinct;
};

// Keys + range check for every input block.
// (also clears ksort, the kept flags by key rank that the norm pass sets)
__global__ void k_keys(const int32_t *brow, const int32_t *bcol, int64_t n, int64_t nbr, int64_t nbc,
                       uint32_t *keys, uint8_t *valid, SetStatus *st, int32_t *ksort) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int32_t i = brow[t], j = bcol[t];
    bool ok = i >= 0 && j >= 0 && i < nbr && j < nbc;
    valid[t] = ok ? 1 : 0;
    keys[t] = ok ? morton2((uint32_t)i, (uint32_t)j) : 0u;
    if (ksort) ksort[t] = 0;
    if (!ok) st->range_err = 1;
}

// Small inputs in one workgroup: the keys, the range check, the duplicate
// check and the rank of every in-range key among the distinct keys (a
// bitmap over the key range and the scan of its words' bit counts, both in
// LDS), in place of the clearing, key, bitmap and scan launches of larger
// inputs.  Writes the whole status; nkept is the distinct count, which is
// the kept count when no block is dropped.
constexpr int kSetSmallThreads = 1024;
constexpr int kSetSmallWords = 8192;            // key range up to 2^18 (block grid side up to 512)
constexpr int64_t kSetSmallBlocks = 16384;

__global__ void __launch_bounds__(kSetSmallThreads) k_set_small(const int32_t *brow, const int32_t *bcol, int64_t n,
                                                                int64_t nbr, int64_t nbc, int nw, uint32_t *keys,
                                                                uint8_t *valid, int32_t *rank, int32_t *ksort,
                                                                SetStatus *st) {
    __shared__ uint32_t bm[kSetSmallWords];
    __shared__ int32_t ws[kSetSmallWords];
    __shared__ int32_t wsum[kSetSmallThreads / 64];
    __shared__ int32_t bad[2];
    for (int w = threadIdx.x; w < nw; w += kSetSmallThreads) bm[w] = 0u;
    if (threadIdx.x < 2) bad[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < n; t += kSetSmallThreads) {
        const int32_t i = brow[t], j = bcol[t];
        const bool ok = i >= 0 && j >= 0 && i < nbr && j < nbc;
        const uint32_t k = ok ? morton2((uint32_t)i, (uint32_t)j) : 0u;
        valid[t] = ok ? 1 : 0;
        keys[t] = k;
        if (ksort) ksort[t] = 0;
        if (ok) {
            const uint32_t bit = 1u << (k & 31u);
            if (atomicOr(&bm[k >> 5], bit) & bit) bad[1] = 1;
        } else {
            bad[0] = 1;
        }
    }
    __syncthreads();
    // exclusive scan of the words' bit counts: `per` consecutive words a thread
    const int per = (nw + kSetSmallThreads - 1) / kSetSmallThreads;
    const int w0 = (int)threadIdx.x * per;
    int32_t own = 0;
    for (int q = 0; q < per; ++q)
        if (w0 + q < nw) own += __popc(bm[w0 + q]);
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    int32_t inc = own;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t v = __shfl_up(inc, o);
        if (lane >= o) inc += v;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t acc = 0;
        for (int q = 0; q < kSetSmallThreads / 64; ++q) {
            const int32_t v = wsum[q];
            wsum[q] = acc;
            acc += v;
        }
        st->range_err = bad[0];
        st->dup = bad[1];
        st->ndistinct = acc;
        st->nkept = acc;
    }
    __syncthreads();
    int32_t run = wsum[wave] + inc - own;
    for (int q = 0; q < per; ++q) {
        if (w0 + q < nw) {
            ws[w0 + q] = run;
            run += __popc(bm[w0 + q]);
        }
    }
    __syncthreads();
    // each thread reads back the keys and flags it wrote itself
    for (int64_t t = threadIdx.x; t < n; t += kSetSmallThreads) {
        const uint32_t k = keys[t];
        rank[t] = valid[t] ? ws[k >> 5] + __popc(bm[k >> 5] & ((1u << (k & 31u)) - 1u)) : -1;
    }
}

// FP64 Frobenius norm of the logical part of each block; keep iff not (norm < tol).
// A kept block also sets ksort[rank] at its key's rank among the distinct
// input keys, so that a scan of ksort ranks the kept keys.
__global__ void __launch_bounds__(256) k_norm_keep(const double *__restrict__ vals, const int32_t *brow,
                                                   const int32_t *bcol, const uint8_t *valid,
                                                   int64_t n, int32_t bs, int64_t nrows,
                                                   int64_t ncols, double tol, uint8_t *keep,
                                                   const int32_t *rank, int32_t *ksort) {
    const int64_t t = blockIdx.x;
    if (t >= n) return;
    __shared__ double red[4];
    double s = 0.0;
    const bool ok = valid[t] != 0;
    if (ok) {
        const int64_t mr = min((int64_t)bs, nrows - (int64_t)brow[t] * bs);
        const int64_t nc = min((int64_t)bs, ncols - (int64_t)bcol[t] * bs);
        const int64_t n2 = (int64_t)bs * bs;
        const double *x = vals + t * n2;
        if (mr == bs && nc == bs && (reinterpret_cast<uintptr_t>(x) & 15) == 0) {
            // whole aligned block: 16-byte loads, several in flight per thread
            const double2 *x2 = reinterpret_cast<const double2 *>(x);
            double s0 = 0.0, s1 = 0.0;
#pragma unroll 8
            for (int64_t e = threadIdx.x; e < n2 / 2; e += 256) {
                const double2 v = x2[e];
                s0 += v.x * v.x;
                s1 += v.y * v.y;
            }
            s = s0 + s1;
        } else {
            const int r = threadIdx.x % bs;  // bs <= 128 divides 256
            for (int c = threadIdx.x / bs; c < bs; c += 256 / bs) {
                if (r < mr && c < nc) {
                    const double v = x[r + (int64_t)c * bs];
                    s += v * v;
                }
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double nrm = sqrt((red[0] + red[1]) + (red[2] + red[3]));
        const bool kp = ok && !(nrm < tol);
        keep[t] = kp ? 1 : 0;
        if (kp && rank[t] >= 0) ksort[rank[t]] = 1;
    }
}

// Scatter kept blocks into Morton order, zeroing the padding: a kept block
// goes to the rank of its key among the kept keys, kscan[rank among all keys]
// (the rank itself when kscan is null: no block dropped).
__global__ void __launch_bounds__(256) k_store_blocks(const double *__restrict__ vals, const int32_t *brow,
                                                      const int32_t *bcol, const uint32_t *keys,
                                                      const uint8_t *keep, const int32_t *rank,
                                                      const int32_t *kscan, int64_t n, int32_t bs,
                                                      int64_t nrows, int64_t ncols, double *__restrict__ pool,
                                                      uint32_t *okeys) {
    int64_t t = blockIdx.x;
    if (t >= n) return;
    if (!keep[t]) return;
    const int32_t r = kscan ? kscan[rank[t]] : rank[t];
    const int64_t mr = min((int64_t)bs, nrows - (int64_t)brow[t] * bs);
    const int64_t nc = min((int64_t)bs, ncols - (int64_t)bcol[t] * bs);
    const int64_t n2 = (int64_t)bs * bs;
    const double *x = vals + t * n2;
    double *y = pool + (int64_t)r * n2;
    if (mr == bs && nc == bs && (reinterpret_cast<uintptr_t>(x) & 15) == 0) {
        // whole aligned block: groups of 8 16-byte loads in flight before their stores
        const double2 *x2 = reinterpret_cast<const double2 *>(x);
        double2 *y2 = reinterpret_cast<double2 *>(y);
        constexpr int G = 8;
        if ((n2 / 2) % (256 * G) == 0) {
            // unconditional loads, so that all G are in flight together
            for (int64_t b0 = 0; b0 < n2 / 2; b0 += 256 * G) {
                double2 v[G];
#pragma unroll
                for (int q = 0; q < G; ++q) v[q] = x2[b0 + q * 256 + threadIdx.x];
#pragma unroll
                for (int q = 0; q < G; ++q) y2[b0 + q * 256 + threadIdx.x] = v[q];
            }
        } else {
            for (int64_t e = threadIdx.x; e < n2 / 2; e += 256) y2[e] = x2[e];
        }
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

// ---- quadtree build, all levels at once.  The leaves are stored in Morton
// order, so the nodes of level l are the runs of equal key prefixes
// key >> 2(D - l) over the leaves, numbered in order.  One pass flags the
// first leaf of every node of every level, one scan over all levels numbers
// them, and one pass writes node keys and child links.
struct LevelPtrs {
    uint32_t *key[17];
    int32_t *child[17];
};

__global__ void k_tree_flags_all(const uint32_t *lkeys, int64_t n, int D, LevelPtrs lp, int32_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = lkeys[i];
    const uint32_t kp = i ? lkeys[i - 1] : 0u;
    for (int l = 0; l < D; ++l) {
        const int sh = 2 * (D - l);
        flags[(int64_t)l * n + i] = (i == 0 || key_above(k, sh) != key_above(kp, sh)) ? 1 : 0;
        // every slot starts nil; the link pass (a later launch) fills the live ones
        reinterpret_cast<int4 *>(lp.child[l])[i] = make_int4(-1, -1, -1, -1);
    }
}

__global__ void k_tree_link_all(const uint32_t *lkeys, int64_t n, int D, LevelPtrs lp, const int32_t *flags,
                                const int32_t *scan, int64_t *counts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = lkeys[i];
    lp.key[D][i] = k;
    // node of leaf i at level l: the number of level-l starts at or before i, minus one
    int32_t below = (int32_t)i;  // the leaf itself at level D
    for (int l = D - 1; l >= 0; --l) {
        const int64_t f = (int64_t)l * n + i;
        const int32_t start = flags[f];
        const int32_t node = scan[f] - scan[(int64_t)l * n] + start - 1;
        const int sh = 2 * (D - l);
        if (start) lp.key[l][node] = key_above(k, sh);
        const bool child_start = l + 1 == D || flags[f + n];
        if (child_start) lp.child[l][(int64_t)node * 4 + ((k >> (sh - 2)) & 3u)] = below;
        below = node;
    }
    if (i == 0) {
        for (int l = 0; l < D; ++l) counts[l] = scan[(int64_t)(l + 1) * n] - scan[(int64_t)l * n];
        counts[D] = n;
    }
}

// Small trees in one workgroup, in place of the flag, scan and link
// launches of larger ones.  A thread takes `per` consecutive leaves; level by
// level from the leaves up, a node starts at a leaf whose key above that
// level differs from the previous leaf's, the workgroup scan of the starts
// numbers the nodes, and `below` (LDS) holds each leaf's node one level
// down, whose slot in its parent is linked where that node starts.
constexpr int kTreeSmallThreads = 1024;
constexpr int64_t kTreeSmallLeaves = 16384;

__global__ void __launch_bounds__(kTreeSmallThreads) k_tree_small(const uint32_t *lkeys, int n, int D, LevelPtrs lp,
                                                                  int64_t *counts) {
    __shared__ int32_t below[kTreeSmallLeaves];
    __shared__ int32_t wsum[kTreeSmallThreads / 64];
    const int per = (n + kTreeSmallThreads - 1) / kTreeSmallThreads;
    const int i0 = (int)threadIdx.x * per;
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    for (int q = 0; q < per; ++q) {
        const int i = i0 + q;
        if (i < n) {
            lp.key[D][i] = lkeys[i];
            below[i] = i;  // the leaf itself at level D
        }
    }
    // every slot starts nil (no level has more nodes than leaves)
    for (int l = 0; l < D; ++l)
        for (int e = (int)threadIdx.x; e < n; e += kTreeSmallThreads)
            reinterpret_cast<int4 *>(lp.child[l])[e] = make_int4(-1, -1, -1, -1);
    if (threadIdx.x == 0) counts[D] = n;
    __syncthreads();
    for (int l = D - 1; l >= 0; --l) {
        const int sh = 2 * (D - l);
        int own = 0;
        for (int q = 0; q < per; ++q) {
            const int i = i0 + q;
            if (i < n && (i == 0 || key_above(lkeys[i], sh) != key_above(lkeys[i - 1], sh))) ++own;
        }
        int inc = own;
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(inc, o);
            if (lane >= o) inc += v;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        if (threadIdx.x == 0) {
            int acc = 0;
            for (int w = 0; w < kTreeSmallThreads / 64; ++w) {
                const int v = wsum[w];
                wsum[w] = acc;
                acc += v;
            }
            counts[l] = acc;
        }
        __syncthreads();
        int node = wsum[wave] + inc - own - 1;  // the last node started before leaf i0
        for (int q = 0; q < per; ++q) {
            const int i = i0 + q;
            if (i >= n) break;
            const uint32_t k = lkeys[i];
            const uint32_t kp = i ? lkeys[i - 1] : 0u;
            if (i == 0 || key_above(k, sh) != key_above(kp, sh)) {
                ++node;
                lp.key[l][node] = key_above(k, sh);
            }
            // leaf i starts its node one level down: link that node
            if (l + 1 == D || i == 0 || (k >> (sh - 2)) != (kp >> (sh - 2)))
                lp.child[l][node * 4 + ((k >> (sh - 2)) & 3u)] = below[i];
            below[i] = node;  // only this thread reads or writes leaf i's entry
        }
        __syncthreads();  // wsum is reused by the next level
    }
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
    static_assert(n2 % 512 == 0, "whole leaf rounds of 16-byte loads");
    // the leaf in LDS with a column stride of bs + 1 doubles: the row-line
    // reads (consecutive rows) and the column-line reads (consecutive pieces
    // and columns) then fall on distinct banks
    constexpr int ld = BS + 1;
    __shared__ double x[ld * BS];
    const int64_t leaf = blockIdx.x;
    using Src2 = typename std::conditional<std::is_same<Src, double>::value, double2, float2>::type;
    const Src2 *g = reinterpret_cast<const Src2 *>(src + leaf * n2);
    Src2 t[n2 / 512];
#pragma unroll
    for (int q = 0; q < n2 / 512; ++q) t[q] = g[threadIdx.x + 256 * q];  // all loads in flight at once
#pragma unroll
    for (int q = 0; q < n2 / 512; ++q) {
        const int i = 2 * (threadIdx.x + 256 * q);  // i and i + 1 lie in one column (BS even)
        x[(i % BS) + (i / BS) * ld] = (double)t[q].x;
        x[(i % BS) + 1 + (i / BS) * ld] = (double)t[q].y;
    }
    __syncthreads();
    const int LB = bk * EB;
    const int ppl = LB / 16;
    const int per_role = (bs / bk) * bs * ppl;
    bool bad_row = false, bad_col = false;
    for (int r = threadIdx.x; r < 2 * per_role; r += 256) {
        const bool col = r >= per_role;
        const int rem = col ? r - per_role : r;
        // consecutive threads write consecutive 16-byte pieces of the pack
        const int piece = rem % ppl;
        const int l = (rem / ppl) % bs;
        const int c = rem / (ppl * bs);
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

// Ozaki splitting on 8-bit integers (Ozaki, Ogita, Oishi and Rump 2012):
// every element of a packed line is truncated to an integer on the exponent
// grid of that line and written as OZ_SLICES balanced digits of OZ_BITS bits;
// the line exponents are stored after the slices of each leaf (OZ_* in
// common.h).

// The exponent of a line with largest finite magnitude m: e with
// m = f 2^e, 0.5 <= f < 1 (0 for m = 0), one more where floor(m 2^(OZ_MANT - e))
// exceeds OZ_MAXM, so that every element's integer has a digit expansion.
__device__ __forceinline__ int oz_line_exponent(double m) {
    int e = 0;
    if (m > 0.0) (void)frexp(m, &e);
    if (m > 0.0 && floor(ldexp(m, OZ_MANT - e)) > (double)OZ_MAXM) ++e;
    return e;
}

// Exponent e of every packed line (a row of a leaf for the left operand);
// a line holding an Inf or NaN gets OZ_NONFINITE.
template <class Src>
__global__ void __launch_bounds__(256) k_oz_exp_row(const Src *src, int64_t nblk, int32_t bs, uint8_t *dst,
                                                    int32_t *nonfinite) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nblk * bs) return;
    const int64_t leaf = t / bs;
    const int l = (int)(t - leaf * bs);
    const Src *x = src + leaf * (int64_t)bs * bs;
    double m = 0.0;
    bool bad = false;
    for (int k = 0; k < bs; ++k) {
        const double v = fabs((double)x[l + (int64_t)k * bs]);
        bad |= !isfinite(v);
        m = v > m ? v : m;
    }
    oz_exponents(dst, leaf, bs)[l] = bad ? OZ_NONFINITE : oz_line_exponent(m);
    if (bad) *nonfinite = 1;
}

// The same for the columns of the leaves (right operand): one wave per
// column, lane r reading row r (a column is contiguous, so the reads are
// coalesced), then a maximum and a non-finite vote over the wave.
template <class Src>
__global__ void __launch_bounds__(256) k_oz_exp_col(const Src *src, int64_t nblk, int32_t bs, uint8_t *dst,
                                                    int32_t *nonfinite) {
    const int64_t line = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int r = (int)(threadIdx.x & 63);
    if (line >= nblk * bs) return;  // the same for every lane of the wave
    const int64_t leaf = line / bs;
    const int64_t c = line - leaf * bs;
    double m = 0.0;
    int bad = 0;
    for (int rr = r; rr < bs; rr += 64) {
        const double v = fabs((double)src[leaf * (int64_t)bs * bs + c * bs + rr]);
        bad |= !isfinite(v);
        m = v > m ? v : m;  // a NaN never wins the comparison; the line is marked anyway
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        m = fmax(m, __shfl_xor(m, o, 64));
        bad |= __shfl_xor(bad, o, 64);
    }
    if (r == 0) {
        oz_exponents(dst, leaf, bs)[c] = bad ? OZ_NONFINITE : oz_line_exponent(m);
        if (bad) *nonfinite = 1;
    }
}

// The digits of 16 elements of one line with exponent e, written as one
// 16-byte piece per slice at o + slice * n2 (zeros for a non-finite line).
__device__ __forceinline__ void oz_store_piece(const double (&v)[16], int e, uint8_t *o, int64_t n2) {
    uint32_t w[OZ_SLICES][4] = {};
    if (e != OZ_NONFINITE) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int64_t n = (int64_t)floor(ldexp(fabs(v[k]), OZ_MANT - e));
            int64_t big = v[k] < 0.0 ? -n : n;
#pragma unroll
            for (int q = OZ_SLICES - 1; q >= 0; --q) {
                const int64_t d = ((big + 128) & 255) - 128;  // two's complement: the floor modulus
                big = (big - d) >> 8;                         // exact: big - d is a multiple of 256
                w[q][k >> 2] |= (uint32_t)(uint8_t)(int8_t)d << (8 * (k & 3));
            }
        }
    }
#pragma unroll
    for (int q = 0; q < OZ_SLICES; ++q)
        *reinterpret_cast<uint4 *>(o + q * n2) = make_uint4(w[q][0], w[q][1], w[q][2], w[q][3]);
}

// One 16-byte piece (16 elements) of one packed line, all slices: element x
// of a line with exponent e becomes M = sign(x) floor(|x| 2^(OZ_MANT - e)),
// |M| <= OZ_MAXM, whose balanced digits are taken from the lowest up:
// d = ((M + 128) mod 256) - 128, M = (M - d) / 256; slice t = 1..OZ_SLICES
// holds the t-th highest digit, so that x = sum_t d_t 2^(e + 1 - 8t) + (less
// than 2^(e - OZ_MANT) in magnitude, toward zero).  A line with an Inf or NaN
// gets zero digits (its products are set to NaN from its exponent).
template <class Src>
__global__ void __launch_bounds__(256) k_pack_oz(const Src *src, int64_t nblk, int32_t bs, int32_t bk, int role,
                                                 uint8_t *dst) {
    constexpr int EPP = 16;
    const int LB = bk;
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
    uint8_t *base = dst + leaf * oz_leaf_bytes(bs);
    const int e = oz_exponents(dst, leaf, bs)[l];
    double v[EPP];
#pragma unroll
    for (int k = 0; k < EPP; ++k) v[k] = role == ROLE_COL ? (double)x[(k0 + k) + l * bs] : (double)x[l + (k0 + k) * bs];
    oz_store_piece(v, e, base + c * (int64_t)bs * LB + l * LB + ((piece ^ piece_swizzle((int)l, LB)) << 4), n2);
}

// Both roles of one matrix of 64 x 64 leaves in one pass (the left and the
// right operand of A * A in the Ozaki mode): one workgroup per leaf reads the
// leaf once into LDS, takes the row and the column maxima, and writes the
// exponents and the digits of the row-line and the column-line packs.
template <class Src>
__global__ void __launch_bounds__(256) k_pack_oz2(const Src *src, uint8_t *dst_row, uint8_t *dst_col,
                                                  int32_t *nf_row, int32_t *nf_col) {
    constexpr int BS = 64, LB = 64, PPL = LB / 16;
    constexpr int64_t n2 = (int64_t)BS * BS;
    constexpr int ld = BS + 1;  // column stride in LDS (rows and columns both read without conflicts)
    __shared__ double x[ld * BS];
    __shared__ int32_t ex[2][BS];  // row, column exponents
    const int64_t leaf = blockIdx.x;
    const int tid = (int)threadIdx.x;
    using Src2 = typename std::conditional<std::is_same<Src, double>::value, double2, float2>::type;
    const Src2 *g = reinterpret_cast<const Src2 *>(src + leaf * n2);
    Src2 t[n2 / 512];
#pragma unroll
    for (int q = 0; q < n2 / 512; ++q) t[q] = g[tid + 256 * q];
#pragma unroll
    for (int q = 0; q < n2 / 512; ++q) {
        const int i = 2 * (tid + 256 * q);
        x[(i % BS) + (i / BS) * ld] = (double)t[q].x;
        x[(i % BS) + 1 + (i / BS) * ld] = (double)t[q].y;
    }
    __syncthreads();
    // threads 0..63: row tid; 64..127: column tid - 64
    if (tid < 2 * BS) {
        const bool col = tid >= BS;
        const int l = col ? tid - BS : tid;
        double m = 0.0;
        bool bad = false;
        for (int k = 0; k < BS; ++k) {
            const double v = fabs(col ? x[k + l * ld] : x[l + k * ld]);
            bad |= !isfinite(v);
            m = isfinite(v) && v > m ? v : m;
        }
        const int e = bad ? OZ_NONFINITE : oz_line_exponent(m);
        ex[col ? 1 : 0][l] = e;
        oz_exponents(col ? dst_col : dst_row, leaf, BS)[l] = e;
        if (bad) *(col ? nf_col : nf_row) = 1;
    }
    __syncthreads();
    // 2 roles x 64 lines x 4 pieces of 16 elements, two per thread
    for (int r = tid; r < 2 * BS * PPL; r += 256) {
        const bool col = r >= BS * PPL;
        const int rem = col ? r - BS * PPL : r;
        const int piece = rem % PPL, l = rem / PPL;
        const int k0 = piece * 16;
        double v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = col ? x[(k0 + k) + l * ld] : x[l + (k0 + k) * ld];
        uint8_t *base = (col ? dst_col : dst_row) + leaf * oz_leaf_bytes(BS);
        oz_store_piece(v, ex[col ? 1 : 0][l], base + l * LB + ((piece ^ piece_swizzle(l, LB)) << 4), n2);
    }
}

size_t mode_elem_bytes(qbsm_mode mode) {
    switch (mode) {
        case QBSM_F64: return 8;
        case QBSM_F32: return 4;
        case QBSM_OZAKI_I8: return 1;
        default: return 2;
    }
}
int mode_parts(qbsm_mode mode) { return mode == QBSM_BF16X3 ? 2 : mode == QBSM_OZAKI_I8 ? OZ_SLICES : 1; }

}  // namespace

int mode_bk(qbsm_mode mode, int bs) {
    // K chunk per packed line: 128-byte lines, except the two-part split mode
    // (64-byte lines) so that two LDS stages of both parts fit in 64 KB
    int bk = (mode == QBSM_BF16X3 || mode == QBSM_OZAKI_I8 ? 64 : 128) / (int)mode_elem_bytes(mode);
    return bk < bs ? bk : bs;
}

int64_t matrix_set_blocks(Matrix &m, int64_t n, const int32_t *brow, const int32_t *bcol,
                          const double *vals, double drop_tol, hipStream_t s) {
    QB_CHECK(n >= 0, QBSM_ERR_ARG, "nblk must be >= 0");
    QB_CHECK(n == 0 || (brow && bcol && vals), QBSM_ERR_ARG, "null block arrays");
    QB_CHECK(!(drop_tol < 0.0) && !std::isnan(drop_tol), QBSM_ERR_ARG, "drop_tol must be >= 0");
    QB_CHECK(n <= (int64_t)INT32_MAX, QBSM_ERR_UNSUPPORTED, "too many blocks");
    matrix_settle(m, s);  // a pack made ahead may still read the old values
    // Without a drop tolerance every in-range block is kept (a repeated or
    // out-of-range one fails the call), so the kept rank is the rank among
    // the distinct keys: no keep flags, no scan of them.
    const bool drop = drop_tol > 0.0;
    DArr<SetStatus> st(1, s);
    DArr<uint32_t> keys(n ? n : 1, s);
    DArr<uint8_t> valid(n ? n : 1, s), keep;
    // rank: of each in-range block's key among the distinct input keys;
    // ksort: kept flags by that rank, whose scan kscan ranks the kept keys
    DArr<int32_t> rank(n ? n : 1, s), ksort, kscan;
    if (drop) {
        keep.alloc(n ? n : 1, s);
        ksort.alloc(n ? n : 1, s);
        kscan.alloc(n + 1, s);
    }
    const uint64_t range = (uint64_t)1 << (2 * ceil_log2(m.nbr > m.nbc ? m.nbr : m.nbc));
    const uint64_t nw = (range + 31) / 32;
    if (n <= kSetSmallBlocks && nw <= (uint64_t)kSetSmallWords) {
        k_set_small<<<1, kSetSmallThreads, 0, s>>>(brow, bcol, n, m.nbr, m.nbc, (int)nw, keys.p, valid.p, rank.p,
                                                   ksort.p, st.p);
        QB_LAUNCH_CHECK();
    } else {
        QB_HIP(hipMemsetAsync(st.p, 0, sizeof(SetStatus), s));
        if (n) {
            k_keys<<<grid_for(n, 256), 256, 0, s>>>(brow, bcol, n, m.nbr, m.nbc, keys.p, valid.p, st.p, ksort.p);
            QB_LAUNCH_CHECK();
        }
        // duplicates among all in-range input blocks
        bitmap_rank(keys.p, valid.p, n, range, rank.p, &st.p->dup, &st.p->ndistinct, s);
    }
    if (n && drop) {
        k_norm_keep<<<(unsigned)n, 256, 0, s>>>(vals, brow, bcol, valid.p, n, m.bs, m.nrows, m.ncols, drop_tol,
                                                keep.p, rank.p, ksort.p);
        QB_LAUNCH_CHECK();
        exclusive_scan_i32(ksort.p, kscan.p, n, &st.p->nkept, s);
    }
    SetStatus h = read_back(st.p, s);
    QB_CHECK(!h.range_err, QBSM_ERR_PATTERN, "block coordinate outside the block grid");
    QB_CHECK(!h.dup, QBSM_ERR_PATTERN, "repeated block coordinate");
    const int64_t nk = drop ? h.nkept : h.ndistinct;
    DArr<double> pool(nk * (int64_t)m.bs * m.bs, s);
    DArr<uint32_t> okeys(nk, s);
    if (n && nk) {
        k_store_blocks<<<(unsigned)n, 256, 0, s>>>(vals, brow, bcol, keys.p, drop ? keep.p : valid.p, rank.p,
                                                   drop ? kscan.p : nullptr, n, m.bs, m.nrows, m.ncols, pool.p,
                                                   okeys.p);
        QB_LAUNCH_CHECK();
    }
    m.v64 = std::move(pool);
    m.v32.reset();
    ++m.storage_id;
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

// FP64 Frobenius norm of each stored leaf (padding is zero, so the whole
// block is summed): one workgroup per leaf.
template <class T>
__global__ void __launch_bounds__(256) k_block_norms(const T *__restrict__ vals, int64_t nblk, int32_t bs,
                                                     double *out) {
    const int64_t t = blockIdx.x;
    if (t >= nblk) return;
    const int64_t n2 = (int64_t)bs * bs;
    const T *x = vals + t * n2;
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < n2; e += 256) {
        const double v = (double)x[e];
        s += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[t] = sqrt((red[0] + red[1]) + (red[2] + red[3]));
}

const double *matrix_norms(Matrix &m, hipStream_t s) {
    QB_CHECK(m.has_blocks, QBSM_ERR_STATE, "matrix has no blocks yet");
    if (m.norms.p && m.norms_version == m.version && m.norms.n == (size_t)(m.nblk ? m.nblk : 1))
        return m.norms.p;
    m.norms.alloc(m.nblk ? m.nblk : 1, s);
    if (m.nblk) {
        if (m.storage == ST_F64)
            k_block_norms<double><<<(unsigned)m.nblk, 256, 0, s>>>(m.v64.p, m.nblk, m.bs, m.norms.p);
        else
            k_block_norms<float><<<(unsigned)m.nblk, 256, 0, s>>>(m.v32.p, m.nblk, m.bs, m.norms.p);
        QB_LAUNCH_CHECK();
    }
    m.norms_version = m.version;
    return m.norms.p;
}

void matrix_store_f32(Matrix &m, hipStream_t s) {
    if (m.storage != ST_F64) return;
    matrix_settle(m, s);
    const int64_t n = m.nblk * (int64_t)m.bs * m.bs;
    DArr<float> v(n ? n : 1, s);
    if (n) {
        const unsigned g = grid_for(n, 256) > 65536 ? 65536 : grid_for(n, 256);
        k_narrow<<<g, 256, 0, s>>>(m.v64.p, v.p, n);
        QB_LAUNCH_CHECK();
    }
    m.v32 = std::move(v);
    m.v64.reset();
    ++m.storage_id;
    m.storage = ST_F32;
    m.version++;
    m.packs.clear();
}

namespace {
// Queues the build of m's depth-D tree.  Level sizes that only the device
// knows are written to counts[0..D] (dev_counts set) for the caller's read.
std::unique_ptr<Tree> tree_queue(Matrix &m, int D, int64_t *counts, hipStream_t s, bool &dev_counts) {
    auto t = std::make_unique<Tree>();
    t->D = D;
    t->n.assign(D + 1, 0);
    t->child.resize(D);
    t->key.resize(D + 1);
    dev_counts = false;
    const int64_t cap = m.nblk;  // nodes of any level <= leaves
    QB_CHECK(D <= 16, QBSM_ERR_UNSUPPORTED, "block grid side above 65536");
    QB_CHECK((int64_t)D * cap < (int64_t)INT32_MAX, QBSM_ERR_UNSUPPORTED, "too many leaves for the tree build");
    LevelPtrs lp{};
    for (int l = 0; l <= D; ++l) {
        t->key[l].alloc(cap ? cap : 1, s);
        lp.key[l] = t->key[l].p;
        if (l < D) {
            t->child[l].alloc((cap ? cap : 1) * 4, s);
            lp.child[l] = t->child[l].p;
        }
    }
    if (cap && D > 0 && cap <= kTreeSmallLeaves) {
        k_tree_small<<<1, kTreeSmallThreads, 0, s>>>(m.keys.p, (int)cap, D, lp, counts);
        QB_LAUNCH_CHECK();
        dev_counts = true;
    } else if (cap && D > 0) {
        DArr<int32_t> flags(D * cap, s), scan(D * cap + 1, s);
        k_tree_flags_all<<<grid_for(cap, 256), 256, 0, s>>>(m.keys.p, cap, D, lp, flags.p);
        QB_LAUNCH_CHECK();
        exclusive_scan_i32(flags.p, scan.p, D * cap, nullptr, s);
        k_tree_link_all<<<grid_for(cap, 256), 256, 0, s>>>(m.keys.p, cap, D, lp, flags.p, scan.p, counts);
        QB_LAUNCH_CHECK();
        dev_counts = true;
    } else if (cap) {  // D == 0: a single leaf is the root
        QB_HIP(hipMemcpyAsync(t->key[0].p, m.keys.p, sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        t->n[0] = cap;
    }
    return t;
}
}  // namespace

void matrix_trees(Matrix *const *ms, int nm, int D, hipStream_t s) {
    std::vector<Matrix *> todo;
    for (int i = 0; i < nm; ++i) {
        Matrix *m = ms[i];
        if (m && m->trees.find(D) == m->trees.end() && std::find(todo.begin(), todo.end(), m) == todo.end())
            todo.push_back(m);
    }
    if (todo.empty()) return;
    const size_t nt = todo.size(), stride = (size_t)D + 1;
    DArr<int64_t> counts(nt * stride, s);
    std::vector<std::unique_ptr<Tree>> built(nt);
    std::vector<char> dev(nt, 0);
    bool any = false;
    for (size_t k = 0; k < nt; ++k) {
        bool d = false;
        built[k] = tree_queue(*todo[k], D, counts.p + k * stride, s, d);
        dev[k] = d;
        any = any || d;
    }
    if (any) {  // one host read for every tree's level sizes
        std::vector<int64_t> h(nt * stride);
        QB_HIP(hipMemcpyAsync(h.data(), counts.p, h.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        QB_HIP(hipStreamSynchronize(s));
        for (size_t k = 0; k < nt; ++k)
            if (dev[k]) std::copy(h.begin() + k * stride, h.begin() + (k + 1) * stride, built[k]->n.begin());
    }
    for (size_t k = 0; k < nt; ++k) todo[k]->trees[D] = std::move(built[k]);
}

Tree &matrix_tree(Matrix &m, int D, hipStream_t s) {
    Matrix *one = &m;
    matrix_trees(&one, 1, D, s);
    return *m.trees.find(D)->second;
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
    pack_into(m, mode, role, pk.buf.p, pk.nonfinite.p, s);
}

void pack_into(Matrix &m, qbsm_mode mode, Role role, uint8_t *dst, int32_t *nonfinite, hipStream_t s) {
    const int bk = mode_bk(mode, m.bs);
    const int ppl = bk * (int)mode_elem_bytes(mode) / 16;
    const int64_t work = m.nblk * (m.bs / bk) * (int64_t)m.bs * ppl;
    if (!work) {
        fill_i32(nonfinite, 0, 1, s);
        return;
    }
    const unsigned g = grid_for(work, 256);
    ProfScope prof(PROF_PACK, s);
    fill_i32(nonfinite, 0, 1, s);
    if (mode == QBSM_OZAKI_I8) {
        QB_CHECK(m.bs == 64, QBSM_ERR_UNSUPPORTED, "the Ozaki mode needs 64 x 64 leaves");
        const unsigned ge = grid_for(m.nblk * m.bs, 256);
        const unsigned gc = grid_for(m.nblk * m.bs * 64, 256);
        if (m.storage == ST_F64) {
            if (role == ROLE_COL)
                k_oz_exp_col<double><<<gc, 256, 0, s>>>(m.v64.p, m.nblk, m.bs, dst, nonfinite);
            else
                k_oz_exp_row<double><<<ge, 256, 0, s>>>(m.v64.p, m.nblk, m.bs, dst, nonfinite);
            k_pack_oz<double><<<g, 256, 0, s>>>(m.v64.p, m.nblk, m.bs, bk, (int)role, dst);
        } else {
            if (role == ROLE_COL)
                k_oz_exp_col<float><<<gc, 256, 0, s>>>(m.v32.p, m.nblk, m.bs, dst, nonfinite);
            else
                k_oz_exp_row<float><<<ge, 256, 0, s>>>(m.v32.p, m.nblk, m.bs, dst, nonfinite);
            k_pack_oz<float><<<g, 256, 0, s>>>(m.v32.p, m.nblk, m.bs, bk, (int)role, dst);
        }
        QB_LAUNCH_CHECK();
        return;
    }
#define QB_PACK(SRC, PTR, MODE) \
    k_pack<SRC, MODE><<<g, 256, 0, s>>>(PTR, m.nblk, m.bs, bk, (int)role, dst, nonfinite)
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

// Both packs from one pass (k_pack2) on stream ks; buffers already sized.
void pack2_launch(Matrix &m, qbsm_mode mode, Pack &pr, Pack &pc, hipStream_t ks) {
    const int bs = m.bs;
    const int bk = mode_bk(mode, bs);
    ProfScope prof(PROF_PACK, ks);
    fill_i32(pr.nonfinite.p, 0, 1, ks);
    fill_i32(pc.nonfinite.p, 0, 1, ks);
    const unsigned g = (unsigned)m.nblk;
#define QB_PACK2(SRC, PTR, MODE)                                                                          \
    if (bs == 32)                                                                                         \
        k_pack2<SRC, MODE, 32><<<g, 256, 0, ks>>>(PTR, bk, pr.buf.p, pc.buf.p, pr.nonfinite.p, pc.nonfinite.p); \
    else                                                                                                  \
        k_pack2<SRC, MODE, 64><<<g, 256, 0, ks>>>(PTR, bk, pr.buf.p, pc.buf.p, pr.nonfinite.p, pc.nonfinite.p)
    if (m.storage == ST_F64) {
        switch (mode) {
            case QBSM_F64: QB_PACK2(double, m.v64.p, QBSM_F64); break;
            case QBSM_F32: QB_PACK2(double, m.v64.p, QBSM_F32); break;
            case QBSM_BF16: QB_PACK2(double, m.v64.p, QBSM_BF16); break;
            case QBSM_BF16X3: QB_PACK2(double, m.v64.p, QBSM_BF16X3); break;
            case QBSM_OZAKI_I8:
                k_pack_oz2<double><<<g, 256, 0, ks>>>(m.v64.p, pr.buf.p, pc.buf.p, pr.nonfinite.p, pc.nonfinite.p);
                break;
            default: break;
        }
    } else {
        switch (mode) {
            case QBSM_F64: QB_PACK2(float, m.v32.p, QBSM_F64); break;
            case QBSM_F32: QB_PACK2(float, m.v32.p, QBSM_F32); break;
            case QBSM_BF16: QB_PACK2(float, m.v32.p, QBSM_BF16); break;
            case QBSM_BF16X3: QB_PACK2(float, m.v32.p, QBSM_BF16X3); break;
            case QBSM_OZAKI_I8:
                k_pack_oz2<float><<<g, 256, 0, ks>>>(m.v32.p, pr.buf.p, pc.buf.p, pr.nonfinite.p, pc.nonfinite.p);
                break;
            default: break;
        }
    }
#undef QB_PACK2
    QB_LAUNCH_CHECK();
}

size_t pack_bytes(const Matrix &m, qbsm_mode mode) {
    if (mode == QBSM_OZAKI_I8) return (size_t)m.nblk * (size_t)oz_leaf_bytes(m.bs);
    return (size_t)m.nblk * m.bs * m.bs * mode_elem_bytes(mode) * mode_parts(mode);
}

PackView pack_view(const Matrix &m, qbsm_mode mode, const void *buf, const int32_t *nonfinite) {
    const int bs = m.bs;
    const int bk = mode_bk(mode, bs);
    const int64_t n2 = (int64_t)bs * bs;
    PackView v;
    v.ptr = buf;
    v.leaf_stride = mode == QBSM_OZAKI_I8 ? oz_leaf_bytes(bs) : n2 * mode_parts(mode);
    v.part_stride = n2;
    v.line_stride = bk;
    v.chunk_stride = (int32_t)((int64_t)bs * bk);
    v.nonfinite = nonfinite;
    return v;
}

namespace {
bool pack_stale(const Matrix &m, qbsm_mode mode, const Pack &pk) {
    return pk.buf.n != pack_bytes(m, mode) || pk.version != m.version || !pk.buf.p;
}
bool pair_ok(const Matrix &m, qbsm_mode mode) {
    return (m.bs == 32 || m.bs == 64) && m.nblk > 0 && (mode != QBSM_OZAKI_I8 || m.bs == 64);
}
// Sizes the buffers of a stale pack (memory taken on s).
void pack_size(const Matrix &m, qbsm_mode mode, Pack &pk, hipStream_t s) {
    const size_t bytes = pack_bytes(m, mode);
    if (pk.buf.n != bytes) pk.buf.alloc(bytes, s);
    if (!pk.nonfinite.p) pk.nonfinite.alloc(1, s);
}
}  // namespace

void matrix_pack_pair(Matrix &m, qbsm_mode mode, hipStream_t s) {
    Pack &pr = m.packs[std::make_pair((int)mode, (int)ROLE_ROW)];
    Pack &pc = m.packs[std::make_pair((int)mode, (int)ROLE_COL)];
    pr.settle(s);
    pc.settle(s);
    if (!pack_stale(m, mode, pr) || !pack_stale(m, mode, pc) || !pair_ok(m, mode))
        return;  // per-role packs do the rest
    pack_size(m, mode, pr, s);
    pack_size(m, mode, pc, s);
    pack2_launch(m, mode, pr, pc, s);
    pr.version = m.version;
    pc.version = m.version;
}

void Pack::settle(hipStream_t s) {
    if (!ready) return;
    QB_HIP(hipStreamWaitEvent(s, ready, 0));
    if (buf.p && buf.s != s) QB_HIP(hipStreamWaitEvent(buf.s, ready, 0));
    if (nonfinite.p && nonfinite.s != s) QB_HIP(hipStreamWaitEvent(nonfinite.s, ready, 0));
    (void)hipEventDestroy(ready);
    ready = nullptr;
}

Pack::~Pack() {
    if (!ready) return;
    // the buffers are returned on their own streams: those wait for the pack
    if (buf.p) (void)hipStreamWaitEvent(buf.s, ready, 0);
    if (nonfinite.p) (void)hipStreamWaitEvent(nonfinite.s, ready, 0);
    (void)hipEventDestroy(ready);
}

void matrix_settle(Matrix &m, hipStream_t s) {
    for (auto &kv : m.packs) {
        Pack &pk = kv.second;
        if (!pk.ready) continue;
        // the pack kernel reads the values: their next free waits for it too
        if (m.v64.p) QB_HIP(hipStreamWaitEvent(m.v64.s, pk.ready, 0));
        if (m.v32.p) QB_HIP(hipStreamWaitEvent(m.v32.s, pk.ready, 0));
        pk.settle(s);
    }
}

hipStream_t side_stream() {
    static std::mutex mu;
    static std::map<int, hipStream_t> streams;
    int dev = 0;
    QB_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    hipStream_t &st = streams[dev];
    if (!st) QB_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));  // default priority
    return st;
}

void matrix_prepack(Matrix &m, qbsm_mode mode, int roles, hipStream_t s) {
    QB_CHECK(m.has_blocks, QBSM_ERR_STATE, "matrix has no blocks yet");
    QB_CHECK(roles >= 1 && roles <= 3, QBSM_ERR_ARG, "roles must be 1 (row lines), 2 (column lines) or 3");
    if (m.nblk == 0) return;
    Pack *pk[2] = {nullptr, nullptr};
    bool stale[2] = {false, false};
    for (int r = 0; r < 2; ++r) {
        if (!(roles & (1 << r))) continue;
        pk[r] = &m.packs[std::make_pair((int)mode, r == 0 ? (int)ROLE_ROW : (int)ROLE_COL)];
        pk[r]->settle(s);
        stale[r] = pack_stale(m, mode, *pk[r]);
    }
    if (!stale[0] && !stale[1]) return;
    for (int r = 0; r < 2; ++r)
        if (stale[r]) pack_size(m, mode, *pk[r], s);
    // the side stream starts after everything queued on s so far (the values
    // and the buffers just taken)
    const hipStream_t side = side_stream();
    hipEvent_t start = nullptr;
    QB_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
    QB_HIP(hipEventRecord(start, s));
    QB_HIP(hipStreamWaitEvent(side, start, 0));
    (void)hipEventDestroy(start);
    if (stale[0] && stale[1] && pair_ok(m, mode)) {
        pack2_launch(m, mode, *pk[0], *pk[1], side);
    } else {
        for (int r = 0; r < 2; ++r)
            if (stale[r]) pack_launch(m, mode, r == 0 ? ROLE_ROW : ROLE_COL, *pk[r], side);
    }
    for (int r = 0; r < 2; ++r) {
        if (!stale[r]) continue;
        QB_HIP(hipEventCreateWithFlags(&pk[r]->ready, hipEventDisableTiming));
        QB_HIP(hipEventRecord(pk[r]->ready, side));
        pk[r]->version = m.version;
    }
}

PackView matrix_pack(Matrix &m, qbsm_mode mode, Role role, hipStream_t s) {
    auto key = std::make_pair((int)mode, (int)role);
    Pack &pk = m.packs[key];
    pk.settle(s);
    if (pack_stale(m, mode, pk)) {
        pack_size(m, mode, pk, s);
        pack_launch(m, mode, role, pk, s);
        pk.version = m.version;
    }
    return pack_view(m, mode, pk.buf.p, pk.nonfinite.p);
}

}  // namespace qbsm
