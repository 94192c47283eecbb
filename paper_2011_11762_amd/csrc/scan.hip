// Device-wide primitives: exclusive scan, fills, unique-key ranking.
#include "common.h"

namespace qbsm {

namespace {

constexpr int SCAN_BLOCK = kScanThreads;
constexpr int SCAN_ITEMS = kScanItems;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

// Exclusive scan of one value per thread over a 256-thread block (4 waves of
// 64).  Returns the exclusive prefix; *block_total receives the block sum.
template <class T>
__device__ T block_exclusive_scan(T v, T *block_total) {
    __shared__ T wsum[SCAN_BLOCK / 64];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    T base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < SCAN_BLOCK / 64; ++w) {
        if (w < wid) base += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *block_total = tot;
    return base + x - v;
}

template <class Tin, class Tacc>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_reduce(const Tin *in, int64_t n, Tacc *partial) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    Tacc s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t idx = base + (int64_t)i * SCAN_BLOCK + threadIdx.x;
        if (idx < n) s += (Tacc)in[idx];
    }
    Tacc tot;
    (void)block_exclusive_scan<Tacc>(s, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

template <class Tacc>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_partials(Tacc *partial, int64_t nb, Tacc *total) {
    Tacc carry = 0;
    for (int64_t c = 0; c < nb; c += SCAN_BLOCK) {
        int64_t idx = c + threadIdx.x;
        Tacc v = idx < nb ? partial[idx] : 0;
        Tacc tot;
        Tacc ex = block_exclusive_scan<Tacc>(v, &tot);
        if (idx < nb) partial[idx] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

template <class Tin, class Tout, class Tacc>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_apply(const Tin *in, Tout *out, int64_t n,
                                                           const Tacc *partial, const Tacc *total,
                                                           int64_t *total64) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    // thread t owns the contiguous run [base + t*ITEMS, base + (t+1)*ITEMS)
    Tacc vals[SCAN_ITEMS];
    Tacc s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t idx = base + (int64_t)threadIdx.x * SCAN_ITEMS + i;
        vals[i] = idx < n ? (Tacc)in[idx] : 0;
        s += vals[i];
    }
    Tacc tot;
    Tacc ex = block_exclusive_scan<Tacc>(s, &tot) + partial[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t idx = base + (int64_t)threadIdx.x * SCAN_ITEMS + i;
        if (idx < n) out[idx] = (Tout)ex;
        ex += vals[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        out[n] = (Tout)(*total);
        if (total64) *total64 = (int64_t)(*total);
    }
}

// The apply pass for up to SCAN_SUM_MAX tiles: each workgroup sums the tile
// totals before its own (at most SCAN_SUM_MAX values) instead of reading a
// scanned partial array, so the scan takes two launches; the last workgroup
// writes the total.
constexpr int64_t SCAN_SUM_MAX = 1024;

template <class Tin, class Tout, class Tacc>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_apply_sum(const Tin *in, Tout *out, int64_t n,
                                                               const Tacc *partial, int64_t *total64,
                                                               int sub = 1) {
    // partial holds `sub` sums per tile (of consecutive parts of it)
    Tacc pre = 0;
    for (int64_t j = threadIdx.x; j < (int64_t)blockIdx.x * sub; j += SCAN_BLOCK) pre += partial[j];
    Tacc before;
    (void)block_exclusive_scan<Tacc>(pre, &before);
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    Tacc vals[SCAN_ITEMS];
    Tacc s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t idx = base + (int64_t)threadIdx.x * SCAN_ITEMS + i;
        vals[i] = idx < n ? (Tacc)in[idx] : 0;
        s += vals[i];
    }
    Tacc tot;
    Tacc ex = block_exclusive_scan<Tacc>(s, &tot) + before;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t idx = base + (int64_t)threadIdx.x * SCAN_ITEMS + i;
        if (idx < n) out[idx] = (Tout)ex;
        ex += vals[i];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        out[n] = (Tout)(before + tot);
        if (total64) *total64 = (int64_t)(before + tot);
    }
}

// The whole scan in one workgroup, for at most SCAN_TILE values (the small
// levels of the symbolic walk): one launch and no scratch array.
template <class Tin, class Tout>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_small(const Tin *in, Tout *out, int64_t n, int64_t *total64) {
    int64_t vals[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t idx = (int64_t)threadIdx.x * SCAN_ITEMS + i;
        vals[i] = idx < n ? (int64_t)in[idx] : 0;
        s += vals[i];
    }
    int64_t tot;
    int64_t ex = block_exclusive_scan<int64_t>(s, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t idx = (int64_t)threadIdx.x * SCAN_ITEMS + i;
        if (idx < n) out[idx] = (Tout)ex;
        ex += vals[i];
    }
    if (threadIdx.x == 0) {
        out[n] = (Tout)tot;
        if (total64) *total64 = tot;
    }
}

template <class Tin, class Tout>
void scan_impl(const Tin *in, Tout *out, int64_t n, int64_t *total64, hipStream_t s) {
    if (n <= SCAN_TILE) {
        k_scan_small<Tin, Tout><<<1, SCAN_BLOCK, 0, s>>>(in, out, n, total64);
        QB_LAUNCH_CHECK();
        return;
    }
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    DArr<int64_t> partial(nb + 1, s);
    k_scan_reduce<Tin, int64_t><<<(unsigned)nb, SCAN_BLOCK, 0, s>>>(in, n, partial.p);
    QB_LAUNCH_CHECK();
    if (nb <= SCAN_SUM_MAX) {
        k_scan_apply_sum<Tin, Tout, int64_t><<<(unsigned)nb, SCAN_BLOCK, 0, s>>>(in, out, n, partial.p, total64);
        QB_LAUNCH_CHECK();
        return;
    }
    k_scan_partials<int64_t><<<1, SCAN_BLOCK, 0, s>>>(partial.p, nb, partial.p + nb);
    QB_LAUNCH_CHECK();
    k_scan_apply<Tin, Tout, int64_t><<<(unsigned)nb, SCAN_BLOCK, 0, s>>>(in, out, n, partial.p,
                                                                         partial.p + nb, total64);
    QB_LAUNCH_CHECK();
}

// Zeroes `head` bytes at p, then n16 16-byte granules (p + head is aligned
// to 16 bytes), then `tail` bytes.
__global__ void k_zero(uint8_t *p, int head, int64_t n16, int tail) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint4 *q = reinterpret_cast<uint4 *>(p + head);
    for (; i < n16; i += stride) q[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0) {
        if ((int)threadIdx.x < head) p[threadIdx.x] = 0;
        if ((int)threadIdx.x < tail) p[head + n16 * 16 + threadIdx.x] = 0;
    }
}

template <class T>
__global__ void k_fill(T *p, T v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_bitmap_set(const uint32_t *keys, const uint8_t *active, int64_t n, uint32_t *bm,
                             int32_t *dup) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (active && !active[i]) return;
    uint32_t k = keys[i];
    uint32_t bit = 1u << (k & 31u);
    uint32_t old = atomicOr(&bm[k >> 5], bit);
    if (old & bit) *dup = 1;
}

__global__ void k_popc(const uint32_t *bm, int64_t nw, int32_t *cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nw) cnt[i] = __popc(bm[i]);
}

__global__ void k_bitmap_rank(const uint32_t *keys, const uint8_t *active, int64_t n,
                              const uint32_t *bm, const int32_t *wscan, int32_t *rank) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (active && !active[i]) { rank[i] = -1; return; }
    uint32_t k = keys[i];
    uint32_t below = bm[k >> 5] & ((1u << (k & 31u)) - 1u);
    rank[i] = wscan[k >> 5] + __popc(below);
}

}  // namespace

void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int64_t *total64, hipStream_t s) {
    scan_impl<int32_t, int32_t>(in, out, n, total64, s);
}

void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
    scan_impl<int64_t, int64_t>(in, out, n, nullptr, s);
}

void exclusive_scan_i32_partials(const int32_t *in, int32_t *out, int64_t n, int64_t *partial, int sub,
                                 int64_t *total64, hipStream_t s) {
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb <= SCAN_SUM_MAX) {
        k_scan_apply_sum<int32_t, int32_t, int64_t><<<(unsigned)nb, SCAN_BLOCK, 0, s>>>(in, out, n, partial, total64,
                                                                                     sub);
        QB_LAUNCH_CHECK();
        return;
    }
    if (sub != 1) {  // a long scan: its own tile sums
        scan_impl<int32_t, int32_t>(in, out, n, total64, s);
        return;
    }
    k_scan_partials<int64_t><<<1, SCAN_BLOCK, 0, s>>>(partial, nb, partial + nb);
    QB_LAUNCH_CHECK();
    k_scan_apply<int32_t, int32_t, int64_t><<<(unsigned)nb, SCAN_BLOCK, 0, s>>>(in, out, n, partial, partial + nb,
                                                                                 total64);
    QB_LAUNCH_CHECK();
}

void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill<int32_t><<<grid_for(n, 256) > 65536 ? 65536 : grid_for(n, 256), 256, 0, s>>>(p, v, n);
    QB_LAUNCH_CHECK();
}

void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill<uint32_t><<<grid_for(n, 256) > 65536 ? 65536 : grid_for(n, 256), 256, 0, s>>>(p, v, n);
    QB_LAUNCH_CHECK();
}

void fill_bytes_zero(void *p, size_t bytes, hipStream_t s) {
    if (!bytes) return;
    // a plain fill kernel (graph-capture friendly): 16-byte granules, the
    // first workgroup also writes the unaligned head and the tail bytes
    size_t head = (16 - (reinterpret_cast<uintptr_t>(p) & 15)) & 15;
    if (head > bytes) head = bytes;
    const int64_t n16 = (int64_t)((bytes - head) / 16);
    const int tail = (int)(bytes - head - (size_t)n16 * 16);
    const int64_t g = grid_for(n16 ? n16 : 1, 256);
    k_zero<<<g > 65536 ? 65536 : g, 256, 0, s>>>(static_cast<uint8_t *>(p), (int)head, n16, tail);
    QB_LAUNCH_CHECK();
}

void bitmap_rank(const uint32_t *keys, const uint8_t *active, int64_t n, uint64_t range, int32_t *rank,
                 int32_t *dup_flag, int64_t *count, hipStream_t s) {
    int64_t nw = (int64_t)((range + 31) / 32);
    if (nw < 1) nw = 1;
    DArr<uint32_t> bm(nw, s);
    DArr<int32_t> cnt(nw, s);
    DArr<int32_t> wscan(nw + 1, s);
    fill_u32(bm.p, 0u, nw, s);
    if (n > 0) {
        k_bitmap_set<<<grid_for(n, 256), 256, 0, s>>>(keys, active, n, bm.p, dup_flag);
        QB_LAUNCH_CHECK();
    }
    k_popc<<<grid_for(nw, 256), 256, 0, s>>>(bm.p, nw, cnt.p);
    QB_LAUNCH_CHECK();
    exclusive_scan_i32(cnt.p, wscan.p, nw, count, s);
    if (n > 0) {
        k_bitmap_rank<<<grid_for(n, 256), 256, 0, s>>>(keys, active, n, bm.p, wscan.p, rank);
        QB_LAUNCH_CHECK();
    }
}

}  // namespace qbsm
