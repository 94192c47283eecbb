// Symbolic phase: level-synchronous walk of two sparse quadtrees.
//
// The paper's multiply task (Sec. 2 and 2.1) handles one quadtree level per
// task: for a non-leaf output quadrant C_ij it registers the child products
// A_ik * B_kj, k in {0,1}, and any product with a nil operand is skipped
// (the nil fallback).  Here all tasks of one level are expanded at once.  A
// "pair" is a live product (L node at (i,k), R node at (k,j)) of one level;
// pairs are kept grouped by output node (Morton order) and, inside a group,
// ordered by the contraction index k.  Expanding a group quadrant by
// quadrant and, inside a quadrant, pair by pair with the child index kb
// ascending keeps both orders at the next level, so no sort is needed: at
// the leaves every output block's products come out contiguous with K
// ascending.
#include <algorithm>

#include "common.h"
#include "trees.h"

namespace qbsm {

namespace {

struct Pairs {
    int64_t n = 0;
    DArr<int32_t> pl, pr, gs, gm, pm;
    DArr<uint32_t> ck;
    // set by the walk: a zero-initialised device block whose first int64 is
    // the exact pair count (*count) followed by kWalkExtra int64 slots, also
    // zero, for the caller's own counts
    DArr<int64_t> book;
    int64_t *count = nullptr;
    void alloc(int64_t cnt, hipStream_t s) {
        const int64_t c = cnt ? cnt : 1;
        n = cnt;
        pl.alloc(c, s); pr.alloc(c, s); gs.alloc(c, s); gm.alloc(c, s); pm.alloc(c, s); ck.alloc(c, s);
    }
};

// Node on the diagonal of C (row coordinate == column coordinate): in a
// Morton key the row bits sit one place above the column bits.
__device__ __forceinline__ bool on_diagonal(uint32_t key) {
    return ((key >> 1) & 0x55555555u) == (key & 0x55555555u);
}

__device__ __forceinline__ int slot_of(int rowbit, int colbit, int trans) {
    return trans ? (colbit * 2 + rowbit) : (rowbit * 2 + colbit);
}

// One walk level: the inputs of item t = 4 p + q (pair p, output quadrant q).
struct WalkLevel {
    const int32_t *pl, *pr, *gs, *gm, *pm;
    const uint32_t *ck;
    const int32_t *chL, *chR, *chM;
    int transL, transR;
    const double *nL, *nR;  // non-null on the step into the leaf level of a sparse approximate multiply
    double tau;
    int upper;
};

struct WalkOut {
    int32_t *pl, *pr, *gs, *gm, *pm;
    uint32_t *ck;
};

// The fields of one pair, read once per item (or once per pair in the
// top-level kernel).
struct PairRec {
    int32_t pl, pr, gs, gm, pm;
    uint32_t ck;
};

__device__ __forceinline__ PairRec pair_at(const WalkLevel &w, int64_t p) {
    return PairRec{w.pl[p], w.pr[p], w.gs[p], w.gm[p], w.chM ? w.pm[p] : -1, w.ck[p]};
}

// The live child pairs of output quadrant q of pair r: bit kb of the result
// is set when both children at contraction index kb exist (and pass the nL
// test on the step into the leaves), with their nodes in cl[kb], cr[kb];
// mchild is the mask tree's child (-1 without a mask).  A quadrant outside
// the mask, or below the diagonal of a diagonal node under `upper`, has none.
// A nL test keeps a leaf pair only when not nL[l] * nR[r] < tau.
__device__ __forceinline__ int quadrant_children(const WalkLevel &w, const PairRec &r, int q, int32_t (&cl)[2],
                                                 int32_t (&cr)[2], int32_t &mchild) {
    const int ib = q >> 1, jb = q & 1;
    mchild = -1;
    if (w.chM) {
        mchild = w.chM[(int64_t)r.pm * 4 + q];
        if (mchild < 0) return 0;
    }
    if (w.upper && ib > jb && on_diagonal(r.ck)) return 0;
    const int64_t a = (int64_t)r.pl * 4, b = (int64_t)r.pr * 4;
    int live = 0;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        cl[kb] = w.chL[a + slot_of(ib, kb, w.transL)];
        cr[kb] = w.chR[b + slot_of(kb, jb, w.transR)];
        if (cl[kb] >= 0 && cr[kb] >= 0 && (!w.nL || !(w.nL[cl[kb]] * w.nR[cr[kb]] < w.tau))) live |= 1 << kb;
    }
    return live;
}

// Slot of item (pair p, quadrant q) in the count layout 4 g + q m + (p - g)
// (g the first pair of p's group, m the group size): the exclusive scan of
// the counts gives every child its position with groups kept together,
// quadrants in order and pairs in order inside them.
__device__ __forceinline__ int64_t item_slot(const PairRec &r, int64_t p, int q) {
    return 4 * (int64_t)r.gs + (int64_t)q * r.gm + (p - r.gs);
}

// Writes the live children of quadrant q of pair r from position pos on
// (Y the scanned counts, for the children's group bounds).
template <class Out>
__device__ __forceinline__ void emit_children(const PairRec &r, int64_t p, int q, int live, const int32_t (&cl)[2],
                                              const int32_t (&cr)[2], int32_t mchild, const int32_t *Y,
                                              int64_t ocap, const Out &o) {
    const int64_t base = 4 * (int64_t)r.gs + (int64_t)q * r.gm;
    int32_t pos = Y[base + (p - r.gs)];
    const int32_t ngs = Y[base];
    const int32_t nge = Y[base + r.gm];
    const uint32_t key = r.ck * 4u + (uint32_t)q;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        if (((live >> kb) & 1) && pos < ocap) {  // pos < ocap always
            o.pl[pos] = cl[kb];
            o.pr[pos] = cr[kb];
            o.gs[pos] = ngs;
            o.gm[pos] = nge - ngs;
            o.pm[pos] = mchild;
            o.ck[pos] = key;
            ++pos;
        }
    }
}

// Writes the child pairs of item t at their scanned positions Y.
__device__ __forceinline__ void walk_fill_item(const WalkLevel &w, int64_t t, const int32_t *Y, int64_t ocap,
                                               const WalkOut &o) {
    const int64_t p = t >> 2;
    const int q = (int)(t & 3);
    const PairRec r = pair_at(w, p);
    int32_t cl[2], cr[2], mchild;
    const int live = quadrant_children(w, r, q, cl, cr, mchild);
    if (live) emit_children(r, p, q, live, cl, cr, mchild, Y, ocap, o);
}

// The pair count np of a level is read from device memory (the previous
// level's scan total); the launches cover the level's capacity, so that the
// next level's count needs no host round trip.
__global__ void k_walk_fill(const int64_t *npp, WalkLevel w, const int32_t *Y, int64_t ocap, WalkOut o) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= *npp * 4) return;
    walk_fill_item(w, t, Y, ocap, o);
}

// Sum of one value per thread over a kScanThreads-thread workgroup (the
// result in every thread).
__device__ __forceinline__ int64_t block_sum(int64_t v) {
    __shared__ int64_t red[kScanThreads / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t t = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / 64; ++k) t += red[k];
    __syncthreads();  // red may be written again by the next call
    return t;
}

// The counts of one walk level by slot of the count layout, one slot per
// thread, each workgroup's sum written to partial[block] for the scan (which
// then needs no reduction pass of its own).  Slot s lies in [4g, 4g + 4m),
// the slots of the group of pair s / 4 (g its first pair, m its size), so
// its item is quadrant (s - 4g) / m of pair g + (s - 4g) % m.  Slots from
// 4 np up to the capacity are zero.
__global__ void __launch_bounds__(kScanThreads) k_walk_count_tile(const int64_t *npp, int64_t cap4, WalkLevel w,
                                                                  int32_t *X, int64_t *partial) {
    const int64_t n4 = *npp * 4;
    const int64_t s = (int64_t)blockIdx.x * kScanThreads + threadIdx.x;
    int32_t c = 0;
    if (s < n4) {
        const int64_t pp = s >> 2;
        const int64_t g = w.gs[pp];
        // a group holds at most 2^16 pairs (one per contraction index)
        const uint32_t m = (uint32_t)w.gm[pp], off = (uint32_t)(s - 4 * g);
        const PairRec r = pair_at(w, g + off % m);
        int32_t cl[2], cr[2], mchild;
        c = __popc(quadrant_children(w, r, (int)(off / m), cl, cr, mchild));
    }
    if (s < cap4) X[s] = c;
    const int64_t tot = block_sum(c);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// The small top levels of the walk in one workgroup: for each level, counts
// into LDS, a workgroup scan, then the fill, with the level's count kept in
// counts[l + 1] as the separate launches do.  Every level's input holds at
// most kTopPairs pairs, one per thread: a thread reads its pair and its
// children's nodes once, before the level's first barrier, so the level's
// output may overwrite its input in place (one LDS copy of the pairs); only
// the last level's pairs go to device memory (out[n - 1]).  The LDS stays
// near 20 KB so that the kernel finds room on a compute unit beside four
// operand-packing workgroups (33 KB each), which the side stream runs at the
// same time.
constexpr int kTopPairs = 512, kTopThreads = kTopPairs, kTopItems = 4 * kTopPairs;
struct TopLevels {
    int n;                    // levels processed: l0 .. l0 + n - 1
    int root;                 // 1: level l0 is the root level (its one pair made here, counts[0] = 1)
    WalkLevel lv[8];          // level inputs (the first one's pair arrays given; the rest filled here)
    WalkOut out[8];           // level outputs (out[i] is the input pairs of lv[i + 1])
    int64_t ocap[8];          // output capacities
};

__global__ void __launch_bounds__(kTopThreads) k_walk_top(TopLevels tl, int64_t *counts) {
    __shared__ int32_t X[kTopItems + 1];
    __shared__ int32_t wsum[kTopThreads / 64];
    __shared__ int32_t pbuf[5][kTopPairs];  // pl, pr, gs, gm, pm
    __shared__ uint32_t kbuf[kTopPairs];    // ck
    const int tid = (int)threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const WalkOut lds{pbuf[0], pbuf[1], pbuf[2], pbuf[3], pbuf[4], kbuf};
    for (int i = 0; i < tl.n; ++i) {
        WalkLevel w = tl.lv[i];
        if (i > 0) {  // the previous level's pairs, in LDS
            w.pl = pbuf[0]; w.pr = pbuf[1]; w.gs = pbuf[2]; w.gm = pbuf[3]; w.pm = pbuf[4];
            w.ck = kbuf;
        }
        const bool last = i + 1 == tl.n;
        const WalkOut o = last ? tl.out[i] : lds;
        const int64_t ocap = last ? tl.ocap[i] : (tl.ocap[i] < kTopPairs ? tl.ocap[i] : kTopPairs);
        const bool root = i == 0 && tl.root;
        // this level's pairs (written by the previous round)
        const int np = root ? 1 : (int)counts[i];
        if (root && tid == 0) counts[0] = 1;
        const bool mine = tid < np;
        PairRec r{};
        int live[4] = {0, 0, 0, 0};
        int32_t cl[4][2], cr[4][2], mch[4];
        if (mine) {
            // the root pair: both trees' (and the mask's) root nodes, one group
            r = root ? PairRec{0, 0, 0, 1, w.chM ? 0 : -1, 0u} : pair_at(w, tid);
#pragma unroll
            for (int q = 0; q < 4; ++q) live[q] = quadrant_children(w, r, q, cl[q], cr[q], mch[q]);
        }
        // counts: the pair's four items go to their slots of [0, 4 np); the rest stay zero
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (mine) X[item_slot(r, tid, q)] = __popc(live[q]);
            else X[4 * tid + q] = 0;
        }
        __syncthreads();
        // exclusive scan of X[0 .. kTopItems), four items per thread
        int32_t v[4], s = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = X[tid * 4 + k];
            s += v[k];
        }
        int32_t x = s;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wid] = x;
        __syncthreads();
        int32_t base = 0, tot = 0;
        for (int k = 0; k < kTopThreads / 64; ++k) {
            base += k < wid ? wsum[k] : 0;
            tot += wsum[k];
        }
        int32_t e = base + x - s;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            X[tid * 4 + k] = e;
            e += v[k];
        }
        if (tid == 0) X[kTopItems] = tot;
        __syncthreads();  // every pair has been read: the output may overwrite it
        if (mine) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (live[q]) emit_children(r, tid, q, live[q], cl[q], cr[q], mch[q], X, ocap, o);
        }
        if (tid == 0) counts[i + 1] = tot;
        __syncthreads();  // the next level reads this level's output and count
        __threadfence_block();
    }
}

// The root pair and its count.
__global__ void k_walk_root(int32_t *pl, int32_t *pr, int32_t *gs, int32_t *gm, int32_t *pm, uint32_t *ck,
                            int64_t *count) {
    pl[0] = 0; pr[0] = 0; gs[0] = 0; gm[0] = 1; pm[0] = 0; ck[0] = 0u;
    *count = 1;
}

// Node keys of levels 1..target of both operand trees, for the level sizing.
struct LevelHistArgs {
    const uint32_t *key[2][17];
    int64_t n[2][17];
    int use_col[2];   // contraction coordinate: column (1) or row (0) of the stored node
    int64_t off[17];  // start of level l's histogram (2^l bins) in each operand's half
    int64_t half;     // size of one operand's half
};

// Histograms of every level's nodes by their contraction coordinate (column
// of a left operand, row of a right one; swapped when transposed): grid
// (nodes, level, operand).
__global__ void k_level_hist(LevelHistArgs a, int32_t *hist) {
    const int l = (int)blockIdx.y + 1, op = (int)blockIdx.z;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n[op][l]) return;
    const uint32_t k = a.key[op][l][t];
    uint32_t c = 0;
    for (int b = 0; b < 16; ++b) c |= ((k >> (2 * b + (a.use_col[op] ? 0 : 1))) & 1u) << b;
    atomicAdd(hist + op * a.half + a.off[l] + c, 1);
}

// Pairs of every level without a mask: sum over the contraction coordinate
// of (left nodes there) * (right nodes there); an upper bound under a mask.
// One workgroup per level.
__global__ void __launch_bounds__(256) k_level_dot(const int32_t *hist, LevelHistArgs a, unsigned long long *cap) {
    const int l = (int)blockIdx.x + 1;
    const int32_t *hL = hist + a.off[l], *hR = hist + a.half + a.off[l];
    unsigned long long v = 0;
    for (int64_t t = threadIdx.x; t < ((int64_t)1 << l); t += 256)
        v += (unsigned long long)hL[t] * (unsigned long long)hR[t];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    __shared__ unsigned long long red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) cap[l] = red[0] + red[1] + red[2] + red[3];
}

// Runs the walk from the root to level `target`; returns the pair list there.
// Every level is sized beforehand from the node histograms (one host read)
// and the levels run back to back.  The exact pair count is left on the
// device in *count (int64); the returned n is its bound (the array size).
// Without a mask the histogram bound is the exact count.  Under a mask it can
// be far above it, so a level whose bound exceeds kMaskedBoundPairs reads its
// exact count back before its arrays are allocated.
constexpr int64_t kMaskedBoundPairs = int64_t(1) << 20;
constexpr int kWalkExtra = 4;
Pairs walk(Tree &tL, int transL, Tree &tR, int transR, Tree *tM, int target, hipStream_t s,
           const double *nL = nullptr, const double *nR = nullptr, double tau = 0.0, int upper = 0) {
    Pairs cur;
    const bool empty = tL.n[0] == 0 || tR.n[0] == 0 || (tM && tM->n[0] == 0);
    if (empty || target == 0) {
        cur.alloc(empty ? 0 : 1, s);
        cur.book.alloc(1 + kWalkExtra, s);
        fill_bytes_zero(cur.book.p, (1 + kWalkExtra) * sizeof(int64_t), s);
        cur.count = cur.book.p;
        if (!empty) {
            k_walk_root<<<1, 1, 0, s>>>(cur.pl.p, cur.pr.p, cur.gs.p, cur.gm.p, cur.pm.p, cur.ck.p, cur.count);
            QB_LAUNCH_CHECK();
        }
        return cur;
    }
    // one zeroed block: counts[0..target] (pairs per level), the caller's
    // slots, the capacities of levels 1..target and the level histograms
    std::vector<int64_t> hoff(target + 1, 0);
    for (int l = 1; l <= target; ++l) hoff[l] = hoff[l - 1] + ((int64_t)1 << (l - 1));
    const int64_t hsize = hoff[target] + ((int64_t)1 << target);
    const int64_t nbook = (target + 1) + kWalkExtra + (target + 1) + (2 * hsize + 1) / 2;
    DArr<int64_t> book(nbook, s);
    fill_bytes_zero(book.p, nbook * sizeof(int64_t), s);
    int64_t *counts = book.p;
    unsigned long long *capd = reinterpret_cast<unsigned long long *>(book.p + (target + 1) + kWalkExtra);
    int32_t *hist = reinterpret_cast<int32_t *>(capd + (target + 1));
    LevelHistArgs ha{};
    ha.use_col[0] = transL ? 0 : 1;
    ha.use_col[1] = transR ? 1 : 0;
    ha.half = hsize;
    int64_t nmax = 1;
    for (int l = 1; l <= target; ++l) {
        ha.key[0][l] = tL.key[l].p;
        ha.key[1][l] = tR.key[l].p;
        ha.n[0][l] = tL.n[l];
        ha.n[1][l] = tR.n[l];
        ha.off[l] = hoff[l];
        nmax = std::max(nmax, std::max(tL.n[l], tR.n[l]));
    }
    k_level_hist<<<dim3(grid_for(nmax, 256), (unsigned)target, 2), 256, 0, s>>>(ha, hist);
    QB_LAUNCH_CHECK();
    k_level_dot<<<(unsigned)target, 256, 0, s>>>(hist, ha, capd);
    QB_LAUNCH_CHECK();
    std::vector<unsigned long long> cap(target + 1, 0);
    QB_HIP(hipMemcpyAsync(cap.data(), capd, (target + 1) * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    QB_HIP(hipStreamSynchronize(s));
    for (int l = 1; l <= target; ++l)
        QB_CHECK(cap[l] <= (unsigned long long)INT32_MAX, QBSM_ERR_UNSUPPORTED, "too many node pairs at one level");

    // counts[l]: pairs at level l (device), written by the scans (a level
    // without pairs keeps its zero)
    cur.alloc(1, s);
    auto level_in = [&](const Pairs &p, int l) {
        WalkLevel w{};
        w.pl = p.pl.p; w.pr = p.pr.p; w.gs = p.gs.p; w.gm = p.gm.p; w.pm = p.pm.p; w.ck = p.ck.p;
        w.chL = tL.child[l].p;
        w.chR = tR.child[l].p;
        w.chM = tM ? tM->child[l].p : nullptr;
        w.transL = transL;
        w.transR = transR;
        // the norm test applies on the step into the leaf level only
        const bool fl = nL && tau > 0.0 && l + 1 == tL.D;
        w.nL = fl ? nL : nullptr;
        w.nR = fl ? nR : nullptr;
        w.tau = tau;
        w.upper = upper;
        return w;
    };
    auto level_out = [](const Pairs &p) {
        WalkOut o{p.pl.p, p.pr.p, p.gs.p, p.gm.p, p.pm.p, p.ck.p};
        return o;
    };
    int64_t capc = 1;  // capacity of the current level
    int l = 0;
    // the top levels whose inputs are small run in one launch (their output
    // capacities are the exact or bounding pair counts from the histograms)
    {
        TopLevels tl{};
        std::vector<Pairs> outs;
        int64_t c = 1;
        while (l + tl.n < target && tl.n < 8 && c * 4 <= kTopItems && cap[l + tl.n + 1] > 0 &&
               (int64_t)cap[l + tl.n + 1] <= kMaskedBoundPairs) {
            outs.emplace_back();
            outs.back().alloc((int64_t)cap[l + tl.n + 1], s);
            c = (int64_t)cap[l + tl.n + 1];
            ++tl.n;
        }
        if (tl.n >= 2) {
            for (int i = 0; i < tl.n; ++i) {
                tl.lv[i] = level_in(i == 0 ? cur : outs[i - 1], l + i);
                tl.out[i] = level_out(outs[i]);
                tl.ocap[i] = outs[i].n;
            }
            tl.root = 1;  // the kernel makes the root pair itself
            k_walk_top<<<1, kTopThreads, 0, s>>>(tl, counts + l);
            QB_LAUNCH_CHECK();
            capc = outs.back().n;
            cur = std::move(outs.back());
            l += tl.n;
        } else {
            k_walk_root<<<1, 1, 0, s>>>(cur.pl.p, cur.pr.p, cur.gs.p, cur.gm.p, cur.pm.p, cur.ck.p, counts);
            QB_LAUNCH_CHECK();
        }
    }
    for (; l < target; ++l) {
        int64_t capn = (int64_t)cap[l + 1];
        Pairs nxt;
        if (capc && capn) {
            DArr<int32_t> X(capc * 4, s), Y(capc * 4 + 1, s);
            const unsigned g = grid_for(capc * 4, 256);
            const WalkLevel w = level_in(cur, l);
            const bool bounded = w.chM || w.nL || upper;
            // counts with their workgroup sums, then the scan's apply pass
            constexpr int sub = (int)(kScanTile / kScanThreads);
            const int64_t nt = (capc * 4 + kScanTile - 1) / kScanTile;
            DArr<int64_t> part(nt * sub + 1, s);
            k_walk_count_tile<<<(unsigned)(nt * sub), kScanThreads, 0, s>>>(counts + l, capc * 4, w, X.p, part.p);
            QB_LAUNCH_CHECK();
            exclusive_scan_i32_partials(X.p, Y.p, capc * 4, part.p, sub, counts + l + 1, s);
            if (bounded && capn > kMaskedBoundPairs) capn = read_back(counts + l + 1, s);
            nxt.alloc(capn, s);
            if (capn) {
                k_walk_fill<<<g, 256, 0, s>>>(counts + l, w, Y.p, capn, level_out(nxt));
                QB_LAUNCH_CHECK();
            }
        } else {
            capn = 0;  // counts[l + 1] stays zero
            nxt.alloc(0, s);
        }
        cur = std::move(nxt);
        capc = capn;
    }
    // the caller's block: the level-`target` count and the slots after it
    // (counts[target + 1 ..] are the zeroed extra slots)
    cur.n = capc;
    cur.book = std::move(book);
    cur.count = cur.book.p + target;
    return cur;
}

// The walk with its exact count read back.
Pairs walk_exact(Tree &tL, int transL, Tree &tR, int transR, Tree *tM, int target, hipStream_t s,
                 const double *nL = nullptr, const double *nR = nullptr, double tau = 0.0, int upper = 0) {
    Pairs pr = walk(tL, transL, tR, transR, tM, target, s, nL, nR, tau, upper);
    const int64_t n = read_back(pr.count, s);
    QB_CHECK(n <= pr.n, QBSM_ERR_STATE, "pair count above its bound");
    pr.n = n;
    return pr;
}

__device__ __forceinline__ void demorton_u32(uint32_t k, uint32_t &i, uint32_t &j) {
    i = 0;
    j = 0;
    for (int b = 0; b < 16; ++b) {
        i |= ((k >> (2 * b + 1)) & 1u) << b;
        j |= ((k >> (2 * b)) & 1u) << b;
    }
}

// First pair of every unit (output group) among the *npp pairs; 0 beyond.
// kScanItems pairs per thread, each workgroup's flag count to partial[block]
// for the scan.
__global__ void __launch_bounds__(kScanThreads) k_unit_flags(const int64_t *npp, int64_t cap, const int32_t *gs,
                                                             int32_t *flags, int64_t *partial) {
    const int64_t np = *npp;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t p = base + i;
        if (p < cap) {
            const int32_t f = (p < np && gs[p] == (int32_t)p) ? 1 : 0;
            flags[p] = f;
            sum += f;
        }
    }
    const int64_t tot = block_sum(sum);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// meta = {pairs, units} on the device; launches cover host-side bounds.
// Also closes ustart (ustart[units] = pairs) and clears the units' output
// leaf masks, which the pair-mask kernel then fills.
__global__ void k_unit_fill(const int64_t *meta, const int32_t *gs, const int32_t *pm, const uint32_t *ck,
                            const int32_t *uscan, int32_t *ustart, uint32_t *ukey, int32_t *umask,
                            int32_t *pu, uint32_t *ucmask) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) ustart[meta[1]] = (int32_t)meta[0];
    if (p >= meta[0]) return;
    const bool start = gs[p] == (int32_t)p;
    const int32_t u = uscan[p] + (start ? 1 : 0) - 1;
    pu[p] = u;
    if (start) {
        ustart[u] = (int32_t)p;
        ukey[u] = ck[p];
        umask[u] = pm[p];
        ucmask[u] = 0u;
    }
}

struct Dims {
    int64_t out_rows, inner, out_cols;
    int32_t bs, s, lpu, transL, transR;
};

__device__ __forceinline__ int64_t ext(int64_t idx, int64_t n, int32_t bs) {
    const int64_t e = n - idx * bs;
    return e < bs ? e : bs;
}

// Leaf-product bits of each unit-level pair, output-leaf bits of each unit,
// product and flop totals.
template <int S>
__device__ __forceinline__ constexpr int msub(int r, int c) {
    // interleave the S low bits of r and c, r's bit above c's
    int q = 0;
    for (int b = 0; b < S; ++b) q |= (((r >> b) & 1) << (2 * b + 1)) | (((c >> b) & 1) << (2 * b));
    return q;
}

// Leaf-product bitmask of every unit-level pair.  The descendant leaves of
// both nodes (and of the mask node) are loaded first; the 2^(3S) candidate
// products are then tested with compile-time indexes.
template <int S>
__global__ void k_pair_masks(const int64_t *meta, const int32_t *pl, const int32_t *pr, const int32_t *pu,
                             const uint32_t *ukey, const int32_t *umask, const int32_t *descL,
                             const int32_t *descR, const int32_t *descM, int hasM, const uint32_t *keyL,
                             Dims d, const double *nL, const double *nR, double tau, int upper,
                             uint64_t *pmask, uint32_t *ucmask, unsigned long long *part) {
    constexpr int LPU = 1 << S, NSUB = LPU * LPU;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = p < meta[0];
    const int32_t a = live ? pl[p] : 0, b = live ? pr[p] : 0;  // node 0 exists whenever np > 0
    const int32_t u = live ? pu[p] : -1;
    const int32_t us = live ? u : 0;
    uint32_t ui, uj, lr, lc;
    demorton_u32(ukey[us], ui, uj);
    demorton_u32(keyL[a], lr, lc);
    const uint32_t uk = d.transL ? lr : lc;  // contraction coordinate of the L node
    int32_t dl[NSUB], dr[NSUB], dm[NSUB];
    if (S == 0) {
        dl[0] = a;
        dr[0] = b;
        dm[0] = hasM ? umask[us] : 0;
    } else {
        const int32_t *xa = descL + (int64_t)a * NSUB;
        const int32_t *xb = descR + (int64_t)b * NSUB;
#pragma unroll
        for (int q = 0; q < NSUB; ++q) {
            dl[q] = xa[q];
            dr[q] = xb[q];
        }
        if (hasM) {
            const int32_t *xm = descM + (int64_t)umask[us] * NSUB;
#pragma unroll
            for (int q = 0; q < NSUB; ++q) dm[q] = xm[q];
        } else {
#pragma unroll
            for (int q = 0; q < NSUB; ++q) dm[q] = 0;
        }
    }
    uint64_t bits = 0;
    uint32_t cm = 0;
    unsigned long long fl = 0;
    if (live) {
#pragma unroll
        for (int kb = 0; kb < LPU; ++kb) {
            const int64_t K = (int64_t)uk * LPU + kb;
            const int64_t ek = ext(K, d.inner, d.bs);
#pragma unroll
            for (int ib = 0; ib < LPU; ++ib) {
                const int32_t la = d.transL ? dl[msub<S>(kb, ib)] : dl[msub<S>(ib, kb)];
                const int64_t ei = ext((int64_t)ui * LPU + ib, d.out_rows, d.bs);
#pragma unroll
                for (int jb = 0; jb < LPU; ++jb) {
                    const int32_t lb = d.transR ? dr[msub<S>(jb, kb)] : dr[msub<S>(kb, jb)];
                    const bool on = la >= 0 && lb >= 0 && dm[msub<S>(ib, jb)] >= 0 &&
                                    (!nL || !(nL[la] * nR[lb] < tau)) && !(upper && ui == uj && ib > jb);
                    if (on) {
                        bits |= 1ull << ((kb * LPU + ib) * LPU + jb);
                        cm |= 1u << (ib * LPU + jb);
                        fl += (unsigned long long)(2 * ei * ek * ext((int64_t)uj * LPU + jb, d.out_cols, d.bs));
                    }
                }
            }
        }
    }
    if (live) pmask[p] = bits;
    // The output mask takes one atomic per unit run inside a wave: the pairs
    // of a unit are contiguous, so a run of lanes with the same unit is
    // OR-reduced onto its first lane.  The product and flop totals go to one
    // slot per block (summed by k_unit_count) rather than to a single address.
    unsigned long long cnt = (unsigned long long)__popcll(bits);
    const int lane = (int)(threadIdx.x & 63);
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t cmo = __shfl_down(cm, o);
        const int32_t uo = __shfl_down(u, o);
        if (lane + o < 64 && uo == u) cm |= cmo;
    }
    for (int o = 32; o > 0; o >>= 1) {
        cnt += __shfl_down(cnt, o);
        fl += __shfl_down(fl, o);
    }
    const int32_t uprev = __shfl_up(u, 1);
    if (live && cm && (lane == 0 || uprev != u)) atomicOr(&ucmask[u], cm);
    __shared__ unsigned long long red[2][4];
    if (lane == 0) {
        red[0][threadIdx.x >> 6] = cnt;
        red[1][threadIdx.x >> 6] = fl;
    }
    __syncthreads();
    if (threadIdx.x < 2)
        part[2 * (int64_t)blockIdx.x + threadIdx.x] =
            red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
}


// Output leaves per unit; zero beyond the units (the scan covers the bound).
// Output leaves of every unit (0 beyond the unit count), kScanItems units
// per thread with each workgroup's sum to partial[block] for the scan; the
// first workgroup also adds up the pair-mask kernel's per-block (products,
// flops) into tot[0..1].
__global__ void __launch_bounds__(kScanThreads) k_unit_count(const int64_t *meta, int64_t cap, const uint32_t *ucmask,
                                                             int32_t *cnt, int64_t *partial,
                                                             const unsigned long long *part, int64_t nblk,
                                                             unsigned long long *tot) {
    const int64_t nu = meta[1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t u = base + i;
        if (u < cap) {
            const int32_t c = u < nu ? __popc(ucmask[u]) : 0;
            cnt[u] = c;
            sum += c;
        }
    }
    const int64_t t = block_sum(sum);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
    if (blockIdx.x == 0) {
        unsigned long long c = 0, f = 0;
        for (int64_t i = threadIdx.x; i < nblk; i += kScanThreads) {
            c += part[2 * i];
            f += part[2 * i + 1];
        }
        const int64_t cs = block_sum((int64_t)c);
        const int64_t fs = block_sum((int64_t)f);
        if (threadIdx.x == 0) {
            tot[0] = (unsigned long long)cs;
            tot[1] = (unsigned long long)fs;
        }
    }
}

// Output leaves of each unit: numbered in Morton order inside the unit
// (unmasked plans), or taken from the mask's leaves (masked plans).
__global__ void k_unit_cdesc(const int64_t *meta, const uint32_t *ucmask, const int32_t *cbase, const uint32_t *ukey,
                             const int32_t *umask, const int32_t *descM, int hasM, int s, int lpu,
                             int32_t *cdesc, uint32_t *okeys) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= meta[1]) return;
    const uint32_t cm = ucmask[u];
    const int nsub = lpu * lpu;
    int32_t next = hasM ? 0 : cbase[u];
    for (int q = 0; q < nsub; ++q) {
        // q is the Morton sub-index; recover (ib, jb)
        int ib = 0, jb = 0;
        for (int b = 0; b < s; ++b) {
            ib |= ((q >> (2 * b + 1)) & 1) << b;
            jb |= ((q >> (2 * b)) & 1) << b;
        }
        const int rm = ib * lpu + jb;
        int32_t v = -1;
        if ((cm >> rm) & 1u) {
            if (hasM) {
                v = descM ? descM[(int64_t)umask[u] * nsub + q] : umask[u];
            } else {
                v = next++;
                okeys[v] = (ukey[u] << (2 * s)) | (uint32_t)q;
            }
        }
        cdesc[u * nsub + rm] = v;
    }
}

// ---- product export (canonical row-major output, K ascending)
__global__ void k_leaf_groups(int64_t np, const int32_t *gs, const uint32_t *ck, int64_t nbc, int32_t *gflag,
                              uint32_t *rmk) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const bool start = gs[p] == (int32_t)p;
    gflag[p] = start ? 1 : 0;
    if (start) {
        uint32_t i, j;
        demorton_u32(ck[p], i, j);
        rmk[p] = (uint32_t)((uint64_t)i * nbc + j);
    }
}

__global__ void k_i32_to_u8(const int32_t *f, uint8_t *a, int64_t n) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = (uint8_t)f[t];
}

__global__ void k_group_sizes(int64_t np, const int32_t *gs, const int32_t *gm, const int32_t *grank,
                              int32_t *size_by_rank) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    if (gs[p] == (int32_t)p) size_by_rank[grank[p]] = gm[p];
}

__global__ void k_emit_products(int64_t np, const int32_t *gs, const int32_t *pl, const uint32_t *ck,
                                const int32_t *grank, const int32_t *off, const uint32_t *keyL, int transL,
                                int32_t *I, int32_t *K, int32_t *J) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int32_t g = gs[p];
    const int32_t pos = off[grank[g]] + (int32_t)(p - g);
    uint32_t i, j, r, c;
    demorton_u32(ck[p], i, j);
    demorton_u32(keyL[pl[p]], r, c);
    I[pos] = (int32_t)i;
    J[pos] = (int32_t)j;
    K[pos] = (int32_t)(transL ? r : c);
}

}  // namespace

// Plans with at most this many unit-level pairs size their unit arrays by the
// pair count and skip the host read of the unit count.
constexpr int64_t kBoundedUnitPairs = int64_t(1) << 20;

std::unique_ptr<Plan> plan_build(Matrix *L, int transL, Matrix *R, int transR, Matrix *M, int unit,
                                 double spamm_tol, int upper,
                                 hipStream_t s) {
    QB_CHECK(L && R, QBSM_ERR_ARG, "null matrix");
    QB_CHECK(L->has_blocks && R->has_blocks && (!M || M->has_blocks), QBSM_ERR_STATE,
             "matrix has no blocks yet");
    QB_CHECK(L->bs == R->bs && (!M || M->bs == L->bs), QBSM_ERR_SHAPE, "leaf sizes differ");
    const int bs = L->bs;
    const int64_t rows = transL ? L->ncols : L->nrows;
    const int64_t inner = transL ? L->nrows : L->ncols;
    const int64_t innerR = transR ? R->ncols : R->nrows;
    const int64_t cols = transR ? R->nrows : R->ncols;
    QB_CHECK(inner == innerR, QBSM_ERR_SHAPE, "inner dimensions differ");
    if (M) QB_CHECK(M->nrows == rows && M->ncols == cols, QBSM_ERR_SHAPE, "mask shape differs from the product");
    if (unit == 0) unit = 128;
    int sl = -1;
    for (int t = 0; t <= 2; ++t)
        if ((bs << t) == unit) sl = t;
    QB_CHECK(sl >= 0 && (unit == 64 || unit == 128 || unit == 256), QBSM_ERR_UNSUPPORTED,
             "unit must be bs*2^s (s<=2) and one of 64, 128, 256");
    const int64_t nbI = (rows + bs - 1) / bs, nbK = (inner + bs - 1) / bs, nbJ = (cols + bs - 1) / bs;
    int64_t nbmax = nbI > nbK ? nbI : nbK;
    nbmax = nbmax > nbJ ? nbmax : nbJ;
    int D = ceil_log2(nbmax < 1 ? 1 : nbmax);
    if (D < sl) D = sl;
    QB_CHECK(D <= 16, QBSM_ERR_UNSUPPORTED, "block grid side above 65536");

    static uint64_t next_id = 0;
    auto p = std::make_unique<Plan>();
    p->id = ++next_id;
    p->L = L; p->R = R; p->M = M;
    p->transL = transL; p->transR = transR;
    p->patL = L->pattern_id; p->patR = R->pattern_id; p->patM = M ? M->pattern_id : 0;
    p->D = D; p->s = sl; p->unit = unit; p->bs = bs; p->lpu = 1 << sl;
    p->out_rows = rows; p->out_cols = cols;
    p->stream = s;

    Matrix *const ops[3] = {L, R, M};
    matrix_trees(ops, 3, D, s);  // the operands' trees behind one host read
    Tree &tL = matrix_tree(*L, D, s);
    Tree &tR = matrix_tree(*R, D, s);
    Tree *tM = M ? &matrix_tree(*M, D, s) : nullptr;
    const int Lw = D - sl;
    const double *nL = spamm_tol > 0.0 ? matrix_norms(*L, s) : nullptr;
    const double *nR = spamm_tol > 0.0 ? matrix_norms(*R, s) : nullptr;
    p->spamm_tol = spamm_tol;
    p->upper = upper;
    Pairs pr = walk(tL, transL, tR, transR, tM, Lw, s, nL, nR, spamm_tol, upper);
    const int64_t cap = pr.n;
    // the counts come back together, in the walk's zeroed block:
    // meta = {pairs, units, leaf products, flops, output leaves}
    int64_t *meta = pr.count;
    static_assert(kWalkExtra >= 4, "units and the three totals follow the pair count");
    struct Tot { unsigned long long nprod, flops; int64_t nout; };
    Tot *totals = reinterpret_cast<Tot *>(meta + 2);
    const int nsub = p->lpu * p->lpu;

    // units = output groups at the unit level
    DArr<int32_t> flags(cap ? cap : 1, s), uscan((cap ? cap : 1) + 1, s), pu(cap ? cap : 1, s);
    if (cap) {
        const int64_t nt = (cap + kScanTile - 1) / kScanTile;
        DArr<int64_t> tsum(nt + 1, s);
        k_unit_flags<<<(unsigned)nt, kScanThreads, 0, s>>>(meta, cap, pr.gs.p, flags.p, tsum.p);
        QB_LAUNCH_CHECK();
        exclusive_scan_i32_partials(flags.p, uscan.p, cap, tsum.p, 1, meta + 1, s);
    }
    // Small plans size their unit arrays by the pair bound (units <= pairs)
    // and read the exact counts back with the totals, in one host read;
    // large ones read the counts first and allocate exactly.
    int64_t np = cap, nu = cap;
    const bool bound = cap <= kBoundedUnitPairs;
    if (!bound) {
        int64_t hm[2];
        QB_HIP(hipMemcpyAsync(hm, meta, sizeof(hm), hipMemcpyDeviceToHost, s));
        QB_HIP(hipStreamSynchronize(s));
        np = hm[0];
        nu = hm[1];
        QB_CHECK(np <= cap && nu <= np, QBSM_ERR_STATE, "pair count above its bound");
    }
    p->ustart.alloc(nu + 1, s);
    p->ukey.alloc(nu ? nu : 1, s);
    p->umask.alloc(nu ? nu : 1, s);
    p->pl = std::move(pr.pl);
    p->pr = std::move(pr.pr);
    p->pmask.alloc(np ? np : 1, s);
    p->cdesc.alloc((nu ? nu : 1) * nsub, s);
    DArr<uint32_t> ucmask(nu ? nu : 1, s);
    DArr<unsigned long long> part;  // per-block (products, flops) of the pair-mask kernel
    int64_t nblk = 0;
    if (np) {
        k_unit_fill<<<grid_for(np, 256), 256, 0, s>>>(meta, pr.gs.p, pr.pm.p, pr.ck.p, uscan.p, p->ustart.p,
                                                     p->ukey.p, p->umask.p, pu.p, ucmask.p);
        QB_LAUNCH_CHECK();
        Dims d{rows, inner, cols, bs, sl, p->lpu, transL, transR};
        const int32_t *dL = tree_desc(*L, tL, sl, s);
        const int32_t *dR = tree_desc(*R, tR, sl, s);
        const int32_t *dM = M ? tree_desc(*M, *tM, sl, s) : nullptr;
#define QB_PAIR_MASKS(S_)                                                                                   \
    k_pair_masks<S_><<<grid_for(np, 256), 256, 0, s>>>(meta, p->pl.p, p->pr.p, pu.p, p->ukey.p, p->umask.p,    \
                                                       dL, dR, dM, M ? 1 : 0, tL.key[Lw].p, d, nL, nR,     \
                                                       spamm_tol, upper, p->pmask.p, ucmask.p, part.p)
        nblk = grid_for(np, 256);
        part.alloc(2 * nblk, s);
        if (sl == 0) QB_PAIR_MASKS(0);
        else if (sl == 1) QB_PAIR_MASKS(1);
        else QB_PAIR_MASKS(2);
#undef QB_PAIR_MASKS
        QB_LAUNCH_CHECK();
    } else {
        int32_t zero = 0;
        QB_HIP(hipMemcpyAsync(p->ustart.p, &zero, sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    // output leaves; their keys go to a bounded array (nu * nsub) first and
    // are trimmed once the count is back with the totals
    DArr<uint32_t> okeys_b;
    if (nu) {
        DArr<int32_t> cnt(nu, s), cbase(nu + 1, s);
        const int64_t nt = (nu + kScanTile - 1) / kScanTile;
        DArr<int64_t> tsum(nt + 1, s);
        // (with the product and flop totals of the pair-mask kernel's blocks)
        k_unit_count<<<(unsigned)nt, kScanThreads, 0, s>>>(meta, nu, ucmask.p, cnt.p, tsum.p, part.p, nblk,
                                                            &totals->nprod);
        QB_LAUNCH_CHECK();
        exclusive_scan_i32_partials(cnt.p, cbase.p, nu, tsum.p, 1, &totals->nout, s);
        if (!M) okeys_b.alloc(nu * nsub, s);
        const int32_t *dM = M ? tree_desc(*M, *tM, sl, s) : nullptr;
        k_unit_cdesc<<<grid_for(nu, 256), 256, 0, s>>>(meta, ucmask.p, cbase.p, p->ukey.p, p->umask.p, dM,
                                                      M ? 1 : 0, sl, p->lpu, p->cdesc.p,
                                                      M ? nullptr : okeys_b.p);
        QB_LAUNCH_CHECK();
    }
    int64_t hm[5];
    QB_HIP(hipMemcpyAsync(hm, meta, sizeof(hm), hipMemcpyDeviceToHost, s));
    QB_HIP(hipStreamSynchronize(s));
    QB_CHECK(hm[0] <= np && hm[1] <= hm[0], QBSM_ERR_STATE, "pair count above its bound");
    np = hm[0];
    nu = hm[1];
    p->npairs = np;
    p->nunits = nu;
    const int64_t nout = nu ? hm[4] : 0;
    QB_CHECK(nout <= nu * nsub, QBSM_ERR_STATE, "output leaf count above its bound");
    // the output keys stay in their bounded array (nout of them are valid)
    if (!M) {
        if (okeys_b.p)
            p->okeys = std::move(okeys_b);
        else
            p->okeys.alloc(1, s);
    }
    p->nprod = (int64_t)hm[2];
    p->flops = (int64_t)hm[3];
    p->nout = M ? M->nblk : nout;
    return p;
}

void plan_get_products(Plan &p, int32_t *I, int32_t *K, int32_t *J, hipStream_t s) {
    if (!p.nprod) return;
    Tree &tL = matrix_tree(*p.L, p.D, s);
    Tree &tR = matrix_tree(*p.R, p.D, s);
    Tree *tM = p.M ? &matrix_tree(*p.M, p.D, s) : nullptr;
    const double *nL = p.spamm_tol > 0.0 ? matrix_norms(*p.L, s) : nullptr;
    const double *nR = p.spamm_tol > 0.0 ? matrix_norms(*p.R, s) : nullptr;
    Pairs lv = walk_exact(tL, p.transL, tR, p.transR, tM, p.D, s, nL, nR, p.spamm_tol, p.upper);
    const int64_t np = lv.n;
    QB_CHECK(np == p.nprod, QBSM_ERR_STATE, "leaf walk disagrees with the plan's product count");
    const int64_t nbc = (p.out_cols + p.bs - 1) / p.bs;
    const int64_t nbr = (p.out_rows + p.bs - 1) / p.bs;
    DArr<int32_t> gflag(np, s), grank(np, s), sizes(np, s), off(np + 1, s), dup(1, s);
    DArr<uint32_t> rmk(np, s);
    DArr<int64_t> cnt(1, s);
    k_leaf_groups<<<grid_for(np, 256), 256, 0, s>>>(np, lv.gs.p, lv.ck.p, nbc, gflag.p, rmk.p);
    QB_LAUNCH_CHECK();
    // rank the groups (output blocks) in row-major order; gflag marks starts
    DArr<uint8_t> act(np, s);
    k_i32_to_u8<<<grid_for(np, 256), 256, 0, s>>>(gflag.p, act.p, np);
    QB_LAUNCH_CHECK();
    bitmap_rank(rmk.p, act.p, np, (uint64_t)nbr * (uint64_t)nbc, grank.p, dup.p, cnt.p, s);
    fill_i32(sizes.p, 0, np, s);
    k_group_sizes<<<grid_for(np, 256), 256, 0, s>>>(np, lv.gs.p, lv.gm.p, grank.p, sizes.p);
    QB_LAUNCH_CHECK();
    exclusive_scan_i32(sizes.p, off.p, np, cnt.p, s);
    k_emit_products<<<grid_for(np, 256), 256, 0, s>>>(np, lv.gs.p, lv.pl.p, lv.ck.p, grank.p, off.p,
                                                     tL.key[p.D].p, p.transL, I, K, J);
    QB_LAUNCH_CHECK();
}

}  // namespace qbsm
