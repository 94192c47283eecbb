// Numeric phase: leaf-block products on MFMA with a segmented, atomic-free
// accumulation.
//
// One workgroup owns one output quadtree node of side U (the "unit", a
// 2^s x 2^s group of leaf blocks; U = 64 or 128 elements) and visits the
// unit's node pairs in contraction order.  For every pair and every leaf
// column kb inside it, the unit's A rows and B columns are staged in LDS
// chunk by chunk (coalesced 16-byte loads of the packed operands) and each
// wave multiplies its 64x64 part of the unit with 16x16 MFMA tiles; a tile
// is skipped when its leaf product is absent (nil operand).  Every output
// block is written once, by its owner, after its last product: no atomics,
// and the order of the additions is fixed (contraction index ascending).
#include "common.h"

namespace qbsm {

namespace {

typedef __attribute__((ext_vector_type(4))) float f4;
typedef __attribute__((ext_vector_type(4))) double d4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf8;

constexpr int LINEB = 144;  // bytes per LDS line: 128 data + 16 pad (bank spread)

template <int MODE>
struct MT;

template <>
struct MT<QBSM_F64> {
    using T = double;
    using Acc = d4;
    using Frag = double;
    using Out = double;
    static constexpr int KSTEP = 4, EPL = 1, PARTS = 1;
    __device__ static Frag frag(const unsigned char *p) { return *reinterpret_cast<const double *>(p); }
    __device__ static void mma(Acc &c, const Frag *a, const Frag *b) {
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
    }
    // accumulator element i of a lane holds row (lane/16) + 4*i
    __device__ static int row_of(int lane, int i) { return (lane >> 4) + 4 * i; }
};

template <>
struct MT<QBSM_F32> {
    using T = float;
    using Acc = f4;
    using Frag = float;
    using Out = float;
    static constexpr int KSTEP = 4, EPL = 1, PARTS = 1;
    __device__ static Frag frag(const unsigned char *p) { return *reinterpret_cast<const float *>(p); }
    __device__ static void mma(Acc &c, const Frag *a, const Frag *b) {
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
    }
    // accumulator element i of a lane holds row 4*(lane/16) + i
    __device__ static int row_of(int lane, int i) { return 4 * (lane >> 4) + i; }
};

template <>
struct MT<QBSM_BF16> {
    using T = uint16_t;
    using Acc = f4;
    using Frag = bf8;
    using Out = float;
    static constexpr int KSTEP = 32, EPL = 8, PARTS = 1;
    __device__ static Frag frag(const unsigned char *p) {
        return __builtin_bit_cast(bf8, *reinterpret_cast<const uint4 *>(p));
    }
    __device__ static void mma(Acc &c, const Frag *a, const Frag *b) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], c, 0, 0, 0);
    }
    __device__ static int row_of(int lane, int i) { return 4 * (lane >> 4) + i; }
};

template <>
struct MT<QBSM_BF16X3> {
    using T = uint16_t;
    using Acc = f4;
    using Frag = bf8;
    using Out = float;
    static constexpr int KSTEP = 32, EPL = 8, PARTS = 2;
    __device__ static Frag frag(const unsigned char *p) {
        return __builtin_bit_cast(bf8, *reinterpret_cast<const uint4 *>(p));
    }
    // a*b ~ hi*lo + lo*hi + hi*hi (the lo*lo term is below FP32 resolution)
    __device__ static void mma(Acc &c, const Frag *a, const Frag *b) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], c, 0, 0, 0);
    }
    __device__ static int row_of(int lane, int i) { return 4 * (lane >> 4) + i; }
};

__device__ __forceinline__ int morton_sub(int r, int c, int s) {
    int q = 0;
    for (int b = 0; b < s; ++b) q |= (((r >> b) & 1) << (2 * b + 1)) | (((c >> b) & 1) << (2 * b));
    return q;
}

__device__ __forceinline__ void demorton(uint32_t k, uint32_t &i, uint32_t &j) {
    i = 0;
    j = 0;
    for (int b = 0; b < 16; ++b) {
        i |= ((k >> (2 * b + 1)) & 1u) << b;
        j |= ((k >> (2 * b)) & 1u) << b;
    }
}

// Consecutive workgroups are dispatched round-robin over the 8 XCDs; give
// each XCD a contiguous run of units so that the units resident on one XCD
// are neighbours in Morton order and share A rows / B columns in its L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int q = n >> 3, r = n & 7;
    const int x = b & 7, i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__device__ __forceinline__ int pick4(const int *v, int i) {
    return i == 0 ? v[0] : i == 1 ? v[1] : i == 2 ? v[2] : v[3];
}

template <int MODE, int U>
__device__ void process_unit(const K5Member &m, int u, unsigned char *smem) {
    using M = MT<MODE>;
    using T = typename M::T;
    constexpr int WPS = U / 64;
    constexpr int NT = 64 * WPS * WPS;
    constexpr int PARTS = M::PARTS;
    constexpr int MAXPPL = 8;  // 16-byte pieces in a 128-byte line
    constexpr int SLOTS = (U * MAXPPL + NT - 1) / NT;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wr = w / WPS, wc = w % WPS;
    const int bs = m.bs, lpu = m.lpu, s = m.s, nsub = lpu * lpu;
    const int bk = (128 / (int)sizeof(T)) < bs ? (128 / (int)sizeof(T)) : bs;
    const int nchunk = bs / bk;
    const int ppl = bk * (int)sizeof(T) / 16;
    const int ksteps = bk / M::KSTEP;
    unsigned char *As = smem;
    unsigned char *Bs = smem + PARTS * U * LINEB;

    typename M::Acc acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = typename M::Acc{};

    const int p0 = m.ustart[u], p1 = m.ustart[u + 1];
    for (int p = p0; p < p1; ++p) {
        const uint64_t pm = m.pmask[p];
        const int a = m.pl[p], b = m.pr[p];
        for (int kb = 0; kb < lpu; ++kb) {
            const uint32_t km = (uint32_t)(pm >> (kb * nsub)) & (uint32_t)((1ull << nsub) - 1ull);
            if (!km) continue;
            int la[4], lb[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                la[i] = -1;
                lb[i] = -1;
                if (i < lpu) {
                    const int qa = m.transL ? morton_sub(kb, i, s) : morton_sub(i, kb, s);
                    la[i] = m.descL ? m.descL[(int64_t)a * nsub + qa] : a;
                    const int qb = m.transR ? morton_sub(i, kb, s) : morton_sub(kb, i, s);
                    lb[i] = m.descR ? m.descR[(int64_t)b * nsub + qb] : b;
                }
            }
            uint32_t en = 0;
#pragma unroll
            for (int tm = 0; tm < 4; ++tm)
#pragma unroll
                for (int tn = 0; tn < 4; ++tn) {
                    const int ib = (64 * wr + 16 * tm) / bs, jb = (64 * wc + 16 * tn) / bs;
                    if ((km >> (ib * lpu + jb)) & 1u) en |= 1u << (tm * 4 + tn);
                }
            for (int c = 0; c < nchunk; ++c) {
                __syncthreads();
                // stage the unit's A lines (rows) and B lines (columns) of chunk c
#pragma unroll
                for (int j = 0; j < SLOTS; ++j) {
                    const int idx = tid + j * NT;
                    if (idx < U * ppl) {
                        const int line = idx / ppl, piece = idx - (idx / ppl) * ppl;
                        const int lbk = line / bs, lr = line - lbk * bs;
                        const int leafA = pick4(la, lbk), leafB = pick4(lb, lbk);
#pragma unroll
                        for (int part = 0; part < PARTS; ++part) {
                            if (leafA >= 0) {
                                const T *src = static_cast<const T *>(m.packL) + (int64_t)leafA * m.leafStrideL +
                                               (int64_t)part * m.partStrideL + (int64_t)c * m.chunkStrideL +
                                               (int64_t)lr * m.lineStrideL + piece * (16 / (int)sizeof(T));
                                *reinterpret_cast<uint4 *>(As + (part * U + line) * LINEB + piece * 16) =
                                    *reinterpret_cast<const uint4 *>(src);
                            }
                            if (leafB >= 0) {
                                const T *src = static_cast<const T *>(m.packR) + (int64_t)leafB * m.leafStrideR +
                                               (int64_t)part * m.partStrideR + (int64_t)c * m.chunkStrideR +
                                               (int64_t)lr * m.lineStrideR + piece * (16 / (int)sizeof(T));
                                *reinterpret_cast<uint4 *>(Bs + (part * U + line) * LINEB + piece * 16) =
                                    *reinterpret_cast<const uint4 *>(src);
                            }
                        }
                    }
                }
                __syncthreads();
                if (!en) continue;
                for (int ks = 0; ks < ksteps; ++ks) {
                    const int kofs = (ks * M::KSTEP + (lane >> 4) * M::EPL) * (int)sizeof(T);
                    typename M::Frag fa[4][PARTS], fb[4][PARTS];
#pragma unroll
                    for (int t = 0; t < 4; ++t)
#pragma unroll
                        for (int part = 0; part < PARTS; ++part) {
                            fa[t][part] = M::frag(As + (part * U + 64 * wr + 16 * t + (lane & 15)) * LINEB + kofs);
                            fb[t][part] = M::frag(Bs + (part * U + 64 * wc + 16 * t + (lane & 15)) * LINEB + kofs);
                        }
#pragma unroll
                    for (int tm = 0; tm < 4; ++tm)
#pragma unroll
                        for (int tn = 0; tn < 4; ++tn)
                            if ((en >> (tm * 4 + tn)) & 1u) M::mma(acc[tm][tn], fa[tm], fb[tn]);
                }
            }
        }
    }

    // write the owned output blocks once (padding beyond the logical size = 0)
    uint32_t ui, uj;
    demorton(m.ukey[u], ui, uj);
    typename M::Out *C = static_cast<typename M::Out *>(m.C);
    const int64_t n2 = (int64_t)bs * bs;
#pragma unroll
    for (int tm = 0; tm < 4; ++tm)
#pragma unroll
        for (int tn = 0; tn < 4; ++tn) {
            const int col = 64 * wc + 16 * tn + (lane & 15);
            const int jb = col / bs, cc = col - jb * bs;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 64 * wr + 16 * tm + M::row_of(lane, i);
                const int ib = row / bs, r = row - ib * bs;
                const int32_t leaf = m.cdesc[(int64_t)u * nsub + ib * lpu + jb];
                if (leaf < 0) continue;
                const int64_t I = (int64_t)ui * lpu + ib, J = (int64_t)uj * lpu + jb;
                const bool ok = (I * bs + r) < m.out_rows && (J * bs + cc) < m.out_cols;
                C[(int64_t)leaf * n2 + r + (int64_t)cc * bs] =
                    ok ? (typename M::Out)acc[tm][tn][i] : (typename M::Out)0;
            }
        }
}

template <int MODE, int U>
__global__ void __launch_bounds__(64 * (U / 64) * (U / 64))
    k5(K5Member single, const K5Member *members, const int2 *items, int64_t nitems, int32_t *counter,
       int persistent) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[MT<MODE>::PARTS * 2 * U * LINEB];
    __shared__ int s_item;
    if (!persistent) {
        const int u = xcd_remap((int)blockIdx.x, single.nunits);
        process_unit<MODE, U>(single, u, smem);
        return;
    }
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if ((int64_t)it >= nitems) break;
        const int2 w = items[it];
        const K5Member mm = members[w.x];
        process_unit<MODE, U>(mm, w.y, smem);
    }
}

template <int MODE, int U>
void launch_one(const K5Member *members, const int2 *items, int64_t nitems, int32_t *counter, int grid,
                int persistent, const K5Member &single, hipStream_t s) {
    constexpr int NT = 64 * (U / 64) * (U / 64);
    k5<MODE, U><<<grid, NT, 0, s>>>(single, members, items, nitems, counter, persistent);
}

template <int MODE>
void launch_mode(int unit, const K5Member *members, const int2 *items, int64_t nitems, int32_t *counter,
                 int grid, int persistent, const K5Member &single, hipStream_t s) {
    switch (unit) {
        case 64: launch_one<MODE, 64>(members, items, nitems, counter, grid, persistent, single, s); break;
        case 128: launch_one<MODE, 128>(members, items, nitems, counter, grid, persistent, single, s); break;
        default: throw Error(QBSM_ERR_UNSUPPORTED, "unit side");
    }
}

}  // namespace

void k5_launch(qbsm_mode mode, int unit, const K5Member *members, int32_t, const int2 *items, int64_t nitems,
               int32_t *counter, int grid, int persistent, const K5Member &single, hipStream_t s) {
    if (grid <= 0) return;
    switch (mode) {
        case QBSM_F64: launch_mode<QBSM_F64>(unit, members, items, nitems, counter, grid, persistent, single, s); break;
        case QBSM_F32: launch_mode<QBSM_F32>(unit, members, items, nitems, counter, grid, persistent, single, s); break;
        case QBSM_BF16: launch_mode<QBSM_BF16>(unit, members, items, nitems, counter, grid, persistent, single, s); break;
        case QBSM_BF16X3: launch_mode<QBSM_BF16X3>(unit, members, items, nitems, counter, grid, persistent, single, s); break;
        default: throw Error(QBSM_ERR_ARG, "mode");
    }
    QB_LAUNCH_CHECK();
}

int k5_occupancy(qbsm_mode mode, int unit) {
    int nb = 0;
    const int NT = 64 * (unit / 64) * (unit / 64);
#define QB_OCC(MD, UU)                                                                                     \
    if (mode == MD && unit == UU)                                                                          \
        QB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(&k5<MD, UU>), NT, 0));
    QB_OCC(QBSM_F64, 64) QB_OCC(QBSM_F64, 128)
    QB_OCC(QBSM_F32, 64) QB_OCC(QBSM_F32, 128)
    QB_OCC(QBSM_BF16, 64) QB_OCC(QBSM_BF16, 128)
    QB_OCC(QBSM_BF16X3, 64) QB_OCC(QBSM_BF16X3, 128)
#undef QB_OCC
    return nb < 1 ? 1 : nb;
}

K5Member make_member(Plan &p, qbsm_mode mode, Matrix &out, hipStream_t s) {
    Tree &tL = matrix_tree(*p.L, p.D, s);
    Tree &tR = matrix_tree(*p.R, p.D, s);
    const PackView vL = matrix_pack(*p.L, mode, p.transL ? ROLE_COL : ROLE_ROW, s);
    const PackView vR = matrix_pack(*p.R, mode, p.transR ? ROLE_ROW : ROLE_COL, s);
    K5Member m{};
    m.ustart = p.ustart.p;
    m.ukey = p.ukey.p;
    m.pl = p.pl.p;
    m.pr = p.pr.p;
    m.pmask = p.pmask.p;
    m.descL = tree_desc(*p.L, tL, p.s, s);
    m.descR = tree_desc(*p.R, tR, p.s, s);
    m.cdesc = p.cdesc.p;
    m.packL = vL.ptr;
    m.packR = vR.ptr;
    m.C = out.storage == ST_F64 ? (void *)out.v64.p : (void *)out.v32.p;
    m.leafStrideL = vL.leaf_stride;
    m.partStrideL = vL.part_stride;
    m.lineStrideL = vL.line_stride;
    m.chunkStrideL = vL.chunk_stride;
    m.leafStrideR = vR.leaf_stride;
    m.partStrideR = vR.part_stride;
    m.lineStrideR = vR.line_stride;
    m.chunkStrideR = vR.chunk_stride;
    m.out_rows = p.out_rows;
    m.out_cols = p.out_cols;
    m.nunits = (int32_t)p.nunits;
    m.bs = p.bs;
    m.s = p.s;
    m.lpu = p.lpu;
    m.transL = p.transL;
    m.transR = p.transR;
    return m;
}

void plan_check_current(const Plan &p) {
    QB_CHECK(p.L->pattern_id == p.patL && p.R->pattern_id == p.patR && (!p.M || p.M->pattern_id == p.patM),
             QBSM_ERR_STATE, "an operand's pattern changed after the symbolic phase");
}

void numeric_prepare_output(Plan &p, qbsm_mode mode, Matrix &out, hipStream_t s) {
    plan_check_current(p);
    QB_CHECK(&out != p.L && &out != p.R && &out != p.M, QBSM_ERR_ARG, "output aliases an operand");
    QB_CHECK(out.nrows == p.out_rows && out.ncols == p.out_cols && out.bs == p.bs, QBSM_ERR_SHAPE,
             "output shape or leaf size differs from the product");
    const Storage want = mode == QBSM_F64 ? ST_F64 : ST_F32;
    const int64_t nout = p.nout;
    // the same plan refilling its own output: pattern and storage are already in place
    // (masked outputs keep their zero blocks: only the plan's products are rewritten)
    if (out.filled_by == p.id && out.storage == want && out.nblk == nout && out.has_blocks) {
        out.version++;
        return;
    }
    DArr<uint32_t> keys(nout ? nout : 1, s);
    const uint32_t *src = p.M ? p.M->keys.p : p.okeys.p;
    if (nout) QB_HIP(hipMemcpyAsync(keys.p, src, nout * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    out.keys = std::move(keys);
    const int64_t elems = nout * (int64_t)p.bs * p.bs;
    if (want == ST_F64) {
        out.v64.alloc(elems ? elems : 1, s);
        out.v32.reset();
        if (p.M) fill_bytes_zero(out.v64.p, elems * sizeof(double), s);
    } else {
        out.v32.alloc(elems ? elems : 1, s);
        out.v64.reset();
        if (p.M) fill_bytes_zero(out.v32.p, elems * sizeof(float), s);
    }
    out.storage = want;
    out.nblk = nout;
    out.has_blocks = true;
    out.version++;
    out.pattern_id++;
    out.filled_by = p.id;
    out.trees.clear();
    out.packs.clear();
    out.stream = s;
}

void numeric_launch(Plan &p, qbsm_mode mode, Matrix &out, hipStream_t s) {
    if (!p.nunits) return;
    K5Member m = make_member(p, mode, out, s);
    ProfScope prof(PROF_NUMERIC, s);
    k5_launch(mode, p.unit, nullptr, 1, nullptr, 0, nullptr, (int)p.nunits, 0, m, s);
}

// ------------------------------------------------------------------ batched
void batch_launch(Batch &b, hipStream_t s) {
    for (auto &j : b.packs) {
        Pack &pk = j.m->packs[std::make_pair((int)j.mode, (int)j.role)];
        pack_launch(*j.m, j.mode, j.role, pk, s);
    }
    fill_i32(b.counter.p, 0, 1, s);
    const int grid = b.num_cus * b.wg_per_cu;
    ProfScope prof(PROF_NUMERIC, s);
    if (b.nitems)
        k5_launch(b.mode, b.unit, b.members.p, b.n, b.items.p, b.nitems, b.counter.p, grid, 1, K5Member{}, s);
}

}  // namespace qbsm
