// Numeric phase: leaf-block products on MFMA with a segmented, atomic-free
// accumulation.
//
// One workgroup owns one output quadtree node of side U (the "unit", a
// 2^s x 2^s group of leaf blocks; U = 64 or 128 elements) and visits the
// unit's node pairs in contraction order.  A "step" is one K chunk of one
// leaf column kb of one pair: the unit's A rows and B columns of that chunk
// are copied from HBM straight into LDS (global_load_lds, 1 KB per wave
// instruction, two LDS stages so the copy of step i+1 overlaps the MFMAs of
// step i; one barrier per step), and each wave multiplies its 64x64 part of
// the unit with 16x16 MFMA tiles.  A tile is skipped when its leaf product
// is absent (nil operand).  Every output block is written once, by its
// owner, after its last product: no atomics, and the order of the additions
// is fixed (contraction index ascending across steps).
//
// Operand layout (written by the pack kernel): per leaf [part][chunk][line]
// with lines of LB = 64 or 128 bytes whose 16-byte pieces are XOR-swizzled
// by the line index, so the LDS copy is a contiguous 1 KB per instruction
// and the MFMA fragment reads of 16 consecutive lines hit distinct banks.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "common.h"
#include "device_math.h"

namespace qbsm {

namespace {

typedef __attribute__((ext_vector_type(4))) float f4;
typedef __attribute__((ext_vector_type(4))) double d4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf8;

#define QB_GAS __attribute__((address_space(1)))
#define QB_LAS __attribute__((address_space(3)))

__device__ __forceinline__ uint4 lds_piece(const uint8_t *arr, int line, int LB, int piece) {
    return *reinterpret_cast<const uint4 *>(arr + line * LB + ((piece ^ piece_swizzle(line, LB)) << 4));
}

// Per-mode traits.  A "read group" is the K range one set of fragment reads
// covers: lane group g = lane/16 reads logical pieces g*SUBS .. g*SUBS+SUBS-1
// of the group; MFMA step j of the group uses element j of those pieces for
// both operands (the same K permutation on A and B leaves the sum unchanged).
template <int MODE>
struct MT;

template <>
struct MT<QBSM_F64> {
    using T = double;
    using Acc = d4;
    using Out = double;
    static constexpr int BK = 16, PARTS = 1, LBMAX = 128, KPG = 16, PPG = 8, SUBS = 2;
    static constexpr bool LEAF_SUMS = false;
    struct Part {};
    struct Frag { uint4 q[2]; };
    __device__ static void mma(Acc &c, const Frag *a, const Frag *b) {
        const double2 a0 = __builtin_bit_cast(double2, a[0].q[0]), a1 = __builtin_bit_cast(double2, a[0].q[1]);
        const double2 b0 = __builtin_bit_cast(double2, b[0].q[0]), b1 = __builtin_bit_cast(double2, b[0].q[1]);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.x, b0.x, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.y, b0.y, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.x, b1.x, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.y, b1.y, c, 0, 0, 0);
    }
    // accumulator element i of a lane holds row (lane/16) + 4*i
    __device__ static int row_of(int lane, int i) { return (lane >> 4) + 4 * i; }
};

template <>
struct MT<QBSM_F32> {
    using T = float;
    using Acc = f4;
    using Out = float;
    static constexpr int BK = 32, PARTS = 1, LBMAX = 128, KPG = 16, PPG = 4, SUBS = 1;
    static constexpr bool LEAF_SUMS = false;
    struct Part {};
    struct Frag { uint4 q[1]; };
    __device__ static void mma(Acc &c, const Frag *a, const Frag *b) {
        const f4 x = __builtin_bit_cast(f4, a[0].q[0]), y = __builtin_bit_cast(f4, b[0].q[0]);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[0], y[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[1], y[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[2], y[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[3], y[3], c, 0, 0, 0);
    }
    // accumulator element i of a lane holds row 4*(lane/16) + i
    __device__ static int row_of(int lane, int i) { return 4 * (lane >> 4) + i; }
};

template <>
struct MT<QBSM_BF16> {
    using T = uint16_t;
    using Acc = f4;
    using Out = float;
    static constexpr int BK = 64, PARTS = 1, LBMAX = 128, KPG = 32, PPG = 4, SUBS = 1;
    static constexpr bool LEAF_SUMS = false;
    struct Part {};
    struct Frag { uint4 q[1]; };
    __device__ static void mma(Acc &c, const Frag *a, const Frag *b) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a[0].q[0]),
                                                    __builtin_bit_cast(bf8, b[0].q[0]), c, 0, 0, 0);
    }
    __device__ static int row_of(int lane, int i) { return 4 * (lane >> 4) + i; }
};

template <>
struct MT<QBSM_BF16X3> {
    using T = uint16_t;
    using Acc = f4;
    using Out = float;
    static constexpr int BK = 32, PARTS = 2, LBMAX = 64, KPG = 32, PPG = 4, SUBS = 1;
    static constexpr bool LEAF_SUMS = false;
    struct Part {};
    struct Frag { uint4 q[1]; };
    // a*b ~ hi*lo + lo*hi + hi*hi (the lo*lo term is below FP32 resolution);
    // a[0]/b[0] are the hi parts, a[1]/b[1] the lo parts
    __device__ static void mma(Acc &c, const Frag *a, const Frag *b) {
        const bf8 ah = __builtin_bit_cast(bf8, a[0].q[0]), al = __builtin_bit_cast(bf8, a[1].q[0]);
        const bf8 bh = __builtin_bit_cast(bf8, b[0].q[0]), bl = __builtin_bit_cast(bf8, b[1].q[0]);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
    }
    __device__ static int row_of(int lane, int i) { return 4 * (lane >> 4) + i; }
};

// Source of the copies of nil leaves on the branch-free path: its LDS lines
// then hold zeros, so the products of a nil leaf add exact zeros.
__device__ __attribute__((aligned(1024))) uint8_t g_zero_page[1024] = {};

// Ozaki slices: OZ_SLICES = 6 balanced 8-bit digits per element (each in
// [-128, 127]), digit t on the grid 2^(e + 1 - 8t) of its line's exponent e.
// The products of digit pairs (t, u) of one pair group g = t + u (2..7; the
// pairs with t + u > 7 are dropped) lie on one grid 2^(e_row + e_col + 2 - 8g)
// per leaf, and over one 64-wide leaf each group's integer MFMA sum S_g is
// exact (|S_g| <= 6 * 64 * 128^2 < 2^23).  The six groups share three int32
// accumulators: P1 = S_2 2^8 + S_3, P2 = S_4 2^8 + S_5, P3 = S_6 2^8 + S_7
// (|P3| <= 5 2^28 + 6 2^20 < 2^31: the accumulator is shifted by 8 bits
// between its two groups).  At the end of every leaf the three are converted
// to FP64, scaled by 2^(e_row + e_col) and added to the FP64 accumulator, so
// the whole FP64 exponent range is covered.
typedef __attribute__((ext_vector_type(4))) int i4;

template <>
struct MT<QBSM_OZAKI_I8> {
    using T = int8_t;
    using Acc = d4;
    using Out = double;
    static constexpr int BK = 64, PARTS = OZ_SLICES, LBMAX = 64, KPG = 64, PPG = 4, SUBS = 1;
    static constexpr bool LEAF_SUMS = true;
    static constexpr int NSUMS = 3;
    static_assert(OZ_SLICES == 6 && OZ_BITS == 8, "the accumulators below combine six 8-bit pair groups");
    struct Part { i4 s[NSUMS]; };
    struct Frag { uint4 q[1]; };
    __device__ static i4 mm(const Frag *a, const Frag *b, int ta, int tb, i4 c) {
        return __builtin_amdgcn_mfma_i32_16x16x64_i8(__builtin_bit_cast(i4, a[ta - 1].q[0]),
                                                     __builtin_bit_cast(i4, b[tb - 1].q[0]), c, 0, 0, 0);
    }
    // the pairs (t, u) of group g into accumulator c
    __device__ static i4 group(const Frag *a, const Frag *b, int g, i4 c) {
#pragma unroll
        for (int ta = 1; ta < g; ++ta)
            if (ta <= OZ_SLICES && g - ta <= OZ_SLICES) c = mm(a, b, ta, g - ta, c);
        return c;
    }
    __device__ static void mma_part(Part &p, const Frag *a, const Frag *b) {
#pragma unroll
        for (int k = 0; k < NSUMS; ++k) {
            p.s[k] = group(a, b, 2 * k + 2, p.s[k]);
            p.s[k] = p.s[k] * 256;  // S_g 2^8, below 2^31
            p.s[k] = group(a, b, 2 * k + 3, p.s[k]);
        }
    }
    // The same for NT tiles of one column tile at once, their MFMAs
    // interleaved tile by tile: consecutive MFMAs on one accumulator are NT
    // instructions apart, so the integer MFMA pipe never waits on a result,
    // and a tile's shift between its two groups overlaps the others' MFMAs.
    template <int NT>
    __device__ static void mma_parts(Part (&p)[NT], const Frag (&a)[NT][OZ_SLICES], const Frag *b) {
#pragma unroll
        for (int k = 0; k < NSUMS; ++k) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int g = 2 * k + 2 + h;
                if (h == 1) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) p[t].s[k] = p[t].s[k] * 256;  // S_g 2^8, below 2^31
                }
#pragma unroll
                for (int ta = 1; ta < g; ++ta)
                    if (ta <= OZ_SLICES && g - ta <= OZ_SLICES) {
#pragma unroll
                        for (int t = 0; t < NT; ++t) p[t].s[k] = mm(a[t], b, ta, g - ta, p[t].s[k]);
                    }
            }
        }
    }
    // c += 2^(er + ec - 22) (P1 + P2 2^-16 + P3 2^-32), element i of a lane
    // being row 4*(lane/16) + i (exponent er[i]) and column lane % 16
    // (exponent ec).  NF: the operands hold non-finite lines, whose products
    // become NaN.
    template <bool NF>
    __device__ static void flush(Acc &c, Part &p, const i4 &er, int ec) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double x = fma((double)p.s[2][i], 0x1p-32, fma((double)p.s[1][i], 0x1p-16, (double)p.s[0][i]));
            const double v = c[i] + ldexp(x, er[i] + ec - 22);
            if constexpr (NF)
                c[i] = (er[i] == OZ_NONFINITE || ec == OZ_NONFINITE) ? __builtin_nan("") : v;
            else
                c[i] = v;
        }
#pragma unroll
        for (int k = 0; k < NSUMS; ++k) p.s[k] = i4{0, 0, 0, 0};
    }
    // the integer MFMA layout: element i of a lane holds row 4*(lane/16) + i
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

// Consecutive workgroups are dispatched round-robin over the 8 XCDs.  The
// units are dealt to the XCDs in chunks of XCD_CHUNK Morton-consecutive
// units, chunk c to XCD c mod 8: the units resident on one XCD are
// neighbours in Morton order (they share A rows / B columns in its L2), and
// a region of costly units (a dense corner of C) is spread over every XCD
// instead of landing on one.  The last partial round keeps the identity.
constexpr int XCD_CHUNK = 64;
__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int full = n / (8 * XCD_CHUNK) * (8 * XCD_CHUNK);
    if (b >= full) return b;
    const int x = b & 7, i = b >> 3;
    return ((i / XCD_CHUNK) * 8 + x) * XCD_CHUNK + i % XCD_CHUNK;
}

// Values that are the same in every lane (read from one LDS address) are
// moved to scalar registers so that the step bookkeeping, the address
// arithmetic and the tile-skip branches run on the scalar unit.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int pick4(const int *v, int i) {
    return i == 0 ? v[0] : i == 1 ? v[1] : i == 2 ? v[2] : v[3];
}

// LDS copy of the metadata of a batch of pairs: product bits and, for every
// leaf column kb, the packed-operand address of each leaf row (A side) and
// leaf column (B side), so that the step loop never waits on a dependent
// global read and needs no stride arithmetic.  A nil leaf has address 0.
// Two workgroups of the smaller units share a compute unit's LDS.
template <int U>
constexpr int k5_meta_bytes = U >= 256 ? 20480 : 15360;

struct Meta {
    uint64_t *pm;  // [cap]
    uint64_t *ad;  // [cap][kb][op][slot]: leaf address, op 0 = left operand
};

__device__ __forceinline__ Meta meta_view(uint8_t *base, int cap) {
    Meta mt;
    mt.pm = reinterpret_cast<uint64_t *>(base);
    mt.ad = mt.pm + cap;
    return mt;
}

// Position in a batch of pairs: pair i, leaf column kb, K chunk c; pm is
// pair i's product bits and km those of leaf column kb.  Every field is
// wave-uniform and kept in scalar registers.
struct Step {
    int i, kb, c;
    uint32_t pm_lo, pm_hi, km;
};

__device__ __forceinline__ Step uni_step(int i, int kb, int c, uint64_t pm, uint32_t km) {
    Step st;
    st.i = uni(i);
    st.kb = uni(kb);
    st.c = uni(c);
    st.pm_lo = (uint32_t)uni((int)(uint32_t)pm);
    st.pm_hi = (uint32_t)uni((int)(uint32_t)(pm >> 32));
    st.km = (uint32_t)uni((int)km);
    return st;
}

__device__ __forceinline__ uint64_t step_pm(const Step &st) { return ((uint64_t)st.pm_hi << 32) | st.pm_lo; }

// Leaf columns of a pair with at least one product (bit kb).
template <int LPU, int NSUB>
__device__ __forceinline__ uint32_t kb_mask(uint64_t pm) {
    uint32_t r = 0;
#pragma unroll
    for (int kb = 0; kb < LPU; ++kb)
        r |= (uint32_t)(((pm >> (kb * NSUB)) & ((1ull << NSUB) - 1ull)) != 0ull) << kb;
    return r;
}

template <int NSUB>
__device__ __forceinline__ uint32_t col_bits(uint64_t pm, int kb) {
    return (uint32_t)(pm >> (kb * NSUB)) & (uint32_t)((1ull << NSUB) - 1ull);
}

// First leaf column with a product at or after pair i (pairs without any
// product are skipped); i == nb at the end of the batch.
template <int LPU, int NSUB>
__device__ __forceinline__ Step first_step(const Meta &mt, int nb, int i) {
    uint64_t pm = 0;
    uint32_t kbm = 0;
    for (; i < nb; i = uni(i + 1)) {
        pm = uni64(mt.pm[i]);
        kbm = kb_mask<LPU, NSUB>(pm);
        if (kbm) break;
    }
    const int kb = kbm ? __builtin_ctz(kbm) : 0;
    return uni_step(i, kb, 0, pm, col_bits<NSUB>(pm, kb));
}

// The step after st (i == nb at the end of the batch).  Only a new pair
// reads its product bits from LDS.
template <int LPU, int NSUB, int NCHUNK>
__device__ __forceinline__ Step next_step(const Meta &mt, int nb, const Step &st) {
    if (st.c + 1 < NCHUNK) return uni_step(st.i, st.kb, st.c + 1, step_pm(st), st.km);
    const uint64_t pm = step_pm(st);
    const uint32_t rest = kb_mask<LPU, NSUB>(pm) & ~((2u << st.kb) - 1u);
    if (rest) {
        const int kb = __builtin_ctz(rest);
        return uni_step(st.i, kb, 0, pm, col_bits<NSUB>(pm, kb));
    }
    return first_step<LPU, NSUB>(mt, nb, st.i + 1);
}

template <int MODE, int U, int BS>
struct Geo {
    using M = MT<MODE>;
    using T = typename M::T;
    static constexpr int LPU = U / BS;                   // leaves per unit side
    static constexpr int S = LPU == 1 ? 0 : LPU == 2 ? 1 : 2;
    static constexpr int NSUB = LPU * LPU;
    static constexpr int BK = M::BK < BS ? M::BK : BS;   // K per chunk (one packed line)
    static constexpr int LB = BK * (int)sizeof(T);       // bytes per line
    static constexpr int NCHUNK = BS / BK;
    static constexpr int NGROUPS = BK / M::KPG;
    static constexpr int LPI = 1024 / LB;                // lines per 1 KB load instruction
    static constexpr int IPA = U / LPI;                  // load instructions per array
    // side of the part one wave computes (Ozaki: four waves of 32 x 32 at
    // unit 64, of one 64 x 64 leaf each at unit 128)
    static constexpr int WT = MODE == QBSM_OZAKI_I8 ? (U >= 128 ? 64 : 32) : U >= 256 ? 128 : 64;
    static constexpr int WPS = U / WT;                   // waves per unit side
    static constexpr int NW = WPS * WPS;
    static constexpr int TPW = WT / 16;                  // 16x16 tiles per wave side
    static constexpr int NLW = WT > BS ? WT / BS : 1;    // leaves per wave side
    static constexpr int TPL = (WT < BS ? WT : BS) / 16; // tiles per leaf side inside a wave
    static constexpr int NARR = 2 * M::PARTS;
    static constexpr int PER_WAVE = NARR * IPA / NW;
    static constexpr int ARRB = U * M::LBMAX;
    static constexpr int STAGEB = NARR * ARRB;
    static constexpr int CAP = k5_meta_bytes<U> / (8 + 16 * NSUB);
    static_assert(NARR * IPA % NW == 0, "load instructions must split evenly over the waves");
    static_assert(LB <= M::LBMAX && LPI <= BS, "line geometry");
    static_assert(NSUB * LPU <= 64, "leaf-product bits of a pair must fit 64 bits");
};

// s_waitcnt immediate for vmcnt(N), other counters left alone (gfx9 layout:
// vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
template <int N>
constexpr int k5_vmcnt = 0x0F70 | (N & 15) | ((N >> 4) << 14);

template <int MODE, int U>
constexpr int k5_wt = MODE == QBSM_OZAKI_I8 ? (U >= 128 ? 64 : 32) : U >= 256 ? 128 : 64;

template <int MODE, int U>
constexpr int k5_nt = 64 * (U / k5_wt<MODE, U>) * (U / k5_wt<MODE, U>);

template <int MODE, int U>
constexpr int k5_stage_bytes = 2 * MT<MODE>::PARTS * U * MT<MODE>::LBMAX;

// Per-lane constants of the copy: lane k < PER_WAVE of wave w issues the
// wave's copy instruction k, which covers array k / IPW (left operand parts,
// then right operand parts) at 1 KB blocks (k % IPW) * NW + w; so the array
// and the LDS destination are compile-time constants plus a scalar.  The lane
// reads the leaf address at index op * LPU + slot of a leaf column's metadata
// and adds its part and line offset.
struct CopyLane {
    int idx;       // op * LPU + slot
    uint32_t off;  // part and line offset inside the leaf, bytes
};

template <int MODE, int U, int BS>
__device__ __forceinline__ CopyLane copy_lane(const K5Member &m, int w) {
    using G = Geo<MODE, U, BS>;
    using T = typename G::T;
    constexpr int IPW = G::IPA / G::NW;
    static_assert(G::IPA % G::NW == 0, "copy blocks of an array must split evenly over the waves");
    static_assert(G::PER_WAVE <= 63, "one lane per copy instruction; vmcnt counts to 63");
    const int k = (threadIdx.x & 63) < G::PER_WAVE ? (threadIdx.x & 63) : 0;
    const int arr = k / IPW;
    const int op = arr / MT<MODE>::PARTS, part = arr - op * MT<MODE>::PARTS;
    const int jj = (k % IPW) * G::NW + w;
    const int line0 = jj * G::LPI;
    const int slot = line0 / BS;
    CopyLane cl;
    cl.idx = op * G::LPU + slot;
    cl.off = (uint32_t)((int64_t)part * m.partStrideL * (int64_t)sizeof(T)) + (uint32_t)((line0 - slot * BS) * G::LB);
    return cl;
}

// Source addresses of one step's copy, one per lane (lane k: the wave's
// instruction k); kept in one 64-bit register pair for the whole step, each
// instruction reads its address back as a scalar.  A nil leaf reads the zero
// page (on the tile-skipping path its lines are never read).
template <int MODE, int U, int BS>
__device__ __forceinline__ uint64_t copy_addr(const Meta &mt, int i, int kb, int c, const CopyLane &cl,
                                              uint32_t chunk_bytes) {
    using G = Geo<MODE, U, BS>;
    const uint64_t b = mt.ad[(int64_t)i * 2 * G::NSUB + kb * 2 * G::LPU + cl.idx];
    const uint64_t zp = reinterpret_cast<uint64_t>(&g_zero_page[0]);
    return b == 0 ? zp : b + cl.off + (uint64_t)c * chunk_bytes;
}

// Copy addresses of the next K chunk of the same leaf column: one chunk
// further in every lane except those reading the zero page.
__device__ __forceinline__ uint64_t next_chunk_addr(uint64_t a, uint32_t chunk_bytes) {
    const uint64_t zp = reinterpret_cast<uint64_t>(&g_zero_page[0]);
    return a == zp ? a : a + chunk_bytes;
}

// Copy instruction k of wave w: 64 lanes x 16 bytes straight into LDS.
template <int MODE, int U, int BS>
__device__ __forceinline__ void issue_one(uint64_t addrs, int k, uint8_t *stage, int w) {
    using G = Geo<MODE, U, BS>;
    constexpr int IPW = G::IPA / G::NW;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)addrs, k);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(addrs >> 32), k);
    const uint64_t a = ((uint64_t)hi << 32) | lo;
    const int arr = k / IPW;
    const int jj = (k % IPW) * G::NW + w;
    // an opaque lane offset keeps the sum "scalar base + 32-bit lane offset"
    // (the instruction's scalar-base form) from being re-associated into a
    // hoisted per-lane 64-bit base
    uint32_t lane16 = (threadIdx.x & 63u) * 16u;
    asm volatile("" : "+v"(lane16));
    __builtin_amdgcn_global_load_lds((const QB_GAS void *)(reinterpret_cast<const uint8_t *>(a) + lane16),
                                     (QB_LAS void *)(stage + arr * G::ARRB + jj * 1024), 16, 0, 0);
}

// Wave-uniform enable bits of the leaves a wave covers in one step: bit
// (a * NLW + b) is set when the product of the wave's leaf row a and leaf
// column b exists in this step.
template <int MODE, int U, int BS>
__device__ __forceinline__ uint32_t wave_leaves(uint32_t km, int wr, int wc) {
    using G = Geo<MODE, U, BS>;
    uint32_t wl = 0;
#pragma unroll
    for (int a = 0; a < G::NLW; ++a)
#pragma unroll
        for (int b = 0; b < G::NLW; ++b) {
            const int ib = (G::WT * wr) / BS + a, jb = (G::WT * wc) / BS + b;
            wl |= ((km >> (ib * G::LPU + jb)) & 1u) << (a * G::NLW + b);
        }
    return (uint32_t)uni((int)wl);
}

// One step on the LDS stage `cur` while the copy of the next step (if any)
// lands in `nxt`.  The two stages are distinct shared arrays, so the
// compiler knows the copy into `nxt` cannot alias the fragment reads of
// `cur` and issues no wait between them: the copy is issued first and runs
// under the whole step.  The step ends with every wave's copies complete and
// a barrier, after which `cur` may be overwritten.
// The step after st and its copy addresses: one chunk on within a leaf
// column, looked up again for a new column (after the last step the copies
// still go out, from the zero page into the stage nobody reads, so that the
// MFMA loop has no branch).
struct Advance {
    Step nx;
    uint64_t addrs;
};

template <int MODE, int U, int BS>
__device__ __forceinline__ Advance advance(const Meta &mt, int nb, const Step &st, uint64_t addrs,
                                           const CopyLane &cl, uint32_t chunk_bytes) {
    using G = Geo<MODE, U, BS>;
    Advance a;
    a.nx = next_step<G::LPU, G::NSUB, G::NCHUNK>(mt, nb, st);
    if (a.nx.i >= nb)
        a.addrs = reinterpret_cast<uint64_t>(&g_zero_page[0]);
    else if (a.nx.c != 0)
        a.addrs = next_chunk_addr(addrs, chunk_bytes);
    else
        a.addrs = copy_addr<MODE, U, BS>(mt, a.nx.i, a.nx.kb, 0, cl, chunk_bytes);
    return a;
}

// Ozaki mode: the line exponents a wave needs for one step -- the rows of its
// row tiles in the left leaf and the columns of its column tiles in the right
// leaf -- read from the exponent block after the leaf's slices.  Loaded one
// step ahead; the step's closing wait covers them.
template <int TPW>
struct OzExp {
    i4 er[TPW];   // rows 4*(lane/16) .. +3 of row tile tm
    int ec[TPW];  // column lane % 16 of column tile tn
};

template <int MODE, int U, int BS>
__device__ __forceinline__ void oz_load_exp(const Meta &mt, int i, int kb, int wr, int wc,
                                            OzExp<Geo<MODE, U, BS>::TPW> &ex) {
    using G = Geo<MODE, U, BS>;
    if constexpr (MODE == QBSM_OZAKI_I8) {
        const int lane = threadIdx.x & 63;
        const uint64_t *d = mt.ad + (int64_t)i * 2 * G::NSUB + kb * 2 * G::LPU;
        constexpr int64_t EXP_OFF = (int64_t)OZ_SLICES * BS * BS;
#pragma unroll
        for (int t = 0; t < G::TPW; ++t) {
            const int r = G::WT * wr + 16 * t, c = G::WT * wc + 16 * t;
            const uint64_t la = uni64(d[r / BS]), lb = uni64(d[G::LPU + c / BS]);
            const int32_t *eA = reinterpret_cast<const int32_t *>(la + EXP_OFF);
            const int32_t *eB = reinterpret_cast<const int32_t *>(lb + EXP_OFF);
            ex.er[t] = *reinterpret_cast<const i4 *>(eA + (r % BS) + 4 * (lane >> 4));
            ex.ec[t] = eB[(c % BS) + (lane & 15)];
        }
    }
}

// One step on stage cur: st is this step, nxa the next one with its copy
// addresses (looked up during the previous step).  The step after next is
// looked up once this step's MFMAs are issued, while the copies land.
// FIRST: the unit's first step, whose successor's copy was issued with the
// step's own copy at the start of the unit; nothing is copied during it.
template <int MODE, int U, int BS, bool DENSE, bool NF, bool FIRST = false>
__device__ __forceinline__ void run_step(const K5Member &m, const Meta &mt, int nb, const uint8_t *cur, uint8_t *nxt,
                                         typename MT<MODE>::Acc (&acc)[Geo<MODE, U, BS>::TPW][Geo<MODE, U, BS>::TPW],
                                         typename MT<MODE>::Part (&part)[Geo<MODE, U, BS>::TPW][Geo<MODE, U, BS>::TPW],
                                         Step &st, Advance &nxa, const CopyLane &cl, uint32_t chunk_bytes, int w,
                                         int wr, int wc, OzExp<Geo<MODE, U, BS>::TPW> &ex) {
    using G = Geo<MODE, U, BS>;
    using M = MT<MODE>;
    constexpr int PARTS = M::PARTS, TPW = G::TPW, TPL = G::TPL, NLW = G::NLW;
    const int lane = threadIdx.x & 63;
    const uint32_t km = st.km;
    // the next step's copy instructions are spread over the column tiles of
    // this step for 64-wide wave parts and on the branch-free path; with
    // 128 x 128 per wave and tile skipping the register file has no room for
    // that schedule and the copy is issued in one go
    constexpr bool SPREAD = (G::WT <= 64 || DENSE) && !FIRST;
    if constexpr (!SPREAD && !FIRST) {
        if (nxa.nx.i < nb) {
#pragma unroll
            for (int k = 0; k < G::PER_WAVE; ++k) issue_one<MODE, U, BS>(nxa.addrs, k, nxt, w);
        }
    }
    OzExp<TPW> ex_next = ex;
    if constexpr (MODE == QBSM_OZAKI_I8) {
        if (nxa.nx.i < nb) oz_load_exp<MODE, U, BS>(mt, nxa.nx.i, nxa.nx.kb, wr, wc, ex_next);
    }
    constexpr int TSPAN = TPW;
    constexpr int KPT = (G::PER_WAVE + TSPAN - 1) / TSPAN;
    const uint32_t wl = wave_leaves<MODE, U, BS>(km, wr, wc);
    if (DENSE || wl) {
        const uint8_t *Ab = cur;
        const uint8_t *Bb = cur + PARTS * G::ARRB;
#pragma unroll
        for (int rg = 0; rg < G::NGROUPS; ++rg) {
            const int pbase = rg * M::PPG + (lane >> 4) * M::SUBS;
            typename M::Frag fa[TPW][PARTS];
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const int la_ = G::WT * wr + 16 * t + (lane & 15);
#pragma unroll
                for (int part = 0; part < PARTS; ++part)
#pragma unroll
                    for (int q = 0; q < M::SUBS; ++q)
                        fa[t][part].q[q] = lds_piece(Ab + part * G::ARRB, la_, G::LB, pbase + q);
            }
            // B fragments of column tile tn + 1 are read while the MFMAs of
            // column tile tn run
            typename M::Frag fb[2][PARTS];
            auto read_b = [&](int tn, typename M::Frag (&dst)[PARTS]) {
                const int lb_ = G::WT * wc + 16 * tn + (lane & 15);
#pragma unroll
                for (int part = 0; part < PARTS; ++part)
#pragma unroll
                    for (int q = 0; q < M::SUBS; ++q)
                        dst[part].q[q] = lds_piece(Bb + part * G::ARRB, lb_, G::LB, pbase + q);
            };
            read_b(0, fb[0]);
#pragma unroll
            for (int tn = 0; tn < TPW; ++tn) {
                if (SPREAD && rg == 0 && tn < TSPAN) {
                    // pinned in place: hoisting the copies' scalar state
                    // across the MFMAs would cost registers
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int j = 0; j < KPT; ++j)
                        if (tn * KPT + j < G::PER_WAVE) issue_one<MODE, U, BS>(nxa.addrs, tn * KPT + j, nxt, w);
                    __builtin_amdgcn_sched_barrier(0);
                }
                if (tn + 1 < TPW) read_b(tn + 1, fb[(tn + 1) & 1]);
#pragma unroll
                for (int tm = 0; tm < TPW; ++tm)
                    if (DENSE || ((wl >> ((tm / TPL) * NLW + tn / TPL)) & 1u)) {
                        if constexpr (M::LEAF_SUMS)
                            M::mma_part(part[tm][tn], fa[tm], fb[tn & 1]);
                        else
                            M::mma(acc[tm][tn], fa[tm], fb[tn & 1]);
                    }
            }
        }
        if constexpr (M::LEAF_SUMS) {
            // the last chunk of the leaf column: its sums are complete (a
            // tile without products adds zeros; a wave without leaves in
            // this column skips the whole block and its sums stay zero)
            if (st.c == G::NCHUNK - 1) {
#pragma unroll
                for (int tm = 0; tm < TPW; ++tm)
#pragma unroll
                    for (int tn = 0; tn < TPW; ++tn)
                        M::template flush<NF>(acc[tm][tn], part[tm][tn], ex.er[tm], ex.ec[tn]);
            }
        }
    } else if constexpr (SPREAD) {
#pragma unroll
        for (int k = 0; k < G::PER_WAVE; ++k) issue_one<MODE, U, BS>(nxa.addrs, k, nxt, w);
    }
    const Advance nn = nxa.nx.i < nb ? advance<MODE, U, BS>(mt, nb, nxa.nx, nxa.addrs, cl, chunk_bytes) : nxa;
    // every wave's copy into nxt has landed and nobody reads cur any more
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    st = nxa.nx;
    nxa = nn;
    if constexpr (MODE == QBSM_OZAKI_I8) ex = ex_next;
}

// Fills the LDS metadata of pairs b0 .. b0 + nb - 1 of a unit: product bits
// and the packed address of every leaf the pair's steps copy.
template <int MODE, int U, int BS>
__device__ __forceinline__ void load_meta(const K5Member &m, const Meta &mt, int b0, int nb) {
    using G = Geo<MODE, U, BS>;
    constexpr int NT = 64 * G::NW;
    constexpr int LPU = G::LPU, NSUB = G::NSUB, S = G::S;
    for (int i = threadIdx.x; i < nb; i += NT) {
        const int p = b0 + i;
        const int a = m.pl[p], b = m.pr[p];
        mt.pm[i] = m.pmask[p];
#pragma unroll
        for (int kb = 0; kb < LPU; ++kb)
#pragma unroll
            for (int q = 0; q < LPU; ++q) {
                const int qa = m.transL ? morton_sub(kb, q, S) : morton_sub(q, kb, S);
                const int qb = m.transR ? morton_sub(q, kb, S) : morton_sub(kb, q, S);
                const int la = m.descL ? m.descL[(int64_t)a * NSUB + qa] : a;
                const int lb = m.descR ? m.descR[(int64_t)b * NSUB + qb] : b;
                uint64_t *d = mt.ad + (int64_t)i * 2 * NSUB + kb * 2 * LPU;
                d[q] = la < 0 ? 0 : reinterpret_cast<uint64_t>(static_cast<const uint8_t *>(m.packL) +
                                                               (int64_t)la * m.leafStrideL * (int64_t)sizeof(typename G::T));
                d[LPU + q] = lb < 0 ? 0 : reinterpret_cast<uint64_t>(static_cast<const uint8_t *>(m.packR) +
                                                                     (int64_t)lb * m.leafStrideR * (int64_t)sizeof(typename G::T));
            }
    }
}

// Where a unit's output goes: its node coordinates and, for each leaf of
// the wave's part, the output leaf index (-1: no output block there).
template <int NLW>
struct UnitOut {
    uint32_t ui, uj;
    int32_t leaves[NLW][NLW];
};

template <int MODE, int U, int BS>
__device__ __forceinline__ UnitOut<Geo<MODE, U, BS>::NLW> unit_out_load(const K5Member &m, int u, int wr, int wc) {
    using G = Geo<MODE, U, BS>;
    constexpr int LPU = G::LPU, NSUB = G::NSUB, NLW = G::NLW;
    UnitOut<NLW> o;
    demorton(m.ukey[u], o.ui, o.uj);
    const int ib0 = (G::WT * wr) / BS, jb0 = (G::WT * wc) / BS;
#pragma unroll
    for (int a = 0; a < NLW; ++a)
#pragma unroll
        for (int b = 0; b < NLW; ++b) o.leaves[a][b] = uni(m.cdesc[(int64_t)u * NSUB + (ib0 + a) * LPU + jb0 + b]);
    return o;
}

// Writes a unit's owned output blocks once (padding beyond the logical size
// = 0) from the wave's accumulators.
template <int MODE, int U, int BS>
__device__ __forceinline__ void store_unit_out(const K5Member &m, const UnitOut<Geo<MODE, U, BS>::NLW> &o,
                                               const typename MT<MODE>::Acc (&acc)[Geo<MODE, U, BS>::TPW][Geo<MODE, U, BS>::TPW],
                                               int wr, int wc) {
    using G = Geo<MODE, U, BS>;
    using M = MT<MODE>;
    constexpr int LPU = G::LPU;
    const int tid = threadIdx.x;
    // leaf by leaf: each stored leaf of the wave's NLW x NLW writes its
    // TPL x TPL tiles
    const int lane = tid & 63;
    typename M::Out *C = static_cast<typename M::Out *>(m.C);
    constexpr int64_t N2 = (int64_t)BS * BS;
    constexpr int NLW = G::NLW, TPL = G::TPL;
    const int ib0 = (G::WT * wr) / BS, jb0 = (G::WT * wc) / BS;
#pragma unroll
    for (int a = 0; a < NLW; ++a)
#pragma unroll
        for (int b = 0; b < NLW; ++b) {
            const int32_t leaf = o.leaves[a][b];
            if (leaf < 0) continue;
            const int ib = ib0 + a, jb = jb0 + b;
            const int64_t I = (int64_t)o.ui * LPU + ib, J = (int64_t)o.uj * LPU + jb;
            const bool interior = (I + 1) * BS <= m.out_rows && (J + 1) * BS <= m.out_cols;
            typename M::Out *Cl = C + (int64_t)leaf * N2;
#pragma unroll
            for (int ta = 0; ta < TPL; ++ta)
#pragma unroll
                for (int tb = 0; tb < TPL; ++tb) {
                    const int tm = a * TPL + ta, tn = b * TPL + tb;
                    // tile origin inside the leaf
                    const int r0 = G::WT * wr + 16 * tm - ib * BS, c0 = G::WT * wc + 16 * tn - jb * BS;
                    const int cc = c0 + (lane & 15);
                    typename M::Out *dst = Cl + (int64_t)cc * BS + r0;
                    if (M::row_of(0, 1) == 1 && interior) {
                        // rows 4*(lane/16) .. +3 of the tile are contiguous in the column
                        if constexpr (sizeof(typename M::Out) == 4) {
                            *reinterpret_cast<float4 *>(dst + 4 * (lane >> 4)) =
                                make_float4(acc[tm][tn][0], acc[tm][tn][1], acc[tm][tn][2], acc[tm][tn][3]);
                        } else {
#pragma unroll
                            for (int i = 0; i < 4; ++i) dst[4 * (lane >> 4) + i] = (typename M::Out)acc[tm][tn][i];
                        }
                    } else {
                        const bool colok = (J * BS + cc) < m.out_cols;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int r = r0 + M::row_of(lane, i);
                            const bool ok = colok && (I * BS + r) < m.out_rows;
                            dst[M::row_of(lane, i)] = ok ? (typename M::Out)acc[tm][tn][i] : (typename M::Out)0;
                        }
                    }
                }
        }
}

template <int MODE, int U, int BS>
__device__ __forceinline__ void store_unit(const K5Member &m, int u,
                                           const typename MT<MODE>::Acc (&acc)[Geo<MODE, U, BS>::TPW][Geo<MODE, U, BS>::TPW],
                                           int wr, int wc) {
    store_unit_out<MODE, U, BS>(m, unit_out_load<MODE, U, BS>(m, u, wr, wc), acc, wr, wc);
}

// A batch of a unit's pairs whose metadata is in LDS and whose first copies
// are in flight: its first step, the next step with its copy addresses, and
// whether that next step's copy went out with the first (pre).
struct BatchGo {
    Step st;
    Advance nxa;
    int nb;
    bool pre;
};

// Reads the metadata of pairs b0 .. min(b0 + CAP, p1) - 1 into LDS and
// issues the copy of the batch's first step and, below unit 256, of its
// second: a unit of two steps (one leaf product of two K chunks) waits for
// one copy latency instead of two.  Only below unit 256: those units are
// short on sparse inputs, while the 256-wide kernels run long units and have
// no registers to spare for a third copy of the step body.
template <int MODE, int U, int BS>
__device__ __forceinline__ BatchGo batch_begin(const K5Member &m, const Meta &mt, int b0, int p1, const CopyLane &cl,
                                               uint32_t chunk_bytes, int w, int wr, int wc, uint8_t *st0,
                                               uint8_t *st1, OzExp<Geo<MODE, U, BS>::TPW> &ex) {
    using G = Geo<MODE, U, BS>;
    BatchGo g;
    g.nb = uni((p1 - b0) < G::CAP ? (p1 - b0) : G::CAP);
    __syncthreads();  // LDS (stages, metadata) of the previous batch or unit is free
    load_meta<MODE, U, BS>(m, mt, b0, g.nb);
    __syncthreads();
    g.st = first_step<G::LPU, G::NSUB>(mt, g.nb, 0);
    g.nxa.nx = g.st;
    g.nxa.addrs = 0;
    constexpr bool PRE2 = U <= 128;
    g.pre = false;
    if (g.st.i < g.nb) {
        const uint64_t addrs = copy_addr<MODE, U, BS>(mt, g.st.i, g.st.kb, 0, cl, chunk_bytes);
#pragma unroll
        for (int k = 0; k < G::PER_WAVE; ++k) issue_one<MODE, U, BS>(addrs, k, st0, w);
        oz_load_exp<MODE, U, BS>(mt, g.st.i, g.st.kb, wr, wc, ex);
        g.nxa = advance<MODE, U, BS>(mt, g.nb, g.st, addrs, cl, chunk_bytes);
        g.pre = PRE2 && g.nxa.nx.i < g.nb;
        if (g.pre) {
#pragma unroll
            for (int k = 0; k < G::PER_WAVE; ++k) issue_one<MODE, U, BS>(g.nxa.addrs, k, st1, w);
        }
    }
    return g;
}

// Runs the steps of a begun batch, from the wait for its first copy on.
// WAIT_ALL: the first wait is for every outstanding memory operation (other
// loads and stores were issued after the batch's copies).
template <int MODE, int U, int BS, bool DENSE, bool NF, bool WAIT_ALL = false>
__device__ __forceinline__ void batch_run(const K5Member &m, const Meta &mt, BatchGo &g, uint8_t *st0, uint8_t *st1,
                                          typename MT<MODE>::Acc (&acc)[Geo<MODE, U, BS>::TPW][Geo<MODE, U, BS>::TPW],
                                          typename MT<MODE>::Part (&part)[Geo<MODE, U, BS>::TPW][Geo<MODE, U, BS>::TPW],
                                          const CopyLane &cl, uint32_t chunk_bytes, int w, int wr, int wc,
                                          OzExp<Geo<MODE, U, BS>::TPW> &ex) {
    using G = Geo<MODE, U, BS>;
    constexpr bool PRE2 = U <= 128;
    const int nb = g.nb;
    Step &st = g.st;
    Advance &nxa = g.nxa;
    if (g.pre && !WAIT_ALL)
        __builtin_amdgcn_s_waitcnt(k5_vmcnt<G::PER_WAVE>);  // the first step's copies (and exponents)
    else
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    // steps alternate between the two stages; unrolled by two so that
    // every access names its stage array at compile time
    if constexpr (PRE2) {
        if (st.i < nb) {
            if (g.pre)
                run_step<MODE, U, BS, DENSE, NF, true>(m, mt, nb, st0, st1, acc, part, st, nxa, cl, chunk_bytes, w,
                                                       wr, wc, ex);
            else
                run_step<MODE, U, BS, DENSE, NF>(m, mt, nb, st0, st1, acc, part, st, nxa, cl, chunk_bytes, w, wr, wc,
                                                 ex);
        }
        while (st.i < nb) {
            run_step<MODE, U, BS, DENSE, NF>(m, mt, nb, st1, st0, acc, part, st, nxa, cl, chunk_bytes, w, wr, wc, ex);
            if (st.i >= nb) break;
            run_step<MODE, U, BS, DENSE, NF>(m, mt, nb, st0, st1, acc, part, st, nxa, cl, chunk_bytes, w, wr, wc, ex);
        }
    } else {
        while (st.i < nb) {
            run_step<MODE, U, BS, DENSE, NF>(m, mt, nb, st0, st1, acc, part, st, nxa, cl, chunk_bytes, w, wr, wc, ex);
            if (st.i >= nb) break;
            run_step<MODE, U, BS, DENSE, NF>(m, mt, nb, st1, st0, acc, part, st, nxa, cl, chunk_bytes, w, wr, wc, ex);
        }
    }
}

template <int MODE, int TPW>
__device__ __forceinline__ void clear_acc(typename MT<MODE>::Acc (&acc)[TPW][TPW],
                                          typename MT<MODE>::Part (&part)[TPW][TPW], OzExp<TPW> &ex) {
    using M = MT<MODE>;
#pragma unroll
    for (int a = 0; a < TPW; ++a)
#pragma unroll
        for (int b = 0; b < TPW; ++b) acc[a][b] = typename M::Acc{};
    if constexpr (M::LEAF_SUMS) {
#pragma unroll
        for (int a = 0; a < TPW; ++a)
#pragma unroll
            for (int b = 0; b < TPW; ++b)
#pragma unroll
                for (int k = 0; k < M::NSUMS; ++k) part[a][b].s[k] = i4{0, 0, 0, 0};
    }
    ex = OzExp<TPW>{};
}

// DENSE: the branch-free path (every tile multiplied, nil leaves copied as
// zeros), valid when neither pack holds Inf or NaN (an infinite value times
// the zero of a nil partner would give NaN where no product exists).
template <int MODE, int U, int BS, bool DENSE, bool NF = false>
__device__ void process_unit(const K5Member &m, int u, uint8_t *st0, uint8_t *st1, uint8_t *meta) {
    using G = Geo<MODE, U, BS>;
    using M = MT<MODE>;
    constexpr int TPW = G::TPW;
    const int tid = threadIdx.x;
    const int w = uni(tid >> 6);
    const int wr = w / G::WPS, wc = w % G::WPS;

    typename M::Acc acc[TPW][TPW];
    typename M::Part part[TPW][TPW];
    OzExp<TPW> ex;
    clear_acc<MODE, TPW>(acc, part, ex);

    // (loaded values are not known to be wave-uniform: say so, or every
    // comparison with the batch size makes the step iterator divergent)
    const int p0 = uni(m.ustart[u]), p1 = uni(m.ustart[u + 1]);
    const Meta mt = meta_view(meta, G::CAP);
    const CopyLane cl = copy_lane<MODE, U, BS>(m, w);
    const uint32_t chunk_bytes = (uint32_t)((int64_t)m.chunkStrideL * (int64_t)sizeof(typename G::T));
    for (int b0 = p0; b0 < p1; b0 += G::CAP) {
        BatchGo g = batch_begin<MODE, U, BS>(m, mt, b0, p1, cl, chunk_bytes, w, wr, wc, st0, st1, ex);
        batch_run<MODE, U, BS, DENSE, NF>(m, mt, g, st0, st1, acc, part, cl, chunk_bytes, w, wr, wc, ex);
    }

    store_unit<MODE, U, BS>(m, u, acc, wr, wc);
}

// Streamed schedule for plans of few leaf products per unit, where a unit
// is a metadata read, a copy, a short MFMA burst and a store, each waiting
// on the one before: one persistent workgroup runs units it, it + G, ...
// (G workgroups; unit xcd_remap(it) as in the one-unit-per-workgroup
// launch).  The next unit's metadata is read and its first copies are issued
// before this unit's output is stored, so the stores drain while those
// copies land, and the next unit's pair range and output leaves are looked
// up while this one runs.  The tile-skipping path only (units below 256).
template <int MODE, int U, int BS>
__device__ void process_stream(const K5Member &m, uint8_t *st0, uint8_t *st1, uint8_t *meta) {
    using G = Geo<MODE, U, BS>;
    using M = MT<MODE>;
    constexpr int TPW = G::TPW, NLW = G::NLW;
    const int n = m.nunits, gsz = (int)gridDim.x;
    int it = (int)blockIdx.x;
    if (it >= n) return;
    const int tid = threadIdx.x;
    const int w = uni(tid >> 6);
    const int wr = w / G::WPS, wc = w % G::WPS;
    const Meta mt = meta_view(meta, G::CAP);
    const CopyLane cl = copy_lane<MODE, U, BS>(m, w);
    const uint32_t chunk_bytes = (uint32_t)((int64_t)m.chunkStrideL * (int64_t)sizeof(typename G::T));

    typename M::Acc acc[TPW][TPW];
    typename M::Part part[TPW][TPW];
    OzExp<TPW> ex;
    clear_acc<MODE, TPW>(acc, part, ex);

    int u = xcd_remap(it, n);
    int p0 = uni(m.ustart[u]), p1 = uni(m.ustart[u + 1]);
    UnitOut<NLW> o = unit_out_load<MODE, U, BS>(m, u, wr, wc);
    BatchGo g{};
    if (p0 < p1) g = batch_begin<MODE, U, BS>(m, mt, p0, p1, cl, chunk_bytes, w, wr, wc, st0, st1, ex);
    for (;;) {
        // the next unit's pair range and output leaves, read under this unit
        const int itn = it + gsz;
        const int un = itn < n ? xcd_remap(itn, n) : 0;
        int q0 = 0, q1 = 0;
        UnitOut<NLW> on = o;
        if (itn < n) {
            q0 = uni(m.ustart[un]);
            q1 = uni(m.ustart[un + 1]);
            on = unit_out_load<MODE, U, BS>(m, un, wr, wc);
        }
        if (p0 < p1) {
            // (the previous unit's stores went out after this batch's copies)
            batch_run<MODE, U, BS, false, false, true>(m, mt, g, st0, st1, acc, part, cl, chunk_bytes, w, wr, wc, ex);
            for (int b0 = p0 + G::CAP; b0 < p1; b0 += G::CAP) {
                g = batch_begin<MODE, U, BS>(m, mt, b0, p1, cl, chunk_bytes, w, wr, wc, st0, st1, ex);
                batch_run<MODE, U, BS, false, false>(m, mt, g, st0, st1, acc, part, cl, chunk_bytes, w, wr, wc, ex);
            }
        }
        // every step of this unit has passed its closing barrier: the stages
        // and the metadata may take the next unit's
        OzExp<TPW> exn{};
        if (itn < n && q0 < q1)
            g = batch_begin<MODE, U, BS>(m, mt, q0, q1, cl, chunk_bytes, w, wr, wc, st0, st1, exn);
        store_unit_out<MODE, U, BS>(m, o, acc, wr, wc);
        if (itn >= n) break;
        clear_acc<MODE, TPW>(acc, part, ex);
        ex = exn;
        it = itn;
        u = un;
        p0 = q0;
        p1 = q1;
        o = on;
    }
}

// Single-stage kernel: one 32 KB LDS stage and a small metadata area, so
// that more workgroups share a compute unit and cover each other's waits.
// Each step copies, waits, computes and leaves the stage with a barrier
// before the next copy; the MFMA order of every accumulator is that of the
// double-buffered kernel, so the results are the same bit for bit.
// - BF16 and BF16X3 at unit 128, for plans of about one leaf product per
//   unit (the HBM-bound random-block multiply, where a unit is a metadata
//   read, one or two copies, a short MFMA burst and a store, each waiting on
//   the one before): at most 128 vector registers, four workgroups per
//   compute unit instead of two.
// - FP64 at unit 128, for every plan: the double-buffered FP64 kernel keeps
//   its accumulators and fragments in 256 + 143 registers and runs one
//   workgroup per compute unit; this one needs 168 and runs three.
constexpr int kMetaSmall = 2048;

template <int MODE, int U, int BS>
__device__ __forceinline__ void compute_step(const uint8_t *cur,
                                             typename MT<MODE>::Acc (&acc)[Geo<MODE, U, BS>::TPW][Geo<MODE, U, BS>::TPW],
                                             const Step &st, int wr, int wc) {
    using G = Geo<MODE, U, BS>;
    using M = MT<MODE>;
    constexpr int PARTS = M::PARTS, TPW = G::TPW, TPL = G::TPL, NLW = G::NLW;
    const int lane = threadIdx.x & 63;
    const uint32_t wl = wave_leaves<MODE, U, BS>(st.km, wr, wc);
    if (!wl) return;
    const uint8_t *Ab = cur;
    const uint8_t *Bb = cur + PARTS * G::ARRB;
#pragma unroll
    for (int rg = 0; rg < G::NGROUPS; ++rg) {
        const int pbase = rg * M::PPG + (lane >> 4) * M::SUBS;
        typename M::Frag fa[TPW][PARTS];
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int la_ = G::WT * wr + 16 * t + (lane & 15);
#pragma unroll
            for (int part = 0; part < PARTS; ++part)
#pragma unroll
                for (int q = 0; q < M::SUBS; ++q)
                    fa[t][part].q[q] = lds_piece(Ab + part * G::ARRB, la_, G::LB, pbase + q);
        }
#pragma unroll
        for (int tn = 0; tn < TPW; ++tn) {
            typename M::Frag fb[PARTS];
            const int lb_ = G::WT * wc + 16 * tn + (lane & 15);
#pragma unroll
            for (int part = 0; part < PARTS; ++part)
#pragma unroll
                for (int q = 0; q < M::SUBS; ++q)
                    fb[part].q[q] = lds_piece(Bb + part * G::ARRB, lb_, G::LB, pbase + q);
#pragma unroll
            for (int tm = 0; tm < TPW; ++tm)
                if ((wl >> ((tm / TPL) * NLW + tn / TPL)) & 1u) M::mma(acc[tm][tn], fa[tm], fb);
        }
    }
}

template <int MODE, int U, int BS>
__device__ void process_unit_serial(const K5Member &m, int u, uint8_t *st0, uint8_t *meta) {
    using G = Geo<MODE, U, BS>;
    using M = MT<MODE>;
    static_assert(!M::LEAF_SUMS, "the integer-digit mode has its own kernels");
    constexpr int TPW = G::TPW, LPU = G::LPU, NSUB = G::NSUB;
    constexpr int CAPS = kMetaSmall / (8 + 16 * NSUB);
    const int w = uni((int)threadIdx.x >> 6);
    const int wr = w / G::WPS, wc = w % G::WPS;
    typename M::Acc acc[TPW][TPW];
#pragma unroll
    for (int a = 0; a < TPW; ++a)
#pragma unroll
        for (int b = 0; b < TPW; ++b) acc[a][b] = typename M::Acc{};
    const int p0 = uni(m.ustart[u]), p1 = uni(m.ustart[u + 1]);
    const Meta mt = meta_view(meta, CAPS);
    const CopyLane cl = copy_lane<MODE, U, BS>(m, w);
    const uint32_t chunk_bytes = (uint32_t)((int64_t)m.chunkStrideL * (int64_t)sizeof(typename G::T));
    for (int b0 = p0; b0 < p1; b0 += CAPS) {
        const int nb = uni((p1 - b0) < CAPS ? (p1 - b0) : CAPS);
        __syncthreads();  // the metadata of the previous batch is no longer read
        load_meta<MODE, U, BS>(m, mt, b0, nb);
        __syncthreads();
        Step st = first_step<LPU, NSUB>(mt, nb, 0);
        while (st.i < nb) {
            const uint64_t addrs = copy_addr<MODE, U, BS>(mt, st.i, st.kb, st.c, cl, chunk_bytes);
#pragma unroll
            for (int k = 0; k < G::PER_WAVE; ++k) issue_one<MODE, U, BS>(addrs, k, st0, w);
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's copies have landed
            __syncthreads();
            compute_step<MODE, U, BS>(st0, acc, st, wr, wc);
            __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this wave's reads of the stage are done
            __syncthreads();
            st = next_step<LPU, NSUB, G::NCHUNK>(mt, nb, st);
        }
    }
    store_unit<MODE, U, BS>(m, u, acc, wr, wc);
}

template <int MODE, int U, int BS>
__global__ void __launch_bounds__((k5_nt<MODE, U>), (MODE == QBSM_F64 ? 2 : 4))
    k5s(K5Member single, const K5Member *members, const int2 *items, int64_t nitems, int32_t *counter) {
    static_assert(U == 128 && (MODE == QBSM_BF16 || MODE == QBSM_BF16X3 || MODE == QBSM_F64),
                  "single-stage kernel: BF16 modes and FP64, unit 128");
    __shared__ __attribute__((aligned(1024))) uint8_t st0[k5_stage_bytes<MODE, U>];
    __shared__ __attribute__((aligned(16))) uint8_t meta[kMetaSmall];
    process_unit_serial<MODE, U, BS>(single, xcd_remap((int)blockIdx.x, single.nunits), st0, meta);
}

// The unit of this workgroup in a single-multiply launch (XCD-aware).
__device__ __forceinline__ int launch_unit(const K5Member &m) { return xcd_remap((int)blockIdx.x, m.nunits); }

// Whether a member takes the branch-free unit-256 path (read from its
// packs' device flags).
__device__ __forceinline__ bool dense_ok(const K5Member &m) { return (*m.nfL | *m.nfR) == 0 && !m.select; }

// Unit 256 takes the branch-free path when both packs are finite; the
// smaller units (two workgroups per compute unit) keep the skipping path.
template <int MODE, int U, int BS>
__device__ __forceinline__ void process_sel(const K5Member &m, int u, uint8_t *st0, uint8_t *st1, uint8_t *meta) {
    if constexpr (U >= 256) {
        // the branch-free path multiplies every pair of stored leaves of a
        // step, so it serves only plans whose products are all such pairs
        if (dense_ok(m)) {
            process_unit<MODE, U, BS, true>(m, u, st0, st1, meta);
            return;
        }
    }
    if constexpr (MODE == QBSM_OZAKI_I8) {
        if ((*m.nfL | *m.nfR) != 0) {
            process_unit<MODE, U, BS, false, true>(m, u, st0, st1, meta);
            return;
        }
    }
    process_unit<MODE, U, BS, false>(m, u, st0, st1, meta);
}

template <int MODE, int U>
__device__ __forceinline__ void process_any(const K5Member &m, int u, uint8_t *st0, uint8_t *st1, uint8_t *meta) {
    // (the Ozaki mode's 64-wide integer MFMA needs 64-wide leaves)
    if constexpr (U <= 128 && MODE != QBSM_OZAKI_I8) {
        if (m.bs == 32) {
            process_sel<MODE, U, 32>(m, u, st0, st1, meta);
            return;
        }
    }
    if (m.bs == 64) {
        process_sel<MODE, U, 64>(m, u, st0, st1, meta);
    } else if constexpr (U >= 128) {
        if (m.bs == 128) process_sel<MODE, U, 128>(m, u, st0, st1, meta);
    }
}

template <int MODE, int U>
constexpr int k5_min_blocks = (MODE == QBSM_F64 || MODE == QBSM_OZAKI_I8 || U >= 256) ? 1 : 2;

// BS > 0: one launch of one multiply with that leaf size, one workgroup per
// unit.  BS == 0: persistent launch over a work list of (member, unit) items
// of members with any leaf size, pulled from a device counter.
// PATH (unit 256, BS > 0): 1 = the branch-free path only, 2 = the
// tile-skipping path only; each workgroup leaves at once when its path does
// not apply, and the host launches both (or only 2 where the plan selects
// products), so neither kernel carries the other path.  0 = both paths in one
// kernel, chosen per unit.  3 (units below 256, BS > 0): the streamed
// schedule, a grid of resident workgroups that each run every G-th unit.
template <int MODE, int U, int BS, int PATH = 0>
__global__ void __launch_bounds__((k5_nt<MODE, U>), (k5_min_blocks<MODE, U>))
    k5(K5Member single, const K5Member *members, const int2 *items, int64_t nitems, int32_t *counter) {
    __shared__ __attribute__((aligned(1024))) uint8_t st0[k5_stage_bytes<MODE, U>];
    __shared__ __attribute__((aligned(1024))) uint8_t st1[k5_stage_bytes<MODE, U>];
    __shared__ __attribute__((aligned(16))) uint8_t meta[k5_meta_bytes<U>];
    if constexpr (BS != 0 && PATH == 1) {
        if (!dense_ok(single)) return;
        process_unit<MODE, U, BS, true>(single, launch_unit(single), st0, st1, meta);
    } else if constexpr (BS != 0 && PATH == 2) {
        if (dense_ok(single)) return;
        process_unit<MODE, U, BS, false>(single, launch_unit(single), st0, st1, meta);
    } else if constexpr (BS != 0 && PATH == 3) {
        static_assert(U <= 128 && MODE != QBSM_OZAKI_I8, "streamed schedule: tile-skipping units below 256");
        process_stream<MODE, U, BS>(single, st0, st1, meta);
    } else if constexpr (BS != 0) {
        process_sel<MODE, U, BS>(single, launch_unit(single), st0, st1, meta);
    } else {
        __shared__ int s_item;
        for (;;) {
            if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
            __syncthreads();
            const int it = s_item;
            __syncthreads();
            if ((int64_t)it >= nitems) break;
            const int2 w = items[it];
            const K5Member mm = members[w.x];
            process_any<MODE, U>(mm, w.y, st0, st1, meta);
        }
    }
}

#ifdef QB_K5_OZAKI_UNIT
// The Ozaki mode at unit 128: 2 x 2 leaves of 64, four waves of one 64 x 64
// output leaf each.  One step (the six slices of two A leaves and two B
// leaves, 96 KB) leaves no LDS for a second stage, so the step's fragments
// are double-buffered in registers instead: every wave reads all of its
// fragments of the step (column tile 0 first), multiplies column tile 0,
// and once every wave's reads are complete (a barrier) the next step's copy
// goes out into the same stage while the other column tiles run from
// registers.  Against unit 64 every copied leaf serves two leaf products,
// which halves the operand traffic.  A wave whose leaf product is absent in
// a step reads nothing and multiplies nothing (its leaves may be nil), but
// issues its share of the copy and meets both barriers.
template <int BS, bool NF>
__device__ void process_unit_oz128(const K5Member &m, int u, uint8_t *stage, uint8_t *meta) {
    constexpr int MODE = QBSM_OZAKI_I8, U = 128;
    using G = Geo<MODE, U, BS>;
    using M = MT<MODE>;
    constexpr int LPU = G::LPU, NSUB = G::NSUB, TPW = G::TPW, PARTS = M::PARTS;
    static_assert(G::WT == BS && G::NCHUNK == 1 && G::NGROUPS == 1 && M::SUBS == 1,
                  "one wave per output leaf, one K chunk per leaf, one read group");
    const int w = uni((int)threadIdx.x >> 6);
    const int wr = w / G::WPS, wc = w % G::WPS;
    const int lane = threadIdx.x & 63, l16 = lane & 15, pc = lane >> 4;
    const int bit = wr * LPU + wc;  // the wave's leaf product among a step's bits

    typename M::Acc acc[TPW][TPW];
#pragma unroll
    for (int a = 0; a < TPW; ++a)
#pragma unroll
        for (int b = 0; b < TPW; ++b) acc[a][b] = typename M::Acc{};
    OzExp<TPW> ex{};

    const int p0 = uni(m.ustart[u]), p1 = uni(m.ustart[u + 1]);
    const Meta mt = meta_view(meta, G::CAP);
    const CopyLane cl = copy_lane<MODE, U, BS>(m, w);
    const uint32_t chunk_bytes = (uint32_t)((int64_t)m.chunkStrideL * (int64_t)sizeof(typename G::T));
    const uint8_t *Ab = stage, *Bb = stage + PARTS * G::ARRB;
    // the four row tiles of column tile tn: integer sums, then their flushes
    auto column = [&](typename M::Frag (&fa)[TPW][PARTS], typename M::Frag (&fb)[TPW][PARTS], int tn) {
        typename M::Part pt[TPW];
#pragma unroll
        for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int k = 0; k < M::NSUMS; ++k) pt[t].s[k] = i4{0, 0, 0, 0};
        M::template mma_parts<TPW>(pt, fa, fb[tn]);
#pragma unroll
        for (int tm = 0; tm < TPW; ++tm) M::template flush<NF>(acc[tm][tn], pt[tm], ex.er[tm], ex.ec[tn]);
    };
    for (int b0 = p0; b0 < p1; b0 += G::CAP) {
        const int nb = uni((p1 - b0) < G::CAP ? (p1 - b0) : G::CAP);
        __syncthreads();  // LDS (stage, metadata) of the previous batch or unit is free
        load_meta<MODE, U, BS>(m, mt, b0, nb);
        __syncthreads();
        Step st = first_step<LPU, NSUB>(mt, nb, 0);
        Advance nxa;
        nxa.nx = st;
        nxa.addrs = 0;
        if (st.i < nb) {
            const uint64_t addrs = copy_addr<MODE, U, BS>(mt, st.i, st.kb, 0, cl, chunk_bytes);
#pragma unroll
            for (int k = 0; k < G::PER_WAVE; ++k) issue_one<MODE, U, BS>(addrs, k, stage, w);
            // exponents only of leaves that exist (a nil leaf has no block)
            if ((st.km >> bit) & 1u) oz_load_exp<MODE, U, BS>(mt, st.i, st.kb, wr, wc, ex);
            nxa = advance<MODE, U, BS>(mt, nb, st, addrs, cl, chunk_bytes);
        }
        while (st.i < nb) {
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this step's copies and exponents
            __syncthreads();
            const bool mine = ((st.km >> bit) & 1u) != 0;
            typename M::Frag fa[TPW][PARTS], fb[TPW][PARTS];
            if (mine) {
#pragma unroll
                for (int t = 0; t < TPW; ++t)
#pragma unroll
                    for (int part = 0; part < PARTS; ++part)
                        fa[t][part].q[0] = lds_piece(Ab + part * G::ARRB, G::WT * wr + 16 * t + l16, G::LB, pc);
#pragma unroll
                for (int t = 0; t < TPW; ++t)
#pragma unroll
                    for (int part = 0; part < PARTS; ++part)
                        fb[t][part].q[0] = lds_piece(Bb + part * G::ARRB, G::WT * wc + 16 * t + l16, G::LB, pc);
                column(fa, fb, 0);
            }
            const bool more = nxa.nx.i < nb;
            OzExp<TPW> exn = ex;
            Advance nn = nxa;
            __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): every read of the stage is complete
            __syncthreads();
            if (more) {
#pragma unroll
                for (int k = 0; k < G::PER_WAVE; ++k) issue_one<MODE, U, BS>(nxa.addrs, k, stage, w);
                if ((nxa.nx.km >> bit) & 1u) oz_load_exp<MODE, U, BS>(mt, nxa.nx.i, nxa.nx.kb, wr, wc, exn);
                nn = advance<MODE, U, BS>(mt, nb, nxa.nx, nxa.addrs, cl, chunk_bytes);
            }
            if (mine) {
#pragma unroll
                for (int tn = 1; tn < TPW; ++tn) column(fa, fb, tn);
            }
            st = nxa.nx;
            nxa = nn;
            ex = exn;
        }
    }
    store_unit<MODE, U, BS>(m, u, acc, wr, wc);
}

__device__ __forceinline__ void oz128_sel(const K5Member &m, int u, uint8_t *stage, uint8_t *meta) {
    if ((*m.nfL | *m.nfR) != 0)
        process_unit_oz128<64, true>(m, u, stage, meta);
    else
        process_unit_oz128<64, false>(m, u, stage, meta);
}

// BS = 64: one launch of one multiply; BS = 0: the persistent work-list form
// (every member has 64 x 64 leaves).
template <int BS>
__global__ void __launch_bounds__(256, 1)
    k5_oz128(K5Member single, const K5Member *members, const int2 *items, int64_t nitems, int32_t *counter) {
    __shared__ __attribute__((aligned(1024))) uint8_t stage[Geo<QBSM_OZAKI_I8, 128, 64>::STAGEB];
    __shared__ __attribute__((aligned(16))) uint8_t meta[k5_meta_bytes<128>];
    if constexpr (BS != 0) {
        oz128_sel(single, launch_unit(single), stage, meta);
    } else {
        __shared__ int s_item;
        for (;;) {
            if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
            __syncthreads();
            const int it = s_item;
            __syncthreads();
            if ((int64_t)it >= nitems) break;
            const int2 wi = items[it];
            const K5Member mm = members[wi.x];
            oz128_sel(mm, wi.y, stage, meta);
        }
    }
}
#endif  // QB_K5_OZAKI_UNIT

template <int MODE, int U>
void launch_u(int bs, const K5Member *members, const int2 *items, int64_t nitems, int32_t *counter, int grid,
              int persistent, const K5Member &single, hipStream_t s) {
    constexpr int NT = k5_nt<MODE, U>;
    if (persistent == 1) {
        k5<MODE, U, 0><<<grid, NT, 0, s>>>(single, members, items, nitems, counter);
        return;
    }
    if (persistent == 3) {
        if constexpr (U == 128 && (MODE == QBSM_BF16 || MODE == QBSM_BF16X3 || MODE == QBSM_F64)) {
            if (bs == 64) {
                k5s<MODE, U, 64><<<grid, NT, 0, s>>>(single, members, items, nitems, counter);
                return;
            }
            if (bs == 128) {
                k5s<MODE, U, 128><<<grid, NT, 0, s>>>(single, members, items, nitems, counter);
                return;
            }
        }
        throw Error(QBSM_ERR_UNSUPPORTED, "single-stage schedule for this mode, unit and leaf size");
    }
    if (persistent == 2) {
        if constexpr (U <= 128 && MODE != QBSM_OZAKI_I8) {
            if (bs == 32) {
                k5<MODE, U, 32, 3><<<grid, NT, 0, s>>>(single, members, items, nitems, counter);
                return;
            }
            if (bs == 64) {
                k5<MODE, U, 64, 3><<<grid, NT, 0, s>>>(single, members, items, nitems, counter);
                return;
            }
            if constexpr (U >= 128) {
                if (bs == 128) {
                    k5<MODE, U, 128, 3><<<grid, NT, 0, s>>>(single, members, items, nitems, counter);
                    return;
                }
            }
        }
        throw Error(QBSM_ERR_UNSUPPORTED, "streamed schedule for this mode, unit and leaf size");
    }
    if constexpr (U <= 128 && MODE != QBSM_OZAKI_I8) {
        if (bs == 32) {
            k5<MODE, U, 32><<<grid, NT, 0, s>>>(single, members, items, nitems, counter);
            return;
        }
    }
    if constexpr (U >= 256) {
        // the two paths as two kernels (the plan's selection is known here;
        // the packs' finiteness is read by each workgroup)
        if (bs == 64 || bs == 128) {
            if (!single.select) {
                if (bs == 64) k5<MODE, U, 64, 1><<<grid, NT, 0, s>>>(single, members, items, nitems, counter);
                else k5<MODE, U, 128, 1><<<grid, NT, 0, s>>>(single, members, items, nitems, counter);
            }
            if (bs == 64) k5<MODE, U, 64, 2><<<grid, NT, 0, s>>>(single, members, items, nitems, counter);
            else k5<MODE, U, 128, 2><<<grid, NT, 0, s>>>(single, members, items, nitems, counter);
            return;
        }
    } else {
        if (bs == 64) {
            k5<MODE, U, 64><<<grid, NT, 0, s>>>(single, members, items, nitems, counter);
            return;
        }
        if constexpr (U >= 128) {
            if (bs == 128) {
                k5<MODE, U, 128><<<grid, NT, 0, s>>>(single, members, items, nitems, counter);
                return;
            }
        }
    }
    throw Error(QBSM_ERR_UNSUPPORTED, "leaf size for this unit side");
}

template <int MODE>
void launch_mode(int unit, int bs, const K5Member *members, const int2 *items, int64_t nitems, int32_t *counter,
                 int grid, int persistent, const K5Member &single, hipStream_t s) {
    switch (unit) {
        case 64: launch_u<MODE, 64>(bs, members, items, nitems, counter, grid, persistent, single, s); break;
        case 128:
            if constexpr (MODE != QBSM_OZAKI_I8) {
                launch_u<MODE, 128>(bs, members, items, nitems, counter, grid, persistent, single, s);
            } else {
#ifdef QB_K5_OZAKI_UNIT
                if (persistent)
                    k5_oz128<0><<<grid, 256, 0, s>>>(single, members, items, nitems, counter);
                else if (bs == 64)
                    k5_oz128<64><<<grid, 256, 0, s>>>(single, members, items, nitems, counter);
                else
                    throw Error(QBSM_ERR_UNSUPPORTED, "leaf size for this unit side");
#endif
            }
            break;
        case 256:
            // the 128 x 128 part of a wave holds 64 KB of accumulators in FP32
            // but twice that in FP64, beyond the register file
            if constexpr (MODE != QBSM_F64 && MODE != QBSM_OZAKI_I8) {
                launch_u<MODE, 256>(bs, members, items, nitems, counter, grid, persistent, single, s);
                break;
            }
            [[fallthrough]];
        default: throw Error(QBSM_ERR_UNSUPPORTED, "unit side for this mode");
    }
}

}  // namespace

#ifdef QB_K5_OZAKI_UNIT
// This translation unit (numeric_oz.hip) holds the Ozaki mode's kernels only.
void k5_launch_ozaki(int unit, int bs, const K5Member *members, const int2 *items, int64_t nitems, int32_t *counter,
                     int grid, int persistent, const K5Member &single, hipStream_t s) {
    launch_mode<QBSM_OZAKI_I8>(unit, bs, members, items, nitems, counter, grid, persistent, single, s);
}

const void *k5_kernel_ozaki(int unit, int bs) {
    if (unit == 64 && bs == 0) return reinterpret_cast<const void *>(&k5<QBSM_OZAKI_I8, 64, 0>);
    if (unit == 64 && bs == 64) return reinterpret_cast<const void *>(&k5<QBSM_OZAKI_I8, 64, 64>);
    if (unit == 128 && bs == 0) return reinterpret_cast<const void *>(&k5_oz128<0>);
    if (unit == 128 && bs == 64) return reinterpret_cast<const void *>(&k5_oz128<64>);
    return nullptr;
}
#else
// The Ozaki mode's kernels are compiled in numeric_oz.hip (see there).
void k5_launch_ozaki(int unit, int bs, const K5Member *members, const int2 *items, int64_t nitems, int32_t *counter,
                     int grid, int persistent, const K5Member &single, hipStream_t s);
const void *k5_kernel_ozaki(int unit, int bs);

void k5_launch(qbsm_mode mode, int unit, const K5Member *members, int32_t, const int2 *items, int64_t nitems,
               int32_t *counter, int grid, int persistent, const K5Member &single, hipStream_t s) {
    if (grid <= 0) return;
    const int bs = single.bs;
    switch (mode) {
        case QBSM_F64: launch_mode<QBSM_F64>(unit, bs, members, items, nitems, counter, grid, persistent, single, s); break;
        case QBSM_F32: launch_mode<QBSM_F32>(unit, bs, members, items, nitems, counter, grid, persistent, single, s); break;
        case QBSM_BF16: launch_mode<QBSM_BF16>(unit, bs, members, items, nitems, counter, grid, persistent, single, s); break;
        case QBSM_BF16X3: launch_mode<QBSM_BF16X3>(unit, bs, members, items, nitems, counter, grid, persistent, single, s); break;
        case QBSM_OZAKI_I8:
            k5_launch_ozaki(unit, bs, members, items, nitems, counter, grid, persistent, single, s);
            break;
        default: throw Error(QBSM_ERR_ARG, "mode");
    }
    QB_LAUNCH_CHECK();
}

// Resident workgroups per CU of the launched variant (bs = 0: persistent
// work-list variant).
int k5_occupancy(qbsm_mode mode, int unit, int bs) {
    int nb = 0;
    const int NT = mode == QBSM_OZAKI_I8 ? 256 : 64 * (unit >= 256 ? 4 : (unit / 64) * (unit / 64));
    const void *fn = nullptr;
#define QB_OCC(MD, UU, BB) \
    if (mode == MD && unit == UU && bs == BB) fn = reinterpret_cast<const void *>(&k5<MD, UU, BB>);
#define QB_OCC_M(MD)                                                                               \
    QB_OCC(MD, 64, 0) QB_OCC(MD, 64, 32) QB_OCC(MD, 64, 64) QB_OCC(MD, 128, 0) QB_OCC(MD, 128, 32) \
    QB_OCC(MD, 128, 64) QB_OCC(MD, 128, 128)
#define QB_OCC2(MD, UU, BB) \
    if (mode == MD && unit == UU && bs == BB) fn = reinterpret_cast<const void *>(&k5<MD, UU, BB, 1>);
#define QB_OCC_256(MD) QB_OCC(MD, 256, 0) QB_OCC2(MD, 256, 64) QB_OCC2(MD, 256, 128)
    QB_OCC_M(QBSM_F64) QB_OCC_M(QBSM_F32) QB_OCC_M(QBSM_BF16) QB_OCC_M(QBSM_BF16X3)
    QB_OCC_256(QBSM_F32) QB_OCC_256(QBSM_BF16) QB_OCC_256(QBSM_BF16X3)
#undef QB_OCC_256
#undef QB_OCC2
#undef QB_OCC_M
#undef QB_OCC
    if (mode == QBSM_OZAKI_I8) fn = k5_kernel_ozaki(unit, bs);
    QB_CHECK(fn, QBSM_ERR_UNSUPPORTED, "no kernel for this mode, unit and leaf size");
    QB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, NT, 0));
    return nb < 1 ? 1 : nb;
}

// The kernel's record of one multiply: the plan's work lists, the operands'
// unit-level descriptor tables and packs, and the output values.
K5Member member_from_views(const Plan &p, const int32_t *descL, const int32_t *descR, const PackView &vL,
                           const PackView &vR, void *C) {
    K5Member m{};
    m.ustart = p.ustart.p;
    m.ukey = p.ukey.p;
    m.pl = p.pl.p;
    m.pr = p.pr.p;
    m.pmask = p.pmask.p;
    m.descL = descL;
    m.descR = descR;
    m.cdesc = p.cdesc.p;
    m.packL = vL.ptr;
    m.packR = vR.ptr;
    m.C = C;
    m.leafStrideL = vL.leaf_stride;
    m.partStrideL = vL.part_stride;
    m.lineStrideL = vL.line_stride;
    m.chunkStrideL = vL.chunk_stride;
    m.leafStrideR = vR.leaf_stride;
    m.partStrideR = vR.part_stride;
    m.lineStrideR = vR.line_stride;
    m.chunkStrideR = vR.chunk_stride;
    QB_CHECK(m.chunkStrideL == m.chunkStrideR && m.partStrideL == m.partStrideR, QBSM_ERR_STATE,
             "operand packs differ in chunk geometry");
    m.nfL = vL.nonfinite;
    m.nfR = vR.nonfinite;
    m.out_rows = p.out_rows;
    m.out_cols = p.out_cols;
    m.nunits = (int32_t)p.nunits;
    m.bs = p.bs;
    m.s = p.s;
    m.lpu = p.lpu;
    m.transL = p.transL;
    m.transR = p.transR;
    m.select = p.spamm_tol > 0.0 ? 1 : 0;
    return m;
}

K5Member make_member(Plan &p, qbsm_mode mode, Matrix &out, hipStream_t s) {
    Tree &tL = matrix_tree(*p.L, p.D, s);
    Tree &tR = matrix_tree(*p.R, p.D, s);
    const Role roleL = p.transL ? ROLE_COL : ROLE_ROW, roleR = p.transR ? ROLE_ROW : ROLE_COL;
    if (p.L == p.R && roleL != roleR) matrix_pack_pair(*p.L, mode, s);
    const PackView vL = matrix_pack(*p.L, mode, roleL, s);
    const PackView vR = matrix_pack(*p.R, mode, roleR, s);
    return member_from_views(p, tree_desc(*p.L, tL, p.s, s), tree_desc(*p.R, tR, p.s, s), vL, vR,
                             out.storage == ST_F64 ? (void *)out.v64.p : (void *)out.v32.p);
}

void plan_check_current(const Plan &p) {
    QB_CHECK(p.L->pattern_id == p.patL && p.R->pattern_id == p.patR && (!p.M || p.M->pattern_id == p.patM),
             QBSM_ERR_STATE, "an operand's pattern changed after the symbolic phase");
}

void numeric_check(const Plan &p, qbsm_mode mode) {
    plan_check_current(p);
    QB_CHECK(!(mode == QBSM_F64 && p.unit >= 256), QBSM_ERR_UNSUPPORTED,
             "unit 256 serves the FP32-accumulating modes only");
    QB_CHECK(mode != QBSM_OZAKI_I8 || ((p.unit == 64 || p.unit == 128) && p.bs == 64), QBSM_ERR_UNSUPPORTED,
             "the Ozaki mode needs 64 x 64 leaves and unit 64 or 128");
}

void numeric_prepare_output(Plan &p, qbsm_mode mode, Matrix &out, hipStream_t s) {
    numeric_check(p, mode);
    QB_CHECK(&out != p.L && &out != p.R && &out != p.M, QBSM_ERR_ARG, "output aliases an operand");
    QB_CHECK(out.nrows == p.out_rows && out.ncols == p.out_cols && out.bs == p.bs, QBSM_ERR_SHAPE,
             "output shape or leaf size differs from the product");
    const Storage want = mode == QBSM_F64 || mode == QBSM_OZAKI_I8 ? ST_F64 : ST_F32;
    const int64_t nout = p.nout;
    // the same plan refilling its own output: pattern and storage are already in place
    // (masked outputs keep their zero blocks: only the plan's products are rewritten)
    matrix_settle(out, s);  // packs of out made ahead still read its values
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
    ++out.storage_id;
    out.nblk = nout;
    out.has_blocks = true;
    out.version++;
    out.pattern_id++;
    out.filled_by = p.id;
    out.trees.clear();
    out.packs.clear();
    out.stream = s;
}

// Resident workgroups per CU of the streamed kernel for (mode, unit, leaf
// size), and the device's CU count, looked up once per device.
static int stream_slots(qbsm_mode mode, int unit, int bs) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int>, int> cache;
    int dev = 0;
    QB_HIP(hipGetDevice(&dev));
    const auto key = std::make_tuple(dev, (int)mode, unit, bs);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    const void *fn = nullptr;
#define QB_ST(MD, UU, BB) \
    if (mode == MD && unit == UU && bs == BB) fn = reinterpret_cast<const void *>(&k5<MD, UU, BB, 3>);
#define QB_ST_M(MD) QB_ST(MD, 64, 32) QB_ST(MD, 64, 64) QB_ST(MD, 128, 32) QB_ST(MD, 128, 64) QB_ST(MD, 128, 128)
    QB_ST_M(QBSM_F64) QB_ST_M(QBSM_F32) QB_ST_M(QBSM_BF16) QB_ST_M(QBSM_BF16X3)
#undef QB_ST_M
#undef QB_ST
    int nb = 0;
    if (fn) {
        const int NT = 64 * (unit / 64) * (unit / 64);
        QB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, NT, 0));
        nb = std::max(nb, 1) * device_cu_count();
        // a multiple of the XCD count keeps every workgroup's units on its XCD
        if (nb >= 8) nb -= nb % 8;
    }
    cache[key] = nb;
    return nb;
}

// Measured on the random-block multiply (N = 65536, 128-wide leaves, about
// one leaf product per unit, where it was meant to pay): the streamed
// schedule is 1% faster in FP64 and 0.5-3.5% slower in FP32, BF16X3 and BF16
// (that kernel moves its L2-side traffic at the rate of a device copy), so
// the automatic choice is one workgroup per unit and the streamed schedule
// is taken only on request.
int numeric_stream_grid(const Plan &p, qbsm_mode mode) {
    if (p.sched != 2 || p.unit > 128 || mode == QBSM_OZAKI_I8 || p.nunits <= 0) return 0;
    const int64_t g = stream_slots(mode, p.unit, p.bs);
    if (g <= 0) return 0;
    return (int)std::min<int64_t>(g, p.nunits);
}

// The automatic schedule takes the single-stage kernel for FP64 plans at
// unit 128 without transposed operands (decay workload 142.8 -> 136.7 ms,
// banded N = 1e5 128.2 -> 116.2 ms, random blocks N = 65536 1.607 -> 1.356
// ms) and for BF16 and BF16X3 plans at unit 128 with at most 1.25
// unit-level pairs per unit (random-block multiply: BF16 0.284 -> 0.256 ms,
// BF16X3 0.371 -> 0.348 ms).  Measured slower, so not taken: the masked
// FP64 adjoints with a transposed operand (1.23 -> 1.33 ms for both), FP32
// (whose 128-wide leaves take four steps) and BF16X3 on dense units (21.1 ->
// 30.7 ms on the decay workload).
bool numeric_single_stage(const Plan &p, qbsm_mode mode) {
    if (p.sched != 0 || p.unit != 128 || (p.bs != 64 && p.bs != 128) || p.nunits <= 0) return false;
    if (mode == QBSM_F64) return !p.transL && !p.transR;
    return (mode == QBSM_BF16 || mode == QBSM_BF16X3) && 4 * p.npairs <= 5 * p.nunits;
}

void numeric_launch(Plan &p, qbsm_mode mode, Matrix &out, hipStream_t s) {
    if (!p.nunits) return;
    K5Member m = make_member(p, mode, out, s);
    ProfScope prof(PROF_NUMERIC, s);
    const int sg = numeric_stream_grid(p, mode);
    if (sg > 0)
        k5_launch(mode, p.unit, nullptr, 1, nullptr, 0, nullptr, sg, 2, m, s);
    else if (numeric_single_stage(p, mode))
        k5_launch(mode, p.unit, nullptr, 1, nullptr, 0, nullptr, (int)p.nunits, 3, m, s);
    else
        k5_launch(mode, p.unit, nullptr, 1, nullptr, 0, nullptr, (int)p.nunits, 0, m, s);
}

// ------------------------------------------------------------------ batched
void batch_settle(Batch &b, hipStream_t s) {
    for (Plan *p : b.plans) plan_check_current(*p);
    for (size_t i = 0; i < b.outs.size(); ++i) {
        const Matrix &o = *b.outs[i];
        const void *v = o.storage == ST_F64 ? (const void *)o.v64.p : (const void *)o.v32.p;
        QB_CHECK(v == b.out_vals[i] && o.pattern_id == b.out_pattern[i], QBSM_ERR_STATE,
                 "a batch output was replaced after the batch was created");
    }
    for (auto &j : b.packs) {
        Pack &pk = j.m->packs[std::make_pair((int)j.mode, (int)j.role)];
        // a re-stored operand may get a buffer at the old address, so the
        // storage counter, not the address, tells whether the values moved
        QB_CHECK(j.m->storage_id == j.storage && pk.buf.p == j.buf && pk.buf.n == j.bytes, QBSM_ERR_STATE,
                 "an operand's values were re-stored after the batch was created (create the batch again)");
        pk.settle(s);
    }
}

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
#endif  // QB_K5_OZAKI_UNIT

}  // namespace qbsm
