// Numeric phase for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid allocation).
//
// The operand packs (the Ozaki mode's line exponents are part of its packs)
// and their non-finite flags go to one file-scope device array per GPU
// instead of allocator memory, and the
// result goes to a caller-owned array.  Everything else is the regular
// numeric phase: the same pack kernels and the same leaf-product kernel.
#include <mutex>

#include "common.h"

namespace qbsm {

namespace {

// The scratch array.  In host code its name is only a stand-in for the
// symbol: the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) uint8_t scratch[QBSM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t *g_scratch[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the
// first call made with that device current).
uint8_t *scratch_ptr() {
    int dev = 0;
    QB_HIP(hipGetDevice(&dev));
    QB_CHECK(dev >= 0 && dev < kMaxDevices, QBSM_ERR_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        QB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        QB_CHECK(p, QBSM_ERR_HIP, "no device address for the scratch array");
        g_scratch[dev] = static_cast<uint8_t *>(p);
    }
    return g_scratch[dev];
}

constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// The plan's unit-level descriptor table of one operand, as made by the
// symbolic phase (nothing is built here).
const int32_t *existing_desc(const Matrix &m, int D, int s) {
    if (s == 0) return nullptr;
    auto it = m.trees.find(D);
    QB_CHECK(it != m.trees.end(), QBSM_ERR_STATE, "an operand's quadtree is gone (run the symbolic phase again)");
    const Tree &t = *it->second;
    if (s == 1) return t.D >= 1 ? t.child[t.D - 1].p : nullptr;
    auto d = t.desc.find(s);
    QB_CHECK(d != t.desc.end(), QBSM_ERR_STATE, "an operand's unit descriptors are gone (run the symbolic phase again)");
    return d->second.p;
}

// Scratch layout of one call: [left pack][right pack][2 flags], each part
// 256-byte aligned; the right pack is absent when both sides use the same
// pack (the same matrix in the same role).
struct Layout {
    size_t packL = 0, packR = 0, flags = 0, total = 0;
};

Layout layout(const Plan &p, qbsm_mode mode, bool shared) {
    Layout l;
    size_t off = 0;
    l.packL = off;
    off += up(pack_bytes(*p.L, mode));
    l.packR = shared ? l.packL : off;
    if (!shared) off += up(pack_bytes(*p.R, mode));
    l.flags = off;
    off += up(2 * sizeof(int32_t));
    l.total = off;
    return l;
}

}  // namespace

}  // namespace qbsm

using namespace qbsm;

extern "C" qbsm_status qbsm_multiply_numeric_noalloc(qbsm_plan plan, qbsm_mode mode, void *out_vals,
                                                     void *stream) {
    try {
        QB_CHECK(plan, QBSM_ERR_ARG, "null plan");
        QB_CHECK(mode == QBSM_F64 || mode == QBSM_F32 || mode == QBSM_BF16 || mode == QBSM_BF16X3 ||
                     mode == QBSM_OZAKI_I8,
                 QBSM_ERR_ARG, "unknown mode");
        QB_CHECK(plan->p, QBSM_ERR_ARG, "null plan");
        Plan &p = *plan->p;
        hipStream_t s = static_cast<hipStream_t>(stream);
        numeric_check(p, mode);
        const int64_t nout = p.nout;
        QB_CHECK(nout == 0 || out_vals, QBSM_ERR_ARG, "null output array");
        const Role roleL = p.transL ? ROLE_COL : ROLE_ROW, roleR = p.transR ? ROLE_ROW : ROLE_COL;
        const bool shared = p.L == p.R && roleL == roleR;
        const Layout l = layout(p, mode, shared);
        QB_CHECK(l.total <= (size_t)QBSM_NOALLOC_SCRATCH_BYTES, QBSM_ERR_UNSUPPORTED,
                 "operand packs of " + std::to_string(l.total) + " bytes exceed the " +
                     std::to_string((size_t)QBSM_NOALLOC_SCRATCH_BYTES) + "-byte scratch array");
        const bool f64out = mode == QBSM_F64 || mode == QBSM_OZAKI_I8;
        const size_t out_bytes = (size_t)nout * p.bs * p.bs * (f64out ? sizeof(double) : sizeof(float));
        // a masked plan's output keeps the mask's pattern: blocks without
        // products read as zero
        if (p.M && out_bytes) fill_bytes_zero(out_vals, out_bytes, s);
        if (!p.nunits) return QBSM_OK;
        const int32_t *dL = existing_desc(*p.L, p.D, p.s);
        const int32_t *dR = existing_desc(*p.R, p.D, p.s);
        // (packs made ahead on the library's side stream write their own
        // buffers and only read the values, so nothing here waits for them)
        for (const Matrix *m : {p.L, p.R})
            QB_CHECK(m->has_blocks && (m->v64.p || m->v32.p), QBSM_ERR_STATE, "operand without values");
        uint8_t *base = scratch_ptr();
        int32_t *flags = reinterpret_cast<int32_t *>(base + l.flags);
        pack_into(*p.L, mode, roleL, base + l.packL, flags, s);
        if (!shared) pack_into(*p.R, mode, roleR, base + l.packR, flags + 1, s);
        const PackView vL = pack_view(*p.L, mode, base + l.packL, flags);
        const PackView vR = pack_view(*p.R, mode, base + l.packR, shared ? flags : flags + 1);
        const K5Member m = member_from_views(p, dL, dR, vL, vR, out_vals);
        QB_CHECK(m.chunkStrideL == m.chunkStrideR && m.partStrideL == m.partStrideR, QBSM_ERR_STATE,
                 "operand packs differ in chunk geometry");
        k5_launch(mode, p.unit, nullptr, 1, nullptr, 0, nullptr, (int)p.nunits, 0, m, s);
        return QBSM_OK;
    } catch (const Error &e) {
        qbsm::set_last_error(e.what());
        return e.st;
    } catch (const std::exception &e) {
        qbsm::set_last_error(e.what());
        return QBSM_ERR_HIP;
    } catch (...) {
        qbsm::set_last_error("unknown failure");
        return QBSM_ERR_HIP;
    }
}
