// Device-side number-format helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace qbsm {

// bfloat16 bits of an FP64 value, round-to-nearest-even straight from FP64
// (no intermediate rounding to binary32).  bfloat16 keeps 8 significant bits
// and the binary32 exponent range: subnormals are multiples of 2^-133 and
// results of magnitude >= 2^128 overflow to infinity.
__device__ __forceinline__ uint16_t bf16_rne_bits(double x) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint16_t sign = (uint16_t)((u >> 48) & 0x8000u);
    if (x != x) return (uint16_t)(sign | 0x7FC0u);
    const double ax = fabs(x);
    if (ax < 0x1p-126) {
        // count of 2^-133 quanta, rounded half-to-even (rint), at most 128
        const double q = rint(ax * 0x1p133);
        return (uint16_t)(sign | (uint16_t)q);
    }
    // keep the top 7 explicit mantissa bits of the binary64 value: round the
    // 45 dropped bits to nearest, ties to even; a carry moves into the exponent
    uint64_t v = u & 0x7FFFFFFFFFFFFFFFull;
    const uint64_t lsb = (v >> 45) & 1ull;
    v += 0x00000FFFFFFFFFFFull + lsb;
    v &= ~0x00001FFFFFFFFFFFull;
    const double r = __longlong_as_double((long long)v);
    if (r >= 0x1p128) return (uint16_t)(sign | 0x7F80u);
    const float f = (float)r;  // exact: 8 significant bits, binary32 range
    return (uint16_t)(sign | (uint16_t)(__float_as_uint(f) >> 16));
}

__device__ __forceinline__ double bf16_bits_to_double(uint16_t h) {
    return (double)__uint_as_float(((uint32_t)h) << 16);
}

// Swizzle of the 16-byte pieces of a packed operand line (64 or 128 bytes):
// piece p of line l is stored at slot p ^ piece_swizzle(l, LB).  Shared by
// the pack kernel (writer) and the leaf-product kernel (LDS reader).
__device__ __forceinline__ int piece_swizzle(int line, int LB) {
    return LB == 128 ? (line & 7) : ((line >> 1) & 3);
}

}  // namespace qbsm
