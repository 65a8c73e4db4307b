// The edge-to-slot hash of the device kernels (Section III-A: the processor of an edge; one
// independent function per group, Section III-B): a degree-3 polynomial over GF(2^61 - 1),
// evaluated in Horner form, mapped to [0, m) by the top bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rept_hash {

constexpr uint64_t kP61 = (1ull << 61) - 1;  // Mersenne prime of the edge hash

__device__ __forceinline__ uint64_t fold61(uint64_t r) {  // r < 2^64 -> [0, p)
    r = (r & kP61) + (r >> 61);
    return r >= kP61 ? r - kP61 : r;
}
// a * b mod p for a, b < 2^61, from the four 32 x 32 -> 64 bit partial products.  With
// 2^61 = 1 and 2^64 = 8 (mod p): a * b = 8 hh + mid 2^32 + ll, and mid 2^32 = (mid >> 29) +
// (mid mod 2^29) 2^32 (mod p); the five terms sum below 2^63.
__device__ __forceinline__ uint64_t mulmod61(uint64_t a, uint64_t b) {
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint64_t ll = (uint64_t)a0 * b0;                       // < 2^64
    const uint64_t mid = (uint64_t)a0 * b1 + (uint64_t)a1 * b0;  // < 2^62
    const uint64_t hh = (uint64_t)a1 * b1;                       // < 2^58
    return fold61((hh << 3) + (mid >> 29) + ((mid & 0x1fffffffull) << 32) + (ll & kP61) + (ll >> 61));
}
// slot of the undirected edge {x, y} for the group whose coefficients are c4[0..3]
__device__ __forceinline__ uint32_t slot_of(const uint64_t* c4, uint32_t m, uint32_t x, uint32_t y) {
    const uint32_t lo = x < y ? x : y, hi = x < y ? y : x;
    const uint64_t key = ((uint64_t)lo << 32) | hi;  // < 2^61 - 1 for ids below 2^29
    uint64_t h = c4[3];
    h = fold61(mulmod61(h, key) + c4[2]);
    h = fold61(mulmod61(h, key) + c4[1]);
    h = fold61(mulmod61(h, key) + c4[0]);
    return (uint32_t)__umul64hi(h << 3, (uint64_t)m);
}

}  // namespace rept_hash
