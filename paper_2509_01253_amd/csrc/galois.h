// galois.h -- the automorphism X -> X^g as an index map of the NTT domain.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fl {

// Slot k of the bit-reversed NTT order holds a(psi^(2 brv(k) + 1)); sigma_g(a) at slot k
// is a at the slot of exponent (2 brv(k) + 1) g mod 2N.  A 16-aligned group of 16
// slots (fixed low bits of the exponent) maps onto another 16-aligned group, and a
// 64-aligned block onto a 64-aligned block.
__device__ __forceinline__ int auto_index(int k, uint32_t g, int log_n) {
    uint32_t b = __builtin_bitreverse32((uint32_t)k) >> (32 - log_n);
    uint32_t e = ((2u * b + 1u) * g) & ((2u << log_n) - 1u);
    return (int)(__builtin_bitreverse32((e - 1u) >> 1) >> (32 - log_n));
}

}  // namespace fl
