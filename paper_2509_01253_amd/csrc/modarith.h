// modarith.h -- exact 64-bit modular arithmetic for gfx950 integer ALUs and host setup.
//
// Device side:
//   shoup_lazy(a, w, w', q)  a * w mod q in [0, 2q) for any a < 2^64, w < q, with the
//                            precomputed w' = floor(w 2^64 / q) (Shoup 2008; Harvey 2014)
//   redc(T)                  Montgomery reduction (Montgomery 1985): T 2^-64 mod q in
//                            [0, q) for T < q 2^64, with mont_neg_inv = -q^-1 mod 2^64
//   mont_mul(a, b~)          a * b mod q when b~ = b 2^64 mod q (Montgomery form)
// Products are built from 32x32->64 multiplies (v_mad_u64_u32 / v_mul_hi_u32).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fl {

typedef unsigned __int128 u128;

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

__device__ __forceinline__ uint64_t shoup_lazy(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    uint64_t h = mulhi64(a, wp);
    return a * w - h * q;
}

__device__ __forceinline__ uint64_t csub(uint64_t a, uint64_t q) { return a >= q ? a - q : a; }

__device__ __forceinline__ uint64_t shoup(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    return csub(shoup_lazy(a, w, wp, q), q);
}

__device__ __forceinline__ uint64_t add_mod(uint64_t a, uint64_t b, uint64_t q) { return csub(a + b, q); }
__device__ __forceinline__ uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }

// 128-bit accumulator as two 64-bit words
struct Acc128 {
    uint64_t lo, hi;
};

__device__ __forceinline__ void mac128(Acc128 &acc, uint64_t a, uint64_t b) {
    uint64_t plo = a * b;
    uint64_t phi = mulhi64(a, b);
    uint64_t nlo = acc.lo + plo;
    acc.hi += phi + (nlo < plo ? 1 : 0);
    acc.lo = nlo;
}

// Montgomery reduction of T = hi*2^64 + lo < q*2^64 -> T*2^-64 mod q in [0, q)
__device__ __forceinline__ uint64_t redc(uint64_t lo, uint64_t hi, uint64_t q, uint64_t ninv) {
    uint64_t m = lo * ninv;             // T + m q = 0 (mod 2^64)
    uint64_t mq_lo = m * q;
    uint64_t mq_hi = mulhi64(m, q);
    uint64_t carry = (lo + mq_lo < lo) ? 1 : 0;  // low word sums to 0 mod 2^64; carry iff lo != 0
    uint64_t t = hi + mq_hi + carry;    // < 2q
    return csub(t, q);
}

__device__ __forceinline__ uint64_t redc(const Acc128 &a, uint64_t q, uint64_t ninv) { return redc(a.lo, a.hi, q, ninv); }

__device__ __forceinline__ uint64_t mont_mul(uint64_t a, uint64_t b_mont, uint64_t q, uint64_t ninv) {
    return redc(a * b_mont, mulhi64(a, b_mont), q, ninv);
}

// ---------------------------------------------------------------------------
// host helpers (context setup only)
// ---------------------------------------------------------------------------
inline uint64_t h_mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
inline uint64_t h_powmod(uint64_t a, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = h_mulmod(r, a, q);
        a = h_mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}
inline uint64_t h_invmod(uint64_t a, uint64_t q) { return h_powmod(a % q, q - 2, q); }  // q prime
inline uint64_t h_shoup(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }
inline uint64_t h_to_mont(uint64_t a, uint64_t q) { return (uint64_t)(((u128)(a % q) << 64) % q); }
inline uint64_t h_neg_inv64(uint64_t q) {
    // Newton iteration for q^-1 mod 2^64 (q odd), then negate
    uint64_t x = q;  // correct to 3 bits
    for (int i = 0; i < 6; ++i) x *= 2 - q * x;
    return (uint64_t)0 - x;
}

}  // namespace fl
