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

// a * w mod q in [0, 2q) for a < 2^52 and w < q < 2^50, with the companion of
// v = floor(w 2^53 / q) < 2^53 stored as (ph << 11) 2^32 + pl (v = ph 2^32 + pl, ph < 2^21).
// With a = ah 2^32 + al (ah < 2^20) and m = hi32(al pl) + ah pl + al ph < 2^54, the
// estimate (ah ph) 2^11 + floor(m / 2^21) drops only the low word of al pl, so it is
// floor(a v / 2^53) or one less; floor(a v / 2^53) is floor(a w / q) or one less since
// a / 2^53 < 1/2.  The estimate is floor(a w / q) or one less -- the 64-bit form's
// [0, 2q) -- from four 32-bit multiplies (the pre-shifted ph makes the last one a
// multiply-add).
//
// The result a w - qe q (mod 2^64) is formed as a w + qe (2^64 - q): the low words as
// two chained 32 x 32 -> 64 multiply-adds, the four cross terms only in the high word.
__device__ __forceinline__ uint64_t shoup53_lazy(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    const uint32_t al = (uint32_t)a, ah = (uint32_t)(a >> 32);
    const uint32_t pl = (uint32_t)wp, ph11 = (uint32_t)(wp >> 32), ph = ph11 >> 11;
    uint64_t m = (uint64_t)ah * pl + __umulhi(al, pl);
    asm("" : "+v"(m));  // keeps the high product as the first multiply-add's addend
    m += (uint64_t)al * ph;
    const uint64_t qe = (uint64_t)ah * ph11 + (m >> 21);
    const uint64_t nq = 0 - q;
    const uint32_t wl = (uint32_t)w, wh = (uint32_t)(w >> 32), nql = (uint32_t)nq, nqh = (uint32_t)(nq >> 32);
    const uint32_t el = (uint32_t)qe, eh = (uint32_t)(qe >> 32);
    const uint64_t lo = (uint64_t)al * wl + (uint64_t)el * nql;
    uint32_t x = ah * wl + al * wh + eh * nql + el * nqh;
    asm("" : "+v"(x));  // a 32-bit add into the high word, not a 64-bit one
    return (uint64_t)(uint32_t)lo | ((uint64_t)((uint32_t)(lo >> 32) + x) << 32);
}

// a - q unless that borrows (the borrow of the subtraction selects, no separate compare)
__device__ __forceinline__ uint64_t csub(uint64_t a, uint64_t q) {
    uint64_t r;
    return __builtin_sub_overflow(a, q, &r) ? a : r;
}

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

// Montgomery reduction of T = hi*2^64 + lo < 2q*2^64 -> T*2^-64 mod q in [0, q):
// (T + m q) / 2^64 < 3q, two conditional subtractions.
__device__ __forceinline__ uint64_t redc_wide(uint64_t lo, uint64_t hi, uint64_t q, uint64_t ninv) {
    uint64_t m = lo * ninv;
    uint64_t mq_lo = m * q;
    uint64_t mq_hi = mulhi64(m, q);
    uint64_t carry = (lo + mq_lo < lo) ? 1 : 0;
    uint64_t t = hi + mq_hi + carry;    // < 3q
    return csub(csub(t, 2 * q), q);
}

// Lazy sums of up to TERMS products a*b, Montgomery-reduced at the end.
//
// Small moduli (every q < 2^55): operands are split once into 28-bit halves packed in
// one word, pack28(a) = a0 | a1 << 32 with a = a0 + a1 2^28.  Then
//   a b = a0 b0 + (a0 b1 + a1 b0) 2^28 + a1 b1 2^56
// and every partial product is below 2^56 (a1 b1 below 2^54), so three 64-bit sums
// take 32 products without carries (s0 < 2^61, s1 < 2^62, s2 < 2^59 plus a restart
// value below 2^63): four 32x32->64 multiply-adds per product and nothing else.
// A reduced value v < q restarts a sum at v 2^64 (v 2^8 in the 2^56 sum; below 2^63).
__device__ __forceinline__ uint64_t pack28(uint64_t a) {
    return (a & 0xFFFFFFFull) | ((a >> 28) << 32);
}

struct Acc28 {
    uint64_t s0, s1, s2;  // weights 1, 2^28, 2^56
};

__device__ __forceinline__ void mac28(Acc28 &A, uint64_t pa, uint64_t pb) {
    const uint32_t a0 = (uint32_t)pa, a1 = (uint32_t)(pa >> 32), b0 = (uint32_t)pb, b1 = (uint32_t)(pb >> 32);
    A.s0 += (uint64_t)a0 * b0;
    A.s1 += (uint64_t)a0 * b1;
    A.s1 += (uint64_t)a1 * b0;
    A.s2 += (uint64_t)a1 * b1;
}

__device__ __forceinline__ uint64_t mont_mul(uint64_t a, uint64_t b_mont, uint64_t q, uint64_t ninv) {
    return redc(a * b_mont, mulhi64(a, b_mont), q, ninv);
}

// T = s0 + s1 2^28 + s2 2^56 < 2q 2^64 -> T 2^-64 mod q
__device__ __forceinline__ uint64_t redc28(const Acc28 &A, uint64_t q, uint64_t ninv) {
    const uint64_t m1 = A.s1 << 28, m2 = A.s2 << 56;
    uint64_t lo = A.s0 + m1;
    uint64_t hi = (A.s1 >> 36) + (A.s2 >> 8) + (lo < m1 ? 1 : 0);
    const uint64_t lo2 = lo + m2;
    hi += lo2 < m2 ? 1 : 0;
    return redc_wide(lo2, hi, q, ninv);
}

// A TERMS-term lazy accumulator over either representation: SMALL (all moduli < 2^55)
// uses Acc28 on packed operands (32 terms), otherwise full 128-bit products on plain
// operands (16 terms, moduli < 2^60).  prep(x) puts an operand in the form mac()
// takes.  set(v) restarts the sum at v 2^64 for a reduced v < q, so the Montgomery
// reduction of (v 2^64 + TERMS products) < 2q 2^64 (TERMS q < 2^64) returns
// v + (products) 2^-64 mod q; value() reads v back after set().
template <bool SMALL>
struct LazyAcc;

template <>
struct LazyAcc<true> {
    static constexpr int TERMS = 32;
    Acc28 a;
    __device__ __forceinline__ static uint64_t prep(uint64_t x) { return pack28(x); }
    __device__ __forceinline__ void zero() { a = Acc28{0, 0, 0}; }
    __device__ __forceinline__ void set(uint64_t v) { a = Acc28{0, 0, v << 8}; }
    __device__ __forceinline__ uint64_t value() const { return a.s2 >> 8; }
    __device__ __forceinline__ void mac(uint64_t px, uint64_t py) { mac28(a, px, py); }
    __device__ __forceinline__ uint64_t reduce(uint64_t q, uint64_t ninv) const { return redc28(a, q, ninv); }
};

template <>
struct LazyAcc<false> {
    static constexpr int TERMS = 16;
    Acc128 a;
    __device__ __forceinline__ static uint64_t prep(uint64_t x) { return x; }
    __device__ __forceinline__ void zero() { a = Acc128{0, 0}; }
    __device__ __forceinline__ void set(uint64_t v) { a = Acc128{0, v}; }
    __device__ __forceinline__ uint64_t value() const { return a.hi; }
    __device__ __forceinline__ void mac(uint64_t x, uint64_t y) { mac128(a, x, y); }
    __device__ __forceinline__ uint64_t reduce(uint64_t q, uint64_t ninv) const {
        return redc_wide(a.lo, a.hi, q, ninv);
    }
};

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
inline uint64_t h_shoup53(uint64_t w, uint64_t q) {
    const uint64_t v = (uint64_t)(((u128)w << 53) / q);  // < 2^53 for w < q
    return ((v >> 32) << 43) | (v & 0xffffffffu);         // high word pre-shifted by 11
}
inline uint64_t h_to_mont(uint64_t a, uint64_t q) { return (uint64_t)(((u128)(a % q) << 64) % q); }
inline uint64_t h_neg_inv64(uint64_t q) {
    // Newton iteration for q^-1 mod 2^64 (q odd), then negate
    uint64_t x = q;  // correct to 3 bits
    for (int i = 0; i < 6; ++i) x *= 2 - q * x;
    return (uint64_t)0 - x;
}

}  // namespace fl
