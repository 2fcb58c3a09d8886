// Host build of the device modular arithmetic (modarith.h) checked against 128-bit
// integers: Montgomery reduction of lazy sums of up to 32 (16) products, restarted at a
// reduced value, for the packed 28-bit accumulator (moduli < 2^55) and the 128-bit one
// (moduli < 2^60), with operands at the edges [0, q); and the Shoup product with the
// 53-bit companion (moduli < 2^50) over inputs in [0, 4q).
#include <cstdint>
#include <cstdio>
#include <random>
#define __device__
#define __forceinline__ inline
#define __host__
static inline uint64_t __umul64hi(uint64_t a, uint64_t b) { return (uint64_t)(((unsigned __int128)a * b) >> 64); }
static inline uint32_t __umulhi(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }
#define HIP_INCLUDE_HIP_HIP_RUNTIME_H
#include "modarith.h"
using namespace fl;

template <bool SMALL>
static long check(uint64_t q, std::mt19937_64 &rng, long *tot) {
    const uint64_t ninv = h_neg_inv64(q);
    const uint64_t rinv = h_invmod(h_powmod(2, 64, q), q);
    long bad = 0;
    for (int it = 0; it < 200000; ++it) {
        const int n = (it & 16) ? LazyAcc<SMALL>::TERMS : 1 + rng() % LazyAcc<SMALL>::TERMS;
        const bool seeded = it & 4;
        const uint64_t v = (it & 8) ? q - 1 : rng() % q;
        LazyAcc<SMALL> A;
        A.zero();
        if (seeded) {
            A.set(v);
            ++*tot;
            if (A.value() != v) ++bad;
        }
        unsigned __int128 ref = 0;
        for (int t = 0; t < n; ++t) {
            const uint64_t a = (it & 1) ? q - 1 - (rng() % 3) : rng() % q, b = (it & 2) ? q - 1 : rng() % q;
            A.mac(LazyAcc<SMALL>::prep(a), LazyAcc<SMALL>::prep(b));
            ref += (unsigned __int128)a * b;
        }
        // expected: v + ref 2^-64 mod q
        uint64_t want = h_mulmod((uint64_t)(ref % q), rinv, q);
        if (seeded) want = (uint64_t)(((unsigned __int128)want + v) % q);
        ++*tot;
        if (A.reduce(q, ninv) != want) ++bad;
    }
    return bad;
}

// Shoup product with the 53-bit companion (moduli < 2^50): a * w mod q in [0, 2q) for
// every a < 4q, w < q, including the edges
static long check53(uint64_t q, std::mt19937_64 &rng, long *tot) {
    long bad = 0;
    for (int it = 0; it < 400000; ++it) {
        const uint64_t w = (it & 1) ? q - 1 - rng() % 3 : (it & 2) ? rng() % 3 : rng() % q;
        const uint64_t a = (it & 4) ? 4 * q - 1 - rng() % 3 : (it & 8) ? rng() % 3 : rng() % (4 * q);
        const uint64_t r = shoup53_lazy(a, w, h_shoup53(w, q), q);
        const uint64_t want = (uint64_t)((unsigned __int128)a * w % q);
        ++*tot;
        if (r >= 2 * q || r % q != want) ++bad;
    }
    return bad;
}

int main() {
    std::mt19937_64 rng(1);
    const uint64_t small_q[] = {(1ull << 55) - 55, 1125899906826241ull, 68719403009ull};
    const uint64_t big_q[] = {(1ull << 56) - 27, 576460752303421441ull /* < 2^60 */, 1125899906826241ull};
    long bad = 0, tot = 0;
    for (uint64_t q : small_q) bad += check<true>(q, rng, &tot);
    for (uint64_t q : big_q) bad += check<false>(q, rng, &tot);
    const uint64_t q50[] = {(1ull << 50) - 27, 1125899906826241ull, 68719403009ull, 65537ull, 3ull};
    for (uint64_t q : q50) bad += check53(q, rng, &tot);
    printf("checked %ld, mismatches %ld\n", tot, bad);
    return bad != 0;
}
