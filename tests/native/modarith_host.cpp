// Host build of the device modular arithmetic (modarith.h) checked against 128-bit
// integers: Montgomery reduction of lazy sums of up to 16 products, restarted at a
// reduced value, for the packed 28-bit accumulator (moduli < 2^55) and the 128-bit one
// (moduli < 2^60), with operands at the edges [0, q).
#include <cstdint>
#include <cstdio>
#include <random>
#define __device__
#define __forceinline__ inline
#define __host__
static inline uint64_t __umul64hi(uint64_t a, uint64_t b) { return (uint64_t)(((unsigned __int128)a * b) >> 64); }
#define HIP_INCLUDE_HIP_HIP_RUNTIME_H
#include "modarith.h"
using namespace fl;

template <bool SMALL>
static long check(uint64_t q, std::mt19937_64 &rng, long *tot) {
    const uint64_t ninv = h_neg_inv64(q);
    const uint64_t rinv = h_invmod(h_powmod(2, 64, q), q);
    long bad = 0;
    for (int it = 0; it < 200000; ++it) {
        const int n = 1 + rng() % 16;
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

int main() {
    std::mt19937_64 rng(1);
    const uint64_t small_q[] = {(1ull << 55) - 55, 1125899906826241ull, 68719403009ull};
    const uint64_t big_q[] = {(1ull << 56) - 27, 576460752303421441ull /* < 2^60 */, 1125899906826241ull};
    long bad = 0, tot = 0;
    for (uint64_t q : small_q) bad += check<true>(q, rng, &tot);
    for (uint64_t q : big_q) bad += check<false>(q, rng, &tot);
    printf("checked %ld, mismatches %ld\n", tot, bad);
    return bad != 0;
}
