// modup.h -- the ModUp tile (centred fast base conversion of one key-switch digit),
// shared by the ModUp kernel and the persistent ModUp + forward-NTT launch.
#pragma once

#include "internal.h"
#include "modarith.h"

namespace fl {

// ModUp of digit j of batch entry t on the 256 coefficients x*256 .. x*256+255 (one
// per thread of a 256-thread workgroup): v_i = [x_i (Q_j/q_i)^-1]_{q_i} centred, and
// for every target modulus r outside the digit y_r = sum_i v_i (Q_j/q_i) mod r minus
// (number of negative v_i) Q_j mod r; the digit's own limbs are copied from `ntt`
// (the caller's choice of domain).  Digits past the entry's count are skipped.
__device__ __forceinline__ void modup_tile(const Batch &b, const ModConst *__restrict__ mods,
                                           const ModUpTab *__restrict__ tabs, const uint64_t *__restrict__ coef,
                                           int64_t coef_es, const uint64_t *__restrict__ ntt, int64_t ntt_es,
                                           uint64_t *__restrict__ digits, int64_t digits_es, int log_n, int L, int K,
                                           int alpha, int dnum, int x, int j, int t) {
    const int l = b.level[t];
    const int beta = (l + alpha - 1) / alpha;
    if (j >= beta) return;
    const int64_t N = (int64_t)1 << log_n;
    const int k = x * 256 + threadIdx.x;
    const ModUpTab &tab = tabs[(l - 1) * dnum + j];
    const int lo = tab.lo, cnt = tab.cnt;
    const uint64_t *xc = coef + t * coef_es;
    const uint64_t *xn = ntt + t * ntt_es;
    uint64_t *y = digits + t * digits_es + (int64_t)j * (L + K) * N;
    uint64_t v[MAX_ALPHA];
    uint64_t nneg = 0;
#pragma unroll
    for (int a = 0; a < MAX_ALPHA; ++a) {
        if (a < cnt) {
            const ModConst mc = mods[lo + a];
            uint64_t w = shoup(xc[(int64_t)(lo + a) * N + k], tab.inv_hat[a], tab.inv_hat_sh[a], mc.q);
            v[a] = w;
            nneg += w > mc.half ? 1 : 0;
            y[(int64_t)(lo + a) * N + k] = xn[(int64_t)(lo + a) * N + k];
        }
    }
    for (int e = 0; e < l + K; ++e) {
        if (e >= lo && e < lo + cnt) continue;
        const int slot = e < l ? e : L + (e - l);
        const ModConst mc = mods[slot];
        Acc128 acc{0, 0};
#pragma unroll
        for (int a = 0; a < MAX_ALPHA; ++a)
            if (a < cnt) mac128(acc, v[a], tab.hat_mont[a][slot]);
        uint64_t r = redc(acc, mc.q, mc.mont_neg_inv);
        if (nneg) r = sub_mod(r, mont_mul(nneg, tab.qj_mont[slot], mc.q, mc.mont_neg_inv), mc.q);
        y[(int64_t)slot * N + k] = r;
    }
}

}  // namespace fl
