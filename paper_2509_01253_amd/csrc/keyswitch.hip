// keyswitch.hip -- hybrid key switching pieces (hot-path rows a5, a6, a8).
//
//   ModUp      digit j of a level-l polynomial (coefficient domain) is extended to
//              every other modulus of B_l = {q_0..q_{l-1}, p_0..p_{K-1}} by the
//              centred fast base conversion: v_i = [x_i (Q_j/q_i)^-1]_{q_i} in
//              (-q_i/2, q_i/2], y_r = sum_i v_i (Q_j/q_i) mod r (Bajard et al. 2016).
//   inner      u_p = sum_j sigma_g(y_j) * evk_g[j].p over B_l in the NTT domain; the
//              automorphism is an index permutation there (hoisting: one ModUp
//              serves every rotation of the same ciphertext; Halevi-Shoup 2018).
//   ModDown    (u_p - conv_{P->q}(u_p)) * P^-1 mod q_i, centred conversion.
//   rescale    c'_i = (c_i - [c]_{q_{l-1}} centred) * q_{l-1}^-1 (coefficient domain).
//
// Layout of per-entry workspace buffers (slot = modulus index):
//   digits [dnum][L+K][N], u [2][L+K][N], md [2][L][N] (stride L), cts [2][stride][N].
// Every kernel maps one thread to one coefficient; grid.z is the batch entry.
#include <cmath>

#include "galois.h"
#include "internal.h"
#include "modarith.h"
#include "modup.h"

namespace fl {

// ---------------------------------------------------------------------------
// ModUp: grid (N/256, beta_max, n); the tile itself is modup_tile (modup.h)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_modup(Batch b, const ModConst *__restrict__ mods,
                                               const ModUpTab *__restrict__ tabs, const uint64_t *__restrict__ coef,
                                               int64_t coef_es, const uint64_t *__restrict__ ntt, int64_t ntt_es,
                                               uint64_t *__restrict__ digits, int64_t digits_es, int log_n, int L,
                                               int K, int alpha, int dnum) {
    modup_tile(b, mods, tabs, coef, coef_es, ntt, ntt_es, digits, digits_es, log_n, L, K, alpha, dnum, blockIdx.x,
               blockIdx.y, blockIdx.z);
}

int launch_modup(const Ctx *c, const Batch &b, const uint64_t *coef, int64_t coef_es, const uint64_t *ntt,
                 int64_t ntt_es, uint64_t *digits, int64_t digits_es, hipStream_t s) {
    if (b.n == 0) return FHELIN_OK;
    int lmax = 0;
    for (int t = 0; t < b.n; ++t) lmax = b.level[t] > lmax ? b.level[t] : lmax;
    int beta = (lmax + c->alpha - 1) / c->alpha;
    double units = 0, bytes = 0;
    for (int t = 0; t < b.n; ++t) {
        const double l = b.level[t];
        units += std::ceil(l / c->alpha) * (l + c->K) * c->N;
        bytes += 8.0 * c->N * (l + std::ceil(l / c->alpha) * (l + c->K));  // read l limbs, write the digits
    }
    ProfScope ps(c, s, PK_MODUP, units, bytes);
    hipLaunchKernelGGL(k_modup, dim3(c->N / 256, beta, b.n), dim3(256), 0, s, b, c->d_mods, c->d_modup, coef, coef_es,
                       ntt, ntt_es, digits, digits_es, c->log_n, c->L, c->K, c->alpha, c->dnum);
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

// ---------------------------------------------------------------------------
// inner product with the evaluation key: grid (N/256, l_max + K, n)
//   u_p[slot] (+)= sum_j sigma_g(y_j)[slot] * evk_g[j].p[slot]  (+ addend for p = 0)
// addend (optional, NTT domain, automorphism applied):
//   add_ext = 0: a Q ciphertext [2][add_stride]; adds P * sigma_g(c0) on the q slots
//   add_ext = 1: an extended ciphertext [2][L+K]; adds sigma_g(c0) on every slot
// ---------------------------------------------------------------------------
struct KsAdd {
    const uint64_t *src;  // null: no addend
    int64_t es;
    int ext;
    int accumulate;
};

// grid (N/256, L + K slots, entry groups of eg): slot s is q_s (entries with s < l)
// or p_{s-L}; the key rows of slot s are the same for every entry of the group, so a
// thread loads them once per key and reuses them.  With a rotation list (rot.n > 0)
// one launch runs every listed rotation of every entry: b.key[t] is then the base of
// the entry's key set, rotation i uses the key at index rot.key[i] of it and writes
// at element offset rot.out[i] of the entry's output; the entries' digits are
// gathered once per rotation while they are still in the caches.

// The digit count of an entry (its beta) is a run-time value; the loads of one entry's
// digits are issued together by dispatching to code compiled for exactly that count
// (no per-digit branches between the loads).
// sum_j d_j kb_j and sum_j d_j ka_j over the nb digits: every digit load is issued
// before the first product
template <bool SMALL, int MAXB>
__device__ __forceinline__ void ks_dot(int nb, LazyAcc<SMALL> &a0, LazyAcc<SMALL> &a1, const uint64_t *d,
                                       int64_t dstride, const uint64_t (&kb)[MAXB], const uint64_t (&ka)[MAXB]) {
    uint64_t v[MAXB];
#pragma unroll
    for (int j = 0; j < MAXB; ++j) {
        v[j] = 0;
        if (j < nb) v[j] = d[j * dstride];
    }
#pragma unroll
    for (int j = 0; j < MAXB; ++j) {
        if (j < nb) {
            const uint64_t dv = LazyAcc<SMALL>::prep(v[j]);
            a0.mac(dv, kb[j]);
            a1.mac(dv, ka[j]);
        }
    }
}

// MAXB >= dnum bounds the digits (the key rows a thread keeps in registers).
template <bool SMALL, int MAXB>
__global__ void __launch_bounds__(256) k_ks_inner(Batch b, const ModConst *__restrict__ mods,
                                                  const ModDownTab *__restrict__ mdt,
                                                  const uint64_t *__restrict__ digits, int64_t digits_es,
                                                  uint64_t *__restrict__ u, int64_t u_es, KsAdd add, KsRot rot,
                                                  int log_n, int L, int K, int alpha, int eg) {
    const int s = blockIdx.y;
    const int64_t N = (int64_t)1 << log_n;
    const int k = blockIdx.x * 256 + threadIdx.x;
    const ModConst mc = mods[s];
    uint64_t kb[MAXB], ka[MAXB];
    const int e_end = min(b.n, (int)(blockIdx.z + 1) * eg);
    const int n_rot = rot.n > 0 ? rot.n : 1;
    for (int ri = 0; ri < n_rot; ++ri) {
    const uint64_t *cur_key = nullptr;
    int cur_beta = 0;
    for (int t = blockIdx.z * eg; t < e_end; ++t) {
        const int l = b.level[t];
        if (s < L && s >= l) continue;
        const int beta = (l + alpha - 1) / alpha;
        const int kl = b.key_level[t];
        const uint64_t *kt = b.key[t];
        if (rot.n > 0) kt += (int64_t)rot.key[ri] * 2 * ((kl + alpha - 1) / alpha) * (kl + K) * N;
        if (kt != cur_key || beta > cur_beta) {
            // key rows of slot s: position s (q) or key_level + (s - L) (p) of each digit/part
            cur_key = kt;
            cur_beta = (kl + alpha - 1) / alpha;
            const int kp = s < L ? s : kl + (s - L);
            const int64_t kpart = (int64_t)(kl + K) * N;
            const uint64_t *key = cur_key + (int64_t)kp * N + k;
            // rows past the key's digits repeat its last one (never used), so every
            // load is unconditional and the loads go out together
#pragma unroll
            for (int j = 0; j < MAXB; ++j) {
                const int jr = j < cur_beta ? j : cur_beta - 1;
                kb[j] = key[(2 * jr) * kpart];
                ka[j] = key[(2 * jr + 1) * kpart];
            }
#pragma unroll
            for (int j = 0; j < MAXB; ++j) {
                kb[j] = LazyAcc<SMALL>::prep(kb[j]);
                ka[j] = LazyAcc<SMALL>::prep(ka[j]);
            }
        }
        const int src = auto_index(k, rot.n > 0 ? rot.g[ri] : b.g[t], log_n);
        const uint64_t *d = digits + t * digits_es + (int64_t)s * N + src;
        uint64_t *ut = u + t * u_es + (rot.n > 0 ? rot.out[ri] : 0);
        uint64_t *o0 = ut + (int64_t)s * N + k, *o1 = ut + ((int64_t)(L + K) + s) * N + k;
        // the addend and the running sum are read before the products so that their
        // loads are in flight together with the digits'
        const bool has_add = add.src && (add.ext || s < L);
        uint64_t addv = 0, prev0 = 0, prev1 = 0;
        if (has_add) addv = add.src[t * add.es + (int64_t)s * N + src];
        if (add.accumulate) {
            prev0 = *o0;
            prev1 = *o1;
        }
        LazyAcc<SMALL> a0, a1;
        a0.zero();
        a1.zero();
        ks_dot<SMALL, MAXB>(beta, a0, a1, d, (int64_t)(L + K) * N, kb, ka);
        uint64_t r0 = a0.reduce(mc.q, mc.mont_neg_inv), r1 = a1.reduce(mc.q, mc.mont_neg_inv);
        if (has_add) {
            if (add.ext) r0 = add_mod(r0, addv, mc.q);
            else r0 = add_mod(r0, mont_mul(addv, mdt->p_mont[s], mc.q, mc.mont_neg_inv), mc.q);
        }
        if (add.accumulate) {
            r0 = add_mod(r0, prev0, mc.q);
            r1 = add_mod(r1, prev1, mc.q);
        }
        *o0 = r0;
        *o1 = r1;
    }
    }
}

// Block coordinates of a 1-D grid of nx * ny * nz blocks in which the nz blocks of
// one (x, y) tile -- they read the same key rows for different entry groups -- are
// dispatched 8 apart: blocks go to the 8 XCDs round-robin, so these share an XCD
// and its L2 and run close together.  Needs nx * ny % 8 == 0 (else plain order).
struct BlockXYZ {
    int x, y, z;
};
__device__ __forceinline__ BlockXYZ xcd_block(int nx, int ny, int nz, bool swizzle) {
    const int lin = blockIdx.x;
    if (!swizzle) return {lin % nx, (lin / nx) % ny, lin / (nx * ny)};
    const int span = 8 * nz, q = lin / span, w = lin % span;
    const int xy = q * 8 + (w & 7);
    return {xy % nx, xy / nx, w >> 3};
}

// Every rotation of a list for every entry (hoisted baby steps): for rotation g and
// entry t, u = (P c0 + <D, evk_g>_0, <D, evk_g>_1) with the digits D and c0 taken at
// sigma_g.  sigma_g(a) at slot k is a at auto_index(k, g), so the value at slot m
// lands at k = auto_index(m, g^-1).  A thread owns one source slot m and EPT entries:
// their digits and addends at m stay in registers across all rotations, while keys
// are read, and outputs written, at k -- a permutation inside m's 64-slot block, so
// each wave still covers whole cache lines.  Each digit is read from memory once
// per launch instead of once per rotation.  The next rotation's key rows are
// loaded while the current one is multiplied.
// Block: 64 slots x 4 entry rows (wave w takes entries w, w + 4, ...); blocks (N/64,
// slots, ceil(n / 4 EPT)) on a 1-D grid (xcd_block).
template <bool SMALL, int MAXB, int EPT>
__global__ void __launch_bounds__(256) k_ks_rot(Batch b, const ModConst *__restrict__ mods,
                                                const ModDownTab *__restrict__ mdt,
                                                const uint64_t *__restrict__ digits, int64_t digits_es,
                                                uint64_t *__restrict__ u, int64_t u_es, KsAdd add, KsRot rot,
                                                int log_n, int L, int K, int alpha, int nz, bool swizzle) {
    const BlockXYZ bk = xcd_block((1 << log_n) / 64, L + K, nz, swizzle);
    const int s = bk.y;
    const int64_t N = (int64_t)1 << log_n;
    const int m = bk.x * 64 + (threadIdx.x & 63);
    // the wave index, known to be uniform: entry metadata is then read with scalar loads
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const ModConst mc = mods[s];
    const int64_t dstride = (int64_t)(L + K) * N;
    const bool has_add = add.src && (add.ext || s < L);
    bool live[EPT];
    int beta[EPT];
    uint64_t dv[EPT][MAXB], pa[EPT];
    int first = -1;
#pragma unroll
    for (int v = 0; v < EPT; ++v) {
        const int t = bk.z * 4 * EPT + w + 4 * v;
        live[v] = t < b.n && !(s < L && s >= b.level[t]);
        beta[v] = live[v] ? (b.level[t] + alpha - 1) / alpha : 0;
        pa[v] = 0;
#pragma unroll
        for (int j = 0; j < MAXB; ++j) dv[v][j] = 0;
        if (!live[v]) continue;
        if (first < 0) first = v;
        const uint64_t *d = digits + t * digits_es + (int64_t)s * N + m;
#pragma unroll
        for (int j = 0; j < MAXB; ++j)
            if (j < beta[v]) dv[v][j] = d[j * dstride];
        if (has_add) pa[v] = add.src[t * add.es + (int64_t)s * N + m];
    }
    if (first < 0) return;
#pragma unroll
    for (int v = 0; v < EPT; ++v) {
#pragma unroll
        for (int j = 0; j < MAXB; ++j) dv[v][j] = LazyAcc<SMALL>::prep(dv[v][j]);
        if (has_add && !add.ext) pa[v] = mont_mul(pa[v], mdt->p_mont[s], mc.q, mc.mont_neg_inv);
    }
    // key rows of slot s: position s (q) or key_level + (s - L) (p) of each digit/part;
    // rows past the key's digits repeat its last one (never used)
    auto key_rows = [&](int v, int ri, int k, uint64_t(&kb)[MAXB], uint64_t(&ka)[MAXB]) {
        const int t = bk.z * 4 * EPT + w + 4 * v;
        const int kl = b.key_level[t];
        const int kbeta = (kl + alpha - 1) / alpha;
        const int64_t kpart = (int64_t)(kl + K) * N;
        const uint64_t *key = b.key[t] + (int64_t)rot.key[ri] * 2 * kbeta * kpart +
                              (int64_t)(s < L ? s : kl + (s - L)) * N + k;
#pragma unroll
        for (int j = 0; j < MAXB; ++j) {
            const int jr = j < kbeta ? j : kbeta - 1;
            kb[j] = key[(2 * jr) * kpart];
            ka[j] = key[(2 * jr + 1) * kpart];
        }
    };
    const int t_first = bk.z * 4 * EPT + w + 4 * first;
    uint64_t nb[MAXB], na[MAXB];
    int k_next = auto_index(m, rot.ginv[0], log_n);
    key_rows(first, 0, k_next, nb, na);
    for (int ri = 0; ri < rot.n; ++ri) {
        const int k = k_next;
        uint64_t kb[MAXB], ka[MAXB];
#pragma unroll
        for (int j = 0; j < MAXB; ++j) {
            kb[j] = LazyAcc<SMALL>::prep(nb[j]);
            ka[j] = LazyAcc<SMALL>::prep(na[j]);
        }
        // the next rotation's keys are in flight during this one's products
        const int rn = ri + 1 < rot.n ? ri + 1 : ri;
        k_next = auto_index(m, rot.ginv[rn], log_n);
        key_rows(first, rn, k_next, nb, na);
        const uint64_t *kt_first = b.key[t_first];
#pragma unroll
        for (int v = 0; v < EPT; ++v) {
            if (!live[v]) continue;
            const int t = bk.z * 4 * EPT + w + 4 * v;
            LazyAcc<SMALL> a0, a1;
            a0.zero();
            a1.zero();
            if (b.key[t] == kt_first && b.key_level[t] == b.key_level[t_first]) {
#pragma unroll
                for (int j = 0; j < MAXB; ++j) {
                    if (j < beta[v]) {
                        a0.mac(dv[v][j], kb[j]);
                        a1.mac(dv[v][j], ka[j]);
                    }
                }
            } else {  // an entry of another key set (several clients in one batch)
                uint64_t ob[MAXB], oa[MAXB];
                key_rows(v, ri, k, ob, oa);
#pragma unroll
                for (int j = 0; j < MAXB; ++j) {
                    if (j < beta[v]) {
                        a0.mac(dv[v][j], LazyAcc<SMALL>::prep(ob[j]));
                        a1.mac(dv[v][j], LazyAcc<SMALL>::prep(oa[j]));
                    }
                }
            }
            uint64_t r0 = a0.reduce(mc.q, mc.mont_neg_inv), r1 = a1.reduce(mc.q, mc.mont_neg_inv);
            if (has_add) r0 = add_mod(r0, pa[v], mc.q);
            uint64_t *ut = u + t * u_es + rot.out[ri];
            ut[(int64_t)s * N + k] = r0;
            ut[((int64_t)(L + K) + s) * N + k] = r1;
        }
    }
}

// Giant-step sum: see KsSum.  Thread = slot k of limb s; a block takes EG entries and
// keeps their two running sums in registers across the terms, so the sum is written
// once instead of read and rewritten per term.  Within a term, every entry's digit
// and addend loads are issued before the first product.
template <bool SMALL, int MAXB, int EG>
__global__ void __launch_bounds__(256) k_ks_sum(Batch b, const ModConst *__restrict__ mods,
                                                const uint64_t *__restrict__ digits, int64_t digits_es,
                                                const uint64_t *__restrict__ add, int64_t add_es,
                                                const uint64_t *__restrict__ init, int64_t init_es,
                                                uint64_t *__restrict__ u, int64_t u_es, KsSum sum, int log_n, int L,
                                                int K, int alpha, int nz, bool swizzle) {
    const BlockXYZ bk = xcd_block((1 << log_n) / 256, L + K, nz, swizzle);
    const int s = bk.y;
    const int64_t N = (int64_t)1 << log_n, E = L + K;
    const int k = bk.x * 256 + threadIdx.x;
    const ModConst mc = mods[s];
    const int t0 = bk.z * EG;
    bool live[EG];
    int beta[EG];
    uint64_t acc[EG][2];
    int first = -1;
#pragma unroll
    for (int v = 0; v < EG; ++v) {
        const int t = t0 + v;
        live[v] = t < b.n && !(s < L && s >= b.level[t]);
        beta[v] = live[v] ? (b.level[t] + alpha - 1) / alpha : 0;
        acc[v][0] = acc[v][1] = 0;
        if (live[v] && init) {
            acc[v][0] = init[t * init_es + (int64_t)s * N + k];
            acc[v][1] = init[t * init_es + (E + s) * N + k];
        }
        if (live[v] && first < 0) first = v;
    }
    if (first < 0) return;
    auto key_rows = [&](int t, int ti, uint64_t(&kb)[MAXB], uint64_t(&ka)[MAXB]) {
        const int kl = b.key_level[t];
        const int kbeta = (kl + alpha - 1) / alpha;
        const int64_t kpart = (int64_t)(kl + K) * N;
        const uint64_t *key = b.key[t] + (int64_t)sum.key[ti] * 2 * kbeta * kpart +
                              (int64_t)(s < L ? s : kl + (s - L)) * N + k;
#pragma unroll
        for (int j = 0; j < MAXB; ++j) {
            const int jr = j < kbeta ? j : kbeta - 1;
            kb[j] = key[(2 * jr) * kpart];
            ka[j] = key[(2 * jr + 1) * kpart];
        }
    };
    const int t_first = t0 + first;
    for (int ti = 0; ti < sum.n; ++ti) {
        const int src = auto_index(k, sum.g[ti], log_n);
        uint64_t kb[MAXB], ka[MAXB];
        key_rows(t_first, ti, kb, ka);
        uint64_t dv[EG][MAXB], addv[EG];
#pragma unroll
        for (int v = 0; v < EG; ++v) {
            addv[v] = 0;
#pragma unroll
            for (int j = 0; j < MAXB; ++j) dv[v][j] = 0;
            if (!live[v]) continue;
            const int t = t0 + v;
            const uint64_t *d = digits + sum.dig_off[ti] + t * digits_es + (int64_t)s * N + src;
#pragma unroll
            for (int j = 0; j < MAXB; ++j)
                if (j < beta[v]) dv[v][j] = d[j * E * N];
            addv[v] = add[sum.add_off[ti] + t * add_es + (int64_t)s * N + src];
        }
#pragma unroll
        for (int j = 0; j < MAXB; ++j) {
            kb[j] = LazyAcc<SMALL>::prep(kb[j]);
            ka[j] = LazyAcc<SMALL>::prep(ka[j]);
        }
#pragma unroll
        for (int v = 0; v < EG; ++v) {
            if (!live[v]) continue;
            const int t = t0 + v;
            LazyAcc<SMALL> a0, a1;
            a0.zero();
            a1.zero();
            if (b.key[t] == b.key[t_first] && b.key_level[t] == b.key_level[t_first]) {
#pragma unroll
                for (int j = 0; j < MAXB; ++j) {
                    if (j < beta[v]) {
                        const uint64_t x = LazyAcc<SMALL>::prep(dv[v][j]);
                        a0.mac(x, kb[j]);
                        a1.mac(x, ka[j]);
                    }
                }
            } else {  // an entry of another key set (several clients in one batch)
                uint64_t ob[MAXB], oa[MAXB];
                key_rows(t, ti, ob, oa);
#pragma unroll
                for (int j = 0; j < MAXB; ++j) {
                    if (j < beta[v]) {
                        const uint64_t x = LazyAcc<SMALL>::prep(dv[v][j]);
                        a0.mac(x, LazyAcc<SMALL>::prep(ob[j]));
                        a1.mac(x, LazyAcc<SMALL>::prep(oa[j]));
                    }
                }
            }
            const uint64_t r0 = add_mod(a0.reduce(mc.q, mc.mont_neg_inv), addv[v], mc.q);
            acc[v][0] = add_mod(acc[v][0], r0, mc.q);
            acc[v][1] = add_mod(acc[v][1], a1.reduce(mc.q, mc.mont_neg_inv), mc.q);
        }
    }
#pragma unroll
    for (int v = 0; v < EG; ++v) {
        if (!live[v]) continue;
        const int t = t0 + v;
        u[t * u_es + (int64_t)s * N + k] = acc[v][0];
        u[t * u_es + (E + s) * N + k] = acc[v][1];
    }
}

// entries of more than one key set (several clients in one batch): the kernels then
// give every wave / block a single entry, so each entry's key rows are prefetched like
// a shared key set's instead of loaded one after another inside the loop
static bool mixed_keys(const Batch &b) {
    for (int t = 1; t < b.n; ++t)
        if (b.key[t] != b.key[0] || b.key_level[t] != b.key_level[0]) return true;
    return false;
}

int launch_ks_sum(const Ctx *c, const Batch &b, const KsSum &sum, const uint64_t *digits, int64_t digits_es,
                  const uint64_t *add, int64_t add_es, const uint64_t *init, int64_t init_es, uint64_t *u,
                  int64_t u_es, hipStream_t s) {
    if (b.n == 0) return FHELIN_OK;
    // work: 2 beta (l + K) N products per entry and term; bytes: per term the digits
    // (beta (l + K) limbs) and the addend (l + K), each distinct key once; the initial
    // value and the sum (2 (l + K) each) once
    double units = 0, bytes = 0;
    const double limb = 8.0 * c->N;
    for (int t = 0; t < b.n; ++t) {
        const double l = b.level[t], beta = std::ceil(l / c->alpha), e = l + c->K;
        units += sum.n * 2.0 * beta * e * c->N;
        bytes += limb * (sum.n * (beta * e + e) + (init ? 2 * e : 0) + 2 * e);
    }
    {
        const uint64_t *seen[MAX_BATCH];
        int n_seen = 0;
        for (int t = 0; t < b.n; ++t) {
            bool dup = false;
            for (int i = 0; i < n_seen; ++i) dup |= seen[i] == b.key[t];
            if (dup) continue;
            seen[n_seen++] = b.key[t];
            const double kl = b.key_level[t];
            bytes += sum.n * limb * 2 * std::ceil(kl / c->alpha) * (kl + c->K);
        }
    }
    ProfScope ps(c, s, PK_KS_SUM, units, bytes);
    const int n_digits = (c->L + c->alpha - 1) / c->alpha;
    const int nxy = c->N / 256 * (c->L + c->K);
#define FL_KSUM(SM, MB, EG) hipLaunchKernelGGL((k_ks_sum<SM, MB, EG>), dim3(nxy * ((b.n + EG - 1) / EG)), dim3(256), 0, s, \
                                               b, c->d_mods, digits, digits_es, add, add_es, init, init_es, u, u_es, sum, \
                                               c->log_n, c->L, c->K, c->alpha, (b.n + EG - 1) / EG, nxy % 8 == 0)
    if (mixed_keys(b)) {
        if (c->small) {
            if (n_digits <= 4) FL_KSUM(true, 4, 1);
            else if (n_digits <= 8) FL_KSUM(true, 8, 1);
            else FL_KSUM(true, 16, 1);
        } else {
            if (n_digits <= 4) FL_KSUM(false, 4, 1);
            else if (n_digits <= 8) FL_KSUM(false, 8, 1);
            else FL_KSUM(false, 16, 1);
        }
    } else if (c->small) {
        if (n_digits <= 4) FL_KSUM(true, 4, 8);
        else if (n_digits <= 8) FL_KSUM(true, 8, 4);
        else FL_KSUM(true, 16, 2);
    } else {
        if (n_digits <= 4) FL_KSUM(false, 4, 8);
        else if (n_digits <= 8) FL_KSUM(false, 8, 4);
        else FL_KSUM(false, 16, 2);
    }
#undef FL_KSUM
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

static uint32_t galois_inverse(uint32_t g, int log_n) {
    // g is odd: Newton's iteration x <- x (2 - g x) doubles the correct low bits
    uint32_t x = g;
    for (int i = 0; i < 5; ++i) x *= 2u - g * x;
    return x & ((2u << log_n) - 1u);
}

static int launch_ks_inner_impl(const Ctx *c, const Batch &b, const uint64_t *digits, int64_t digits_es, uint64_t *u,
                                int64_t u_es, KsAdd add, hipStream_t s, int eg, const KsRot &rot) {
    if (b.n == 0) return FHELIN_OK;
    const int n_rot = rot.n > 0 ? rot.n : 1;
    // work: 2 beta (l + K) N products per entry; bytes: digits beta (l + K) limbs, the
    // addend (l + K limbs extended, l limbs lifted), the accumulated sum read back, two
    // output polynomials, and each distinct key once (2 beta_k (l_k + K) limbs)
    double units = 0, bytes = 0;
    const double limb = 8.0 * c->N;
    const uint64_t *seen[MAX_BATCH];
    int n_seen = 0;
    for (int t = 0; t < b.n; ++t) {
        const double l = b.level[t], beta = std::ceil(l / c->alpha), e = l + c->K;
        units += n_rot * 2.0 * beta * e * c->N;
        // the digits are read once per launch (rotations of one launch re-read them from cache)
        bytes += limb * (beta * e + n_rot * 2 * e);
        if (add.src) bytes += limb * (add.ext ? e : l);
        if (add.accumulate) bytes += n_rot * limb * 2 * e;
        bool dup = false;
        for (int i = 0; i < n_seen; ++i) dup |= seen[i] == b.key[t];
        if (!dup) {
            seen[n_seen++] = b.key[t];
            const double kl = b.key_level[t];
            bytes += n_rot * limb * 2 * std::ceil(kl / c->alpha) * (kl + c->K);
        }
    }
    ProfScope ps(c, s, rot.n > 0 ? PK_KS_ROT : PK_KS_INNER, units, bytes);
    const int n_digits = (c->L + c->alpha - 1) / c->alpha;  // at most 16 (checked at context creation)
    if (rot.n > 0) {
        KsRot r = rot;
        for (int i = 0; i < r.n; ++i) r.ginv[i] = galois_inverse(r.g[i], c->log_n);
        const int nxy = c->N / 64 * (c->L + c->K);
#define FL_KR(SM, MB, E) hipLaunchKernelGGL((k_ks_rot<SM, MB, E>), dim3(nxy * ((b.n + 4 * E - 1) / (4 * E))), dim3(256), \
                                            0, s, b, c->d_mods, c->d_moddown, digits, digits_es, u, u_es, add, r, c->log_n, \
                                            c->L, c->K, c->alpha, (b.n + 4 * E - 1) / (4 * E), nxy % 8 == 0)
        const bool one = mixed_keys(b);
        if (c->small) {
            if (n_digits <= 4) { if (one) FL_KR(true, 4, 1); else FL_KR(true, 4, 4); }
            else if (n_digits <= 8) { if (one) FL_KR(true, 8, 1); else FL_KR(true, 8, 2); }
            else FL_KR(true, 16, 1);
        } else {
            if (n_digits <= 4) { if (one) FL_KR(false, 4, 1); else FL_KR(false, 4, 4); }
            else if (n_digits <= 8) { if (one) FL_KR(false, 8, 1); else FL_KR(false, 8, 2); }
            else FL_KR(false, 16, 1);
        }
#undef FL_KR
        FL_TRY_HIP(hipGetLastError());
        return FHELIN_OK;
    }
    if (eg < 1 || mixed_keys(b)) eg = 1;
    dim3 grid(c->N / 256, c->L + c->K, (b.n + eg - 1) / eg);
#define FL_KS(SM, MB) hipLaunchKernelGGL((k_ks_inner<SM, MB>), grid, dim3(256), 0, s, b, c->d_mods, c->d_moddown, \
                                         digits, digits_es, u, u_es, add, rot, c->log_n, c->L, c->K, c->alpha, eg)
    if (c->small) {
        if (n_digits <= 4) FL_KS(true, 4);
        else if (n_digits <= 8) FL_KS(true, 8);
        else FL_KS(true, 16);
    } else {
        if (n_digits <= 4) FL_KS(false, 4);
        else if (n_digits <= 8) FL_KS(false, 8);
        else FL_KS(false, 16);
    }
#undef FL_KS
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

int launch_ks_inner(const Ctx *c, const Batch &b, const uint64_t *digits, int64_t digits_es, uint64_t *u, int64_t u_es,
                    hipStream_t s, int eg) {
    return launch_ks_inner_impl(c, b, digits, digits_es, u, u_es, KsAdd{nullptr, 0, 0, 0}, s, eg, KsRot{});
}

int launch_ks_inner_add(const Ctx *c, const Batch &b, const uint64_t *digits, int64_t digits_es, uint64_t *u,
                        int64_t u_es, const uint64_t *add, int64_t add_es, int add_ext, int accumulate, hipStream_t s,
                        int eg) {
    return launch_ks_inner_impl(c, b, digits, digits_es, u, u_es, KsAdd{add, add_es, add_ext, accumulate}, s, eg,
                                KsRot{});
}

int launch_ks_inner_rot(const Ctx *c, const Batch &b, const KsRot &rot, const uint64_t *digits, int64_t digits_es,
                        uint64_t *u, int64_t u_es, const uint64_t *add, int64_t add_es, int add_ext, hipStream_t s,
                        int eg) {
    return launch_ks_inner_impl(c, b, digits, digits_es, u, u_es, KsAdd{add, add_es, add_ext, 0}, s, eg, rot);
}

// ---------------------------------------------------------------------------
// extended-basis helpers (NTT domain): dst[p][slot] over slots of B_l
//   lift:  dst = P * src for a Q ciphertext src [2][src_stride] (0 on the p slots)
//   add:   dst (+)= src for extended ciphertexts [2][L+K]
// grid (N/256, 2 (l_max + K), n)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_ext_lift_add(Batch b, const ModConst *__restrict__ mods,
                                                      const ModDownTab *__restrict__ mdt,
                                                      const uint64_t *__restrict__ src, int64_t src_es,
                                                      int src_stride, int lift, int accumulate,
                                                      uint64_t *__restrict__ dst, int64_t dst_es, int log_n, int L,
                                                      int K) {
    const int t = blockIdx.z;
    const int l = b.level[t];
    const int r = blockIdx.y;
    if (r >= 2 * (l + K)) return;
    const int p = r / (l + K), e = r % (l + K);
    const int slot = e < l ? e : L + (e - l);
    const int64_t N = (int64_t)1 << log_n;
    const int k = blockIdx.x * 256 + threadIdx.x;
    const ModConst mc = mods[slot];
    uint64_t v;
    if (lift) {
        v = e < l ? mont_mul(src[t * src_es + ((int64_t)p * src_stride + e) * N + k], mdt->p_mont[e], mc.q,
                             mc.mont_neg_inv)
                  : 0;
    } else {
        v = src[t * src_es + ((int64_t)p * (L + K) + slot) * N + k];
    }
    uint64_t *o = dst + t * dst_es + ((int64_t)p * (L + K) + slot) * N + k;
    if (accumulate) v = add_mod(v, *o, mc.q);
    *o = v;
}

int launch_ext_lift_add(const Ctx *c, const Batch &b, const uint64_t *src, int64_t src_es, int src_stride, int lift,
                        int accumulate, uint64_t *dst, int64_t dst_es, hipStream_t s) {
    if (b.n == 0) return FHELIN_OK;
    int lmax = 0;
    double units = 0;
    for (int t = 0; t < b.n; ++t) {
        lmax = b.level[t] > lmax ? b.level[t] : lmax;
        units += 2.0 * (b.level[t] + c->K) * c->N;
    }
    // bytes: each output element written once and its source read once (lift: the p slots
    // are written without a read), plus the read-back of an accumulated destination
    double bytes = 0;
    for (int t = 0; t < b.n; ++t)
        bytes += 8.0 * 2 * c->N * ((b.level[t] + c->K) + (lift ? b.level[t] : b.level[t] + c->K) +
                                   (accumulate ? b.level[t] + c->K : 0));
    ProfScope ps(c, s, PK_COPY, units, bytes);
    hipLaunchKernelGGL(k_ext_lift_add, dim3(c->N / 256, 2 * (lmax + c->K), b.n), dim3(256), 0, s, b, c->d_mods,
                       c->d_moddown, src, src_es, src_stride, lift, accumulate, dst, dst_es, c->log_n, c->L, c->K);
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

// ---------------------------------------------------------------------------
// ModDown base conversion P -> q_i: grid (N/256, 2, n); u P-slots in coefficient domain
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_moddown_fbc(Batch b, const ModConst *__restrict__ mods,
                                                     const ModDownTab *__restrict__ tab,
                                                     const uint64_t *__restrict__ u, int64_t u_es,
                                                     uint64_t *__restrict__ md, int64_t md_es, int log_n, int L,
                                                     int K) {
    const int t = blockIdx.z, p = blockIdx.y;
    const int l = b.level[t];
    const int64_t N = (int64_t)1 << log_n;
    const int k = blockIdx.x * 256 + threadIdx.x;
    const uint64_t *up = u + t * u_es + (int64_t)p * (L + K) * N;
    uint64_t *out = md + t * md_es + (int64_t)p * L * N;
    uint64_t v[MAX_P];
    uint64_t nneg = 0;
#pragma unroll
    for (int a = 0; a < MAX_P; ++a) {
        if (a < K) {
            const ModConst mc = mods[L + a];
            uint64_t w = shoup(up[(int64_t)(L + a) * N + k], tab->inv_hat[a], tab->inv_hat_sh[a], mc.q);
            v[a] = w;
            nneg += w > mc.half ? 1 : 0;
        }
    }
    for (int i = 0; i < l; ++i) {
        const ModConst mc = mods[i];
        Acc128 acc{0, 0};
#pragma unroll
        for (int a = 0; a < MAX_P; ++a)
            if (a < K) mac128(acc, v[a], tab->hat_mont[a][i]);
        uint64_t r = redc(acc, mc.q, mc.mont_neg_inv);
        if (nneg) r = sub_mod(r, mont_mul(nneg, tab->p_mont[i], mc.q, mc.mont_neg_inv), mc.q);
        out[(int64_t)i * N + k] = r;
    }
}

int launch_moddown_fbc(const Ctx *c, const Batch &b, const uint64_t *u, int64_t u_es, uint64_t *md, int64_t md_es,
                       hipStream_t s, int n_parts) {
    if (b.n == 0) return FHELIN_OK;
    double units = 0;
    for (int t = 0; t < b.n; ++t) {
        const double l = b.level[t];
        units += 2.0 * l * c->N;
    }
    // reads K limbs per part per entry, writes l limbs per part: (K + l) N 8 bytes per part
    double bytes = 0;
    for (int t = 0; t < b.n; ++t) bytes += 8.0 * c->N * (c->K + b.level[t]) * n_parts;
    ProfScope ps(c, s, PK_MODDOWN_FBC, units * n_parts / 2, bytes);
    hipLaunchKernelGGL(k_moddown_fbc, dim3(c->N / 256, n_parts, b.n), dim3(256), 0, s, b, c->d_mods, c->d_moddown, u,
                       u_es, md, md_es, c->log_n, c->L, c->K);
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

// ---------------------------------------------------------------------------
// ModDown in the coefficient domain, conversion and combination in one pass:
// grid (N/256, 1, n); u is one polynomial [L+K] (slot-indexed) per entry
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_moddown_coef(Batch b, const ModConst *__restrict__ mods,
                                                      const ModDownTab *__restrict__ tab,
                                                      const uint64_t *__restrict__ u, int64_t u_es,
                                                      uint64_t *__restrict__ out, int64_t out_es, int log_n, int L,
                                                      int K) {
    const int t = blockIdx.z;
    const int l = b.level[t];
    const int64_t N = (int64_t)1 << log_n;
    const int k = blockIdx.x * 256 + threadIdx.x;
    const uint64_t *up = u + t * u_es;
    uint64_t *o = out + t * out_es;
    uint64_t v[MAX_P];
    uint64_t nneg = 0;
#pragma unroll
    for (int a = 0; a < MAX_P; ++a) {
        if (a < K) {
            const ModConst mc = mods[L + a];
            uint64_t w = shoup(up[(int64_t)(L + a) * N + k], tab->inv_hat[a], tab->inv_hat_sh[a], mc.q);
            v[a] = w;
            nneg += w > mc.half ? 1 : 0;
        }
    }
    for (int i = 0; i < l; ++i) {
        const ModConst mc = mods[i];
        Acc128 acc{0, 0};
#pragma unroll
        for (int a = 0; a < MAX_P; ++a)
            if (a < K) mac128(acc, v[a], tab->hat_mont[a][i]);
        uint64_t r = redc(acc, mc.q, mc.mont_neg_inv);
        if (nneg) r = sub_mod(r, mont_mul(nneg, tab->p_mont[i], mc.q, mc.mont_neg_inv), mc.q);
        const uint64_t x = up[(int64_t)i * N + k];
        o[(int64_t)i * N + k] = shoup(sub_mod(x, r, mc.q), tab->pinv[i], tab->pinv_sh[i], mc.q);
    }
}

int launch_moddown_coef(const Ctx *c, const Batch &b, const uint64_t *u, int64_t u_es, uint64_t *out, int64_t out_es,
                        hipStream_t s) {
    if (b.n == 0) return FHELIN_OK;
    double units = 0, bytes = 0;
    for (int t = 0; t < b.n; ++t) {
        const double l = b.level[t];
        units += l * c->N;
        bytes += 8.0 * c->N * (c->K + 2 * l);  // reads K + l limbs, writes l
    }
    ProfScope ps(c, s, PK_MODDOWN_FBC, units, bytes);
    hipLaunchKernelGGL(k_moddown_coef, dim3(c->N / 256, 1, b.n), dim3(256), 0, s, b, c->d_mods, c->d_moddown, u, u_es,
                       out, out_es, c->log_n, c->L, c->K);
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

// ---------------------------------------------------------------------------
// ModDown combine (NTT domain): grid (N/256, 2*l_max, n)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_moddown_combine(Batch b, const ModConst *__restrict__ mods,
                                                         const ModDownTab *__restrict__ tab,
                                                         const uint64_t *__restrict__ u, int64_t u_es,
                                                         const uint64_t *__restrict__ md, int64_t md_es,
                                                         uint64_t *__restrict__ dst, int64_t dst_es, int dst_stride,
                                                         const uint64_t *__restrict__ c0, int64_t c0_es,
                                                         int c0_stride, int accumulate, int n_parts, int log_n, int L,
                                                         int K) {
    const int t = blockIdx.z;
    const int l = b.level[t];
    const int r = blockIdx.y;
    if (r >= n_parts * l) return;
    const int p = r / l, i = r % l;
    const int64_t N = (int64_t)1 << log_n;
    const int k = blockIdx.x * 256 + threadIdx.x;
    const ModConst mc = mods[i];
    uint64_t x = u[t * u_es + ((int64_t)p * (L + K) + i) * N + k];
    uint64_t y = md[t * md_es + ((int64_t)p * L + i) * N + k];
    uint64_t v = shoup(sub_mod(x, y, mc.q), tab->pinv[i], tab->pinv_sh[i], mc.q);
    if (p == 0 && c0) v = add_mod(v, c0[t * c0_es + (int64_t)i * N + auto_index(k, b.g[t], log_n)], mc.q);
    uint64_t *o = dst + t * dst_es + ((int64_t)p * dst_stride + i) * N + k;
    if (accumulate) v = add_mod(v, *o, mc.q);
    *o = v;
}

int launch_moddown_combine(const Ctx *c, const Batch &b, const uint64_t *u, int64_t u_es, const uint64_t *md,
                           int64_t md_es, uint64_t *dst, int64_t dst_es, int dst_stride, const uint64_t *c0,
                           int64_t c0_es, int c0_stride, int accumulate, hipStream_t s, int n_parts) {
    if (b.n == 0) return FHELIN_OK;
    int lmax = 0;
    for (int t = 0; t < b.n; ++t) lmax = b.level[t] > lmax ? b.level[t] : lmax;
    double units = 0;
    for (int t = 0; t < b.n; ++t) {
        const double l = b.level[t];
        units += 2.0 * l * c->N;
    }
    ProfScope ps(c, s, PK_COMBINE, units * n_parts / 2, 8.0 * units * n_parts / 2 * (c0 ? 4 : 3));
    hipLaunchKernelGGL(k_moddown_combine, dim3(c->N / 256, n_parts * lmax, b.n), dim3(256), 0, s, b, c->d_mods,
                       c->d_moddown, u, u_es, md, md_es, dst, dst_es, dst_stride, c0, c0_es, c0_stride, accumulate,
                       n_parts, c->log_n, c->L, c->K);
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

// ---------------------------------------------------------------------------
// rescale (coefficient domain): grid (N/256, 2*(l_max-1), n)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_rescale(Batch b, const ModConst *__restrict__ mods,
                                                 const uint64_t *__restrict__ rs_inv,
                                                 const uint64_t *__restrict__ rs_inv_sh,
                                                 const uint64_t *__restrict__ in, int64_t in_es, int in_stride,
                                                 uint64_t *__restrict__ out, int64_t out_es, int out_stride,
                                                 int log_n, int L) {
    const int t = blockIdx.z;
    const int l = b.level[t];
    const int r = blockIdx.y;
    if (r >= 2 * (l - 1)) return;
    const int p = r / (l - 1), i = r % (l - 1);
    const int64_t N = (int64_t)1 << log_n;
    const int k = blockIdx.x * 256 + threadIdx.x;
    const ModConst mt = mods[l - 1], mc = mods[i];
    const uint64_t *ip = in + t * in_es + (int64_t)p * in_stride * N;
    uint64_t top = ip[(int64_t)(l - 1) * N + k];
    uint64_t vi;  // centred top residue, reduced mod q_i
    if (top <= mt.half) {
        vi = csub(shoup_lazy(top, 1, mc.one_sh, mc.q), mc.q);
    } else {
        uint64_t m = csub(shoup_lazy(mt.q - top, 1, mc.one_sh, mc.q), mc.q);
        vi = m ? mc.q - m : 0;
    }
    uint64_t x = ip[(int64_t)i * N + k];
    const int64_t ti = (int64_t)(l - 1) * L + i;
    out[t * out_es + ((int64_t)p * out_stride + i) * N + k] = shoup(sub_mod(x, vi, mc.q), rs_inv[ti], rs_inv_sh[ti], mc.q);
}

int launch_rescale(const Ctx *c, const Batch &b, const uint64_t *in, int64_t in_es, int in_stride, uint64_t *out,
                   int64_t out_es, int out_stride, hipStream_t s) {
    if (b.n == 0) return FHELIN_OK;
    int lmax = 0;
    for (int t = 0; t < b.n; ++t) lmax = b.level[t] > lmax ? b.level[t] : lmax;
    if (lmax < 2) return FHELIN_OK;
    double units = 0;
    for (int t = 0; t < b.n; ++t) {
        const double l = b.level[t];
        units += 2.0 * (l - 1) * c->N;
    }
    ProfScope ps(c, s, PK_RESCALE, units, 16.0 * units);
    hipLaunchKernelGGL(k_rescale, dim3(c->N / 256, 2 * (lmax - 1), b.n), dim3(256), 0, s, b, c->d_mods, c->d_rs_inv,
                       c->d_rs_inv_sh, in, in_es, in_stride, out, out_es, out_stride, c->log_n, c->L);
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

// ---------------------------------------------------------------------------
// row copy between two row maps of identical shape: grid (N/256 capped, rows, n)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_copy_rows(RowMap dst, RowMap src) {
    const int t = blockIdx.z, r = blockIdx.y;
    if (r >= rowmap_rows(dst, t)) return;
    int64_t od, os;
    int md, ms;
    rowmap_get(dst, t, r, &od, &md);
    rowmap_get(src, t, r, &os, &ms);
    const int N = 1 << dst.log_n;
    const uint64_t *a = src.base + os;
    uint64_t *o = dst.base + od;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < N; e += gridDim.x * 256) o[e] = a[e];
}

int launch_copy_rows(const Ctx *c, const RowMap &dst, const RowMap &src, hipStream_t s) {
    int rows = rowmap_max_rows(dst);
    if (rows == 0 || dst.n_ct == 0) return FHELIN_OK;
    int bx = c->N / 256 < 32 ? c->N / 256 : 32;
    double units = 0;
    for (int t = 0; t < dst.n_ct; ++t) units += (double)rowmap_rows(dst, t) * c->N;
    ProfScope ps(c, s, PK_COPY, units, 16.0 * units);
    hipLaunchKernelGGL(k_copy_rows, dim3(bx, rows, dst.n_ct), dim3(256), 0, s, dst, src);
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

}  // namespace fl
