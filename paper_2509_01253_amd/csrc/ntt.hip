// ntt.hip -- batched negacyclic NTT / INTT over RNS limbs (hot-path row a4).
//
// Forward: merged-psi Cooley-Tukey (natural order in, bit-reversed out), stage m
// (m = 1, 2, ..., N/2 groups, butterfly distance t = N/2m) multiplies by
// psi^{brv(m+i)} in group i (Longa-Naehrig 2016).  Inverse: Gentleman-Sande with
// psi^{-brv(m+i)}, then N^{-1}.  Butterflies are lazy (Harvey 2014): values stay
// in [0, 4q) (forward) or [0, 2q) (inverse) between stages; rows are canonical
// [0, q) on entry and exit.
//
// Blocking for gfx950 (256 threads per workgroup, 16 elements per thread):
//   N <= 2^12: one workgroup holds a whole limb in LDS and runs every stage.
//   N >= 2^13: two passes through HBM.  N = N1 * 256.  The first forward pass
//   runs the log2(N1) stages with distance >= 256 on tiles of 4096/N1 adjacent
//   columns (element c + 256 r, r < N1); the second runs the last 8 stages on
//   tiles of 16 contiguous 256-element blocks.  The inverse runs them mirrored.
//   Inside a pass, butterflies run on registers in two rounds (radix 16 x 2^(S-4))
//   with one LDS exchange; global accesses are 128-byte contiguous per 16 lanes.
// Grid: x = tile within the limb, y = row within a batch entry, z = batch entry.
#include "internal.h"
#include "modarith.h"
#include "modup.h"

namespace fl {

constexpr int NTT_THREADS = 256;  // single-pass kernels (N <= 4096)
// Two-pass kernels: NT threads per workgroup, 16 elements each (a tile of 16 NT
// elements: 16 NT / 256 blocks of 256 in the row passes, NT / T columns in the column
// passes).  NT in {128, 256, 512} is a tile choice of the plan (autotuned); results
// do not depend on it.
static thread_local int tl_ntt_threads = 256;

// row r of batch entry t: its address and modulus index (false past the entry's rows)
__device__ __forceinline__ bool row_at(const RowMap &m, int t, int r, uint64_t *&ptr, int &mod) {
    if (r >= rowmap_rows(m, t)) return false;
    int64_t off;
    rowmap_get(m, t, r, &off, &mod);
    ptr = m.base + off;
    return true;
}

__device__ __forceinline__ bool row_of(const RowMap &m, uint64_t *&ptr, int &mod) {
    return row_at(m, blockIdx.z, blockIdx.y, ptr, mod);
}

// out-of-place first pass: the same row of the source map (same row enumeration,
// its own layout), or the destination itself when the map is empty
__device__ __forceinline__ const uint64_t *src_row_at(const RowMap &src, int t, int r, const uint64_t *dst) {
    if (!src.base) return dst;
    int64_t off;
    int mod;
    rowmap_get(src, t, r, &off, &mod);
    return src.base + off;
}

__device__ __forceinline__ const uint64_t *src_row(const RowMap &src, const uint64_t *dst) {
    return src_row_at(src, blockIdx.z, blockIdx.y, dst);
}

// twiddle products: F53 (every modulus < 2^50) takes the 53-bit companions
template <bool F53>
__device__ __forceinline__ uint64_t tw_mul(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    if constexpr (F53) return shoup53_lazy(a, w, wp, q);
    else return shoup_lazy(a, w, wp, q);
}

// forward CT butterfly, lazy: X, Y in [0, 4q) -> [0, 4q)
template <bool F53>
__device__ __forceinline__ void ct_bfly(uint64_t &X, uint64_t &Y, uint64_t w, uint64_t wp, uint64_t q) {
    uint64_t q2 = 2 * q;
    uint64_t x;  // X - 2q unless that borrows
    if (__builtin_sub_overflow(X, q2, &x)) x = X;
    uint64_t t = tw_mul<F53>(Y, w, wp, q);
    X = x + t;
    Y = x - t + q2;
}

// inverse GS butterfly, lazy: U, V in [0, 2q) -> [0, 2q)
template <bool F53>
__device__ __forceinline__ void gs_bfly(uint64_t &U, uint64_t &V, uint64_t w, uint64_t wp, uint64_t q) {
    uint64_t q2 = 2 * q;
    uint64_t u = U, v = V;
    uint64_t s = u + v, r;
    U = __builtin_sub_overflow(s, q2, &r) ? s : r;
    V = tw_mul<F53>(u - v + q2, w, wp, q);
}

__device__ __forceinline__ uint64_t reduce4q(uint64_t x, uint64_t q) { return csub(csub(x, 2 * q), q); }

// ---------------------------------------------------------------------------
// single pass (N <= 4096)
// ---------------------------------------------------------------------------
template <int LOGN, bool F53>
__global__ void __launch_bounds__(NTT_THREADS) k_ntt_fwd_1(RowMap rm, const ModConst *__restrict__ mods,
                                                           const uint64_t *__restrict__ tw,
                                                           const uint64_t *__restrict__ twp) {
    constexpr int N = 1 << LOGN;
    __shared__ uint64_t s[N];
    uint64_t *x;
    int mi;
    if (!row_of(rm, x, mi)) return;
    const uint64_t q = mods[mi].q;
    const uint64_t *w = tw + (size_t)mi * N, *wp = twp + (size_t)mi * N;
    for (int e = threadIdx.x; e < N; e += NTT_THREADS) s[e] = x[e];
    __syncthreads();
    for (int lt = LOGN - 1, m = 1; lt >= 0; --lt, m <<= 1) {
        const int t = 1 << lt;
        for (int b = threadIdx.x; b < N / 2; b += NTT_THREADS) {
            int i = b >> lt;
            int j = (i << (lt + 1)) + (b & (t - 1));
            uint64_t X = s[j], Y = s[j + t];
            ct_bfly<F53>(X, Y, w[m + i], wp[m + i], q);
            s[j] = X;
            s[j + t] = Y;
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < N; e += NTT_THREADS) x[e] = reduce4q(s[e], q);
}

template <int LOGN, bool F53>
__global__ void __launch_bounds__(NTT_THREADS) k_ntt_inv_1(RowMap rm, const ModConst *__restrict__ mods,
                                                           const uint64_t *__restrict__ itw,
                                                           const uint64_t *__restrict__ itwp) {
    constexpr int N = 1 << LOGN;
    __shared__ uint64_t s[N];
    uint64_t *x;
    int mi;
    if (!row_of(rm, x, mi)) return;
    const ModConst mc = mods[mi];
    const uint64_t q = mc.q;
    const uint64_t *w = itw + (size_t)mi * N, *wp = itwp + (size_t)mi * N;
    for (int e = threadIdx.x; e < N; e += NTT_THREADS) s[e] = x[e];
    __syncthreads();
    for (int lt = 0, m = N / 2; lt < LOGN; ++lt, m >>= 1) {
        const int t = 1 << lt;
        for (int b = threadIdx.x; b < N / 2; b += NTT_THREADS) {
            int i = b >> lt;
            int j = (i << (lt + 1)) + (b & (t - 1));
            uint64_t U = s[j], V = s[j + t];
            gs_bfly<F53>(U, V, w[m + i], wp[m + i], q);
            s[j] = U;
            s[j + t] = V;
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < N; e += NTT_THREADS) x[e] = shoup(s[e], mc.ninv, mc.ninv_sh, q);
}

// ---------------------------------------------------------------------------
// two passes (N >= 8192), N = N1 * 256, register-blocked
//
// Each pass runs the stages of 2^S-point sub-transforms (columns of N1 = 2^S
// elements with stride 256 in pass 1, contiguous 256-blocks in pass 2).  A thread
// holds 16 elements of one sub-transform in registers, T = 2^(S-4) threads per
// sub-transform.  Round A: element u sits at local index rho = r + T u and the
// four stages with distances 8T, 4T, 2T, T pair u with u + 8, 4, 2, 1.  Round B:
// rho = 16 r + u and the S-4 remaining stages (distances 2^(S-5) .. 1) pair u
// with u + h inside the thread.  One LDS exchange separates the rounds.
// The twiddle of stage distance t for the pair at rho is psi^brv(idx),
// idx = (M + gb 2^S + rho) / 2t, with M = 2^S in pass 1 (first stages of the
// transform, gb = 0) and M = N in pass 2 (gb = global 256-block index).
// ---------------------------------------------------------------------------
// The twiddles of a round are loaded before its butterflies, in the order they are
// used, so that their loads are in flight together (and with the data's) rather
// than one stage at a time.
struct Tw {
    uint64_t w[15], wp[15];  // at most 1 + 2 + 4 + 8 pairs
};

// round A twiddles: stages lh = 3..0 (forward) or 0..3 (inverse), groups g < 8 / 2^lh
template <int S, bool FWD>
__device__ __forceinline__ void tw_load_a(Tw &t, int64_t base, const uint64_t *__restrict__ w,
                                          const uint64_t *__restrict__ wp) {
    constexpr int T = 1 << (S - 4);
    int k = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int lh = FWD ? 3 - i : i;
        const int h = 1 << lh, lt = lh + (S - 4);  // log2 of the distance t = h T
#pragma unroll
        for (int g = 0; g < 8 / h; ++g, ++k) {
            const int64_t idx = (base + (int64_t)T * (g * 2 * h)) >> (lt + 1);
            t.w[k] = w[idx];
            t.wp[k] = wp[idx];
        }
    }
}

// round B twiddles: stages lh = S-5..0 (forward) or 0..S-5 (inverse)
template <int S, bool FWD>
__device__ __forceinline__ void tw_load_b(Tw &t, int64_t base, const uint64_t *__restrict__ w,
                                          const uint64_t *__restrict__ wp) {
    int k = 0;
#pragma unroll
    for (int i = 0; i <= S - 5; ++i) {
        const int lh = FWD ? S - 5 - i : i;
        const int h = 1 << lh;
#pragma unroll
        for (int g = 0; g < 8 / h; ++g, ++k) {
            const int64_t idx = (base + g * 2 * h) >> (lh + 1);
            t.w[k] = w[idx];
            t.wp[k] = wp[idx];
        }
    }
}

template <int S, bool F53>
__device__ __forceinline__ void fwd_round_a(uint64_t (&X)[16], const Tw &t, uint64_t q) {
    int k = 0;
#pragma unroll
    for (int lh = 3; lh >= 0; --lh) {
        const int h = 1 << lh;
#pragma unroll
        for (int g = 0; g < 8 / h; ++g, ++k)
#pragma unroll
            for (int v = 0; v < h; ++v) ct_bfly<F53>(X[g * 2 * h + v], X[g * 2 * h + v + h], t.w[k], t.wp[k], q);
    }
}

template <int S, bool F53>
__device__ __forceinline__ void fwd_round_b(uint64_t (&X)[16], const Tw &t, uint64_t q) {
    int k = 0;
#pragma unroll
    for (int lh = S - 5; lh >= 0; --lh) {
        const int h = 1 << lh;
#pragma unroll
        for (int g = 0; g < 8 / h; ++g, ++k)
#pragma unroll
            for (int v = 0; v < h; ++v) ct_bfly<F53>(X[g * 2 * h + v], X[g * 2 * h + v + h], t.w[k], t.wp[k], q);
    }
}

// inverse rounds: stages in increasing distance
template <int S, bool F53>
__device__ __forceinline__ void inv_round_b(uint64_t (&X)[16], const Tw &t, uint64_t q) {
    int k = 0;
#pragma unroll
    for (int lh = 0; lh <= S - 5; ++lh) {
        const int h = 1 << lh;
#pragma unroll
        for (int g = 0; g < 8 / h; ++g, ++k)
#pragma unroll
            for (int v = 0; v < h; ++v) gs_bfly<F53>(X[g * 2 * h + v], X[g * 2 * h + v + h], t.w[k], t.wp[k], q);
    }
}

template <int S, bool F53>
__device__ __forceinline__ void inv_round_a(uint64_t (&X)[16], const Tw &t, uint64_t q) {
    int k = 0;
#pragma unroll
    for (int lh = 0; lh <= 3; ++lh) {
        const int h = 1 << lh;
#pragma unroll
        for (int g = 0; g < 8 / h; ++g, ++k)
#pragma unroll
            for (int v = 0; v < h; ++v) gs_bfly<F53>(X[g * 2 * h + v], X[g * 2 * h + v + h], t.w[k], t.wp[k], q);
    }
}

// forward pass 1: stages with distance >= 256 on columns c + 256 rho, rho < N1 = 2^S;
// column tile bx of the row at x (read from xs), LDS scratch s of (2^S)(NT/T + 1) words
template <int LOGN, bool F53, int NT>
__device__ __forceinline__ void fwd_cols_tile(uint64_t *x, const uint64_t *xs, int mi, int bx,
                                              const ModConst *__restrict__ mods, const uint64_t *__restrict__ tw,
                                              const uint64_t *__restrict__ twp, uint64_t *s) {
    constexpr int N = 1 << LOGN, S = LOGN - 8, T = 1 << (S - 4), C = NT / T, CP = C + 1;
    const uint64_t q = mods[mi].q;
    const uint64_t *w = tw + (size_t)mi * N, *wp = twp + (size_t)mi * N;
    const int c = threadIdx.x % C, r = threadIdx.x / C;
    uint64_t *xc = x + bx * C + c;
    const uint64_t *xsc = xs + bx * C + c;
    uint64_t X[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) X[u] = xsc[256 * (r + T * u)];
    {
        Tw ta;
        tw_load_a<S, true>(ta, 1 << S, w, wp);
        fwd_round_a<S, F53>(X, ta, q);
    }
    Tw tb;
    tw_load_b<S, true>(tb, (1 << S) + 16 * r, w, wp);
#pragma unroll
    for (int u = 0; u < 16; ++u) s[(r + T * u) * CP + c] = X[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) X[u] = s[(16 * r + u) * CP + c];
    fwd_round_b<S, F53>(X, tb, q);
#pragma unroll
    for (int u = 0; u < 16; ++u) xc[256 * (16 * r + u)] = X[u];  // lazy [0, 4q)
}

template <int LOGN, bool F53, int NT>
__global__ void __launch_bounds__(NT) k_ntt_fwd_cols(RowMap rm, RowMap src,
                                                     const ModConst *__restrict__ mods,
                                                     const uint64_t *__restrict__ tw,
                                                     const uint64_t *__restrict__ twp) {
    constexpr int S = LOGN - 8, T = 1 << (S - 4), C = NT / T, CP = C + 1;
    __shared__ uint64_t s[(1 << S) * CP];
    uint64_t *x;
    int mi;
    if (!row_of(rm, x, mi)) return;
    fwd_cols_tile<LOGN, F53, NT>(x, src_row(src, x), mi, blockIdx.x, mods, tw, twp, s);
}

// forward pass 2: the last 8 stages inside contiguous 256-blocks; NT/16 blocks per
// workgroup (tile bx of the row at x, LDS scratch s of (NT/16) 272 words);
// MONT: outputs in Montgomery form (one Shoup product by 2^64 mod q replaces the final reduction)
template <int LOGN, bool MONT, bool F53, int NT>
__device__ __forceinline__ void fwd_rows_tile(uint64_t *x, int mi, int bx, const ModConst *__restrict__ mods,
                                              const uint64_t *__restrict__ tw, const uint64_t *__restrict__ twp,
                                              uint64_t *s) {
    constexpr int N = 1 << LOGN, BS = 272;  // padded block stride in LDS (one pad word per 16)
    constexpr int NB = NT / 16, TILE = 16 * NT;  // 256-blocks per workgroup, elements per workgroup
    const uint64_t q = mods[mi].q;
    const uint64_t *w = tw + (size_t)mi * N, *wp = twp + (size_t)mi * N;
    const int blk = threadIdx.x >> 4, r = threadIdx.x & 15;
    const int gb = bx * NB + blk;
    uint64_t *xt = x + (size_t)bx * TILE;
    uint64_t X[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) X[u] = xt[blk * 256 + r + 16 * u];
    const int64_t base = N + (int64_t)gb * 256;
    {
        Tw ta;
        tw_load_a<8, true>(ta, base, w, wp);
        fwd_round_a<8, F53>(X, ta, q);
    }
    Tw tb;
    tw_load_b<8, true>(tb, base + 16 * r, w, wp);
    uint64_t *sb = s + blk * BS;
#pragma unroll
    for (int u = 0; u < 16; ++u) sb[r + 17 * u] = X[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) X[u] = sb[17 * r + u];
    fwd_round_b<8, F53>(X, tb, q);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        if constexpr (MONT) sb[17 * r + u] = shoup(X[u], mods[mi].r1, mods[mi].r1_sh, q);
        else sb[17 * r + u] = reduce4q(X[u], q);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < TILE; e += NT) xt[e] = s[(e >> 8) * BS + (e & 255) + ((e & 255) >> 4)];
}

template <int LOGN, bool MONT, bool F53, int NT>
__global__ void __launch_bounds__(NT) k_ntt_fwd_rows(RowMap rm, const ModConst *__restrict__ mods,
                                                     const uint64_t *__restrict__ tw,
                                                     const uint64_t *__restrict__ twp) {
    __shared__ uint64_t s[(NT / 16) * 272];
    uint64_t *x;
    int mi;
    if (!row_of(rm, x, mi)) return;
    fwd_rows_tile<LOGN, MONT, F53, NT>(x, mi, blockIdx.x, mods, tw, twp, s);
}

// inverse pass 1: the first 8 stages (distance 1 .. 128) inside contiguous 256-blocks
template <int LOGN, bool F53, int NT>
__global__ void __launch_bounds__(NT) k_ntt_inv_rows(RowMap rm, RowMap src, const ModConst *__restrict__ mods,
                                                     const uint64_t *__restrict__ itw,
                                                     const uint64_t *__restrict__ itwp) {
    constexpr int N = 1 << LOGN, BS = 272;
    constexpr int NB = NT / 16, TILE = 16 * NT;
    __shared__ uint64_t s[NB * BS];
    uint64_t *x;
    int mi;
    if (!row_of(rm, x, mi)) return;
    const uint64_t *xst = src_row(src, x) + (size_t)blockIdx.x * TILE;
    const uint64_t q = mods[mi].q;
    const uint64_t *w = itw + (size_t)mi * N, *wp = itwp + (size_t)mi * N;
    const int blk = threadIdx.x >> 4, r = threadIdx.x & 15;
    const int gb = blockIdx.x * NB + blk;
    uint64_t *xt = x + (size_t)blockIdx.x * TILE;
    const int64_t base = N + (int64_t)gb * 256;
    uint64_t X[16];
    {
        Tw tb;
        tw_load_b<8, false>(tb, base + 16 * r, w, wp);
        // the thread's 16 contiguous inputs as eight 16-byte loads (measured faster
        // than staging the tile through LDS; the forward pass's outputs, by contrast,
        // are faster staged)
        const ulonglong2 *in = reinterpret_cast<const ulonglong2 *>(xst + blk * 256 + 16 * r);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const ulonglong2 v = in[u];
            X[2 * u] = v.x;
            X[2 * u + 1] = v.y;
        }
        inv_round_b<8, F53>(X, tb, q);
    }
    Tw ta;
    tw_load_a<8, false>(ta, base, w, wp);
    uint64_t *sb = s + blk * BS;
#pragma unroll
    for (int u = 0; u < 16; ++u) sb[17 * r + u] = X[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) X[u] = sb[r + 17 * u];
    inv_round_a<8, F53>(X, ta, q);
#pragma unroll
    for (int u = 0; u < 16; ++u) xt[blk * 256 + r + 16 * u] = X[u];  // lazy [0, 2q)
}

// inverse pass 2: stages with distance >= 256 on columns, then N^{-1}
template <int LOGN, bool F53, int NT>
__global__ void __launch_bounds__(NT) k_ntt_inv_cols(RowMap rm, const ModConst *__restrict__ mods,
                                                     const uint64_t *__restrict__ itw,
                                                     const uint64_t *__restrict__ itwp) {
    constexpr int N = 1 << LOGN, S = LOGN - 8, T = 1 << (S - 4), C = NT / T, CP = C + 1;
    __shared__ uint64_t s[(1 << S) * CP];
    uint64_t *x;
    int mi;
    if (!row_of(rm, x, mi)) return;
    const ModConst mc = mods[mi];
    const uint64_t q = mc.q;
    const uint64_t *w = itw + (size_t)mi * N, *wp = itwp + (size_t)mi * N;
    const int c = threadIdx.x % C, r = threadIdx.x / C;
    uint64_t *xc = x + blockIdx.x * C + c;
    uint64_t X[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) X[u] = xc[256 * (16 * r + u)];
    {
        Tw tb;
        tw_load_b<S, false>(tb, (1 << S) + 16 * r, w, wp);
        inv_round_b<S, F53>(X, tb, q);
    }
    Tw ta;
    tw_load_a<S, false>(ta, 1 << S, w, wp);
#pragma unroll
    for (int u = 0; u < 16; ++u) s[(16 * r + u) * CP + c] = X[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) X[u] = s[(r + T * u) * CP + c];
    inv_round_a<S, F53>(X, ta, q);
#pragma unroll
    for (int u = 0; u < 16; ++u) xc[256 * (r + T * u)] = shoup(X[u], mc.ninv, mc.ninv_sh, q);
}

// ---------------------------------------------------------------------------
// Montgomery-form conversion over rows
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_to_mont(RowMap rm, const ModConst *__restrict__ mods, int to) {
    uint64_t *x;
    int mi;
    if (!row_of(rm, x, mi)) return;
    const ModConst mc = mods[mi];
    const int N = 1 << rm.log_n;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < N; e += gridDim.x * 256) {
        uint64_t v = x[e];
        x[e] = to ? mont_mul(v, mc.r2, mc.q, mc.mont_neg_inv) : redc(v, 0, mc.q, mc.mont_neg_inv);
    }
}

template <int LOGN, bool F53, int NT>
static void launch_two_pass(const Ctx *c, const RowMap &rm, const RowMap &src, int rows, int inverse, bool to_mont,
                            hipStream_t s, double bfly_per_stage, double row_bytes) {
    dim3 g((1 << LOGN) / (16 * NT), rows, rm.n_ct);
    if (!inverse) {
        {
            ProfScope ps(c, s, PK_NTT_FWD_COLS, bfly_per_stage * (LOGN - 8), row_bytes);
            hipLaunchKernelGGL((k_ntt_fwd_cols<LOGN, F53, NT>), g, dim3(NT), 0, s, rm, src, c->d_mods, c->d_tw, c->d_twp);
        }
        ProfScope ps(c, s, PK_NTT_FWD_ROWS, bfly_per_stage * 8, row_bytes);
        if (to_mont)
            hipLaunchKernelGGL((k_ntt_fwd_rows<LOGN, true, F53, NT>), g, dim3(NT), 0, s, rm, c->d_mods, c->d_tw, c->d_twp);
        else
            hipLaunchKernelGGL((k_ntt_fwd_rows<LOGN, false, F53, NT>), g, dim3(NT), 0, s, rm, c->d_mods, c->d_tw, c->d_twp);
    } else {
        {
            ProfScope ps(c, s, PK_NTT_INV_ROWS, bfly_per_stage * 8, row_bytes);
            hipLaunchKernelGGL((k_ntt_inv_rows<LOGN, F53, NT>), g, dim3(NT), 0, s, rm, src, c->d_mods, c->d_itw,
                               c->d_itwp);
        }
        ProfScope ps(c, s, PK_NTT_INV_COLS, bfly_per_stage * (LOGN - 8), row_bytes);
        hipLaunchKernelGGL((k_ntt_inv_cols<LOGN, F53, NT>), g, dim3(NT), 0, s, rm, c->d_mods, c->d_itw, c->d_itwp);
    }
}

template <int LOGN, bool F53>
static void launch_ntt_t(const Ctx *c, const RowMap &rm, const RowMap &src, int rows, int inverse, bool to_mont,
                         hipStream_t s) {
    const int M = 1 << LOGN;
    double total_rows = 0;
    for (int t = 0; t < rm.n_ct; ++t) total_rows += rowmap_rows(rm, t);
    const double bfly_per_stage = total_rows * (M / 2);
    const double row_bytes = total_rows * 16.0 * M;  // each row read and written once per pass
    if (LOGN <= 12) {
        dim3 g(1, rows, rm.n_ct);
        if (!inverse) {
            ProfScope ps(c, s, PK_NTT_FWD_1, bfly_per_stage * LOGN, row_bytes);
            hipLaunchKernelGGL((k_ntt_fwd_1<(LOGN <= 12 ? LOGN : 12), F53>), g, dim3(NTT_THREADS), 0, s, rm, c->d_mods, c->d_tw,
                               c->d_twp);
        } else {
            ProfScope ps(c, s, PK_NTT_INV_1, bfly_per_stage * LOGN, row_bytes);
            hipLaunchKernelGGL((k_ntt_inv_1<(LOGN <= 12 ? LOGN : 12), F53>), g, dim3(NTT_THREADS), 0, s, rm, c->d_mods, c->d_itw,
                               c->d_itwp);
        }
    } else {
        constexpr int L2 = LOGN > 12 ? LOGN : 13;
        if (tl_ntt_threads == 128) launch_two_pass<L2, F53, 128>(c, rm, src, rows, inverse, to_mont, s, bfly_per_stage, row_bytes);
        else if (tl_ntt_threads == 512) launch_two_pass<L2, F53, 512>(c, rm, src, rows, inverse, to_mont, s, bfly_per_stage, row_bytes);
        else launch_two_pass<L2, F53, 256>(c, rm, src, rows, inverse, to_mont, s, bfly_per_stage, row_bytes);
    }
}

// ---------------------------------------------------------------------------
// persistent ModUp + forward NTT (one launch for a key switch's digit
// decomposition and its transform)
// ---------------------------------------------------------------------------
// Work items, claimed in ticket order from a counter: every ModUp chunk (entry, digit,
// 256 coefficients), then every column tile of every digit row, then every row tile.
// A column tile waits until all ModUp chunks of its digit are done; a row tile until
// all column tiles of its row are.  An item only ever waits for items with smaller
// tickets, which workgroups already running have claimed and which wait only for
// smaller tickets still, so the launch drains whatever the number of resident
// workgroups.  Waits are bounded: past spin_limit polls the workgroup sets the
// context's fault word and goes on (the result is then wrong and the host reports
// it), so no launch can hang.  Completion counters are released and acquired at
// device scope (stores of a tile written back before its counter moves, caches
// invalidated before the dependent tile reads).
// Every wave fences at device scope on both sides: a tile's stores are written back
// (the 8 L2s of the chip are not coherent with each other) before its counter moves,
// and every wave of a dependent tile invalidates its caches before reading.  (Fencing
// once per workgroup after a barrier was measured to leave stale data: the barrier
// does not make the other waves' stores visible at device scope.)
__device__ __forceinline__ void persist_wait(const uint32_t *ctr, uint32_t target, uint32_t *fault,
                                             uint32_t spin_limit) {
    if (threadIdx.x == 0) {
        uint32_t spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > spin_limit) {
                atomicOr(fault, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
    __threadfence();
}

__device__ __forceinline__ void persist_done(uint32_t *ctr) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int LOGN, bool F53>
__global__ void __launch_bounds__(256, 3) k_modup_ntt(Batch b, const ModConst *__restrict__ mods,
                                                   const ModUpTab *__restrict__ tabs, const uint64_t *__restrict__ coef,
                                                   int64_t coef_es, const uint64_t *__restrict__ ntt, int64_t ntt_es,
                                                   uint64_t *__restrict__ digits, int64_t digits_es, RowMap rm,
                                                   const uint64_t *__restrict__ tw, const uint64_t *__restrict__ twp,
                                                   uint32_t *ctl, uint32_t *fault, int L, int K, int alpha, int dnum,
                                                   int beta_max, int rows_max, uint32_t spin_limit) {
    constexpr int N = 1 << LOGN, NT = 256, S = LOGN - 8, T = 1 << (S - 4), CP = NT / T + 1;
    constexpr int TILES = N / (16 * NT), CHUNKS = N / 256;
    constexpr int LDS_COLS = (1 << S) * CP, LDS_ROWS = (NT / 16) * 272;
    __shared__ uint64_t s[LDS_COLS > LDS_ROWS ? LDS_COLS : LDS_ROWS];
    __shared__ uint32_t item;
    const uint32_t n = (uint32_t)b.n;
    const uint32_t n_m = n * beta_max * CHUNKS, n_c = n * rows_max * TILES, total = n_m + 2 * n_c;
    uint32_t *ticket = ctl, *cnt_m = ctl + 1, *cnt_c = cnt_m + n * PERSIST_DIGITS;
    for (;;) {
        __syncthreads();  // the previous item's readers of `item` and of the LDS are done
        if (threadIdx.x == 0) item = atomicAdd(ticket, 1u);
        __syncthreads();
        const uint32_t it = item;
        if (it >= total) break;
        if (it < n_m) {
            const int x = (int)(it % CHUNKS), j = (int)((it / CHUNKS) % beta_max), t = (int)(it / (CHUNKS * beta_max));
            if (j >= (b.level[t] + alpha - 1) / alpha) continue;
            modup_tile(b, mods, tabs, coef, coef_es, ntt, ntt_es, digits, digits_es, LOGN, L, K, alpha, dnum, x, j,
                       t);
            persist_done(&cnt_m[t * PERSIST_DIGITS + j]);
            continue;
        }
        const bool row_pass = it >= n_m + n_c;
        const uint32_t i2 = row_pass ? it - n_m - n_c : it - n_m;
        const int x = (int)(i2 % TILES), r = (int)((i2 / TILES) % rows_max), t = (int)(i2 / (TILES * rows_max));
        uint64_t *px;
        int mi;
        if (!row_at(rm, t, r, px, mi)) continue;
        if (!row_pass) {
            // digit of the row: its offset in the entry's digit buffer is (j (L+K) + slot) N
            const int j = (int)(((px - rm.base) - (int64_t)t * rm.ct_stride) / N / (L + K));
            persist_wait(&cnt_m[t * PERSIST_DIGITS + j], CHUNKS, fault, spin_limit);
            fwd_cols_tile<LOGN, F53, NT>(px, px, mi, x, mods, tw, twp, s);
            persist_done(&cnt_c[t * rows_max + r]);
        } else {
            persist_wait(&cnt_c[t * rows_max + r], TILES, fault, spin_limit);
            fwd_rows_tile<LOGN, false, F53, NT>(px, mi, x, mods, tw, twp, s);
        }
    }
}

__global__ void __launch_bounds__(256) k_zero_u32(uint32_t *p, int n) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0;
}

template <int LOGN, bool F53>
static int launch_modup_ntt_t(const Ctx *c, const Batch &b, const uint64_t *coef, int64_t coef_es,
                              const uint64_t *ntt, int64_t ntt_es, uint64_t *digits, int64_t digits_es,
                              const RowMap &rm, uint32_t *ctl, hipStream_t s) {
    int lmax = 0;
    for (int t = 0; t < b.n; ++t) lmax = b.level[t] > lmax ? b.level[t] : lmax;
    const int beta_max = (lmax + c->alpha - 1) / c->alpha;
    const int rows_max = rowmap_max_rows(rm);
    FL_CHECK(b.n <= MAX_BATCH && beta_max <= PERSIST_DIGITS && rows_max <= PERSIST_ROWS, FHELIN_E_UNSUPPORTED_PARAM,
             "persistent ModUp/NTT: batch beyond its counters");
    const int n_ctl = 1 + b.n * PERSIST_DIGITS + b.n * rows_max;
    hipLaunchKernelGGL(k_zero_u32, dim3((n_ctl + 255) / 256), dim3(256), 0, s, ctl, n_ctl);
    constexpr int N = 1 << LOGN;
    double rows = 0, units = 0, bytes = 0;
    for (int t = 0; t < b.n; ++t) {
        const double l = b.level[t], beta = std::ceil(l / c->alpha);
        rows += rowmap_rows(rm, t);
        units += beta * (l + c->K) * c->N;
        bytes += 8.0 * c->N * (l + beta * (l + c->K));
    }
    // work: the transforms' butterflies (the ModUp's conversions ride along); bytes: the
    // ModUp's input and output once (the transforms' passes over the digits stay in the
    // same launch)
    (void)units;
    ProfScope ps(c, s, PK_MODUP_NTT, rows * (N / 2) * LOGN, bytes);
    const uint32_t total = (uint32_t)b.n * beta_max * (N / 256) + 2u * (uint32_t)b.n * rows_max * (N / 4096);
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
    // three workgroups per compute unit are resident at this kernel's register count
    const uint32_t grid = std::min<uint32_t>(total, (uint32_t)cus * 3);
    hipLaunchKernelGGL((k_modup_ntt<LOGN, F53>), dim3(grid), dim3(256), 0, s, b, c->d_mods, c->d_modup, coef, coef_es,
                       ntt, ntt_es, digits, digits_es, rm, c->d_tw, c->d_twp, ctl, c->d_fault, c->L, c->K, c->alpha,
                       c->dnum, beta_max, rows_max, (uint32_t)PERSIST_SPIN_LIMIT);
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

int launch_modup_ntt(const Ctx *c, const Batch &b, const uint64_t *coef, int64_t coef_es, const uint64_t *ntt,
                     int64_t ntt_es, uint64_t *digits, int64_t digits_es, const RowMap &rm, uint32_t *ctl,
                     hipStream_t s) {
    if (b.n == 0) return FHELIN_OK;
    switch (c->log_n) {
    case 13: return c->ntt53 ? launch_modup_ntt_t<13, true>(c, b, coef, coef_es, ntt, ntt_es, digits, digits_es, rm, ctl, s)
                             : launch_modup_ntt_t<13, false>(c, b, coef, coef_es, ntt, ntt_es, digits, digits_es, rm, ctl, s);
    case 14: return c->ntt53 ? launch_modup_ntt_t<14, true>(c, b, coef, coef_es, ntt, ntt_es, digits, digits_es, rm, ctl, s)
                             : launch_modup_ntt_t<14, false>(c, b, coef, coef_es, ntt, ntt_es, digits, digits_es, rm, ctl, s);
    case 15: return c->ntt53 ? launch_modup_ntt_t<15, true>(c, b, coef, coef_es, ntt, ntt_es, digits, digits_es, rm, ctl, s)
                             : launch_modup_ntt_t<15, false>(c, b, coef, coef_es, ntt, ntt_es, digits, digits_es, rm, ctl, s);
    case 16: return c->ntt53 ? launch_modup_ntt_t<16, true>(c, b, coef, coef_es, ntt, ntt_es, digits, digits_es, rm, ctl, s)
                             : launch_modup_ntt_t<16, false>(c, b, coef, coef_es, ntt, ntt_es, digits, digits_es, rm, ctl, s);
    }
    return set_error(FHELIN_E_UNSUPPORTED_PARAM, "persistent ModUp/NTT needs N >= 2^13");
}

int ntt_threads_set(int nt) {
    const int prev = tl_ntt_threads;
    tl_ntt_threads = (nt == 128 || nt == 512) ? nt : 256;
    return prev;
}

static int launch_mont(const Ctx *c, const RowMap &rm, int to, hipStream_t s);

int launch_ntt(const Ctx *c, const RowMap &rm, int inverse, hipStream_t s, bool to_mont) {
    RowMap none{};
    return launch_ntt_from(c, rm, none, inverse, s, to_mont);
}

int launch_ntt_from(const Ctx *c, const RowMap &rm, const RowMap &src, int inverse, hipStream_t s, bool to_mont) {
    int rows = rowmap_max_rows(rm);
    if (rows == 0 || rm.n_ct == 0) return FHELIN_OK;
    if (src.base && c->log_n <= 12) {
        // one-pass sizes: copy, then transform in place
        FL_RET(launch_copy_rows(c, rm, src, s));
        RowMap none{};
        return launch_ntt_from(c, rm, none, inverse, s, to_mont);
    }
    // the two-pass forward transform converts in its last pass; the one-pass one is followed by a conversion
    const bool fused = to_mont && !inverse && c->log_n > 12;
    switch (c->log_n) {
    case 10: c->ntt53 ? launch_ntt_t<10, true>(c, rm, src, rows, inverse, fused, s)
                      : launch_ntt_t<10, false>(c, rm, src, rows, inverse, fused, s); break;
    case 11: c->ntt53 ? launch_ntt_t<11, true>(c, rm, src, rows, inverse, fused, s)
                      : launch_ntt_t<11, false>(c, rm, src, rows, inverse, fused, s); break;
    case 12: c->ntt53 ? launch_ntt_t<12, true>(c, rm, src, rows, inverse, fused, s)
                      : launch_ntt_t<12, false>(c, rm, src, rows, inverse, fused, s); break;
    case 13: c->ntt53 ? launch_ntt_t<13, true>(c, rm, src, rows, inverse, fused, s)
                      : launch_ntt_t<13, false>(c, rm, src, rows, inverse, fused, s); break;
    case 14: c->ntt53 ? launch_ntt_t<14, true>(c, rm, src, rows, inverse, fused, s)
                      : launch_ntt_t<14, false>(c, rm, src, rows, inverse, fused, s); break;
    case 15: c->ntt53 ? launch_ntt_t<15, true>(c, rm, src, rows, inverse, fused, s)
                      : launch_ntt_t<15, false>(c, rm, src, rows, inverse, fused, s); break;
    case 16: c->ntt53 ? launch_ntt_t<16, true>(c, rm, src, rows, inverse, fused, s)
                      : launch_ntt_t<16, false>(c, rm, src, rows, inverse, fused, s); break;
    default: return set_error(FHELIN_E_UNSUPPORTED_PARAM, "unsupported ring degree");
    }
    FL_TRY_HIP(hipGetLastError());
    if (to_mont && !fused) return launch_mont(c, rm, 1, s);
    return FHELIN_OK;
}

static int launch_mont(const Ctx *c, const RowMap &rm, int to, hipStream_t s) {
    int rows = rowmap_max_rows(rm);
    if (rows == 0 || rm.n_ct == 0) return FHELIN_OK;
    int bx = c->N / 256 < 64 ? c->N / 256 : 64;
    double units = 0;
    for (int t = 0; t < rm.n_ct; ++t) units += (double)rowmap_rows(rm, t) * c->N;
    ProfScope ps(c, s, PK_MONT, units, 16.0 * units);
    hipLaunchKernelGGL(k_to_mont, dim3(bx, rows, rm.n_ct), dim3(256), 0, s, rm, c->d_mods, to);
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

int launch_to_mont(const Ctx *c, const RowMap &rm, hipStream_t s) { return launch_mont(c, rm, 1, s); }

// ---------------------------------------------------------------------------
// issue-rate probe of the forward butterfly (diagnostics): 16 register values per
// thread, each round 16 butterflies (two radix-2 layers of 8 independent ones) with
// the 53-bit companions, no memory traffic inside the loop
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NTT_THREADS) k_diag_bfly(uint64_t *__restrict__ sink, uint64_t *__restrict__ stamps,
                                                           int iters, uint64_t q, uint64_t w, uint64_t wp) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = (tid * 0x9E3779B97F4A7C15ull + i) % q;
    const uint64_t c0 = clock64(), r0 = wall_clock64();
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int b = 0; b < 8; ++b) ct_bfly<true>(x[b], x[b + 8], w, wp, q);
#pragma unroll
        for (int b = 0; b < 8; ++b) ct_bfly<true>(x[(b & 3) + (b >> 2) * 8], x[(b & 3) + (b >> 2) * 8 + 4], w, wp, q);
    }
    const uint64_t c1 = clock64(), r1 = wall_clock64();
    if ((threadIdx.x & 63) == 0) {
        const int wave = tid >> 6;
        stamps[2 * wave] = c1 - c0;
        stamps[2 * wave + 1] = r1 - r0;
    }
    uint64_t acc = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc ^= x[i];
    sink[tid] = acc;
}

void launch_diag_bfly(int blocks, uint64_t *sink, uint64_t *stamps, int iters, uint64_t q, uint64_t w, uint64_t wp) {
    hipLaunchKernelGGL(k_diag_bfly, dim3(blocks), dim3(NTT_THREADS), 0, 0, sink, stamps, iters, q, w, wp);
}
int launch_from_mont(const Ctx *c, const RowMap &rm, hipStream_t s) { return launch_mont(c, rm, 0, s); }

}  // namespace fl
