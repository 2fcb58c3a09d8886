// ntt.hip -- batched negacyclic NTT / INTT over RNS limbs (hot-path row a4).
//
// Forward: merged-psi Cooley-Tukey (natural order in, bit-reversed out), stage m
// (m = 1, 2, ..., N/2 groups, butterfly distance t = N/2m) multiplies by
// psi^{brv(m+i)} in group i (Longa-Naehrig 2016).  Inverse: Gentleman-Sande with
// psi^{-brv(m+i)}, then N^{-1}.  Butterflies are lazy (Harvey 2014): values stay
// in [0, 4q) (forward) or [0, 2q) (inverse) between stages; rows are canonical
// [0, q) on entry and exit.
//
// Blocking for gfx950 (64 KiB LDS per workgroup here, 256 threads):
//   N <= 2^12: one workgroup holds a whole limb in LDS and runs every stage.
//   N >= 2^13: two passes through HBM.  N = N1 * 256.  The first forward pass
//   runs the log2(N1) stages with distance >= 256 on tiles of 4096/N1 adjacent
//   columns (element c + 256 r, r < N1); the second runs the last 8 stages on
//   tiles of 16 contiguous 256-element blocks.  The inverse runs them mirrored.
// Grid: x = tile within the limb, y = row within a batch entry, z = batch entry.
#include "internal.h"
#include "modarith.h"

namespace fl {

constexpr int NTT_THREADS = 256;
constexpr int TILE = 4096;  // elements per workgroup in the two-pass kernels

__device__ __forceinline__ bool row_of(const RowMap &m, uint64_t *&ptr, int &mod) {
    int t = blockIdx.z, r = blockIdx.y;
    if (r >= rowmap_rows(m, t)) return false;
    int64_t off;
    rowmap_get(m, t, r, &off, &mod);
    ptr = m.base + off;
    return true;
}

// forward CT butterfly, lazy: X, Y in [0, 4q) -> [0, 4q)
__device__ __forceinline__ void ct_bfly(uint64_t &X, uint64_t &Y, uint64_t w, uint64_t wp, uint64_t q) {
    uint64_t q2 = 2 * q;
    uint64_t x = X >= q2 ? X - q2 : X;
    uint64_t t = shoup_lazy(Y, w, wp, q);
    X = x + t;
    Y = x - t + q2;
}

// inverse GS butterfly, lazy: U, V in [0, 2q) -> [0, 2q)
__device__ __forceinline__ void gs_bfly(uint64_t &U, uint64_t &V, uint64_t w, uint64_t wp, uint64_t q) {
    uint64_t q2 = 2 * q;
    uint64_t u = U, v = V;
    uint64_t s = u + v;
    U = s >= q2 ? s - q2 : s;
    V = shoup_lazy(u - v + q2, w, wp, q);
}

__device__ __forceinline__ uint64_t reduce4q(uint64_t x, uint64_t q) {
    uint64_t q2 = 2 * q;
    x = x >= q2 ? x - q2 : x;
    return x >= q ? x - q : x;
}

// ---------------------------------------------------------------------------
// single pass (N <= 4096)
// ---------------------------------------------------------------------------
template <int LOGN>
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
            ct_bfly(X, Y, w[m + i], wp[m + i], q);
            s[j] = X;
            s[j + t] = Y;
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < N; e += NTT_THREADS) x[e] = reduce4q(s[e], q);
}

template <int LOGN>
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
            gs_bfly(U, V, w[m + i], wp[m + i], q);
            s[j] = U;
            s[j + t] = V;
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < N; e += NTT_THREADS) x[e] = shoup(s[e], mc.ninv, mc.ninv_sh, q);
}

// ---------------------------------------------------------------------------
// two passes (N >= 8192), N = N1 * 256
// ---------------------------------------------------------------------------
// forward pass 1: stages m = 1 .. N1/2 on columns
template <int LOGN>
__global__ void __launch_bounds__(NTT_THREADS) k_ntt_fwd_cols(RowMap rm, const ModConst *__restrict__ mods,
                                                              const uint64_t *__restrict__ tw,
                                                              const uint64_t *__restrict__ twp) {
    constexpr int N = 1 << LOGN, LOGN1 = LOGN - 8, N1 = 1 << LOGN1, C = TILE / N1, LOGC = 12 - LOGN1;
    __shared__ uint64_t s[TILE];
    uint64_t *x;
    int mi;
    if (!row_of(rm, x, mi)) return;
    const uint64_t q = mods[mi].q;
    const uint64_t *w = tw + (size_t)mi * N, *wp = twp + (size_t)mi * N;
    const int col0 = blockIdx.x * C;
    for (int e = threadIdx.x; e < TILE; e += NTT_THREADS) {
        int c = e & (C - 1), r = e >> LOGC;
        s[e] = x[col0 + c + 256 * r];
    }
    __syncthreads();
    for (int lt = LOGN1 - 1, m = 1; lt >= 0; --lt, m <<= 1) {
        const int t = 1 << lt;  // column-local distance
        for (int b = threadIdx.x; b < TILE / 2; b += NTT_THREADS) {
            int c = b & (C - 1), pb = b >> LOGC;
            int i = pb >> lt;
            int r = (i << (lt + 1)) + (pb & (t - 1));
            uint64_t X = s[(r << LOGC) + c], Y = s[((r + t) << LOGC) + c];
            ct_bfly(X, Y, w[m + i], wp[m + i], q);
            s[(r << LOGC) + c] = X;
            s[((r + t) << LOGC) + c] = Y;
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < TILE; e += NTT_THREADS) {
        int c = e & (C - 1), r = e >> LOGC;
        x[col0 + c + 256 * r] = s[e];  // lazy [0, 4q)
    }
}

// forward pass 2: stages m = N1 .. N/2 inside contiguous 256-blocks
template <int LOGN>
__global__ void __launch_bounds__(NTT_THREADS) k_ntt_fwd_rows(RowMap rm, const ModConst *__restrict__ mods,
                                                              const uint64_t *__restrict__ tw,
                                                              const uint64_t *__restrict__ twp) {
    constexpr int N = 1 << LOGN, N1 = N >> 8;
    __shared__ uint64_t s[TILE];
    uint64_t *x;
    int mi;
    if (!row_of(rm, x, mi)) return;
    const uint64_t q = mods[mi].q;
    const uint64_t *w = tw + (size_t)mi * N, *wp = twp + (size_t)mi * N;
    uint64_t *xt = x + (size_t)blockIdx.x * TILE;
    const int blk0 = blockIdx.x * (TILE / 256);
    for (int e = threadIdx.x; e < TILE; e += NTT_THREADS) s[e] = xt[e];
    __syncthreads();
    for (int lt = 7, m = N1; lt >= 0; --lt, m <<= 1) {
        const int t = 1 << lt;
        for (int b = threadIdx.x; b < TILE / 2; b += NTT_THREADS) {
            int blk = b >> 7, pb = b & 127;
            int il = pb >> lt;
            int l = (il << (lt + 1)) + (pb & (t - 1));
            int i = (blk0 + blk) * (128 >> lt) + il;
            int j = (blk << 8) + l;
            uint64_t X = s[j], Y = s[j + t];
            ct_bfly(X, Y, w[m + i], wp[m + i], q);
            s[j] = X;
            s[j + t] = Y;
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < TILE; e += NTT_THREADS) xt[e] = reduce4q(s[e], q);
}

// inverse pass 1: stages t = 1 .. 128 inside contiguous 256-blocks
template <int LOGN>
__global__ void __launch_bounds__(NTT_THREADS) k_ntt_inv_rows(RowMap rm, const ModConst *__restrict__ mods,
                                                              const uint64_t *__restrict__ itw,
                                                              const uint64_t *__restrict__ itwp) {
    constexpr int N = 1 << LOGN;
    __shared__ uint64_t s[TILE];
    uint64_t *x;
    int mi;
    if (!row_of(rm, x, mi)) return;
    const uint64_t q = mods[mi].q;
    const uint64_t *w = itw + (size_t)mi * N, *wp = itwp + (size_t)mi * N;
    uint64_t *xt = x + (size_t)blockIdx.x * TILE;
    const int blk0 = blockIdx.x * (TILE / 256);
    for (int e = threadIdx.x; e < TILE; e += NTT_THREADS) s[e] = xt[e];
    __syncthreads();
    for (int lt = 0, m = N / 2; lt < 8; ++lt, m >>= 1) {
        const int t = 1 << lt;
        for (int b = threadIdx.x; b < TILE / 2; b += NTT_THREADS) {
            int blk = b >> 7, pb = b & 127;
            int il = pb >> lt;
            int l = (il << (lt + 1)) + (pb & (t - 1));
            int i = (blk0 + blk) * (128 >> lt) + il;
            int j = (blk << 8) + l;
            uint64_t U = s[j], V = s[j + t];
            gs_bfly(U, V, w[m + i], wp[m + i], q);
            s[j] = U;
            s[j + t] = V;
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < TILE; e += NTT_THREADS) xt[e] = s[e];  // lazy [0, 2q)
}

// inverse pass 2: stages with distance >= 256 on columns, then N^{-1}
template <int LOGN>
__global__ void __launch_bounds__(NTT_THREADS) k_ntt_inv_cols(RowMap rm, const ModConst *__restrict__ mods,
                                                              const uint64_t *__restrict__ itw,
                                                              const uint64_t *__restrict__ itwp) {
    constexpr int N = 1 << LOGN, LOGN1 = LOGN - 8, N1 = 1 << LOGN1, C = TILE / N1, LOGC = 12 - LOGN1;
    __shared__ uint64_t s[TILE];
    uint64_t *x;
    int mi;
    if (!row_of(rm, x, mi)) return;
    const ModConst mc = mods[mi];
    const uint64_t q = mc.q;
    const uint64_t *w = itw + (size_t)mi * N, *wp = itwp + (size_t)mi * N;
    const int col0 = blockIdx.x * C;
    for (int e = threadIdx.x; e < TILE; e += NTT_THREADS) {
        int c = e & (C - 1), r = e >> LOGC;
        s[e] = x[col0 + c + 256 * r];
    }
    __syncthreads();
    for (int lt = 0, m = N1 / 2; lt < LOGN1; ++lt, m >>= 1) {
        const int t = 1 << lt;
        for (int b = threadIdx.x; b < TILE / 2; b += NTT_THREADS) {
            int c = b & (C - 1), pb = b >> LOGC;
            int i = pb >> lt;
            int r = (i << (lt + 1)) + (pb & (t - 1));
            uint64_t U = s[(r << LOGC) + c], V = s[((r + t) << LOGC) + c];
            gs_bfly(U, V, w[m + i], wp[m + i], q);
            s[(r << LOGC) + c] = U;
            s[((r + t) << LOGC) + c] = V;
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < TILE; e += NTT_THREADS) {
        int c = e & (C - 1), r = e >> LOGC;
        x[col0 + c + 256 * r] = shoup(s[e], mc.ninv, mc.ninv_sh, q);
    }
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

template <int LOGN>
static void launch_ntt_t(const Ctx *c, const RowMap &rm, int rows, int inverse, hipStream_t s) {
    const int M = 1 << LOGN;
    if (LOGN <= 12) {
        dim3 g(1, rows, rm.n_ct);
        if (!inverse)
            hipLaunchKernelGGL(k_ntt_fwd_1<(LOGN <= 12 ? LOGN : 12)>, g, dim3(NTT_THREADS), 0, s, rm, c->d_mods, c->d_tw,
                               c->d_twp);
        else
            hipLaunchKernelGGL(k_ntt_inv_1<(LOGN <= 12 ? LOGN : 12)>, g, dim3(NTT_THREADS), 0, s, rm, c->d_mods, c->d_itw,
                               c->d_itwp);
    } else {
        constexpr int L2 = LOGN > 12 ? LOGN : 13;
        dim3 g(M / TILE, rows, rm.n_ct);
        if (!inverse) {
            hipLaunchKernelGGL(k_ntt_fwd_cols<L2>, g, dim3(NTT_THREADS), 0, s, rm, c->d_mods, c->d_tw, c->d_twp);
            hipLaunchKernelGGL(k_ntt_fwd_rows<L2>, g, dim3(NTT_THREADS), 0, s, rm, c->d_mods, c->d_tw, c->d_twp);
        } else {
            hipLaunchKernelGGL(k_ntt_inv_rows<L2>, g, dim3(NTT_THREADS), 0, s, rm, c->d_mods, c->d_itw, c->d_itwp);
            hipLaunchKernelGGL(k_ntt_inv_cols<L2>, g, dim3(NTT_THREADS), 0, s, rm, c->d_mods, c->d_itw, c->d_itwp);
        }
    }
}

int launch_ntt(const Ctx *c, const RowMap &rm, int inverse, hipStream_t s) {
    int rows = rowmap_max_rows(rm);
    if (rows == 0 || rm.n_ct == 0) return FHELIN_OK;
    switch (c->log_n) {
    case 10: launch_ntt_t<10>(c, rm, rows, inverse, s); break;
    case 11: launch_ntt_t<11>(c, rm, rows, inverse, s); break;
    case 12: launch_ntt_t<12>(c, rm, rows, inverse, s); break;
    case 13: launch_ntt_t<13>(c, rm, rows, inverse, s); break;
    case 14: launch_ntt_t<14>(c, rm, rows, inverse, s); break;
    case 15: launch_ntt_t<15>(c, rm, rows, inverse, s); break;
    case 16: launch_ntt_t<16>(c, rm, rows, inverse, s); break;
    default: return set_error(FHELIN_E_UNSUPPORTED_PARAM, "unsupported ring degree");
    }
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

static int launch_mont(const Ctx *c, const RowMap &rm, int to, hipStream_t s) {
    int rows = rowmap_max_rows(rm);
    if (rows == 0 || rm.n_ct == 0) return FHELIN_OK;
    int bx = c->N / 256 < 64 ? c->N / 256 : 64;
    hipLaunchKernelGGL(k_to_mont, dim3(bx, rows, rm.n_ct), dim3(256), 0, s, rm, c->d_mods, to);
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

int launch_to_mont(const Ctx *c, const RowMap &rm, hipStream_t s) { return launch_mont(c, rm, 1, s); }
int launch_from_mont(const Ctx *c, const RowMap &rm, hipStream_t s) { return launch_mont(c, rm, 0, s); }

}  // namespace fl
