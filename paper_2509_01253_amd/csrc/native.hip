// native.hip -- the paper's own server pipeline (Sec. 2.1-2.4, 4.2, 4.4): RLWE over the
// discrete torus q = 2^64 in Z_q[X]/Phi_M, M = t^alpha, N = phi(M).
//
//   extraction  for every chunk and coefficient i, E_i = u sum_d ct(m(X^d))
//               (X^(d (M-i)) - X^(d (M/t - r))), r = i mod M/t, u = M^-1 mod p
//               (the lemma on partial trace extraction with the two-term dual basis
//               element M conj(Omega*_i)); the client sent the powers m(X^d).
//   linear      F_o = sum_i W[o][i] E_i (integer weights, CSR), the shuffle folded
//               into W's rows.
//   packing     phi(t^beta) rows into one ciphertext of sum_o y_o X^(o M/t^beta):
//               leaves l_e = sum_j X^(j M/t^gamma) F_(e + j t^(beta-gamma)); per level
//               i = gamma..beta-1 a merge of t sub-packs y_k, v_m = sum_k
//               X^(k (M/t^(i+1) - m M/t)) y_k, S = v_(t-1), S = v_m + tau_i(S); then
//               Tr_{K/K_beta} as, per level j = alpha-1 down to beta, S = P,
//               S = P + tau_j(S) (t - 1 times); tau_i = sigma_(1 + t^i).
//   tau(S)      automorphism then key switch with a gadget of base D (2^log_d, or an even
//               base such as the paper's 310), depth l:
//               a' = sigma(a), b' = sigma(b), digits d_i of a' (balanced, stored with
//               the offset D/2), a'' = -sum_i d_i k_i.a, b'' = b' - sum_i d_i k_i.b.
//               The products d_i k_i modulo Phi_M are one matrix product per key:
//               K[j][i N + m] = coefficient j of X^m k_i, precomputed at key load, so a
//               batch of ciphertexts switches as C = A K^T (A = digits).
//
// Polynomials are N uint64 coefficients of the power basis; ciphertexts [2][N] (a, b).
// Reduction of a cyclic index x < M: X^(N + r) = -sum_{k < t-1} X^(k M/t + r), so
// coefficient j of a polynomial given modulo X^M - 1 as c is c[j] - c[N + j mod M/t].
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "native.h"

namespace fl {

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
struct NatDims {
    int M, N, Mt;
};

// coefficient x (< M) of X^e c taken modulo X^M - 1 (c has N coefficients)
__device__ __forceinline__ uint64_t cyc_at(const uint64_t *__restrict__ c, int x, int e, const NatDims &d) {
    int s = x - e;
    s += s < 0 ? d.M : 0;
    return s < d.N ? c[s] : 0;
}

// coefficient j (< N) of X^e c modulo Phi_M
__device__ __forceinline__ uint64_t mono_at(const uint64_t *__restrict__ c, int j, int e, const NatDims &d) {
    return cyc_at(c, j, e, d) - cyc_at(c, d.N + j % d.Mt, e, d);
}

// coefficient x (< M) of c(X^g) modulo X^M - 1: c at g^-1 x mod M (ginv = g^-1 mod M)
__device__ __forceinline__ uint64_t aut_cyc(const uint64_t *__restrict__ c, int x, int ginv, const NatDims &d) {
    const int s = (int)(((int64_t)x * ginv) % d.M);
    return s < d.N ? c[s] : 0;
}

__device__ __forceinline__ uint64_t aut_at(const uint64_t *__restrict__ c, int j, int ginv, const NatDims &d) {
    return aut_cyc(c, j, ginv, d) - aut_cyc(c, d.N + j % d.Mt, ginv, d);
}

// a mask coefficient as a torus value rounded to a multiple of 1 / D^l: floor((a D^l +
// 2^63) / 2^64), at most D^l (for D = 2^log_d: the top l log_d bits of a, rounded)
__device__ __forceinline__ uint64_t gadget_top(uint64_t a, const NatGadget &g) {
    if (g.log_d) {
        const int sh = 64 - g.log_d * g.l;
        return (a >> sh) + ((a >> (sh - 1)) & 1);
    }
    return __umul64hi(a, g.Dl) + ((a * g.Dl) >> 63);
}

// the next balanced base-D digit of top (least significant first), in [-D/2, D/2); a
// carry out of the top digit is dropped by the caller (the torus wraps)
__device__ __forceinline__ int gadget_digit(uint64_t &top, const NatGadget &g) {
    int64_t d;
    if (g.log_d) {
        d = (int64_t)(top & (g.D - 1));
        top >>= g.log_d;
    } else {
        const uint64_t q = top / g.D;
        d = (int64_t)(top - q * g.D);
        top = q;
    }
    if (d >= (int64_t)(g.D >> 1)) {
        d -= (int64_t)g.D;
        top += 1;
    }
    return (int)d;
}

// ---------------------------------------------------------------------------
// extraction: the rows of each chunk from the encryptions of its powers
// ---------------------------------------------------------------------------
struct NatPowers {
    int n;
    int32_t d[NAT_MAX_POW];
};

// The t - 1 rows i = r + q M/t (q < t - 1) share r = i mod M/t and with it the second
// term X^(d (M/t - r)) of every power: a thread gathers that term's coefficients once
// for up to EXT_Q rows and the first term's for each of them.
// grid (ceil(N / 256), M/t * ceil((t - 1) / EXT_Q), chunks).
constexpr int EXT_Q = 8;
__global__ void __launch_bounds__(256) k_nat_extract(const uint64_t *__restrict__ pows, uint64_t *__restrict__ rows,
                                                     NatDims dm, NatPowers pw, uint64_t u, int t) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= dm.N) return;
    const int r = blockIdx.y % dm.Mt, q0 = blockIdx.y / dm.Mt * EXT_Q, ch = blockIdx.z;
    const int nq = min(EXT_Q, t - 1 - q0);
    const int64_t ct = 2 * (int64_t)dm.N;
    const uint64_t *src = pows + (int64_t)ch * pw.n * ct;
    uint64_t acc0[EXT_Q], acc1[EXT_Q], g0 = 0, g1 = 0;
#pragma unroll
    for (int q = 0; q < EXT_Q; ++q) acc0[q] = acc1[q] = 0;
    for (int k = 0; k < pw.n; ++k) {
        const int d = pw.d[k];
        const uint64_t *a = src + k * ct, *b = a + dm.N;
        const int e2 = (int)(((int64_t)d * (dm.Mt - r)) % dm.M);
        g0 += mono_at(a, j, e2, dm);
        g1 += mono_at(b, j, e2, dm);
#pragma unroll
        for (int q = 0; q < EXT_Q; ++q)
            if (q < nq) {
                const int i = r + (q0 + q) * dm.Mt;
                const int e1 = (int)(((int64_t)d * (dm.M - i)) % dm.M);
                acc0[q] += mono_at(a, j, e1, dm);
                acc1[q] += mono_at(b, j, e1, dm);
            }
    }
#pragma unroll
    for (int q = 0; q < EXT_Q; ++q)
        if (q < nq) {
            uint64_t *o = rows + ((int64_t)ch * dm.N + r + (q0 + q) * dm.Mt) * ct;
            o[j] = (acc0[q] - g0) * u;
            o[dm.N + j] = (acc1[q] - g1) * u;
        }
}

// The same rows with the chunk's powers staged in LDS once per workgroup: a workgroup
// computes `rpg` consecutive rows of one chunk, every gather then reading LDS instead
// of the caches (each power polynomial serves all N rows of its chunk).  Thread t owns
// columns t, t + 512, ...  grid (ceil(N / rpg), chunks), 512 threads; dynamic LDS
// pw.n 2 N 8 bytes.
constexpr int EXT_T = 512;  // threads per workgroup
constexpr int EXT_J = 4;    // columns per thread at most (N <= EXT_J EXT_T)
__global__ void __launch_bounds__(EXT_T) k_nat_extract_lds(const uint64_t *__restrict__ pows,
                                                         uint64_t *__restrict__ rows, NatDims dm, NatPowers pw,
                                                         uint64_t u, int rpg) {
    extern __shared__ uint64_t sp[];  // [pw.n][2][N]
    const int ch = blockIdx.y;
    const int64_t ct = 2 * (int64_t)dm.N;
    const uint64_t *src = pows + (int64_t)ch * pw.n * ct;
    {  // eight loads in flight per thread, then their stores
        const int total = pw.n * (int)ct;
        for (int e0 = 0; e0 < total; e0 += 8 * EXT_T) {
            uint64_t v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = e0 + q * EXT_T + threadIdx.x;
                v[q] = e < total ? src[e] : 0;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = e0 + q * EXT_T + threadIdx.x;
                if (e < total) sp[e] = v[q];
            }
        }
    }
    __syncthreads();
    int jx[EXT_J], jy[EXT_J];  // the thread's columns and their partners N + j mod M/t
#pragma unroll
    for (int q = 0; q < EXT_J; ++q) {
        jx[q] = threadIdx.x + EXT_T * q;
        jy[q] = dm.N + jx[q] % dm.Mt;
    }
    auto cyc = [&](const uint64_t *c, int x, int e) {
        int s = x - e;
        s += s < 0 ? dm.M : 0;
        return s < dm.N ? c[s] : (uint64_t)0;
    };
    const int i1 = min(dm.N, (int)(blockIdx.x + 1) * rpg);
    for (int i = blockIdx.x * rpg; i < i1; ++i) {
        const int r = i % dm.Mt;
        uint64_t acc0[EXT_J], acc1[EXT_J];
#pragma unroll
        for (int q = 0; q < EXT_J; ++q) acc0[q] = acc1[q] = 0;
        for (int k = 0; k < pw.n; ++k) {
            const int d = pw.d[k];
            const int e1 = (int)(((int64_t)d * (dm.M - i)) % dm.M), e2 = (int)(((int64_t)d * (dm.Mt - r)) % dm.M);
            const uint64_t *a = sp + k * ct, *b = a + dm.N;
#pragma unroll
            for (int q = 0; q < EXT_J; ++q) {
                if (jx[q] >= dm.N) break;
                acc0[q] += (cyc(a, jx[q], e1) - cyc(a, jy[q], e1)) - (cyc(a, jx[q], e2) - cyc(a, jy[q], e2));
                acc1[q] += (cyc(b, jx[q], e1) - cyc(b, jy[q], e1)) - (cyc(b, jx[q], e2) - cyc(b, jy[q], e2));
            }
        }
        uint64_t *o = rows + ((int64_t)ch * dm.N + i) * ct;
#pragma unroll
        for (int q = 0; q < EXT_J; ++q) {
            if (jx[q] >= dm.N) break;
            o[jx[q]] = acc0[q] * u;
            o[dm.N + jx[q]] = acc1[q] * u;
        }
    }
}

// The rows streamed through LDS one power polynomial at a time, for rings with M <= 4096
// whose powers do not fit LDS whole.  A workgroup computes the rows i = r + q M/t,
// q0 <= q < q0 + nq, of one chunk and accumulates them in the cyclic ring Z[X]/(X^M - 1)
// at all M positions (the reduction modulo Phi_M, coefficient j minus coefficient
// N + j mod M/t, is linear and taken once at the end): a gather per position and row
// instead of two per coefficient, the second term X^(d (M/t - r)) gathered once for the
// nq rows.  Units u = b n_pow + k (polynomial b of power k) pass through two LDS slots
// of EXS_SLOT words, [0, N) the unit's coefficients and [N, M) zeros; the next unit's
// loads are in registers while the current one is read.  Thread x owns positions
// x + EXS_T p, p < X (M <= X EXS_T); rows per workgroup Q at most.
// grid (M/t ceil((t - 1) / Q), chunks), EXS_T threads, 64 KiB of static LDS.
constexpr int EXS_T = 512;
constexpr int EXS_SLOT = 4096;  // words per slot: M <= 4096
template <int X, int Q>
__global__ void __launch_bounds__(EXS_T, 2) k_nat_extract_stream(const uint64_t *__restrict__ pows,
                                                                 uint64_t *__restrict__ rows, NatDims dm,
                                                                 NatPowers pw, uint64_t u, int t) {
    __shared__ uint64_t L[2 * EXS_SLOT];
    const int tid = threadIdx.x;
    const int r = blockIdx.x % dm.Mt, q0 = blockIdx.x / dm.Mt * Q, ch = blockIdx.y;
    const int nq = min(Q, t - 1 - q0);
    const int64_t ct = 2 * (int64_t)dm.N;
    const uint64_t *src = pows + (int64_t)ch * pw.n * ct;
    const int U = 2 * pw.n;
    uint64_t acc[Q][X], g[X], pre[X];
#pragma unroll
    for (int p = 0; p < X; ++p) {
        g[p] = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) acc[q][p] = 0;
    }
    // unit u into the staging registers: coefficient x of polynomial b of power k, zero
    // for N <= x < M
    auto load = [&](int b, int k) {
        const uint64_t *c = src + k * ct + b * dm.N;
#pragma unroll
        for (int p = 0; p < X; ++p) {
            const int x = tid + EXS_T * p;
            pre[p] = x < dm.N ? c[x] : 0;
        }
    };
    // positions M <= x < X EXS_T (at most EXS_SLOT) hold zeros and gather in-slot values
    // that are never read back
    auto store = [&](int slot) {
#pragma unroll
        for (int p = 0; p < X; ++p) L[slot * EXS_SLOT + tid + EXS_T * p] = pre[p];
    };
    // x mod M for x < 2^26 by a multiply: mmag = floor(2^44 / M) + 1 overshoots 1 / M by
    // under 2^-44, so x mmag / 2^44 exceeds x / M by under 2^-18, less than the gap
    // 1 / M >= 2^-13 between x / M's fraction and 1
    const uint64_t mmag = (1ull << 44) / (uint64_t)dm.M + 1;
    auto mod_m = [&](uint32_t x) { return x - (uint32_t)(((uint64_t)x * mmag) >> 44) * (uint32_t)dm.M; };
    uint32_t xb[X];  // byte offsets of the thread's positions
#pragma unroll
    for (int p = 0; p < X; ++p) xb[p] = 8u * (uint32_t)(tid + EXS_T * p);
    const uint32_t mb = 8u * (uint32_t)dm.M;
    // coefficient x of X^e c modulo X^M - 1 is c at (x + M - e) mod M: with ob = 8 (M - e),
    // M - e in [1, M], and x < EXS_SLOT the byte index xb + ob is below 8 (EXS_SLOT + M),
    // and the unsigned minimum of it and itself less 8 M is the remainder's (below
    // 8 EXS_SLOT)
    auto gather = [&](const char *base, uint32_t x8, uint32_t ob) {
        const uint32_t sb = x8 + ob;
        return *(const uint64_t *)(base + min(sb, sb - mb));
    };
    auto compute = [&](int slot, int k) {
        const char *base = (const char *)(L + slot * EXS_SLOT);
        const uint32_t d = (uint32_t)pw.d[k];
        const uint32_t e2 = mod_m(d * (uint32_t)(dm.Mt - r));
        // e1 of row r + (q0 + q) M/t is d (M - r - q0 M/t) - q d M/t modulo M
        uint32_t e1 = mod_m(d * (uint32_t)(dm.M - r - q0 * dm.Mt));
        const uint32_t step = mod_m(d * (uint32_t)dm.Mt);
        {
            const uint32_t ob = 8u * ((uint32_t)dm.M - e2);
#pragma unroll
            for (int p = 0; p < X; ++p) g[p] += gather(base, xb[p], ob);
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (q >= nq) break;
            const uint32_t ob = 8u * ((uint32_t)dm.M - e1);
#pragma unroll
            for (int p = 0; p < X; ++p) acc[q][p] += gather(base, xb[p], ob);
            e1 = e1 >= step ? e1 - step : e1 + (uint32_t)dm.M - step;
        }
    };
    // polynomial b of the rows done: the coefficients at N <= x < M through the free slot,
    // then coefficient j of row i is (F(j) - F(N + j mod M/t)) u
    auto fold = [&](int slot, int b) {
        uint64_t *w = L + slot * EXS_SLOT;  // [q][M/t]
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (q >= nq) break;
#pragma unroll
            for (int p = 0; p < X; ++p) {
                const int x = tid + EXS_T * p;
                if (x >= dm.N && x < dm.M) w[q * dm.Mt + x - dm.N] = acc[q][p] - g[p];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (q >= nq) break;
            uint64_t *o = rows + ((int64_t)ch * dm.N + r + (q0 + q) * dm.Mt) * ct + (int64_t)b * dm.N;
#pragma unroll
            for (int p = 0; p < X; ++p) {
                const int x = tid + EXS_T * p;
                if (x < dm.N) o[x] = (acc[q][p] - g[p] - w[q * dm.Mt + x % dm.Mt]) * u;
            }
        }
#pragma unroll
        for (int p = 0; p < X; ++p) {
            g[p] = 0;
#pragma unroll
            for (int q = 0; q < Q; ++q) acc[q][p] = 0;
        }
        __syncthreads();
    };
    // units counted without divisions: (bc, kc) the one computed, (bl, kl) the one last
    // loaded into registers
    int bc = 0, kc = 0, bl = 0, kl = 0;
    auto next = [&](int &b, int &k) {
        if (++k == pw.n) {
            k = 0;
            ++b;
        }
    };
    // one unit from `slot`; the next goes to the other slot, the one after into registers
    auto step = [&](int slot, int uu) {
        compute(slot, kc);
        if (kc == pw.n - 1) fold(1 - slot, bc);
        if (uu + 1 < U) store(1 - slot);
        if (uu + 2 < U) {
            next(bl, kl);
            load(bl, kl);
        }
        next(bc, kc);
        __syncthreads();
    };
    load(bl, kl);
    store(0);
    next(bl, kl);
    load(bl, kl);  // U = 2 n_pow >= 2
    __syncthreads();
    for (int uu = 0; uu < U; uu += 2) {
        step(0, uu);
        step(1, uu + 1);
    }
}

// ---------------------------------------------------------------------------
// integer layer on rows (CSR): grid (ceil(2N / 256), n_out)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_nat_linear(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                                    const int32_t *__restrict__ val, const uint64_t *__restrict__ rows,
                                                    uint64_t *__restrict__ out, int n2) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int o = blockIdx.y;
    if (c >= n2) return;
    const int k0 = row_ptr[o], k1 = row_ptr[o + 1];
    uint64_t acc = 0;
    int k = k0;
    // four independent loads in flight
    for (; k + 4 <= k1; k += 4) {
        uint64_t v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = rows[(int64_t)col[k + q] * n2 + c];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc += (uint64_t)(int64_t)val[k + q] * v[q];
    }
    for (; k < k1; ++k) acc += (uint64_t)(int64_t)val[k] * rows[(int64_t)col[k] * n2 + c];
    out[(int64_t)o * n2 + c] = acc;
}

// ---------------------------------------------------------------------------
// packing pieces
// ---------------------------------------------------------------------------
// leaves: grid (ceil(N / 256), T, packs); out [packs][T][2][N]
__global__ void __launch_bounds__(256) k_nat_leaves(const uint64_t *__restrict__ F, int n_rows, uint64_t *__restrict__ out,
                                                    NatDims dm, int n_pack, int T, int phig, int estep) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= dm.N) return;
    const int e = blockIdx.y, g = blockIdx.z;
    const int64_t ct = 2 * (int64_t)dm.N;
    uint64_t a0 = 0, a1 = 0;
    for (int q = 0; q < phig; ++q) {
        const int row = g * n_pack + e + q * T;
        if (row >= n_rows) break;
        const uint64_t *f = F + row * ct;
        a0 += mono_at(f, j, q * estep, dm);
        a1 += mono_at(f + dm.N, j, q * estep, dm);
    }
    uint64_t *o = out + ((int64_t)g * T + e) * ct;
    o[j] = a0;
    o[dm.N + j] = a1;
}

// merge terms: grid (ceil(N / 256), step * t, packs); cur [packs][t step][2][N] ->
// v [packs][step][t][2][N], v[r][m] = sum_k X^(k (th - m Mt)) cur[r + k step]
__global__ void __launch_bounds__(256) k_nat_merge_v(const uint64_t *__restrict__ cur, uint64_t *__restrict__ v,
                                                     NatDims dm, int t, int step, int th) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= dm.N) return;
    const int r = blockIdx.y / t, m = blockIdx.y % t, g = blockIdx.z;
    const int64_t ct = 2 * (int64_t)dm.N;
    const uint64_t *base = cur + (int64_t)g * t * step * ct;
    uint64_t a0 = 0, a1 = 0;
    int em = th - m * dm.Mt;
    em %= dm.M;
    em += em < 0 ? dm.M : 0;
    for (int k = 0; k < t; ++k) {
        const uint64_t *y = base + (int64_t)(r + k * step) * ct;
        const int e = (int)(((int64_t)k * em) % dm.M);
        a0 += mono_at(y, j, e, dm);
        a1 += mono_at(y + dm.N, j, e, dm);
    }
    uint64_t *o = v + (((int64_t)g * step + r) * t + m) * ct;
    o[j] = a0;
    o[dm.N + j] = a1;
}

// The same merge terms with the t sub-packs of a merge read once: a workgroup takes one
// (r, pack), stages polynomial b of cur[r + k step] in LDS for k = 0..t-1 and
// accumulates all t terms m in registers in the cyclic ring Z[X]/(X^M - 1) at all M
// positions, reduced modulo Phi_M (coefficient j minus coefficient N + j mod M/t) once
// at the end through LDS, as the streamed extraction does.  Thread x owns positions
// x + MGS_T p, p < X (M <= X MGS_T <= MGS_SLOT); the slot holds the staged polynomial at
// [0, N), zeros up to X MGS_T.  grid (step, packs), MGS_T threads, 32 KiB of LDS.
constexpr int MGS_T = 512;
constexpr int MGS_SLOT = 4096;
template <int X, int TT>
__global__ void __launch_bounds__(MGS_T) k_nat_merge_s(const uint64_t *__restrict__ cur, uint64_t *__restrict__ v,
                                                       NatDims dm, int step, int th) {
    __shared__ uint64_t L[MGS_SLOT];
    const int r = blockIdx.x, g = blockIdx.y, tid = threadIdx.x;
    const int64_t ct = 2 * (int64_t)dm.N;
    const uint64_t *base = cur + (int64_t)g * TT * step * ct;
    // term m shifts sub-pack k by k (th - m M/t) modulo M
    int em[TT];
#pragma unroll
    for (int m = 0; m < TT; ++m) {
        int e = (th - m * dm.Mt) % dm.M;
        em[m] = e < 0 ? e + dm.M : e;
    }
    uint32_t xb[X];  // byte offsets of the thread's positions
#pragma unroll
    for (int p = 0; p < X; ++p) xb[p] = 8u * (uint32_t)(tid + MGS_T * p);
    const uint32_t mb = 8u * (uint32_t)dm.M;
    const char *lb = (const char *)L;
#pragma unroll 1
    for (int b = 0; b < 2; ++b) {
        uint64_t F[TT][X];
        int e[TT];  // k em[m] modulo M for the current k
#pragma unroll
        for (int m = 0; m < TT; ++m) {
            e[m] = 0;
#pragma unroll
            for (int p = 0; p < X; ++p) F[m][p] = 0;
        }
#pragma unroll 1
        for (int k = 0; k < TT; ++k) {
            const uint64_t *y = base + (int64_t)(r + k * step) * ct + (int64_t)b * dm.N;
            __syncthreads();  // the previous polynomial's (or fold's) readers are done
#pragma unroll
            for (int p = 0; p < X; ++p) {
                const int x = tid + MGS_T * p;
                L[x] = x < dm.N ? y[x] : 0;
            }
            __syncthreads();
            // coefficient x of X^e y modulo X^M - 1 is y at (x + M - e) mod M; with
            // o = M - e in [1, M] and x < MGS_SLOT the byte index xb + 8 o is below
            // 8 (MGS_SLOT + M), and the unsigned minimum of it and itself less 8 M is the
            // remainder's for x < M and in the slot for the rest
#pragma unroll
            for (int m = 0; m < TT; ++m) {
                const uint32_t ob = 8u * (uint32_t)(dm.M - e[m]);
#pragma unroll
                for (int p = 0; p < X; ++p) {
                    const uint32_t sb = xb[p] + ob;
                    F[m][p] += *(const uint64_t *)(lb + min(sb, sb - mb));
                }
                e[m] += em[m];
                e[m] -= e[m] >= dm.M ? dm.M : 0;
            }
        }
        // the coefficients at N <= x < M of every term through the slot, then
        // coefficient j of term m is F_m(j) - F_m(N + j mod M/t)
        __syncthreads();
#pragma unroll
        for (int m = 0; m < TT; ++m)
#pragma unroll
            for (int p = 0; p < X; ++p) {
                const int x = tid + MGS_T * p;
                if (x >= dm.N && x < dm.M) L[m * dm.Mt + x - dm.N] = F[m][p];
            }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < TT; ++m) {
            uint64_t *o = v + (((int64_t)g * step + r) * TT + m) * ct + (int64_t)b * dm.N;
#pragma unroll
            for (int p = 0; p < X; ++p) {
                const int x = tid + MGS_T * p;
                if (x < dm.N) o[x] = F[m][p] - L[m * dm.Mt + x % dm.Mt];
            }
        }
    }
}

// automorphism + gadget digits of a batch, and the output's start value: grid
// (ceil(N / 256), n); S [n] (s_es apart); digits [n][l][N] (offset by D/2, < D);
// out[c] = (add_a + corr_a, add_b + sigma(b) + corr_b), to which the product kernel
// adds -sum_k A K.  out must not overlap S or add.
__global__ void __launch_bounds__(256) k_nat_aut_decomp(const uint64_t *__restrict__ S, int64_t s_es,
                                                        const uint64_t *__restrict__ add, int64_t add_es,
                                                        uint64_t *__restrict__ out, int64_t out_es,
                                                        const uint64_t *__restrict__ corr_a,
                                                        const uint64_t *__restrict__ corr_b, uint32_t *__restrict__ dig,
                                                        NatDims dm, int ginv, NatGadget g) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= dm.N) return;
    const int c = blockIdx.y;
    const uint64_t *a = S + c * s_es, *b = a + dm.N;
    const uint64_t av = aut_at(a, j, ginv, dm), bv = aut_at(b, j, ginv, dm);
    const uint64_t *ad = add + c * add_es;
    uint64_t *o = out + c * out_es;
    o[j] = ad[j] + corr_a[j];
    o[dm.N + j] = ad[dm.N + j] + bv + corr_b[j];
    // rounded, then balanced digits from the least significant
    uint64_t top = gadget_top(av, g);
    uint32_t *dg = dig + (int64_t)c * g.l * dm.N + j;
    for (int i = g.l - 1; i >= 0; --i) dg[(int64_t)i * dm.N] = (uint32_t)(gadget_digit(top, g) + (int)(g.D >> 1));
}

// out[c][p][j] -= sum_k A[c][k] K_p[j][k] (mod 2^64) for both key parts, A[c][k] = digit +
// D/2 < 2^16 (the offset is removed by corr_p[j] = (D/2) sum_k K_p[j][k], added by the
// digits kernel).  Each product: v_mad_u64_u32 on the key's low word and a 32-bit
// multiply-add of its high word.  Tile: 32 ciphertexts x 128 coefficients per workgroup,
// thread (tc, tj) owns ciphertexts tc, tc + 16 and coefficients tj + 16 q (q < 8); K
// chunks of 16 staged in LDS.  grid.z splits K into slices of kc (small batches): the
// slices' sums are added with 64-bit atomics (exact modulo 2^64 in any order).
constexpr int KS_TC = 32, KS_TJ = 128, KS_TK = 16;

__global__ void __launch_bounds__(256) k_nat_ksprod(const uint32_t *__restrict__ A, const uint64_t *__restrict__ Ka,
                                                    const uint64_t *__restrict__ Kb, uint64_t *__restrict__ out,
                                                    int64_t out_es, int n, int N, int KD, int kc) {
    __shared__ uint32_t As[KS_TK][KS_TC + 1];
    __shared__ uint64_t Ks[2][KS_TK][KS_TJ + 1];
    const int c0 = blockIdx.y * KS_TC, j0 = blockIdx.x * KS_TJ;
    const int kb = blockIdx.z * kc, ke = min(KD, kb + kc);
    const int tc = threadIdx.x >> 4, tj = threadIdx.x & 15;
    uint64_t lo[2][2][8];
    uint32_t hi[2][2][8];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                lo[p][x][q] = 0;
                hi[p][x][q] = 0;
            }
    for (int k0 = kb; k0 < ke; k0 += KS_TK) {
        __syncthreads();
        // A tile: 32 x 16 digits (two per thread)
        for (int e = threadIdx.x; e < KS_TC * KS_TK; e += 256) {
            const int cc = e / KS_TK, kk = e % KS_TK;
            const int c = c0 + cc, k = k0 + kk;
            As[kk][cc] = c < n && k < ke ? A[(int64_t)c * KD + k] : 0u;
        }
        // K tiles: 128 x 16 per part
        for (int e = threadIdx.x; e < KS_TJ * KS_TK; e += 256) {
            const int jj = e / KS_TK, kk = e % KS_TK;
            const int j = j0 + jj, k = k0 + kk;
            const bool ok = j < N && k < ke;
            Ks[0][kk][jj] = ok ? Ka[(int64_t)j * KD + k] : 0;
            Ks[1][kk][jj] = ok ? Kb[(int64_t)j * KD + k] : 0;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < KS_TK; ++kk) {
            const uint32_t a[2] = {As[kk][tc], As[kk][tc + 16]};
#pragma unroll
            for (int q = 0; q < 8; ++q) {
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const uint64_t kv = Ks[p][kk][tj + 16 * q];
                    const uint32_t kl = (uint32_t)kv, kh = (uint32_t)(kv >> 32);
#pragma unroll
                    for (int x = 0; x < 2; ++x) {
                        lo[p][x][q] += (uint64_t)a[x] * kl;
                        hi[p][x][q] += a[x] * kh;
                    }
                }
            }
        }
    }
    const bool split = gridDim.z > 1;
#pragma unroll
    for (int x = 0; x < 2; ++x) {
        const int c = c0 + tc + 16 * x;
        if (c >= n) continue;
        uint64_t *o = out + c * out_es;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = j0 + tj + 16 * q;
            if (j >= N) continue;
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const uint64_t sum = lo[p][x][q] + ((uint64_t)hi[p][x][q] << 32);
                uint64_t *dst = o + p * N + j;
                if (split) atomicAdd((unsigned long long *)dst, (unsigned long long)(0 - sum));
                else *dst -= sum;
            }
        }
    }
}

// convolution on rows (channels-last inputs, index (y w + x) c_in + ci; zero padding
// k / 2): computed output (position, co) = sum over the window of wts[co][ci][dy][dx]
// times input row, written to out row out_row[position c_out + co] (the shuffle).  A
// thread owns one of the 2N columns and 16 output channels: each input value is read
// once for all 16, whose weights (transposed to wT[ci][dy][dx][cop], cop = c_out
// rounded up to 16, zero past c_out) are one 64-byte uniform load.  The weights are
// stored offset by 2^31 (sign bit flipped), u = W + 2^31 in [0, 2^32), so that with
// v = v_lo + 2^32 v_hi every product is two unsigned 32 x 32 -> 64 multiply-adds:
//   sum W v = sum u v_lo + 2^32 sum u v_hi - 2^31 sum v   (mod 2^64),
// the last sum (over the window's inputs) shared by the 16 channels.
// grid (ceil(2N / 256), output positions, cop / 16).
constexpr int CONV_CO = 16;

__global__ void __launch_bounds__(256) k_nat_conv_wt(const int32_t *__restrict__ wts, int32_t *__restrict__ wT,
                                                     int c_in, int c_out, int k, int cop) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= c_in * k * k * cop) return;
    const int co = idx % cop, t = idx / cop, ci = t / (k * k), r = t % (k * k);
    const uint32_t wv = co < c_out ? (uint32_t)wts[((int64_t)co * c_in + ci) * k * k + r] : 0u;
    wT[idx] = (int32_t)(wv ^ 0x80000000u);
}

__global__ void __launch_bounds__(256) k_nat_conv(const uint64_t *__restrict__ rows, const int32_t *__restrict__ wT,
                                                  const int32_t *__restrict__ out_row, uint64_t *__restrict__ out,
                                                  int c_in, int c_out, int cop, int h, int w, int k, int stride, int wo,
                                                  int n2) {
    const int col = blockIdx.x * 256 + threadIdx.x;
    if (col >= n2) return;
    const int pos = blockIdx.y, yo = pos / wo, xo = pos % wo, co0 = blockIdx.z * CONV_CO;
    uint64_t acc[CONV_CO], acc_hi[CONV_CO], sum = 0;
#pragma unroll
    for (int q = 0; q < CONV_CO; ++q) acc[q] = acc_hi[q] = 0;
    const int64_t ci_stride = (int64_t)k * k * cop;
    for (int dy = 0; dy < k; ++dy) {
        const int y = stride * yo + dy - k / 2;
        if (y < 0 || y >= h) continue;
        for (int dx = 0; dx < k; ++dx) {
            const int x = stride * xo + dx - k / 2;
            if (x < 0 || x >= w) continue;
            const uint64_t *in = rows + ((int64_t)(y * w + x) * c_in) * n2 + col;
            const int32_t *wp = wT + (int64_t)(dy * k + dx) * cop + co0;
            // input ci times the 16 channels' weights
            auto mac = [&](uint64_t v, int ci) {
                const uint32_t vl = (uint32_t)v, vh = (uint32_t)(v >> 32);
                sum += v;
                const int4 *w4 = (const int4 *)(wp + ci * ci_stride);
                uint32_t wv[CONV_CO];
#pragma unroll
                for (int q4 = 0; q4 < CONV_CO / 4; ++q4) {
                    const int4 t4 = w4[q4];
                    wv[4 * q4] = (uint32_t)t4.x;
                    wv[4 * q4 + 1] = (uint32_t)t4.y;
                    wv[4 * q4 + 2] = (uint32_t)t4.z;
                    wv[4 * q4 + 3] = (uint32_t)t4.w;
                }
#pragma unroll
                for (int q = 0; q < CONV_CO; ++q) {
                    acc[q] += (uint64_t)wv[q] * vl;
                    acc_hi[q] += (uint64_t)wv[q] * vh;
                }
            };
            // inputs two at a time, the next two loaded while these are multiplied; the
            // loads past the last input re-read it (clamped index, no branch between a
            // load and its use)
            const int last = c_in - 1;
            uint64_t va = in[0], vb = in[(int64_t)min(1, last) * n2];
            for (int ci = 0; ci < c_in; ci += 2) {
                const uint64_t a = va, b = vb;
                va = in[(int64_t)min(ci + 2, last) * n2];
                vb = in[(int64_t)min(ci + 3, last) * n2];
                mac(a, ci);
                if (ci + 1 < c_in) mac(b, ci + 1);
            }
        }
    }
    const uint64_t corr = sum << 31;
#pragma unroll
    for (int q = 0; q < CONV_CO; ++q)
        if (co0 + q < c_out) out[(int64_t)out_row[pos * c_out + co0 + q] * n2 + col] = acc[q] + (acc_hi[q] << 32) - corr;
}

// ---------------------------------------------------------------------------
// int8 matrix-core engine.  A balanced digit d in [-D/2, D/2) is split into H int8
// pieces: for D <= 2^9, d = p0 + 16 p1 with p0 in [-8, 8), p1 in [-16, 16] (H = 2); up
// to D = 2^16, d = p0 + 32 p1 + 1024 p2 with p0, p1 in [-16, 16), p2 in [-32, 32]
// (H = 3).  A key entry K (mod 2^64) is sum_b 2^(8b) s_b with balanced bytes s_b in
// [-128, 128).  Then
//   sum_k d_k K_k = sum_b 2^(8b) sum_h w_h (sum_k p_hk s_bk)   (mod 2^64),  w_h = 16^h or 32^h,
// and each inner sum is an int8 matrix product with an exact int32 sum (|sum| <= 32
// 128 K < 2^31 for K <= 2^19).
// ---------------------------------------------------------------------------
typedef int v4i __attribute__((ext_vector_type(4)));

// Operand layout of the int8 product (digit halves and key byte planes alike): rows
// in tiles of 64 (padded), each tile's K in 64-byte chunks, each chunk as four 1 KiB
// blocks of 16 rows, so that one block is one contiguous load of 64 lanes x 16 bytes.
// Within a block, quarter q (16 bytes) of row r sits in slot 4 r + (q ^ k8_swz(r)):
// the 16 (or 8) lanes that one LDS read cycle serves then hit distinct banks.
__device__ __forceinline__ int k8_swz(int r) { return ((r >> 2) & 1) | ((((r >> 1) ^ (r >> 3)) & 1) << 1); }

// byte offset of (row, k) in one operand part with nkc 64-byte chunks per row
__device__ __forceinline__ int64_t k8_at(int row, int k, int nkc) {
    const int rr = row & 15, q = (k >> 4) & 3;
    return (((int64_t)(row >> 6) * nkc + (k >> 6)) * 4 + ((row >> 4) & 3)) * 1024 + (4 * rr + (q ^ k8_swz(rr))) * 16 +
           (k & 15);
}

// digits of a batch as H int8 planes (the pieces of each digit, least significant
// first), row c, k = i N + m (zero past l N), in the tiled operand layout (a_half bytes
// per plane), and the output's start value out = (add_a, add_b + sigma(b)); grid
// (ceil(N / 256), n)
template <int H>
__global__ void __launch_bounds__(256) k_nat_aut_decomp8(const uint64_t *__restrict__ S, int64_t s_es,
                                                         const uint64_t *__restrict__ add, int64_t add_es,
                                                         uint64_t *__restrict__ out, int64_t out_es,
                                                         int8_t *__restrict__ A8, int64_t a_half, NatDims dm, int ginv,
                                                         NatGadget g, int KDp) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y, nkc = KDp >> 6, l = g.l;
    if (j < KDp - l * dm.N) {  // the padding of the row
        const int64_t o = k8_at(c, l * dm.N + j, nkc);
#pragma unroll
        for (int h = 0; h < H; ++h) A8[h * a_half + o] = 0;
    }
    if (j >= dm.N) return;
    const uint64_t *a = S + c * s_es, *b = a + dm.N;
    const uint64_t av = aut_at(a, j, ginv, dm), bv = aut_at(b, j, ginv, dm);
    const uint64_t *ad = add + c * add_es;
    uint64_t *o = out + c * out_es;
    o[j] = ad[j];
    o[dm.N + j] = ad[dm.N + j] + bv;
    uint64_t top = gadget_top(av, g);
    for (int i = l - 1; i >= 0; --i) {
        const int d = gadget_digit(top, g);
        const int64_t o = k8_at(c, i * dm.N + j, nkc);
        if constexpr (H == 2) {  // d = p0 + 16 p1, p0 in [-8, 8), p1 in [-16, 16] (|d| <= 256)
            const int p1 = (d + 8) >> 4;
            A8[o] = (int8_t)(d - 16 * p1);
            A8[a_half + o] = (int8_t)p1;
        } else {  // d = p0 + 32 p1 + 1024 p2, p0, p1 in [-16, 16), p2 in [-32, 32] (|d| <= 2^15)
            const int p0 = ((d + 16) & 31) - 16, d1 = (d - p0) >> 5;
            const int p1 = ((d1 + 16) & 31) - 16, p2 = (d1 - p1) >> 5;
            A8[o] = (int8_t)p0;
            A8[a_half + o] = (int8_t)p1;
            A8[2 * a_half + o] = (int8_t)p2;
        }
    }
}

// out[c][p][j] -= sum_k d[c][k] K_p[j][k] (mod 2^64) on the matrix cores.  Workgroup:
// 64 ciphertexts x 64 coefficients, four waves of 32 x 32 (2 x 2 tiles of 16 x 16),
// v_mfma_i32_16x16x64_i8: lane l feeds row (or column) l mod 16 with the 16 bytes at
// k0 + 16 (l / 16), the same k positions for both operands, so the product is
// independent of how the instruction orders k; result lane l, register r: row
// 4 (l / 16) + r, column l mod 16.  Byte planes go one at a time (b outer), each
// folded into the 64-bit results after its K loop.
//
// Staging: a stage is one 64-byte K chunk of both operands (the digit pieces of 64
// ciphertexts and both key parts of 64 coefficients: 4 H + 8 blocks of 1 KiB holding 16
// rows each, contiguous in the tiled operand layout and copied to LDS as they are).
// The chunks of all planes form one sequence; their loads go straight from global
// memory into a ring of K8_NS stages in LDS (global_load_lds, 16 bytes per lane, no
// registers), one stage fewer than the ring ahead of the products.  Each wave fills a
// quarter of every stage's blocks and waits only for its own loads of the stage it
// reads next (vmcnt); a barrier then tells every wave that all loads of that stage have
// landed and that the slot it refills next has been read.  With two pieces the
// fragments are double-buffered in registers, so a stage's products run while the next
// stage's fragments are read.
// Rows past the batch or the ring (the padding of the last tile) hold any values and
// only feed outputs that are not written.  grid.z splits K as in k_nat_ksprod.
constexpr int K8_NS = 4;  // stages in the LDS ring (two digit pieces)

typedef __attribute__((address_space(3))) void *lds_ptr_t;

// wait until at most N vector-memory operations of this wave are outstanding and all
// of its LDS operations are done
template <int N>
__device__ __forceinline__ void k8_wait() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (0 << 8));
}

// Tile of this workgroup.  Workgroups go to the eight XCDs round-robin by linear id;
// each XCD is given a contiguous run of tiles instead, ordered in groups of K8_GROUP
// ciphertext tiles (coefficient tiles outer within a group), so that the workgroups
// resident on one XCD at a time share their digit and key chunks in its L2.  The K
// split is outermost.
constexpr int K8_GROUP = 8;
__device__ __forceinline__ void k8_tile(int &tc, int &tj, int &tz) {
    const int gx = gridDim.x, gy = gridDim.y, G = gx * gy * gridDim.z;
    const int pid = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const int xcd = pid & 7, q = G >> 3, r = G & 7;
    const int L = xcd * q + min(xcd, r) + (pid >> 3);
    const int per_z = gx * gy;
    tz = L / per_z;
    const int m = L - tz * per_z, span = K8_GROUP * gx;
    const int grp = m / span, first = grp * K8_GROUP, gsize = min(gy - first, K8_GROUP);
    const int in = m - grp * span;
    tc = first + in % gsize;
    tj = in / gsize;
}

// H digit pieces (2 for D <= 512: d = p0 + 16 p1; 3 for larger D up to 2^16: d = p0 +
// 32 p1 + 1024 p2), each an int8 plane of the tiled layout; a stage holds 4 H + 8
// blocks.  Three pieces take a three-stage ring and single-buffered fragments (the
// accumulators grow by half).
template <int H>
struct K8Cfg {
    static constexpr int NS = H == 2 ? K8_NS : 3;   // stages in the ring
    static constexpr int NB = 4 * H + 8;            // 1 KiB blocks per stage
    static constexpr int BPW = NB / 4;              // blocks each wave loads
    static constexpr int STAGE = NB * 1024;
    static constexpr int NF = H == 2 ? 2 : 1;       // fragment buffers
    static constexpr int SHIFT = H == 2 ? 4 : 5;    // piece h weighs 2^(SHIFT h)
};

template <int H>
__global__ void __launch_bounds__(256, 2) k_nat_ksprod8(const int8_t *__restrict__ A8, int64_t a_half,
                                                     const int8_t *__restrict__ B8, uint64_t *__restrict__ out,
                                                     int64_t out_es, int n, int N, int KDp, int kc) {
    using C = K8Cfg<H>;
    constexpr int NS = C::NS, NB = C::NB, BPW = C::BPW, STAGE = C::STAGE, NF = C::NF;
    __shared__ __attribute__((aligned(16))) int8_t ring[NS * STAGE];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int tc, tj, tz;
    k8_tile(tc, tj, tz);
    const int c0 = tc * 64, j0 = tj * 64;
    const int wc = (w & 1) * 32, wj = (w >> 1) * 32;
    const int kb = tz * kc, ke = min(KDp, kb + kc);
    const int nk = (ke - kb) >> 6, total = 8 * nk;  // chunks per plane, stages in all
    const int r16 = lane & 15, g = lane >> 4;
    const int64_t plane = (int64_t)((N + 63) & ~63) * KDp;  // bytes per key byte plane
    // loads: wave w fills blocks BPW w .. BPW w + BPW - 1 of a stage; block 4 h + t holds
    // rows 16 t .. 16 t + 15 of digit piece h, block 4 H + 4 p + t those of key part p;
    // lane l the 16 bytes at 16 l of the block
    const int nkc = KDp >> 6;
    const int8_t *src[BPW];
    bool keyb[BPW];
#pragma unroll
    for (int i = 0; i < BPW; ++i) {
        const int bl = BPW * w + i;
        keyb[i] = bl >= 4 * H;
        const int part = (keyb[i] ? bl - 4 * H : bl) >> 2, t = bl & 3;
        src[i] = (keyb[i] ? B8 + (int64_t)part * 8 * plane + ((int64_t)tj * nkc * 4 + t) * 1024
                          : A8 + part * a_half + ((int64_t)tc * nkc * 4 + t) * 1024) +
                 16 * lane;
    }
    auto issue = [&](int st) {
        const int b = st / nk, kcs = (kb >> 6) + (st - b * nk);
        int8_t *dst = ring + (st % NS) * STAGE + w * BPW * 1024;
#pragma unroll
        for (int i = 0; i < BPW; ++i)
            __builtin_amdgcn_global_load_lds(
                (const void *)(src[i] + (keyb[i] ? (int64_t)b * plane : 0) + (int64_t)kcs * 4096),
                (lds_ptr_t)(dst + i * 1024), 16, 0, 0);
    };
    uint64_t res[2][2][2][4];
    v4i acc[2][H][2][2];  // [part][piece][c tile][j tile]
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int bq = 0; bq < 2; ++bq) {
#pragma unroll
                for (int r = 0; r < 4; ++r) res[p][a][bq][r] = 0;
#pragma unroll
                for (int h = 0; h < H; ++h) acc[p][h][a][bq] = v4i{0, 0, 0, 0};
            }
    const int slot = 16 * (4 * r16 + (g ^ k8_swz(r16)));
    v4i fa[NF][H][2], fb[NF][2][2];
    auto frags = [&](int f, int st) {
        const int8_t *stg = ring + (st % NS) * STAGE + slot;
#pragma unroll
        for (int t2 = 0; t2 < 2; ++t2) {
#pragma unroll
            for (int h = 0; h < H; ++h) fa[f][h][t2] = *(const v4i *)(stg + 1024 * (4 * h + (wc >> 4) + t2));
#pragma unroll
            for (int p = 0; p < 2; ++p) fb[f][p][t2] = *(const v4i *)(stg + 1024 * (4 * H + 4 * p + (wj >> 4) + t2));
        }
    };
    auto products = [&](int f) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int h = 0; h < H; ++h)
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int bq = 0; bq < 2; ++bq)
                        acc[p][h][a][bq] =
                            __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[f][h][a], fb[f][p][bq], acc[p][h][a][bq], 0, 0, 0);
    };
    auto fold = [&](int it) {  // after the last chunk of plane b: fold and restart
        if ((it + 1) % nk) return;
        const int b = it / nk;
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int bq = 0; bq < 2; ++bq) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        int64_t v = 0;
#pragma unroll
                        for (int h = 0; h < H; ++h) v += (int64_t)acc[p][h][a][bq][r] << (C::SHIFT * h);
                        res[p][a][bq][r] += (uint64_t)v << (8 * b);
                    }
#pragma unroll
                    for (int h = 0; h < H; ++h) acc[p][h][a][bq] = v4i{0, 0, 0, 0};
                }
    };
    // every wave's loads of stage it + 1 are in LDS and every wave has its fragments of
    // stage it in registers (own LDS reads drained), so stage it's slot can be refilled
    auto sync_next = [&](int it) {
        if (it + NS - 1 < total) k8_wait<BPW * (NS - 2)>();
        else k8_wait<0>();
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    };
    // the ring starts full; stage it's products run while stage it + 1's fragments are
    // read (into the other buffer when there are two) and stage it + NS is loaded into
    // the slot stage it left
    for (int st = 0; st < NS && st < total; ++st) issue(st);
    if (NS - 1 < total) k8_wait<BPW * (NS - 1)>();
    else k8_wait<0>();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    frags(0, 0);
    for (int it = 0; it < total; it += 2) {
        products(0);
        if (it + 1 < total) {
            sync_next(it);
            if (it + NS < total) issue(it + NS);
            frags(1 % NF, it + 1);
        }
        fold(it);
        if (it + 1 >= total) break;
        products(1 % NF);
        if (it + 2 < total) {
            sync_next(it + 1);
            if (it + 1 + NS < total) issue(it + 1 + NS);
            frags(0, it + 2);
        }
        fold(it + 1);
    }
    const bool split = gridDim.z > 1;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = c0 + wc + a * 16 + 4 * g + r;
            if (c >= n) continue;
            uint64_t *o = out + c * out_es;
#pragma unroll
            for (int bq = 0; bq < 2; ++bq) {
                const int j = j0 + wj + bq * 16 + r16;
                if (j >= N) continue;
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    uint64_t *dst = o + p * N + j;
                    if (split) atomicAdd((unsigned long long *)dst, (unsigned long long)(0 - res[p][a][bq][r]));
                    else *dst -= res[p][a][bq][r];
                }
            }
        }
}

// balanced byte planes of the key product matrices: plane B8[lv][p][b] holds s_b of
// coefficient j of X^m k_(lv, i, p) at row j, k = i N + m (zero for k >= l N and for
// the padding rows j >= N) in the tiled operand layout; grid (ceil(JP / 256), KDp,
// levels * 2), JP = N rounded up to 64
__global__ void __launch_bounds__(256) k_nat_kmat8(const uint64_t *__restrict__ ksk, int8_t *__restrict__ B8, NatDims dm,
                                                   int l, int KDp) {
    const int JP = (dm.N + 63) & ~63;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= JP) return;
    const int km = blockIdx.y;
    const int lv = blockIdx.z >> 1, p = blockIdx.z & 1;
    uint64_t v = 0;
    if (km < l * dm.N && j < dm.N) {
        const int i = km / dm.N, m = km % dm.N;
        v = mono_at(ksk + (((int64_t)lv * l + i) * 2 + p) * dm.N, j, m, dm);
    }
    const int64_t plane = (int64_t)JP * KDp;
    int8_t *o = B8 + ((int64_t)(lv * 2 + p) * 8) * plane + k8_at(j, km, KDp >> 6);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        int s = (int)(v & 0xff);
        s -= s >= 128 ? 256 : 0;
        v = (v - (uint64_t)(int64_t)s) >> 8;
        o[b * plane] = (int8_t)s;
    }
}

// key product matrices: K[lv][p][j][i N + m] = coefficient j of X^m k_(lv, i, p);
// grid (ceil(N / 256), l N, levels * 2)
__global__ void __launch_bounds__(256) k_nat_kmat(const uint64_t *__restrict__ ksk, uint64_t *__restrict__ K, NatDims dm,
                                                  int l) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= dm.N) return;
    const int km = blockIdx.y, i = km / dm.N, m = km % dm.N;
    const int lv = blockIdx.z >> 1, p = blockIdx.z & 1;
    const uint64_t *k = ksk + (((int64_t)lv * l + i) * 2 + p) * dm.N;
    const int64_t KD = (int64_t)l * dm.N;
    K[(((int64_t)lv * 2 + p) * dm.N + j) * KD + km] = mono_at(k, j, m, dm);
}

// corr[lv][p][j] = (D/2) sum_k K[lv][p][j][k]; one workgroup per row (lv, p, j)
__global__ void __launch_bounds__(256) k_nat_kcorr(const uint64_t *__restrict__ K, uint64_t *__restrict__ corr,
                                                   int64_t KD, uint64_t half_d) {
    __shared__ uint64_t part[256];
    const uint64_t *row = K + (int64_t)blockIdx.x * KD;
    uint64_t s = 0;
    for (int64_t k = threadIdx.x; k < KD; k += 256) s += row[k];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) corr[blockIdx.x] = part[0] * half_d;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
const char *const NAT_KIND_NAMES[NK_COUNT] = {"extract", "linear", "leaves", "merge", "aut_decomp", "ksprod", "kmat"};

NatProf::NatProf(Native *n_, hipStream_t s_, int k, double u, double by) : n(n_), s(s_), kind(k), units(u), bytes(by) {
    if (!n->prof) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventRecord(a, s) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
    }
    on = true;
}

NatProf::~NatProf() {
    if (!on) return;
    hipEvent_t b;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
    }
    (void)hipEventRecord(b, s);
    n->pending.push_back(Native::Rec{kind, a, b, units, bytes});
}

static void nat_prof_drain(Native *n) {
    for (auto &r : n->pending) {
        float ms = 0;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            n->sum_ms[r.kind] += ms;
            n->sum_units[r.kind] += r.units;
            n->sum_bytes[r.kind] += r.bytes;
            n->launches[r.kind] += 1;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    n->pending.clear();
}

int native_profile_enable(Native *n, bool on) {
    nat_prof_drain(n);
    for (int k = 0; k < NK_COUNT; ++k) {
        n->sum_ms[k] = n->sum_units[k] = n->sum_bytes[k] = 0;
        n->launches[k] = 0;
    }
    n->prof = on;
    return FHELIN_OK;
}

int native_profile_read(Native *n, const char *kind, int64_t *launches, double *ms, double *units, double *bytes) {
    FL_CHECK(kind, FHELIN_E_INVALID_ARG, "null kernel class");
    nat_prof_drain(n);
    for (int k = 0; k < NK_COUNT; ++k) {
        if (std::strcmp(kind, NAT_KIND_NAMES[k]) != 0) continue;
        if (launches) *launches = n->launches[k];
        if (ms) *ms = n->sum_ms[k];
        if (units) *units = n->sum_units[k];
        if (bytes) *bytes = n->sum_bytes[k];
        return FHELIN_OK;
    }
    return set_error(FHELIN_E_INVALID_ARG, std::string("unknown native kernel class: ") + kind);
}
static bool is_odd_prime(int t) {
    if (t < 3 || t % 2 == 0) return false;
    for (int f = 3; f * f <= t; f += 2)
        if (t % f == 0) return false;
    return true;
}

static int64_t ipow(int64_t b, int e) {
    int64_t r = 1;
    while (e-- > 0) r *= b;
    return r;
}

static int64_t inv_mod(int64_t a, int64_t m) {
    // extended Euclid; a and m coprime
    int64_t g = m, x = 0, x1 = 1, aa = a % m;
    if (aa < 0) aa += m;
    while (aa) {
        const int64_t q = g / aa;
        int64_t t = g - q * aa;
        g = aa;
        aa = t;
        t = x - q * x1;
        x = x1;
        x1 = t;
    }
    x %= m;
    return x < 0 ? x + m : x;
}

int native_create(const fhelin_native_params *prm, Native **out) {
    FL_CHECK(prm && out, FHELIN_E_INVALID_ARG, "native_create: null argument");
    const fhelin_native_params &q = *prm;
    FL_CHECK(is_odd_prime(q.t), FHELIN_E_UNSUPPORTED_PARAM, "t must be an odd prime");
    FL_CHECK(q.alpha >= 2 && ipow(q.t, q.alpha) <= NAT_MAX_M, FHELIN_E_UNSUPPORTED_PARAM,
             "M = t^alpha must satisfy alpha >= 2 and M <= " + std::to_string(NAT_MAX_M));
    FL_CHECK(q.gamma >= 1 && q.gamma <= 2 && q.gamma <= q.beta && q.beta <= q.alpha - 1, FHELIN_E_UNSUPPORTED_PARAM,
             "need 1 <= gamma <= 2 and gamma <= beta <= alpha - 1");
    NatGadget gad;
    gad.l = q.l;
    FL_CHECK(q.l >= 1 && q.l <= 8, FHELIN_E_UNSUPPORTED_PARAM, "gadget: 1 <= l <= 8");
    if (q.base == 0) {
        FL_CHECK(q.log_d >= 1 && q.log_d <= 16 && q.log_d * q.l < 64, FHELIN_E_UNSUPPORTED_PARAM,
                 "gadget: 1 <= log_d <= 16, log_d l < 64");
        gad.log_d = q.log_d;
        gad.D = 1ull << q.log_d;
    } else {
        FL_CHECK(q.base >= 4 && q.base <= 65536 && q.base % 2 == 0, FHELIN_E_UNSUPPORTED_PARAM,
                 "gadget base: even, 4..65536");
        gad.D = (uint64_t)q.base;
    }
    if (q.base != 0) {  // D^l, the scale of the rounding (a power of two rounds by shifts)
        gad.Dl = 1;
        for (int i = 0; i < q.l; ++i) {
            FL_CHECK(gad.Dl <= ((1ull << 63) - 1) / gad.D, FHELIN_E_UNSUPPORTED_PARAM, "gadget: D^l must be below 2^63");
            gad.Dl *= gad.D;
        }
    }
    FL_CHECK(q.log_p >= 1 && q.log_p <= 31, FHELIN_E_UNSUPPORTED_PARAM, "message modulus: 1 <= log_p <= 31");
    FL_CHECK(q.engine == 0 || q.engine == 1, FHELIN_E_UNSUPPORTED_PARAM, "engine: 0 (int8 matrix cores) or 1 (ALU)");
    FL_CHECK(q.engine == 1 || (gad.D <= 65536 && (int64_t)q.l * ipow(q.t, q.alpha) <= (1 << 19)),
             FHELIN_E_UNSUPPORTED_PARAM, "the int8 engine splits digits into int8 pieces: D <= 2^16");
    std::unique_ptr<Native> n(new Native());
    n->prm = q;
    n->gad = gad;
    n->M = (int)ipow(q.t, q.alpha);
    n->Mt = n->M / q.t;
    n->N = n->M - n->Mt;
    n->n_pack = (int)((q.t - 1) * ipow(q.t, q.beta - 1));
    n->T = (int)ipow(q.t, q.beta - q.gamma);
    n->phig = (int)((q.t - 1) * ipow(q.t, q.gamma - 1));
    n->KDp = (q.l * n->N + 63) / 64 * 64;
    const int64_t p = 1ll << q.log_p;
    int64_t u = inv_mod(n->M, p);
    if (u > p / 2) u -= p;
    n->u = (uint64_t)u;
    FL_CHECK(n->phig <= NAT_MAX_POW, FHELIN_E_UNSUPPORTED_PARAM, "too many powers at this gamma");
    if (q.gamma == 1) {
        for (int k = 1; k < q.t; ++k) n->powers.push_back(k);
    } else {
        for (int k = 1; k < q.t; ++k)
            for (int j = 0; j < q.t; ++j) n->powers.push_back((int)(((int64_t)k * (j * q.t + 1)) % n->M));
    }
    for (int i = q.gamma; i < q.alpha; ++i) {
        const int g = (int)((1 + ipow(q.t, i)) % n->M);
        n->tau.push_back(g);
        n->tau_inv.push_back((int)inv_mod(g, n->M));
    }
    FL_TRY_HIP(hipGetDevice(&n->device));
    FL_TRY_HIP(hipDeviceGetAttribute(&n->cus, hipDeviceAttributeMultiprocessorCount, n->device));
    FL_TRY_HIP(hipDeviceGetAttribute(&n->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, n->device));
    *out = n.release();
    return FHELIN_OK;
}

void native_destroy(Native *n) {
    if (!n) return;
    (void)hipSetDevice(n->device);
    (void)hipDeviceSynchronize();
    nat_prof_drain(n);
    if (n->kmat) (void)hipFree(n->kmat);
    if (n->kmat8) (void)hipFree(n->kmat8);
    if (n->wt) (void)hipFree(n->wt);
    if (n->kcorr) (void)hipFree(n->kcorr);
    if (n->ws) (void)hipFree(n->ws);
    delete n;
}

static int nat_workspace(Native *n, size_t bytes, hipStream_t s, uint8_t **out) {
    if (n->ws_bytes < bytes) {
        if (n->ws) {
            FL_TRY_HIP(hipStreamSynchronize(s));
            FL_TRY_HIP(hipFree(n->ws));
            n->ws = nullptr;
            n->ws_bytes = 0;
        }
        if (hipMalloc(&n->ws, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(FHELIN_E_OOM, "native workspace: device allocation failed");
        }
        n->ws_bytes = bytes;
    }
    *out = (uint8_t *)n->ws;
    return FHELIN_OK;
}

static NatDims dims(const Native *n) { return NatDims{n->M, n->N, n->Mt}; }

int native_keys_load(Native *n, const uint64_t *ksk, hipStream_t s) {
    FL_CHECK(n && ksk, FHELIN_E_INVALID_ARG, "native_keys_load: null argument");
    const int levels = (int)n->tau.size(), l = n->prm.l;
    const int64_t KD = (int64_t)l * n->N;
    const NatDims dm = dims(n);
    if (n->prm.engine == 0) {
        const int JP = (n->N + 63) & ~63;
        const size_t bytes8 = (size_t)levels * 2 * 8 * JP * n->KDp;
        if (!n->kmat8 && hipMalloc((void **)&n->kmat8, bytes8) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(FHELIN_E_OOM, "native keys: device allocation failed");
        }
        NatProf ps(n, s, NK_KMAT, (double)levels * 2 * n->N * n->KDp, (double)bytes8 + levels * l * 2.0 * n->N * 8);
        hipLaunchKernelGGL(k_nat_kmat8, dim3((JP + 255) / 256, (unsigned)n->KDp, levels * 2), dim3(256), 0, s, ksk,
                           n->kmat8, dm, l, n->KDp);
        FL_TRY_HIP(hipGetLastError());
        n->keys = true;
        return FHELIN_OK;
    }
    const size_t kbytes = (size_t)levels * 2 * n->N * KD * sizeof(uint64_t);
    if (!n->kmat) {
        if (hipMalloc((void **)&n->kmat, kbytes) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(FHELIN_E_OOM, "native keys: device allocation failed");
        }
        if (hipMalloc((void **)&n->kcorr, (size_t)levels * 2 * n->N * sizeof(uint64_t)) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(FHELIN_E_OOM, "native keys: device allocation failed");
        }
    }
    {
        NatProf ps(n, s, NK_KMAT, (double)levels * 2 * n->N * KD, (double)kbytes + levels * l * 2.0 * n->N * 8);
        hipLaunchKernelGGL(k_nat_kmat, dim3((n->N + 255) / 256, (unsigned)KD, levels * 2), dim3(256), 0, s, ksk, n->kmat,
                           dm, l);
        FL_TRY_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_nat_kcorr, dim3(levels * 2 * n->N), dim3(256), 0, s, n->kmat, n->kcorr, KD, n->gad.D >> 1);
        FL_TRY_HIP(hipGetLastError());
    }
    n->keys = true;
    return FHELIN_OK;
}

// the streamed kernel's instance for M (positions per thread X = ceil(M / EXS_T)) and t
// (rows per workgroup Q: 2 for t <= 5, else 3; with more, the accumulators leave room for
// one workgroup per compute unit only, measured slower: 16.0 against 15.1 ms of
// extraction per ResNet-20 inference for M = 7^4 at gamma = 2 with Q = 6 and 3)
using ExsKernel = void (*)(const uint64_t *, uint64_t *, NatDims, NatPowers, uint64_t, int);
template <int Q>
static ExsKernel exs_kernel_q(int X) {
    switch (X) {
    case 1: return k_nat_extract_stream<1, Q>;
    case 2: return k_nat_extract_stream<2, Q>;
    case 3: return k_nat_extract_stream<3, Q>;
    case 4: return k_nat_extract_stream<4, Q>;
    case 5: return k_nat_extract_stream<5, Q>;
    case 6: return k_nat_extract_stream<6, Q>;
    case 7: return k_nat_extract_stream<7, Q>;
    case 8: return k_nat_extract_stream<8, Q>;
    default: return nullptr;
    }
}
static int exs_rows(int t) { return t <= 5 ? 2 : 3; }
static ExsKernel exs_kernel(int M, int t) {
    const int X = (M + EXS_T - 1) / EXS_T;
    switch (exs_rows(t)) {
    case 2: return exs_kernel_q<2>(X);
    case 3: return exs_kernel_q<3>(X);
    default: return nullptr;
    }
}

// the LDS-staged merge kernel's instance for M and t (nullptr: the gather kernel)
using MgsKernel = void (*)(const uint64_t *, uint64_t *, NatDims, int, int);
template <int TT>
static MgsKernel mgs_kernel_t(int X) {
    switch (X) {
    case 1: return k_nat_merge_s<1, TT>;
    case 2: return k_nat_merge_s<2, TT>;
    case 3: return k_nat_merge_s<3, TT>;
    case 4: return k_nat_merge_s<4, TT>;
    case 5: return k_nat_merge_s<5, TT>;
    case 6: return k_nat_merge_s<6, TT>;
    case 7: return k_nat_merge_s<7, TT>;
    case 8: return k_nat_merge_s<8, TT>;
    default: return nullptr;
    }
}
static MgsKernel mgs_kernel(int M, int t) {
    const int X = (M + MGS_T - 1) / MGS_T;
    if (M > MGS_SLOT) return nullptr;
    switch (t) {
    case 3: return mgs_kernel_t<3>(X);
    case 5: return mgs_kernel_t<5>(X);
    case 7: return mgs_kernel_t<7>(X);
    default: return nullptr;
    }
}

int native_extract(Native *n, const uint64_t *pows, int n_chunks, uint64_t *rows, hipStream_t s) {
    FL_CHECK(n && pows && rows && n_chunks >= 0, FHELIN_E_INVALID_ARG, "native_extract: null argument");
    FL_CHECK(n_chunks <= 65535, FHELIN_E_INVALID_ARG, "native_extract: at most 65535 chunks per call");
    if (n_chunks == 0) return FHELIN_OK;
    NatPowers pw{};
    pw.n = (int)n->powers.size();
    for (int k = 0; k < pw.n; ++k) pw.d[k] = n->powers[k];
    // bytes: the chunks' powers read once, the rows written
    const double ctb = 16.0 * n->N;
    NatProf ps(n, s, NK_EXTRACT, (double)n_chunks * n->N, n_chunks * (pw.n * ctb + (double)n->N * ctb));
    const size_t lds = (size_t)pw.n * 2 * n->N * sizeof(uint64_t);
    // the staged kernel needs two workgroups per compute unit to hide its staging (with
    // one, the gather kernel measured faster: 5.5 against 8.0 ms per ResNet-20
    // inference at M = 3^7, gamma = 2) and keeps its dynamic LDS within 64 KiB
    if (n->N <= EXT_T * EXT_J && 2 * lds <= (size_t)n->lds_max && lds <= 65536) {
        // about two workgroups per resident slot (a slot per compute unit and whole
        // copy of the powers that fits its LDS): each copy serves as many rows as can be
        const int per_cu = std::max(1, (int)(std::max(n->lds_max, 1) / std::max<size_t>(lds, 1)));
        const int groups = std::max(1, (2 * std::max(n->cus, 1) * per_cu + n_chunks - 1) / n_chunks);
        const int rpg = std::max(4, (n->N + groups - 1) / groups);
        hipLaunchKernelGGL(k_nat_extract_lds, dim3((n->N + rpg - 1) / rpg, n_chunks), dim3(EXT_T), lds, s, pows, rows,
                           dims(n), pw, n->u, rpg);
    } else if (n->M <= EXS_SLOT) {
        const int Q = exs_rows(n->prm.t), passes = (n->prm.t - 1 + Q - 1) / Q;
        hipLaunchKernelGGL(exs_kernel(n->M, n->prm.t), dim3(n->Mt * passes, n_chunks), dim3(EXS_T), 0, s, pows,
                           rows, dims(n), pw, n->u, n->prm.t);
    } else {
        const int passes = (n->prm.t - 2) / EXT_Q + 1;  // ceil((t - 1) / EXT_Q)
        hipLaunchKernelGGL(k_nat_extract, dim3((n->N + 255) / 256, n->Mt * passes, n_chunks), dim3(256), 0, s, pows,
                           rows, dims(n), pw, n->u, n->prm.t);
    }
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

int native_linear(Native *n, const int32_t *row_ptr, const int32_t *col, const int32_t *val, int n_out,
                  const uint64_t *rows, uint64_t *out, hipStream_t s) {
    FL_CHECK(n && row_ptr && col && val && rows && out && n_out >= 0, FHELIN_E_INVALID_ARG,
             "native_linear: null argument");
    FL_CHECK(n_out <= 65535, FHELIN_E_INVALID_ARG, "native_linear: at most 65535 outputs per call");
    if (n_out == 0) return FHELIN_OK;
    const int n2 = 2 * n->N;
    // units: products; bytes: every referenced row once and the outputs (the rows shared
    // between outputs are read again from the caches)
    int32_t nnz = 0;
    if (n->prof) FL_TRY_HIP(hipMemcpy(&nnz, row_ptr + n_out, sizeof(nnz), hipMemcpyDeviceToHost));
    NatProf ps(n, s, NK_LINEAR, (double)nnz * n2, (double)n_out * n2 * 8.0);
    hipLaunchKernelGGL(k_nat_linear, dim3((n2 + 255) / 256, n_out), dim3(256), 0, s, row_ptr, col, val, rows, out, n2);
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

size_t native_pack_workspace(const Native *n, int n_rows) {
    const size_t packs = (size_t)(n_rows + n->n_pack - 1) / n->n_pack;
    const size_t ct = 2 * (size_t)n->N * sizeof(uint64_t);
    const size_t nmax = packs * n->T;  // the leaves: the widest level
    // current sub-packs, merge terms (t per merge), results, and the digits of a
    // key-switch batch
    const size_t dig = std::max(nmax * (size_t)n->prm.l * n->N * sizeof(uint32_t), 3 * ((nmax + 63) & ~(size_t)63) * n->KDp);
    return 3 * nmax * ct + dig;
}

// K chunks per workgroup of the int8 product for `tiles` output tiles, `chunks` 64-byte
// K chunks and `slots` resident workgroups: the split whose rounds of workgroups times
// chunks per workgroup (plus a few chunks' worth of set-up and atomics per split) is
// least, fewest splits on ties, at most 32 splits.
static int k8_split(int tiles, int chunks, int slots) {
    int best = chunks;
    double best_cost = 1e300;
    for (int s = 1; s <= 32 && s <= chunks; ++s) {
        const int per = (chunks + s - 1) / s, gz = (chunks + per - 1) / per;
        const double rounds = std::ceil((double)tiles * gz / slots);
        const double cost = rounds * (per + 4.0) + (gz > 1 ? 1.0 : 0.0);
        if (cost < best_cost - 1e-9) {
            best_cost = cost;
            best = per;
        }
    }
    return best;
}

// out = add + tau(S) for a batch of cnt ciphertexts with the key of tower level lv; out
// overlaps neither S nor add.
static int nat_ks_step(Native *n, int lv, const uint64_t *S, int64_t s_es, const uint64_t *add, int64_t add_es,
                       uint64_t *out, int64_t out_es, int cnt, uint32_t *dig, hipStream_t s) {
    const NatDims dm = dims(n);
    const int l = n->prm.l;
    const int64_t KD = (int64_t)l * n->N;
    for (int c0 = 0; c0 < cnt; c0 += 65535) {
        const int c = std::min(cnt - c0, 65535);
        if (n->prm.engine == 0) {
            int8_t *A8 = (int8_t *)dig;
            const bool three = n->gad.D > 512;  // digit pieces: 2, or 3 beyond D = 2^9
            const int64_t a_half = (int64_t)((c + 63) & ~63) * n->KDp;
            {
                NatProf pa(n, s, NK_AUT_DECOMP, (double)c * n->N, (double)c * n->N * (2 * 8.0 + 2 * 8.0 + 2 * 8.0 + 2.0 * l));
                const dim3 gd((std::max(n->N, n->KDp - (int)KD) + 255) / 256, c);
                if (three)
                    hipLaunchKernelGGL(k_nat_aut_decomp8<3>, gd, dim3(256), 0, s, S + c0 * s_es, s_es, add + c0 * add_es,
                                       add_es, out + c0 * out_es, out_es, A8, a_half, dm, n->tau_inv[lv], n->gad, n->KDp);
                else
                    hipLaunchKernelGGL(k_nat_aut_decomp8<2>, gd, dim3(256), 0, s, S + c0 * s_es, s_es, add + c0 * add_es,
                                       add_es, out + c0 * out_es, out_es, A8, a_half, dm, n->tau_inv[lv], n->gad, n->KDp);
                FL_TRY_HIP(hipGetLastError());
            }
            const int gx = (n->N + 63) / 64, gy = (c + 63) / 64;
            const int kc = 64 * k8_split(gx * gy, n->KDp / 64, 2 * std::max(n->cus, 1));
            const int gz = (n->KDp + kc - 1) / kc;
            const int8_t *B8 = n->kmat8 + (int64_t)lv * 2 * 8 * ((n->N + 63) & ~63) * n->KDp;
            // units: 64-bit products (both key parts); bytes: the digit planes and the
            // sixteen key planes once per launch, the output read and written
            NatProf pk(n, s, NK_KSPROD, 2.0 * c * n->N * (double)KD,
                       (three ? 3.0 : 2.0) * c * n->KDp + 16.0 * n->N * n->KDp + (double)c * n->N * 8 * 4);
            if (three)
                hipLaunchKernelGGL(k_nat_ksprod8<3>, dim3(gx, gy, gz), dim3(256), 0, s, A8, a_half, B8, out + c0 * out_es,
                                   out_es, c, n->N, n->KDp, kc);
            else
                hipLaunchKernelGGL(k_nat_ksprod8<2>, dim3(gx, gy, gz), dim3(256), 0, s, A8, a_half, B8, out + c0 * out_es,
                                   out_es, c, n->N, n->KDp, kc);
            FL_TRY_HIP(hipGetLastError());
            continue;
        }
        const uint64_t *Ka = n->kmat + (int64_t)lv * 2 * n->N * KD, *Kb = Ka + (int64_t)n->N * KD;
        const uint64_t *ca = n->kcorr + (int64_t)lv * 2 * n->N, *cb = ca + n->N;
        {
            NatProf pa(n, s, NK_AUT_DECOMP, (double)c * n->N, (double)c * n->N * (2 * 8.0 + 2 * 8.0 + 2 * 8.0 + 4.0 * l));
            hipLaunchKernelGGL(k_nat_aut_decomp, dim3((n->N + 255) / 256, c), dim3(256), 0, s, S + c0 * s_es, s_es,
                               add + c0 * add_es, add_es, out + c0 * out_es, out_es, ca, cb, dig, dm, n->tau_inv[lv],
                               n->gad);
            FL_TRY_HIP(hipGetLastError());
        }
        // a small batch splits K so that about 1024 workgroups run
        const int gx = (n->N + KS_TJ - 1) / KS_TJ, gy = (c + KS_TC - 1) / KS_TC;
        const int splits = std::max(1, std::min(16, 1024 / (gx * gy)));
        const int kc = (int)(((KD + splits - 1) / splits + KS_TK - 1) / KS_TK * KS_TK);
        const int gz = (int)((KD + kc - 1) / kc);
        // units: 64-bit products (both key parts); bytes: digits, both key matrices (once
        // per launch) and the output read and written
        NatProf pk(n, s, NK_KSPROD, 2.0 * c * n->N * (double)KD,
                   (double)c * KD * 4 + 2.0 * n->N * KD * 8 + (double)c * n->N * 8 * 4);
        hipLaunchKernelGGL(k_nat_ksprod, dim3(gx, gy, gz), dim3(256), 0, s, dig, Ka, Kb, out + c0 * out_es, out_es, c, n->N,
                           (int)KD, kc);
        FL_TRY_HIP(hipGetLastError());
    }
    return FHELIN_OK;
}

int native_pack(Native *n, const uint64_t *rows, int n_rows, uint64_t *packed, hipStream_t s) {
    FL_CHECK(n && rows && packed && n_rows >= 0, FHELIN_E_INVALID_ARG, "native_pack: null argument");
    FL_CHECK(n->keys, FHELIN_E_MISSING_GALOIS_KEY, "native_pack: keys not loaded");
    if (n_rows == 0) return FHELIN_OK;
    const int t = n->prm.t, packs = (n_rows + n->n_pack - 1) / n->n_pack;
    FL_CHECK(packs <= 65535 && (int64_t)packs * n->T <= (1 << 22), FHELIN_E_INVALID_ARG,
             "native_pack: too many rows per call");
    const NatDims dm = dims(n);
    const int64_t ct = 2 * (int64_t)n->N;
    uint8_t *ws;
    FL_RET(nat_workspace(n, native_pack_workspace(n, n_rows), s, &ws));
    const int64_t nmax = (int64_t)packs * n->T;
    uint64_t *cur = (uint64_t *)ws, *v = cur + nmax * ct, *S = v + nmax * ct;
    uint32_t *dig = (uint32_t *)(S + nmax * ct);
    const unsigned gx = (n->N + 255) / 256;
    // leaves
    {
        NatProf ps(n, s, NK_LEAVES, (double)nmax * n->N, (double)(n_rows + nmax) * ct * 8);
        hipLaunchKernelGGL(k_nat_leaves, dim3(gx, n->T, packs), dim3(256), 0, s, rows, n_rows, cur, dm, n->n_pack, n->T,
                           n->phig, (int)(n->M / ipow(t, n->prm.gamma)));
        FL_TRY_HIP(hipGetLastError());
    }
    // merges up the tower: level i has len = t^(beta - i) sub-packs per pack
    int len = n->T;
    for (int i = n->prm.gamma; i < n->prm.beta; ++i) {
        const int lv = i - n->prm.gamma, step = len / t, th = (int)(n->M / ipow(t, i + 1));
        {
            NatProf pm(n, s, NK_MERGE, (double)packs * len * n->N, (double)packs * len * ct * 8 * 2);
            // the staged kernel when it has a workgroup per compute unit at least (with
            // fewer, the gather kernel's many small workgroups finish sooner)
            const MgsKernel mk = mgs_kernel(n->M, t);
            if (mk && (int64_t)step * packs >= std::max(n->cus, 1))
                hipLaunchKernelGGL(mk, dim3(step, packs), dim3(MGS_T), 0, s, cur, v, dm, step, th);
            else
                hipLaunchKernelGGL(k_nat_merge_v, dim3(gx, step * t, packs), dim3(256), 0, s, cur, v, dm, t, step, th);
            FL_TRY_HIP(hipGetLastError());
        }
        // S = v_(t-1); S = v_m + tau_i(S) for m = t-2 .. 0 (a merge's t terms are ct apart);
        // the results alternate between S and cur (consumed by the merge terms above)
        const int cnt = packs * step;
        const uint64_t *src = v + (int64_t)(t - 1) * ct;
        int64_t src_es = (int64_t)t * ct;
        uint64_t *dst = S, *other = cur;
        for (int m = t - 2; m >= 0; --m) {
            FL_RET(nat_ks_step(n, lv, src, src_es, v + (int64_t)m * ct, (int64_t)t * ct, dst, ct, cnt, dig, s));
            src = dst;
            src_es = ct;
            std::swap(dst, other);
        }
        // the level's result is in src; the other buffer is free
        cur = (uint64_t *)src;
        S = dst;
        len = step;
    }
    // Tr_{K/K_beta}: per level j = alpha-1 down to beta, T_j = P, T_j = P + tau_j(T_j)
    // (t - 1 times); the partial results alternate between the two free buffers
    uint64_t *fa = S, *fb = v;
    for (int j = n->prm.alpha - 1; j >= n->prm.beta; --j) {
        const int lv = j - n->prm.gamma;
        const uint64_t *src = cur;
        uint64_t *dst = fa, *other = fb;
        for (int k = 0; k < t - 1; ++k) {
            FL_RET(nat_ks_step(n, lv, src, ct, cur, ct, dst, ct, packs, dig, s));
            src = dst;
            std::swap(dst, other);
        }
        // result in src; the old P and the other buffer are free
        uint64_t *old = cur;
        cur = (uint64_t *)src;
        fa = old;
        fb = dst;
    }
    FL_TRY_HIP(hipMemcpyAsync(packed, cur, (size_t)packs * ct * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    return FHELIN_OK;
}

int native_conv(Native *n, int c_in, int c_out, int h, int w, int k, int stride, const int32_t *wts,
                const int32_t *out_row, const uint64_t *rows, uint64_t *out, hipStream_t s) {
    FL_CHECK(n && wts && out_row && rows && out, FHELIN_E_INVALID_ARG, "native_conv: null argument");
    FL_CHECK(c_in >= 1 && c_out >= 1 && h >= 1 && w >= 1 && k >= 1 && k % 2 == 1 && stride >= 1,
             FHELIN_E_INVALID_ARG, "native_conv: need positive sizes, an odd kernel and a positive stride");
    const int ho = (h - 1) / stride + 1, wo = (w - 1) / stride + 1;
    const int cop = (c_out + CONV_CO - 1) / CONV_CO * CONV_CO;
    FL_CHECK(ho * wo <= 65535 && cop / CONV_CO <= 65535 && (int64_t)c_in * k * k * cop <= (1 << 26),
             FHELIN_E_INVALID_ARG, "native_conv: layer too large");
    // the transposed weights live in the handle (calls sharing the handle must not overlap)
    const size_t wbytes = (size_t)c_in * k * k * cop * sizeof(int32_t);
    if (n->wt_bytes < wbytes) {
        if (n->wt) {
            FL_TRY_HIP(hipStreamSynchronize(s));
            FL_TRY_HIP(hipFree(n->wt));
            n->wt = nullptr;
            n->wt_bytes = 0;
        }
        if (hipMalloc((void **)&n->wt, wbytes) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(FHELIN_E_OOM, "native_conv: device allocation failed");
        }
        n->wt_bytes = wbytes;
    }
    hipLaunchKernelGGL(k_nat_conv_wt, dim3((unsigned)((wbytes / 4 + 255) / 256)), dim3(256), 0, s, wts, n->wt, c_in, c_out,
                       k, cop);
    FL_TRY_HIP(hipGetLastError());
    const int n2 = 2 * n->N;
    // units: products over the taps inside the image; bytes: every input row once and
    // the outputs (a row shared by overlapping windows is read again from the caches)
    auto taps = [&](int len, int olen) {
        double t = 0;
        for (int o = 0; o < olen; ++o)
            for (int d = 0; d < k; ++d) {
                const int v = stride * o + d - k / 2;
                t += v >= 0 && v < len;
            }
        return t;
    };
    NatProf ps(n, s, NK_LINEAR, taps(h, ho) * taps(w, wo) * c_out * c_in * n2,
               ((double)c_in * h * w + (double)c_out * ho * wo) * n2 * 8.0);
    hipLaunchKernelGGL(k_nat_conv, dim3((n2 + 255) / 256, ho * wo, cop / CONV_CO), dim3(256), 0, s, rows, n->wt, out_row,
                       out, c_in, c_out, cop, h, w, k, stride, wo, n2);
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

}  // namespace fl
