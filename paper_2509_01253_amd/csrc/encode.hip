// encode.hip -- plaintext weights: diagonal / multiplexed slot vectors with the
// shuffle folded in, CKKS encoding, RNS and NTT (hot-path row a3).
//
// Encoding (Cheon-Kim-Kim-Song 2017): m_k = round(Delta (2/N) Re sum_j z_j zeta^(-5^j k)),
// zeta = exp(i pi / N).  Over all odd exponents e (z_j at 5^j, conj z_j at -5^j)
// this is (Delta/N) Re(zeta^(-k) sum_t Z_t w^(-tk)) with e = 2t+1, w = exp(2 pi i/N):
// one forward complex FFT of length N per plaintext: radix-2 decimation in time
// (Cooley-Tukey 1965) on bit-reversed input, natural-order output, in two passes
// through HBM with the butterflies of each pass in LDS (the stages inside 256-element
// blocks, then the stages across them, column-wise).  Rounding is rint (ties to even).
#include "internal.h"
#include "modarith.h"

namespace fl {

// Z[p][(5^j-1)/2] = z_j, Z[p][(2N-5^j-1)/2] = z_j (real slots: conj z = z); every index
// once, stored at its bit-reversed position (the FFT's input order)
__global__ void __launch_bounds__(256) k_encode_scatter(const double *__restrict__ slots, double2 *__restrict__ Z,
                                                        const int32_t *__restrict__ slot_idx, int log_n) {
    const int64_t N = (int64_t)1 << log_n, S = N / 2;
    const int p = blockIdx.y;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= S) return;
    double z = slots[(int64_t)p * S + j];
    const uint32_t t = (uint32_t)slot_idx[j];
    double2 *zp = Z + (int64_t)p * N;
    zp[__brev(t) >> (32 - log_n)] = make_double2(z, 0.0);
    zp[__brev((uint32_t)(N - 1) - t) >> (32 - log_n)] = make_double2(z, 0.0);
}

// one decimation-in-time butterfly: (u, v) -> (u + w v, u - w v), w = exp(-2 pi i idx / N)
__device__ __forceinline__ void dit_bfly(double2 *x, int i0, int i1, const double *__restrict__ tw, int64_t idx) {
    const double wr = tw[2 * idx], wi = tw[2 * idx + 1];
    const double2 a = x[i0], b = x[i1];
    const double br = b.x * wr - b.y * wi, bi = b.x * wi + b.y * wr;
    x[i0] = make_double2(a.x + br, a.y + bi);
    x[i1] = make_double2(a.x - br, a.y - bi);
}

constexpr int FFT_TILE = 1024;   // complex elements per workgroup of the first pass (16 KiB of LDS)
constexpr int FFT_CTILE = 2048;  // at most, of the second (32 KiB): 8 columns of 128 bytes at N = 2^16

// columns per workgroup of the second pass
__host__ __device__ inline int fft_cols(int log_n) {
    const int c = FFT_CTILE >> (log_n - 8);
    return c < 256 ? c : 256;
}

// pass 1: stages m = 2 .. 256 inside each contiguous 256-element block; grid (N / 1024, n)
__global__ void __launch_bounds__(256) k_fft_rows(double2 *__restrict__ A, const double *__restrict__ tw, int log_n) {
    __shared__ double2 x[FFT_TILE];
    const int64_t N = (int64_t)1 << log_n;
    double2 *a = A + (int64_t)blockIdx.y * N + (int64_t)blockIdx.x * FFT_TILE;
    for (int e = threadIdx.x; e < FFT_TILE; e += 256) x[e] = a[e];
    __syncthreads();
    for (int lm = 1; lm <= 8; ++lm) {
        const int half = 1 << (lm - 1);
        for (int b = threadIdx.x; b < FFT_TILE / 2; b += 256) {
            const int jj = b & (half - 1), i0 = ((b >> (lm - 1)) << lm) + jj;
            dit_bfly(x, i0, i0 + half, tw, (int64_t)jj << (log_n - lm));
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < FFT_TILE; e += 256) a[e] = x[e];
}

// pass 2: stages m = 512 .. N across the blocks: element c + 256 r is row r of column
// c; a workgroup transforms fft_cols adjacent columns of N1 = N / 256 rows, each a
// DIT FFT over r whose twiddles also depend on c; grid (256 / columns, n)
__global__ void __launch_bounds__(256) k_fft_cols(double2 *__restrict__ A, const double *__restrict__ tw, int log_n) {
    __shared__ double2 x[FFT_CTILE];
    const int64_t N = (int64_t)1 << log_n;
    const int log_n1 = log_n - 8, cols = fft_cols(log_n), tile = cols << log_n1;
    const int c0 = blockIdx.x * cols;
    double2 *a = A + (int64_t)blockIdx.y * N + c0;
    // LDS element (r, cc) at r * cols + cc: consecutive threads read consecutive columns
    for (int e = threadIdx.x; e < tile; e += 256) x[e] = a[(int64_t)(e / cols) * 256 + e % cols];
    __syncthreads();
    for (int lm = 1; lm <= log_n1; ++lm) {
        const int half = 1 << (lm - 1);
        for (int b = threadIdx.x; b < tile / 2; b += 256) {
            const int cc = b % cols, rb = b / cols;
            const int jj = rb & (half - 1), r0 = ((rb >> (lm - 1)) << lm) + jj;
            // exp(-2 pi i (c + 256 jj) / (256 m)), m = 2^lm
            const int64_t idx = ((int64_t)(c0 + cc) + 256 * (int64_t)jj) << (log_n1 - lm);
            dit_bfly(x, r0 * cols + cc, (r0 + half) * cols + cc, tw, idx);
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < tile; e += 256) a[(int64_t)(e / cols) * 256 + e % cols] = x[e];
}

// m_k = rint(scale/N * Re(X_k zeta^-k)); residues mod q_0..q_{level-1}, p_0..p_{K-1}
// -> pt[p][row][k] (coefficient domain)
__global__ void __launch_bounds__(256) k_encode_finish(const double2 *__restrict__ X, uint64_t *__restrict__ pt,
                                                       const ModConst *__restrict__ mods,
                                                       const double *__restrict__ zeta, int level, int L, int K,
                                                       double scale, int log_n) {
    const int64_t N = (int64_t)1 << log_n;
    const int p = blockIdx.y;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double2 v = X[(int64_t)p * N + k];
    // zeta^-k = cos(pi k/N) - i sin(pi k/N)
    const double re = v.x * zeta[2 * k] + v.y * zeta[2 * k + 1];
    const double m = rint(re * (scale / (double)N));
    const int64_t mi = (int64_t)m;
    const bool neg = mi < 0;
    const uint64_t mag = neg ? (uint64_t)(-mi) : (uint64_t)mi;
    uint64_t *o = pt + (int64_t)p * (level + K) * N + k;
    for (int r = 0; r < level + K; ++r) {
        const ModConst mc = mods[r < level ? r : L + (r - level)];
        uint64_t v = csub(shoup_lazy(mag, 1, mc.one_sh, mc.q), mc.q);
        o[(int64_t)r * N] = (neg && v) ? mc.q - v : v;
    }
}

// ---------------------------------------------------------------------------
// weights -> slot vectors for a plan
// ---------------------------------------------------------------------------
// FC: entry (j, b), i = n1 j + b: value[s] = W'[(s - n1 j) mod n][(s - n1 j + i) mod n]
__global__ void __launch_bounds__(256) k_diag_fc(const double *__restrict__ W, const int32_t *__restrict__ perm_out,
                                                 const int32_t *__restrict__ perm_in, int fc_out, int fc_in, int n,
                                                 int n1, int S, int p0, double *__restrict__ out) {
    const int pidx = p0 + blockIdx.y;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= S) return;
    const int j = pidx / n1, b = pidx % n1, i = n1 * j + b;
    const int row = ((s - n1 * j) % n + n) % n;
    const int col = (row + i) % n;
    double v = 0.0;
    if (row < fc_out && col < fc_in) {
        int ro = perm_out ? perm_out[row] : row;
        int ci = perm_in ? perm_in[col] : col;
        v = W[(int64_t)ro * fc_in + ci];
    }
    out[(int64_t)blockIdx.y * S + s] = v;
}

// conv: with n1 channel baby steps, entry (o, i, j, b), b = k1 k^2 + (spatial offset),
// holds rot_{-n1 j h w}(d) for channel offset kc = k1 + n1 j, where
// d[s] = W'[o c + co(s)][i c + (co(s) + kc) mod c][dy + r][dx + r] * [inside]
__global__ void __launch_bounds__(256) k_diag_conv(const double *__restrict__ W, const int32_t *__restrict__ perm_out,
                                                   const int32_t *__restrict__ perm_in, int c_out, int c_in, int h,
                                                   int w, int ks, int n_in, int n1, int S, int p0,
                                                   double *__restrict__ out) {
    const int pidx = p0 + blockIdx.y;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= S) return;
    const int hw = h * w, cct = S / hw, KK = ks * ks, B = n1 * KK, G = cct / n1, r = ks / 2;
    const int b = pidx % B, j = (pidx / B) % G, ii = (pidx / B / G) % n_in, o = pidx / B / G / n_in;
    const int k1 = b / KK, bo = b % KK, kc = k1 + n1 * j;
    const int dy = bo / ks - r, dx = bo % ks - r;
    const int sp = ((s - n1 * j * hw) % S + S) % S;
    const int co = sp / hw, y = (sp % hw) / w, x = sp % w;
    const int cog = o * cct + co, cig = ii * cct + (co + kc) % cct;
    double v = 0.0;
    if (cog < c_out && cig < c_in && y + dy >= 0 && y + dy < h && x + dx >= 0 && x + dx < w) {
        int a = perm_out ? perm_out[cog] : cog;
        int c = perm_in ? perm_in[cig] : cig;
        v = W[(((int64_t)a * c_in + c) * ks + (dy + r)) * ks + (dx + r)];
    }
    out[(int64_t)blockIdx.y * S + s] = v;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int ptset_new(Ctx *c, int n_pt, int level, PtSet **out) {
    FL_CHECK(n_pt >= 1 && level >= 1 && level <= c->L, FHELIN_E_INVALID_ARG, "bad plaintext set shape");
    std::unique_ptr<PtSet> p(new PtSet());
    p->ctx = c;
    p->n_pt = n_pt;
    p->level = level;
    p->bytes = (size_t)n_pt * (level + c->K) * c->N * sizeof(uint64_t);
    FL_RET(dev_alloc(c, (void **)&p->data, p->bytes));
    *out = p.release();
    return FHELIN_OK;
}

void ptset_free(PtSet *p) {
    if (!p) return;
    dev_free(p->ctx, p->data, p->bytes);
    delete p;
}

// rows of plaintexts p0 .. p0+n-1 of a [n_pt][level+K][N] buffer: row e < level -> q_e,
// else p_{e-level}
static RowMap pt_rows(const Ctx *c, uint64_t *data, int n, int level) {
    RowMap m{};
    m.base = data;
    m.kind = ROWS_KEY;
    m.n_part = n;
    m.n_ct = 1;
    m.L = c->L;
    m.K = c->K;
    m.alpha = c->alpha;
    m.log_n = c->log_n;
    m.level[0] = (uint8_t)level;
    return m;
}

// coefficient domain -> NTT domain, Montgomery form, in place
static int pt_to_internal(Ctx *c, PtSet *p, hipStream_t s) {
    const int64_t rows = p->level + c->K;
    for (int p0 = 0; p0 < p->n_pt; p0 += 64) {
        RowMap e = pt_rows(c, p->data + (int64_t)p0 * rows * c->N, std::min(64, p->n_pt - p0), p->level);
        FL_RET(launch_ntt(c, e, 0, s, true));
    }
    return p->ready.record(s);
}

int pt_import(Ctx *c, const uint64_t *src, int n_pt, int level, int on_device, hipStream_t s, PtSet **out) {
    FL_CHECK(c && src && out, FHELIN_E_INVALID_ARG, "pt_import: null argument");
    PtSet *p;
    FL_RET(ptset_new(c, n_pt, level, &p));
    hipError_t e = hipMemcpyAsync(p->data, src, p->bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        ptset_free(p);
        return set_error(FHELIN_E_HIP, std::string("pt_import copy: ") + hipGetErrorString(e));
    }
    if (!on_device) {  // the host source may be reused by the caller as soon as we return
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            ptset_free(p);
            return set_error(FHELIN_E_HIP, std::string("pt_import sync: ") + hipGetErrorString(e));
        }
    }
    int rc = pt_to_internal(c, p, s);
    if (rc) {
        ptset_free(p);
        return rc;
    }
    *out = p;
    return FHELIN_OK;
}

int pt_export(Ctx *c, const PtSet *p, int level, uint64_t *dst, hipStream_t s) {
    FL_CHECK(c && p && dst, FHELIN_E_INVALID_ARG, "pt_export: null argument");
    FL_CHECK(level >= 1 && level <= p->level, FHELIN_E_LEVEL_MISMATCH, "pt_export: level above the set's level");
    const int64_t N = c->N, K = c->K;
    const size_t row = (size_t)N * sizeof(uint64_t);
    FL_RET(p->ready.wait(s));
    // q rows 0..level-1, then the K special rows
    FL_TRY_HIP(hipMemcpy2DAsync(dst, (level + K) * row, p->data, (p->level + K) * row, level * row, p->n_pt,
                                hipMemcpyDeviceToDevice, s));
    FL_TRY_HIP(hipMemcpy2DAsync(dst + level * N, (level + K) * row, p->data + (int64_t)p->level * N,
                                (p->level + K) * row, K * row, p->n_pt, hipMemcpyDeviceToDevice, s));
    for (int p0 = 0; p0 < p->n_pt; p0 += 64) {
        RowMap e = pt_rows(c, dst + (int64_t)p0 * (level + K) * N, std::min(64, p->n_pt - p0), level);
        FL_RET(launch_from_mont(c, e, s));
        FL_RET(launch_ntt(c, e, 1, s));
    }
    return FHELIN_OK;
}

// encode n real slot vectors (device [n][S]) into coefficient-domain rows dst[n][level+K][N]
static int encode_into(Ctx *c, const double *slots, int n, int level, double scale, uint64_t *dst, hipStream_t s) {
    const int64_t N = c->N;
    uint64_t *ws;
    FL_RET(workspace_get(c, s, (size_t)n * N * sizeof(double2), &ws));
    double2 *a = (double2 *)ws;
    hipLaunchKernelGGL(k_encode_scatter, dim3((unsigned)(N / 2 + 255) / 256, n), dim3(256), 0, s, slots, a,
                       c->d_slot_idx, c->log_n);
    // N >= 2^10: 256-element blocks, then the 256 columns of N / 256 rows
    hipLaunchKernelGGL(k_fft_rows, dim3((unsigned)(N / FFT_TILE), n), dim3(256), 0, s, a, c->d_fft_tw, c->log_n);
    hipLaunchKernelGGL(k_fft_cols, dim3((unsigned)(256 / fft_cols(c->log_n)), n), dim3(256), 0, s, a, c->d_fft_tw,
                       c->log_n);
    hipLaunchKernelGGL(k_encode_finish, dim3((unsigned)N / 256, n), dim3(256), 0, s, a, dst, c->d_mods, c->d_zeta,
                       level, c->L, c->K, scale, c->log_n);
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

int pt_encode(Ctx *c, const double *slots, int n_pt, int level, double scale, hipStream_t s, PtSet **out) {
    FL_CHECK(c && slots && out, FHELIN_E_INVALID_ARG, "pt_encode: null argument");
    FL_CHECK(scale > 0 && scale < 0x1p62, FHELIN_E_INVALID_ARG, "pt_encode: scale out of range");
    PtSet *p;
    FL_RET(ptset_new(c, n_pt, level, &p));
    const int64_t N = c->N;
    int rc = FHELIN_OK;
    for (int p0 = 0; p0 < n_pt && rc == FHELIN_OK; p0 += 64) {
        const int n = std::min(64, n_pt - p0);
        rc = encode_into(c, slots + (int64_t)p0 * (N / 2), n, level, scale,
                         p->data + (int64_t)p0 * (level + c->K) * N, s);
    }
    if (rc == FHELIN_OK) rc = pt_to_internal(c, p, s);
    if (rc) {
        ptset_free(p);
        return rc;
    }
    *out = p;
    return FHELIN_OK;
}

int plan_encode_weights(Ctx *c, const Plan *pl, const double *W, const int32_t *perm_out, const int32_t *perm_in,
                        int level, double scale, hipStream_t s, PtSet **out) {
    FL_CHECK(c && pl && W && out, FHELIN_E_INVALID_ARG, "encode_weights: null argument");
    FL_CHECK(scale > 0 && scale < 0x1p62, FHELIN_E_INVALID_ARG, "encode_weights: scale out of range");
    const int S = c->N / 2, n_pt = pl->n_pt();
    const int64_t N = c->N;
    const int chunk = std::min(n_pt, 64);
    double *slots = nullptr;
    FL_RET(dev_alloc(c, (void **)&slots, (size_t)chunk * S * sizeof(double)));
    PtSet *p = nullptr;
    int rc = ptset_new(c, n_pt, level, &p);
    const fhelin_layer_desc &d = pl->desc;
    for (int p0 = 0; p0 < n_pt && rc == FHELIN_OK; p0 += chunk) {
        const int n = std::min(chunk, n_pt - p0);
        if (pl->kind == FHELIN_LAYER_FC)
            hipLaunchKernelGGL(k_diag_fc, dim3((S + 255) / 256, n), dim3(256), 0, s, W, perm_out, perm_in, d.fc_out,
                               d.fc_in, d.fc_n, d.n1, S, p0, slots);
        else
            hipLaunchKernelGGL(k_diag_conv, dim3((S + 255) / 256, n), dim3(256), 0, s, W, perm_out, perm_in, d.c_out,
                               d.c_in, d.h, d.w, d.k, pl->n_in, d.n1 > 1 ? d.n1 : 1, S, p0, slots);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) rc = set_error(FHELIN_E_HIP, std::string("encode_weights: ") + hipGetErrorString(e));
        if (rc == FHELIN_OK)
            rc = encode_into(c, slots, n, level, scale, p->data + (int64_t)p0 * (level + c->K) * N, s);
    }
    if (rc == FHELIN_OK) rc = pt_to_internal(c, p, s);
    (void)hipStreamSynchronize(s);  // the slot buffer is read by queued kernels
    dev_free(c, slots, (size_t)chunk * S * sizeof(double));
    if (rc) {
        ptset_free(p);
        return rc;
    }
    *out = p;
    return FHELIN_OK;
}

}  // namespace fl
