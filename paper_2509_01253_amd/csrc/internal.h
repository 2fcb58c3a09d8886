// internal.h -- shared declarations of the fhelin HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fhelin.h"

namespace fl {

typedef unsigned __int128 u128;

constexpr int MAX_MODS = 40;   // n_q + n_p
constexpr int MAX_Q = 32;
constexpr int MAX_P = 8;
constexpr int MAX_ALPHA = 8;   // primes per key-switch digit
constexpr int MAX_BATCH = 64;  // ciphertexts per launch descriptor
constexpr int MIN_LOGN = 10;
constexpr int MAX_LOGN = 16;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
int set_error(int code, const std::string &msg);
const char *status_string(int code);

#define FL_TRY_HIP(expr)                                                                     \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess)                                                                \
            return ::fl::set_error(FHELIN_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

#define FL_CHECK(cond, code, msg)                  \
    do {                                           \
        if (!(cond)) return ::fl::set_error((code), (msg)); \
    } while (0)

#define FL_RET(expr)             \
    do {                         \
        int _rc = (expr);        \
        if (_rc != FHELIN_OK) return _rc; \
    } while (0)

// ---------------------------------------------------------------------------
// per-modulus device constants
// ---------------------------------------------------------------------------
struct ModConst {
    uint64_t q;
    uint64_t mont_neg_inv;  // -q^{-1} mod 2^64
    uint64_t r2;            // 2^128 mod q: REDC(a * r2) = a * 2^64 mod q
    uint64_t ninv, ninv_sh; // N^{-1} mod q and its Shoup companion
    uint64_t half;          // (q - 1) / 2: largest non-negative centred residue
    uint64_t one_sh;        // floor(2^64 / q): x mod q = csub(shoup_lazy(x, 1, one_sh, q))
    uint64_t r1, r1_sh;     // 2^64 mod q and its Shoup companion: Montgomery form in one Shoup product
};

// Base conversion constants of ModUp for (level l, digit j): digit primes
// q_lo .. q_lo+cnt-1.  inv_hat[i] = (Q_j/q_i)^{-1} mod q_i (Shoup pair);
// hat_mont[i][m] = (Q_j/q_i mod r_m) * 2^64 mod r_m;  qj_mont[m] = (Q_j mod r_m) * 2^64 mod r_m.
struct ModUpTab {
    int32_t lo, cnt, pad0, pad1;
    uint64_t inv_hat[MAX_ALPHA], inv_hat_sh[MAX_ALPHA];
    uint64_t hat_mont[MAX_ALPHA][MAX_MODS];
    uint64_t qj_mont[MAX_MODS];
};

// ModDown constants (level independent): inv_hat[k] = (P/p_k)^{-1} mod p_k (Shoup);
// hat_mont[k][i] = (P/p_k mod q_i) Montgomery; p_mont[i] = (P mod q_i) Montgomery;
// pinv[i] = P^{-1} mod q_i (Shoup pair).
struct ModDownTab {
    uint64_t inv_hat[MAX_P], inv_hat_sh[MAX_P];
    uint64_t hat_mont[MAX_P][MAX_Q];
    uint64_t p_mont[MAX_Q];
    uint64_t pinv[MAX_Q], pinv_sh[MAX_Q];
};

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct Workspace;

// Optional per-kernel timing with HIP events on the launching stream (diagnostics).
enum ProfKind : int {
    PK_NTT_FWD_COLS = 0, PK_NTT_FWD_ROWS, PK_NTT_INV_ROWS, PK_NTT_INV_COLS, PK_NTT_FWD_1, PK_NTT_INV_1,
    PK_MAC, PK_KS_INNER, PK_MODUP, PK_MODDOWN_FBC, PK_COMBINE, PK_RESCALE, PK_COPY, PK_MONT, PK_ENCODE, PK_KS_ROT,
    PK_KS_SUM, PK_MODUP_NTT, PK_ROT_MAC, PK_COUNT
};
extern const char *const PROF_NAMES[PK_COUNT];

struct Profiler {
    bool on = false;
    std::mutex mu;
    struct Rec {
        int kind;
        hipEvent_t a, b;
        double units;  // algorithmic work of the launch (butterflies, multiply-adds, elements)
        double bytes;  // algorithmic HBM bytes of the launch (each stream read or written once)
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get();
};

struct Ctx {
    int device = 0;
    int log_n = 0, N = 0, L = 0, K = 0, dnum = 0, alpha = 0;
    bool small = false;              // every modulus < 2^55: cheaper lazy accumulation
    bool ntt53 = false;              // every modulus < 2^50: NTT twiddle companions floor(w 2^53 / q)
    std::vector<uint64_t> mods;      // q_0..q_{L-1}, p_0..p_{K-1}
    std::vector<uint64_t> psi;       // minimal primitive 2N-th root per modulus
    std::vector<ModConst> h_mods;
    // device tables
    ModConst *d_mods = nullptr;
    uint64_t *d_tw = nullptr, *d_twp = nullptr;    // [M][N]  psi^{brv(i)}, Shoup
    uint64_t *d_itw = nullptr, *d_itwp = nullptr;  // [M][N]  psi^{-brv(i)}, Shoup
    ModUpTab *d_modup = nullptr;                   // [L][dnum], index (l-1)*dnum + j
    ModDownTab *d_moddown = nullptr;
    uint64_t *d_rs_inv = nullptr, *d_rs_inv_sh = nullptr;  // [L][L]: q_{l-1}^{-1} mod q_i at [l-1][i]
    double *d_fft_tw = nullptr;                    // encode FFT twiddles exp(-2 pi i k/N): [N/2] (re, im)
    double *d_zeta = nullptr;                      // exp(i pi k / N), k < N: [N] (re, im)
    int32_t *d_slot_idx = nullptr;                 // (5^j mod 2N - 1) / 2, j < N/2
    uint64_t *d_zero = nullptr;                    // 256 zero bytes (padding source of tile loads)
    uint32_t *d_fault = nullptr;                   // bounded waits that gave up (persistent launches)
    // memory accounting
    uint64_t budget = 0;
    uint64_t used = 0;
    // freed device blocks kept for reuse by an allocation of the same size (not
    // charged to `used`), so steady-state loads and releases call neither hipMalloc
    // nor hipFree; flushed on an allocation failure, by fhelin_ctx_trim and on destroy
    std::multimap<size_t, void *> cache;
    uint64_t cached = 0;
    std::mutex mu;
    std::map<void *, std::unique_ptr<Workspace>> ws;  // per stream
    std::unique_ptr<Profiler> prof{new Profiler()};
    ~Ctx();
};

int ctx_create(const fhelin_params *prm, Ctx **out);
void ctx_destroy(Ctx *c);
int dev_alloc(Ctx *c, void **p, size_t bytes);    // charged to the budget
void cache_flush(Ctx *c);                         // return the cached free blocks to HIP
void dev_free(Ctx *c, void *p, size_t bytes);

// ---------------------------------------------------------------------------
// row descriptors for batched per-limb kernels
// ---------------------------------------------------------------------------
enum RowKind : int32_t {
    ROWS_LIST = 0,  // row r at base + r*N, modulus list[r]
    ROWS_CT = 1,    // ct buffer [2][stride]: polys poly_lo..poly_lo+poly_cnt-1, limbs 0..l-1
    ROWS_EXT_P = 2, // extended buffer [n_part][L+K] slots: the K special slots of each part
    ROWS_MODUP = 3, // digit buffer [dnum][L+K]: every slot of each digit except the digit's own q's
    ROWS_EXT_Q = 4, // extended buffer [n_part][L+K]: Q slots 0..l-1 of each part
    ROWS_KEY = 5,   // compact key rows [n_part][l+K]: position e < l -> q_e, else p_{e-l}
    ROWS_EXT = 6,   // extended buffer [n_part][L+K]: Q slots 0..l-1 and the K special slots of each part
    ROWS_DIGITS = 7,// digit buffer [dnum][L+K]: Q slots 0..l-1 and the special slots of each of the beta digits
};

struct RowMap {
    uint64_t *base;
    const int32_t *list;  // ROWS_LIST moduli (device)
    int64_t ct_stride;    // elements between consecutive batch entries
    int32_t kind;
    int32_t n_ct;
    int32_t stride;       // ROWS_CT limb stride
    int32_t poly_lo, poly_cnt;
    int32_t n_part;       // ROWS_EXT_*: parts
    int32_t L, K, alpha;
    int32_t n_list;
    int32_t log_n;
    int32_t level[MAX_BATCH];  // 32-bit: a uniform index then reads it with a scalar load
};

// Number of rows of batch entry t.
__host__ __device__ inline int rowmap_rows(const RowMap &m, int t) {
    int l = m.level[t];
    switch (m.kind) {
    case ROWS_LIST: return m.n_list;
    case ROWS_CT: return m.poly_cnt * l;
    case ROWS_EXT_P: return m.n_part * m.K;
    case ROWS_EXT_Q: return m.n_part * l;
    case ROWS_KEY: return m.n_part * (l + m.K);
    case ROWS_EXT: return m.n_part * (l + m.K);
    case ROWS_DIGITS: return (l + m.alpha - 1) / m.alpha * (l + m.K);
    case ROWS_MODUP: {
        int beta = (l + m.alpha - 1) / m.alpha;
        return beta * (l + m.K) - l;
    }
    }
    return 0;
}

// Row r of batch entry t: element offset of the row and its modulus index.
__host__ __device__ inline void rowmap_get(const RowMap &m, int t, int r, int64_t *off, int *mod) {
    const int64_t N = (int64_t)1 << m.log_n;
    const int l = m.level[t];
    const int64_t base = (int64_t)t * m.ct_stride;
    switch (m.kind) {
    case ROWS_LIST:
        *off = (int64_t)r * N;
        *mod = m.list[r];
        return;
    case ROWS_CT: {
        int p = m.poly_lo + r / l, i = r % l;
        *off = base + ((int64_t)p * m.stride + i) * N;
        *mod = i;
        return;
    }
    case ROWS_EXT_P: {
        int p = r / m.K, k = r % m.K;
        *off = base + ((int64_t)p * (m.L + m.K) + m.L + k) * N;
        *mod = m.L + k;
        return;
    }
    case ROWS_EXT_Q: {
        int p = r / l, i = r % l;
        *off = base + ((int64_t)p * (m.L + m.K) + i) * N;
        *mod = i;
        return;
    }
    case ROWS_KEY: {
        int e = r % (l + m.K);
        *off = base + (int64_t)r * N;
        *mod = e < l ? e : m.L + (e - l);
        return;
    }
    case ROWS_EXT:
    case ROWS_DIGITS: {
        // part (or digit) r / (l + K), position e < l -> q_e, else p_{e-l}; slot-indexed layout
        int p = r / (l + m.K), e = r % (l + m.K);
        int slot = e < l ? e : m.L + (e - l);
        *off = base + ((int64_t)p * (m.L + m.K) + slot) * N;
        *mod = slot;
        return;
    }
    case ROWS_MODUP: {
        // digit j has (l + K - cnt_j) target rows; cnt_j = min(alpha, l - j*alpha)
        int j = 0, rr = r;
        for (;;) {
            int cnt = l - j * m.alpha;
            if (cnt > m.alpha) cnt = m.alpha;
            int rows_j = l + m.K - cnt;
            if (rr < rows_j) {
                int lo = j * m.alpha;
                int e = rr < lo ? rr : rr + cnt;  // skip the digit's own limbs
                int slot = e < l ? e : m.L + (e - l);
                *off = base + ((int64_t)j * (m.L + m.K) + slot) * N;
                *mod = slot;
                return;
            }
            rr -= rows_j;
            ++j;
        }
    }
    }
    *off = 0;
    *mod = 0;
}

inline int rowmap_max_rows(const RowMap &m) {
    int mx = 0;
    for (int t = 0; t < m.n_ct; ++t) {
        int r = rowmap_rows(m, t);
        if (r > mx) mx = r;
    }
    return mx;
}

// per-entry metadata of a batched key-switch / combine launch
struct Batch {
    int32_t n;
    // 32-bit entries: a byte read at a run-time index is a vector load, which waits
    // for every store and load the wave still has in flight
    int32_t level[MAX_BATCH];
    int32_t key_level[MAX_BATCH];  // level the entry's key set was loaded at
    uint32_t g[MAX_BATCH];         // Galois element (1 = none)
    const uint64_t *key[MAX_BATCH];// the entry's evaluation key for g (digit 0, part 0, row 0)
};

// device buffers of a loaded key set (compact layout, Montgomery form, NTT domain):
// key t, digit j, part p, position e: evk + ((t*beta + j)*2 + p)*(level+K)*N + e*N,
// position e < level -> q_e, else p_{e-level}
// Completion of an asynchronous load (key set, plaintext set): recorded on the loading
// stream; a call on another stream waits for it before its first kernel.
struct Ready {
    hipEvent_t ev = nullptr;
    int record(hipStream_t s);           // create on first use, record on s
    int wait(hipStream_t s) const;       // stream wait (skipped while s is capturing)
    int host_wait() const;               // host-side wait
    Ready() = default;
    Ready(const Ready &) = delete;
    Ready &operator=(const Ready &) = delete;
    ~Ready();
};

// The streams a key or plaintext set was used on, each with an event recorded after
// its last use enqueued there: a release waits for these uses, not for the whole
// device.  note() is skipped while the stream is capturing (a graph launch notes its
// own uses).
struct UseLog {
    std::mutex mu;
    std::vector<std::pair<hipStream_t, hipEvent_t>> ev;
    void note(hipStream_t s);
    void host_wait();
    UseLog() = default;
    UseLog(const UseLog &) = delete;
    UseLog &operator=(const UseLog &) = delete;
    ~UseLog();
};

struct KeySet {
    Ctx *ctx = nullptr;
    int level = 0, beta = 0, n_keys = 0;
    std::vector<uint32_t> galois;
    uint64_t *evk = nullptr;
    size_t bytes = 0;
    Ready ready;
    mutable UseLog uses;
    int64_t key_stride() const { return (int64_t)beta * 2 * (level + ctx->K) * ctx->N; }
    const uint64_t *key_ptr(int idx) const { return evk + (int64_t)idx * key_stride(); }
    int find(uint32_t g) const {
        for (int i = 0; i < n_keys; ++i)
            if (galois[i] == g) return i;
        return -1;
    }
};

struct PtSet {
    Ctx *ctx = nullptr;
    int n_pt = 0, level = 0;
    uint64_t *data = nullptr;  // [n_pt][level][N], NTT domain, Montgomery form
    size_t bytes = 0;
    Ready ready;
    mutable UseLog uses;
};

// Tile and chunk choices of a layer schedule (results do not depend on them).  The
// defaults are the autotuner's choice on the batched N = 2^16 FC workload.
struct Tune {
    int chunk = 0;    // requests per chunk (0: as many as fit MAX_BATCH ciphertexts)
    int ks_eg = 16;   // batch entries per key-switch inner-product workgroup
    int mac_my = 2;   // requests per thread in the multiply-accumulate
    int ntt_threads = 256;  // workgroup size of the two-pass NTT kernels (128, 256, 512)
    int persistent = 0;     // 1: each key switch's ModUp and forward NTT in one persistent launch
    int fuse_baby = 0;      // 1: double-hoisted baby rotations computed inside the multiply-accumulate
};
bool tune_valid(const Tune &t);

struct Plan {
    int kind = 0;
    fhelin_layer_desc desc{};
    int n_in = 0, n_out = 0;
    std::vector<int32_t> rb, gk;  // baby / giant rotation amounts
    std::vector<uint32_t> galois; // distinct Galois elements needed
    Tune tune;
    int n_pt() const { return n_out * n_in * (int)gk.size() * (int)rb.size(); }
};

// A workspace buffer.  Shared: the stream's workspace slot holds one reference and every
// graph captured against it holds another, so a regrow of the slot never frees memory a
// captured graph still points at.
struct WsBuf {
    Ctx *ctx = nullptr;
    void *buf = nullptr;
    size_t bytes = 0;
    ~WsBuf() {
        if (buf) dev_free(ctx, buf, bytes);
    }
};
struct Workspace {
    std::shared_ptr<WsBuf> cur;
};
// workspace of at least `bytes` for `stream` (grows; synchronises the stream before a regrow
// that frees the old buffer); `hold`, if given, receives a reference that keeps it alive
int workspace_get(Ctx *c, hipStream_t s, size_t bytes, uint64_t **out, std::shared_ptr<WsBuf> *hold = nullptr);

uint32_t galois_of_rotation(int64_t r, int log_n);

// Bracket one launch with profiling events when enabled and the stream is not capturing.
struct ProfScope {
    Profiler *p = nullptr;
    hipStream_t s;
    int kind;
    double units, bytes;
    hipEvent_t a{};
    ProfScope(const Ctx *c, hipStream_t st, int k, double u, double by = 0);
    ~ProfScope();
};

// ---------------------------------------------------------------------------
// kernel launchers (each .hip file owns its kernels)
// ---------------------------------------------------------------------------
// NTT over the rows of a RowMap; inverse = 0 forward (natural -> bit-reversed),
// 1 inverse.  Rows hold canonical residues on entry and exit.
// to_mont (forward only): the outputs leave in Montgomery form (x 2^64 mod q)
int launch_ntt(const Ctx *c, const RowMap &rows, int inverse, hipStream_t s, bool to_mont = false);
// out of place: rows of `src` (same row enumeration as `rows`, its own layout) transformed into `rows`
int launch_ntt_from(const Ctx *c, const RowMap &rows, const RowMap &src, int inverse, hipStream_t s,
                    bool to_mont = false);
// persistent ModUp + forward NTT (one launch): digits of the entries' ModUp written to
// `digits` and transformed over the rows of `rm` (ROWS_MODUP or ROWS_DIGITS); ctl is a
// control block of PERSIST_CTL_WORDS words (zeroed by the launch itself); N >= 2^13
constexpr int PERSIST_DIGITS = 16;  // ModUp counters per entry (digits)
constexpr int PERSIST_ROWS = 640;   // transform counters per entry (digit rows)
constexpr int PERSIST_CTL_WORDS = 1 + MAX_BATCH * (PERSIST_DIGITS + PERSIST_ROWS);
constexpr uint32_t PERSIST_SPIN_LIMIT = 1u << 20;  // polls before a wait gives up
int launch_modup_ntt(const Ctx *c, const Batch &b, const uint64_t *coef, int64_t coef_es, const uint64_t *ntt,
                     int64_t ntt_es, uint64_t *digits, int64_t digits_es, const RowMap &rm, uint32_t *ctl,
                     hipStream_t s);
// workgroup size of the two-pass NTT kernels for launches from the calling thread
// (128, 256 or 512; anything else = 256); returns the previous setting
int ntt_threads_set(int nt);
// to/from Montgomery form over the rows (canonical in, canonical out)
int launch_to_mont(const Ctx *c, const RowMap &rows, hipStream_t s);
int launch_from_mont(const Ctx *c, const RowMap &rows, hipStream_t s);
// copy rows between two row maps of the same shape
int launch_copy_rows(const Ctx *c, const RowMap &dst, const RowMap &src, hipStream_t s);
// ModDown of one polynomial of extended entries in the coefficient domain:
// out[i] = (u[i] - conv_P->q_i(u[P])) * P^{-1} mod q_i, i < level
int launch_moddown_coef(const Ctx *c, const Batch &b, const uint64_t *u, int64_t u_es, uint64_t *out, int64_t out_es,
                        hipStream_t s);

// key switching (keyswitch.hip); all pointers are bases of batch entry 0, *_es = elements per entry
int launch_modup(const Ctx *c, const Batch &b, const uint64_t *coef, int64_t coef_es, const uint64_t *ntt,
                 int64_t ntt_es, uint64_t *digits, int64_t digits_es, hipStream_t s);
int launch_ks_inner(const Ctx *c, const Batch &b, const uint64_t *digits, int64_t digits_es, uint64_t *u, int64_t u_es,
                    hipStream_t s, int eg = 8);
int launch_moddown_fbc(const Ctx *c, const Batch &b, const uint64_t *u, int64_t u_es, uint64_t *md, int64_t md_es,
                       hipStream_t s, int n_parts = 2);
// inner product with an addend: add_ext = 0 adds P * sigma_g(c0) of a Q ciphertext [2][L] on the
// q slots, add_ext = 1 adds sigma_g(c0) of an extended ciphertext [2][L+K]; accumulate adds into u
int launch_ks_inner_add(const Ctx *c, const Batch &b, const uint64_t *digits, int64_t digits_es, uint64_t *u,
                        int64_t u_es, const uint64_t *add, int64_t add_es, int add_ext, int accumulate, hipStream_t s,
                        int eg = 8);
// a list of rotations run by one inner-product launch (see k_ks_inner)
constexpr int MAX_ROT = 64;
struct KsRot {
    int32_t n;               // 0: one rotation per entry from Batch.g / Batch.key
    uint32_t g[MAX_ROT];     // Galois element of rotation i
    int32_t key[MAX_ROT];    // its key index in every entry's key set
    int64_t out[MAX_ROT];    // element offset of its output from the entry's output
    uint32_t ginv[MAX_ROT];  // g^-1 mod 2N (filled by the launcher)
};
// A sum of key switches per entry (giant steps): entry t gets
//   init_t + sum_i (add_i,t(sigma_i) + <D_i,t(sigma_i), evk_i>_0, <D_i,t(sigma_i), evk_i>_1)
// on the extended basis, each rotation with its own digits and addend.
constexpr int MAX_SUM = 16;
struct KsSum {
    int32_t n;
    uint32_t g[MAX_SUM];        // Galois element of term i
    int32_t key[MAX_SUM];       // its key index in every entry's key set
    int64_t dig_off[MAX_SUM];   // element offset of term i's digits from `digits`
    int64_t add_off[MAX_SUM];   // element offset of term i's addend from `add`
};
int launch_ks_sum(const Ctx *c, const Batch &b, const KsSum &sum, const uint64_t *digits, int64_t digits_es,
                  const uint64_t *add, int64_t add_es, const uint64_t *init, int64_t init_es, uint64_t *u,
                  int64_t u_es, hipStream_t s);
// every rotation of `rot` for every entry of b (b.key[t] = base of the entry's key set)
int launch_ks_inner_rot(const Ctx *c, const Batch &b, const KsRot &rot, const uint64_t *digits, int64_t digits_es,
                        uint64_t *u, int64_t u_es, const uint64_t *add, int64_t add_es, int add_ext, hipStream_t s,
                        int eg);
// extended ciphertexts [2][L+K]: dst (+)= P * src (lift, src a Q ciphertext [2][src_stride]) or dst (+)= src
int launch_ext_lift_add(const Ctx *c, const Batch &b, const uint64_t *src, int64_t src_es, int src_stride, int lift,
                        int accumulate, uint64_t *dst, int64_t dst_es, hipStream_t s);
// dst[p][i] (+)= (u[p][i] - md[p][i]) P^-1 (+ sigma_g(c0)[i] for p = 0); dst/c0 are [2][stride] ct buffers
int launch_moddown_combine(const Ctx *c, const Batch &b, const uint64_t *u, int64_t u_es, const uint64_t *md,
                           int64_t md_es, uint64_t *dst, int64_t dst_es, int dst_stride, const uint64_t *c0,
                           int64_t c0_es, int c0_stride, int accumulate, hipStream_t s, int n_parts = 2);
// coefficient-domain rescale of [2][in_stride] -> [2][out_stride]
int launch_rescale(const Ctx *c, const Batch &b, const uint64_t *in, int64_t in_es, int in_stride, uint64_t *out,
                   int64_t out_es, int out_stride, hipStream_t s);

// diagnostics: issue-rate probes (diag.hip; the butterfly probe lives beside the
// butterfly in ntt.hip)
int primes_generate(int log_n, int bits, int count, uint64_t *out);
void launch_diag_bfly(int blocks, uint64_t *sink, uint64_t *stamps, int iters, uint64_t q, uint64_t w, uint64_t wp);
int diag_alu_rate(int op, int waves_per_simd, int iters, double *ghz, double *clk_per_op, double *ops_per_s);

}  // namespace fl
