// context.hip -- parameter validation and one-time context tables (hot-path row a1).
//
// Tables: minimal primitive 2N-th roots, merged-psi NTT twiddles in bit-reversed
// order with Shoup companions (Longa-Naehrig 2016 layout), Montgomery constants,
// and the constants of the centred fast base conversion (Bajard et al. 2016) used
// by ModUp, ModDown and rescale.
#include <cmath>
#include <cstring>

#include "internal.h"
#include "modarith.h"

namespace fl {

static thread_local std::string g_last_error;

int set_error(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

const char *last_error() { return g_last_error.c_str(); }

const char *status_string(int code) {
    switch (code) {
    case FHELIN_OK: return "ok";
    case FHELIN_E_INVALID_ARG: return "invalid argument";
    case FHELIN_E_UNSUPPORTED_PARAM: return "unsupported parameter";
    case FHELIN_E_LEVEL_MISMATCH: return "level mismatch";
    case FHELIN_E_MISSING_GALOIS_KEY: return "missing Galois key";
    case FHELIN_E_OOM: return "device out of memory";
    case FHELIN_E_BUDGET: return "HBM budget exceeded";
    case FHELIN_E_HIP: return "HIP runtime error";
    case FHELIN_E_UNIMPLEMENTED: return "unimplemented";
    }
    return "unknown status";
}

// Deterministic Miller-Rabin for 64-bit n (the first 12 prime bases suffice).
static bool is_prime64(uint64_t n) {
    static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return false;
    for (uint64_t b : bases) {
        if (n == b) return true;
        if (n % b == 0) return false;
    }
    uint64_t d = n - 1;
    int r = 0;
    while (!(d & 1)) {
        d >>= 1;
        ++r;
    }
    for (uint64_t b : bases) {
        uint64_t x = h_powmod(b, d, n);
        if (x == 1 || x == n - 1) continue;
        bool composite = true;
        for (int i = 1; i < r && composite; ++i) {
            x = h_mulmod(x, x, n);
            if (x == n - 1) composite = false;
        }
        if (composite) return false;
    }
    return true;
}

int primes_generate(int log_n, int bits, int count, uint64_t *out) {
    FL_CHECK(out && count > 0 && log_n >= 1 && log_n <= 30 && bits > log_n + 1 && bits <= 62, FHELIN_E_INVALID_ARG,
             "primes_generate: bad arguments");
    const uint64_t step = (uint64_t)2 << log_n;
    uint64_t k = (((uint64_t)1 << bits) - 2) / step;  // largest k with k*2N + 1 < 2^bits
    int got = 0;
    for (; k > 0 && got < count; --k) {
        uint64_t cand = k * step + 1;
        if (is_prime64(cand)) out[got++] = cand;
    }
    FL_CHECK(got == count, FHELIN_E_UNSUPPORTED_PARAM, "primes_generate: range exhausted");
    return FHELIN_OK;
}

// minimal x with x^N = -1 (mod q): the smallest primitive 2N-th root of unity
static uint64_t minimal_root(uint64_t q, int log_n) {
    const uint64_t n = (uint64_t)1 << log_n, two_n = 2 * n;
    uint64_t r = 0;
    for (uint64_t g = 2; g < q && !r; ++g) {
        uint64_t c = h_powmod(g, (q - 1) / two_n, q);
        if (h_powmod(c, n, q) == q - 1) r = c;
    }
    if (!r) return 0;
    uint64_t r2 = h_mulmod(r, r, q), cur = r, best = r;
    for (uint64_t k = 3; k < two_n; k += 2) {
        cur = h_mulmod(cur, r2, q);
        if (cur < best) best = cur;
    }
    return best;
}

static inline uint32_t brv(uint32_t x, int bits) { return __builtin_bitreverse32(x) >> (32 - bits); }

constexpr uint64_t CACHE_CAP = 32ull << 30;  // most bytes of freed blocks kept for reuse

void cache_flush(Ctx *c) {
    std::multimap<size_t, void *> blocks;
    {
        std::lock_guard<std::mutex> g(c->mu);
        blocks.swap(c->cache);
        c->cached = 0;
    }
    for (auto &b : blocks) (void)hipFree(b.second);
}

int dev_alloc(Ctx *c, void **p, size_t bytes) {
    {
        std::lock_guard<std::mutex> g(c->mu);
        if (c->budget && c->used + bytes > c->budget)
            return set_error(FHELIN_E_BUDGET, "allocation of " + std::to_string(bytes) + " bytes exceeds the HBM budget");
        c->used += bytes;
        auto it = c->cache.find(bytes);
        if (it != c->cache.end()) {
            *p = it->second;
            c->cache.erase(it);
            c->cached -= bytes;
            return FHELIN_OK;
        }
    }
    hipError_t e = hipMalloc(p, bytes ? bytes : 256);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        cache_flush(c);  // blocks of other sizes may be what is missing
        e = hipMalloc(p, bytes ? bytes : 256);
    }
    if (e != hipSuccess) {
        std::lock_guard<std::mutex> g(c->mu);
        c->used -= bytes;
        (void)hipGetLastError();
        return set_error(FHELIN_E_OOM, "hipMalloc(" + std::to_string(bytes) + ") failed: " + hipGetErrorString(e));
    }
    return FHELIN_OK;
}

void dev_free(Ctx *c, void *p, size_t bytes) {
    if (!p) return;
    // like hipFree: no queued work may still use the block once it is handed out again
    (void)hipDeviceSynchronize();
    bool keep;
    {
        std::lock_guard<std::mutex> g(c->mu);
        c->used -= bytes;
        keep = c->cached + bytes <= CACHE_CAP;
        if (keep) {
            c->cache.emplace(bytes, p);
            c->cached += bytes;
        }
    }
    if (!keep) (void)hipFree(p);
}

template <class T>
static int upload(Ctx *c, T **dst, const std::vector<T> &src) {
    FL_RET(dev_alloc(c, (void **)dst, src.size() * sizeof(T)));
    FL_TRY_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return FHELIN_OK;
}

uint32_t galois_of_rotation(int64_t r, int log_n) {
    const int64_t slots = (int64_t)1 << (log_n - 1);
    const uint64_t two_n = (uint64_t)2 << log_n;
    uint64_t e = (uint64_t)(((r % slots) + slots) % slots);
    return (uint32_t)h_powmod(5, e, two_n);
}

int ctx_create(const fhelin_params *prm, Ctx **out) {
    FL_CHECK(prm && out, FHELIN_E_INVALID_ARG, "ctx_create: null argument");
    FL_CHECK(prm->q && prm->p, FHELIN_E_INVALID_ARG, "ctx_create: null modulus arrays");
    FL_CHECK(prm->log_n >= MIN_LOGN && prm->log_n <= MAX_LOGN, FHELIN_E_UNSUPPORTED_PARAM,
             "log_n must be in [10, 16]");
    FL_CHECK(prm->n_q >= 1 && prm->n_q <= MAX_Q, FHELIN_E_UNSUPPORTED_PARAM, "n_q must be in [1, 32]");
    FL_CHECK(prm->n_p >= 1 && prm->n_p <= MAX_P, FHELIN_E_UNSUPPORTED_PARAM, "n_p must be in [1, 8]");
    FL_CHECK(prm->dnum >= 1 && prm->dnum <= prm->n_q, FHELIN_E_UNSUPPORTED_PARAM, "dnum must be in [1, n_q]");
    const int L = prm->n_q, K = prm->n_p, alpha = (L + prm->dnum - 1) / prm->dnum;
    FL_CHECK(alpha <= MAX_ALPHA, FHELIN_E_UNSUPPORTED_PARAM, "digits hold at most 8 primes (raise dnum)");
    FL_CHECK((L + alpha - 1) / alpha <= 16, FHELIN_E_UNSUPPORTED_PARAM, "at most 16 key-switch digits (lower dnum)");
    const uint64_t two_n = (uint64_t)2 << prm->log_n;
    std::vector<uint64_t> mods(prm->q, prm->q + L);
    mods.insert(mods.end(), prm->p, prm->p + K);
    for (size_t i = 0; i < mods.size(); ++i) {
        uint64_t q = mods[i];
        FL_CHECK(q < ((uint64_t)1 << 60), FHELIN_E_UNSUPPORTED_PARAM, "moduli must be below 2^60");
        FL_CHECK(q % two_n == 1, FHELIN_E_UNSUPPORTED_PARAM, "moduli must be 1 mod 2N");
        FL_CHECK(is_prime64(q), FHELIN_E_UNSUPPORTED_PARAM, "moduli must be prime");
        for (size_t j = 0; j < i; ++j) FL_CHECK(mods[j] != q, FHELIN_E_UNSUPPORTED_PARAM, "moduli must be distinct");
    }
    // P must exceed every digit modulus Q_j (compared in log2)
    long double logP = 0;
    for (int k = 0; k < K; ++k) logP += log2l((long double)mods[L + k]);
    for (int j = 0; j * alpha < L; ++j) {
        long double lq = 0;
        for (int i = j * alpha; i < L && i < (j + 1) * alpha; ++i) lq += log2l((long double)mods[i]);
        FL_CHECK(logP > lq, FHELIN_E_UNSUPPORTED_PARAM, "the special modulus P must exceed every digit modulus");
    }
    int dev = 0;
    FL_TRY_HIP(hipGetDevice(&dev));

    std::unique_ptr<Ctx> c(new Ctx());
    c->device = dev;
    c->log_n = prm->log_n;
    c->N = 1 << prm->log_n;
    c->L = L;
    c->K = K;
    c->dnum = prm->dnum;
    c->alpha = alpha;
    c->mods = mods;
    c->small = true;
    for (uint64_t q : mods) c->small = c->small && q < ((uint64_t)1 << 55);
    c->ntt53 = true;
    for (uint64_t q : mods) c->ntt53 = c->ntt53 && q < ((uint64_t)1 << 50);
    const int M = L + K, N = c->N;

    // per-modulus constants, roots and twiddles
    std::vector<uint64_t> tw((size_t)M * N), twp((size_t)M * N), itw((size_t)M * N), itwp((size_t)M * N);
    for (int m = 0; m < M; ++m) {
        uint64_t q = mods[m];
        uint64_t psi = minimal_root(q, c->log_n);
        FL_CHECK(psi != 0, FHELIN_E_UNSUPPORTED_PARAM, "no primitive 2N-th root");
        c->psi.push_back(psi);
        ModConst mc;
        mc.q = q;
        mc.mont_neg_inv = h_neg_inv64(q);
        mc.r2 = (uint64_t)((((u128)1 << 64) % q) * (u128)(((u128)1 << 64) % q) % q);
        mc.ninv = h_invmod((uint64_t)N % q, q);
        mc.ninv_sh = h_shoup(mc.ninv, q);
        mc.half = (q - 1) / 2;
        mc.one_sh = h_shoup(1, q);
        mc.r1 = (uint64_t)((((u128)1) << 64) % q);
        mc.r1_sh = h_shoup(mc.r1, q);
        c->h_mods.push_back(mc);
        uint64_t psi_inv = h_invmod(psi, q);
        std::vector<uint64_t> pw(N), ipw(N);
        pw[0] = ipw[0] = 1;
        for (int k = 1; k < N; ++k) {
            pw[k] = h_mulmod(pw[k - 1], psi, q);
            ipw[k] = h_mulmod(ipw[k - 1], psi_inv, q);
        }
        for (int k = 0; k < N; ++k) {
            uint32_t b = brv((uint32_t)k, c->log_n);
            size_t o = (size_t)m * N + k;
            tw[o] = pw[b];
            twp[o] = c->ntt53 ? h_shoup53(pw[b], q) : h_shoup(pw[b], q);
            itw[o] = ipw[b];
            itwp[o] = c->ntt53 ? h_shoup53(ipw[b], q) : h_shoup(ipw[b], q);
        }
    }
    FL_RET(upload(c.get(), &c->d_mods, c->h_mods));
    FL_RET(upload(c.get(), &c->d_tw, tw));
    FL_RET(upload(c.get(), &c->d_twp, twp));
    FL_RET(upload(c.get(), &c->d_itw, itw));
    FL_RET(upload(c.get(), &c->d_itwp, itwp));

    // ModUp conversion tables per (level, digit)
    std::vector<ModUpTab> mu((size_t)L * c->dnum);
    memset(mu.data(), 0, mu.size() * sizeof(ModUpTab));
    for (int l = 1; l <= L; ++l) {
        int beta = (l + alpha - 1) / alpha;
        for (int j = 0; j < beta; ++j) {
            ModUpTab &t = mu[(size_t)(l - 1) * c->dnum + j];
            t.lo = j * alpha;
            t.cnt = std::min(alpha, l - j * alpha);
            for (int a = 0; a < t.cnt; ++a) {
                int i = t.lo + a;
                uint64_t qi = mods[i], hat = 1;
                for (int b = 0; b < t.cnt; ++b)
                    if (b != a) hat = h_mulmod(hat, mods[t.lo + b] % qi, qi);
                t.inv_hat[a] = h_invmod(hat, qi);
                t.inv_hat_sh[a] = h_shoup(t.inv_hat[a], qi);
                for (int m = 0; m < M; ++m) {
                    uint64_t r = mods[m], h = 1;
                    for (int b = 0; b < t.cnt; ++b)
                        if (b != a) h = h_mulmod(h, mods[t.lo + b] % r, r);
                    t.hat_mont[a][m] = h_to_mont(h, r);
                }
            }
            for (int m = 0; m < M; ++m) {
                uint64_t r = mods[m], h = 1;
                for (int b = 0; b < t.cnt; ++b) h = h_mulmod(h, mods[t.lo + b] % r, r);
                t.qj_mont[m] = h_to_mont(h, r);
            }
        }
    }
    FL_RET(upload(c.get(), &c->d_modup, mu));

    // ModDown tables
    std::vector<ModDownTab> md(1);
    memset(md.data(), 0, sizeof(ModDownTab));
    ModDownTab &d = md[0];
    for (int k = 0; k < K; ++k) {
        uint64_t pk = mods[L + k], hat = 1;
        for (int s = 0; s < K; ++s)
            if (s != k) hat = h_mulmod(hat, mods[L + s] % pk, pk);
        d.inv_hat[k] = h_invmod(hat, pk);
        d.inv_hat_sh[k] = h_shoup(d.inv_hat[k], pk);
        for (int i = 0; i < L; ++i) {
            uint64_t qi = mods[i], h = 1;
            for (int s = 0; s < K; ++s)
                if (s != k) h = h_mulmod(h, mods[L + s] % qi, qi);
            d.hat_mont[k][i] = h_to_mont(h, qi);
        }
    }
    for (int i = 0; i < L; ++i) {
        uint64_t qi = mods[i], P = 1;
        for (int k = 0; k < K; ++k) P = h_mulmod(P, mods[L + k] % qi, qi);
        d.p_mont[i] = h_to_mont(P, qi);
        d.pinv[i] = h_invmod(P, qi);
        d.pinv_sh[i] = h_shoup(d.pinv[i], qi);
    }
    FL_RET(upload(c.get(), &c->d_moddown, md));

    // rescale: q_{l-1}^{-1} mod q_i
    std::vector<uint64_t> rs((size_t)L * L, 0), rss((size_t)L * L, 0);
    for (int l = 2; l <= L; ++l)
        for (int i = 0; i < l - 1; ++i) {
            uint64_t qi = mods[i];
            uint64_t v = h_invmod(mods[l - 1] % qi, qi);
            rs[(size_t)(l - 1) * L + i] = v;
            rss[(size_t)(l - 1) * L + i] = h_shoup(v, qi);
        }
    FL_RET(upload(c.get(), &c->d_rs_inv, rs));
    FL_RET(upload(c.get(), &c->d_rs_inv_sh, rss));

    // encode FFT twiddles exp(-2 pi i k / N), k < N/2, from long double
    std::vector<double> ft((size_t)N);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < N / 2; ++k) {
        long double a = -2.0L * pi * (long double)k / (long double)N;
        ft[2 * k] = (double)cosl(a);
        ft[2 * k + 1] = (double)sinl(a);
    }
    FL_RET(upload(c.get(), &c->d_fft_tw, ft));
    std::vector<double> zt((size_t)2 * N);
    for (int k = 0; k < N; ++k) {
        long double a = pi * (long double)k / (long double)N;
        zt[2 * k] = (double)cosl(a);
        zt[2 * k + 1] = (double)sinl(a);
    }
    FL_RET(upload(c.get(), &c->d_zeta, zt));
    std::vector<int32_t> si((size_t)N / 2);
    {
        uint64_t e = 1, two_n = (uint64_t)2 * N;
        for (int j = 0; j < N / 2; ++j) {
            si[j] = (int32_t)((e - 1) / 2);
            e = e * 5 % two_n;
        }
    }
    FL_RET(upload(c.get(), &c->d_slot_idx, si));
    FL_RET(upload(c.get(), &c->d_zero, std::vector<uint64_t>(32, 0)));
    FL_RET(upload(c.get(), &c->d_fault, std::vector<uint32_t>(64, 0)));

    *out = c.release();
    return FHELIN_OK;
}

const char *const PROF_NAMES[PK_COUNT] = {"ntt_fwd_cols", "ntt_fwd_rows", "ntt_inv_rows", "ntt_inv_cols",
                                          "ntt_fwd_1",    "ntt_inv_1",    "mac",          "ks_inner",
                                          "modup",        "moddown_fbc",  "combine",      "rescale",
                                          "copy",         "mont",         "encode",       "ks_rot",
                                          "ks_sum",       "modup_ntt",    "rot_mac"};

hipEvent_t Profiler::get() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ProfScope::ProfScope(const Ctx *c, hipStream_t st, int k, double u, double by)
    : s(st), kind(k), units(u), bytes(by) {
    Profiler *pr = c->prof.get();
    if (!pr->on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    std::lock_guard<std::mutex> g(pr->mu);
    a = pr->get();
    if (!a) return;
    if (hipEventRecord(a, st) != hipSuccess) return;
    p = pr;
}

ProfScope::~ProfScope() {
    if (!p) return;
    std::lock_guard<std::mutex> g(p->mu);
    hipEvent_t b = p->get();
    if (!b || hipEventRecord(b, s) != hipSuccess) return;
    p->recs.push_back({kind, a, b, units, bytes});
}

int Ready::record(hipStream_t s) {
    if (!ev) FL_TRY_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    FL_TRY_HIP(hipEventRecord(ev, s));
    return FHELIN_OK;
}

int Ready::wait(hipStream_t s) const {
    if (!ev) return FHELIN_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    FL_TRY_HIP(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) return FHELIN_OK;  // the capture call waited on the host
    FL_TRY_HIP(hipStreamWaitEvent(s, ev, 0));
    return FHELIN_OK;
}

int Ready::host_wait() const {
    if (ev) FL_TRY_HIP(hipEventSynchronize(ev));
    return FHELIN_OK;
}

Ready::~Ready() {
    if (ev) (void)hipEventDestroy(ev);
}

void UseLog::note(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    std::lock_guard<std::mutex> g(mu);
    for (auto &e : ev)
        if (e.first == s) {
            (void)hipEventRecord(e.second, s);
            return;
        }
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    (void)hipEventRecord(e, s);
    ev.emplace_back(s, e);
}

void UseLog::host_wait() {
    std::lock_guard<std::mutex> g(mu);
    for (auto &e : ev) (void)hipEventSynchronize(e.second);
}

UseLog::~UseLog() {
    for (auto &e : ev) (void)hipEventDestroy(e.second);
}

Ctx::~Ctx() {
    ws.clear();
    for (auto &b : cache) (void)hipFree(b.second);
    cache.clear();
    if (prof) {
        for (auto &r : prof->recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : prof->pool) (void)hipEventDestroy(e);
    }
    (void)hipFree(d_mods);
    (void)hipFree(d_tw);
    (void)hipFree(d_twp);
    (void)hipFree(d_itw);
    (void)hipFree(d_itwp);
    (void)hipFree(d_modup);
    (void)hipFree(d_moddown);
    (void)hipFree(d_rs_inv);
    (void)hipFree(d_rs_inv_sh);
    (void)hipFree(d_fft_tw);
    (void)hipFree(d_zeta);
    (void)hipFree(d_slot_idx);
    (void)hipFree(d_zero);
    (void)hipFree(d_fault);
}

void ctx_destroy(Ctx *c) { delete c; }

}  // namespace fl
