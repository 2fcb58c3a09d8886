/*
 * ckks_oracle.c -- plain, slow CPU oracle for the encrypted linear-layer path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * What it computes (each function names the passage or published definition
 * it follows):
 *   - the ring R_q = Z_q[X]/(X^N+1) and its arithmetic, coefficient by
 *     coefficient, with every modular product written as (a*b) mod q on
 *     128-bit integers;
 *   - the negacyclic NTT by its defining sum (bit-reversed evaluation order);
 *   - ring automorphisms X -> X^g (paper Sec. 2.2: automorphisms change the
 *     key from s(X) to s(X^d));
 *   - hybrid key switching (paper Sec. 2.2 and the key form of Sec. 4.2,
 *     realised with the special-modulus / digit-decomposition method of
 *     Gentry-Halevi-Smart 2012 and Han-Ki 2020, with the centred fast base
 *     conversion of Bajard-Eynard-Hasan-Zucca 2016);
 *   - rescale (full-RNS CKKS, Cheon-Han-Kim-Kim-Song 2018);
 *   - client-side key generation, encryption and decryption (paper Sec. 2.1
 *     and 4.2), used only to build test inputs and to check decryptions.
 *
 * Ring products default to an exact O(N log N) evaluation (twist by psi^j,
 * recursive radix-2 cyclic transform over Z_q, pointwise product, inverse,
 * untwist: Cooley-Tukey 1965 applied to the negacyclic convolution).  The
 * schoolbook definition is kept beside it; the tests pin the fast product to
 * the schoolbook one and can switch every high-level routine to schoolbook
 * with or_set_schoolbook(1).
 *
 * Layout conventions (shared with the C-ABI only by definition, not by code):
 *   a polynomial limb is N uint64 values in [0, q), coefficient order;
 *   a ciphertext at level l is [2][l][N] (c0 then c1), decrypting as c0+c1*s;
 *   the modulus list is q_0..q_{L-1} followed by p_0..p_{K-1}.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* scalar modular arithmetic                                           */
/* ------------------------------------------------------------------ */
static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
static uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) { uint64_t s = a + b; return s >= q ? s - q : s; }
static uint64_t submod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }
static uint64_t powmod(uint64_t a, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q; a %= q;
    while (e) { if (e & 1) r = mulmod(r, a, q); a = mulmod(a, a, q); e >>= 1; }
    return r;
}
/* q prime: Fermat inverse */
static uint64_t invmod(uint64_t a, uint64_t q) { return powmod(a % q, q - 2, q); }
/* signed integer -> [0,q) */
static uint64_t from_signed(int64_t v, uint64_t q) {
    if (v >= 0) return (uint64_t)v % q;
    uint64_t m = (uint64_t)(-(v + 1)) + 1; /* |v| without overflow */
    m %= q;
    return m ? q - m : 0;
}

uint64_t or_mulmod(uint64_t a, uint64_t b, uint64_t q) { return mulmod(a, b, q); }
uint64_t or_powmod(uint64_t a, uint64_t e, uint64_t q) { return powmod(a, e, q); }
uint64_t or_invmod(uint64_t a, uint64_t q) { return invmod(a, q); }

/* Deterministic Miller-Rabin; the first 12 prime bases decide every n < 3.3e24. */
int or_is_prime(uint64_t n) {
    static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) { if (n == bases[i]) return 1; if (n % bases[i] == 0) return 0; }
    uint64_t d = n - 1; int r = 0;
    while ((d & 1) == 0) { d >>= 1; r++; }
    for (int i = 0; i < 12; i++) {
        uint64_t x = powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int comp = 1;
        for (int k = 1; k < r; k++) { x = mulmod(x, x, n); if (x == n - 1) { comp = 0; break; } }
        if (comp) return 0;
    }
    return 1;
}

/* Primes q = 1 (mod 2N) below 2^bits, in descending order (the first `count`
 * found).  Returns the number written. */
int or_gen_primes(int log_n, int bits, int count, uint64_t *out) {
    uint64_t two_n = (uint64_t)2 << log_n;
    uint64_t top = (bits >= 64) ? UINT64_MAX : (((uint64_t)1 << bits) - 1);
    uint64_t k = (top - 1) / two_n;
    int got = 0;
    while (got < count && k > 0) {
        uint64_t cand = k * two_n + 1;
        if (or_is_prime(cand)) out[got++] = cand;
        k--;
    }
    return got;
}

/* Smallest x in [2,q) with x^N = -1 (mod q), i.e. the minimal primitive
 * 2N-th root of unity.  Finds one primitive root r from g^((q-1)/2N), then
 * takes the minimum over r^k, k odd (these are exactly all the primitive
 * 2N-th roots). */
uint64_t or_min_root(uint64_t q, int log_n) {
    uint64_t n = (uint64_t)1 << log_n, two_n = 2 * n;
    if ((q - 1) % two_n) return 0;
    uint64_t r = 0;
    for (uint64_t g = 2; g < q; g++) {
        uint64_t c = powmod(g, (q - 1) / two_n, q);
        if (powmod(c, n, q) == q - 1) { r = c; break; }
    }
    if (!r) return 0;
    uint64_t r2 = mulmod(r, r, q), best = r, cur = r;
    for (uint64_t k = 3; k < two_n; k += 2) {
        cur = mulmod(cur, r2, q);
        if (cur < best) best = cur;
    }
    return best;
}

static unsigned brv(unsigned x, int bits) {
    unsigned y = 0;
    for (int i = 0; i < bits; i++) { y = (y << 1) | (x & 1); x >>= 1; }
    return y;
}

/* ------------------------------------------------------------------ */
/* NTT by its definition                                               */
/*   A[k] = sum_j a_j psi^(j(2 brv(k)+1))   (bit-reversed evaluation)    */
/* ------------------------------------------------------------------ */
void or_ntt_naive(const uint64_t *a, uint64_t *out, int log_n, uint64_t q, uint64_t psi) {
    size_t n = (size_t)1 << log_n;
    for (size_t k = 0; k < n; k++) {
        uint64_t e = 2 * (uint64_t)brv((unsigned)k, log_n) + 1;
        uint64_t w = powmod(psi, e, q), x = 1, acc = 0;
        for (size_t j = 0; j < n; j++) { acc = addmod(acc, mulmod(a[j], x, q), q); x = mulmod(x, w, q); }
        out[k] = acc;
    }
}
/* one output of the definition (for sampled checks at large N) */
uint64_t or_ntt_naive_at(const uint64_t *a, size_t k, int log_n, uint64_t q, uint64_t psi) {
    size_t n = (size_t)1 << log_n;
    uint64_t e = 2 * (uint64_t)brv((unsigned)k, log_n) + 1;
    uint64_t w = powmod(psi, e, q), x = 1, acc = 0;
    for (size_t j = 0; j < n; j++) { acc = addmod(acc, mulmod(a[j], x, q), q); x = mulmod(x, w, q); }
    return acc;
}
/* inverse: a_j = N^-1 sum_k A[k] psi^(-j(2 brv(k)+1)) */
void or_intt_naive(const uint64_t *A, uint64_t *out, int log_n, uint64_t q, uint64_t psi) {
    size_t n = (size_t)1 << log_n;
    uint64_t psi_inv = invmod(psi, q), n_inv = invmod(n % q, q);
    for (size_t j = 0; j < n; j++) {
        uint64_t acc = 0;
        for (size_t k = 0; k < n; k++) {
            uint64_t e = (2 * (uint64_t)brv((unsigned)k, log_n) + 1) * (uint64_t)j % (2 * n);
            acc = addmod(acc, mulmod(A[k], powmod(psi_inv, e, q), q), q);
        }
        out[j] = mulmod(acc, n_inv, q);
    }
}

/* ------------------------------------------------------------------ */
/* ring products in Z_q[X]/(X^N+1)                                     */
/* ------------------------------------------------------------------ */
static int g_schoolbook = 0;
void or_set_schoolbook(int on) { g_schoolbook = on; }

/* schoolbook negacyclic product: X^N = -1 */
void or_polymul_schoolbook(const uint64_t *a, const uint64_t *b, uint64_t *out, int log_n, uint64_t q) {
    size_t n = (size_t)1 << log_n;
    uint64_t *acc = (uint64_t *)calloc(n, sizeof(uint64_t));
    for (size_t i = 0; i < n; i++) {
        if (!a[i]) continue;
        for (size_t j = 0; j < n; j++) {
            uint64_t t = mulmod(a[i], b[j], q);
            size_t k = i + j;
            if (k < n) acc[k] = addmod(acc[k], t, q);
            else acc[k - n] = submod(acc[k - n], t, q);
        }
    }
    memcpy(out, acc, n * sizeof(uint64_t));
    free(acc);
}

/* one coefficient of the negacyclic product: sum_{i+j=k} a_i b_j - sum_{i+j=k+N} a_i b_j */
uint64_t or_polymul_at(const uint64_t *a, const uint64_t *b, size_t k, int log_n, uint64_t q) {
    size_t n = (size_t)1 << log_n;
    uint64_t acc = 0;
    for (size_t i = 0; i < n; i++) {
        if (i <= k) acc = addmod(acc, mulmod(a[i], b[k - i], q), q);
        else acc = submod(acc, mulmod(a[i], b[k + n - i], q), q);
    }
    return acc;
}

/* recursive radix-2 cyclic DFT over Z_q: X[k] = sum_t x[t] w^(tk), length n
 * (decimation in time: X[k] = E[k] + w^k O[k], X[k+n/2] = E[k] - w^k O[k]) */
static void dft_rec(uint64_t *x, size_t n, uint64_t w, uint64_t q, uint64_t *scratch) {
    if (n == 1) return;
    size_t h = n / 2;
    uint64_t *ev = scratch, *od = scratch + h;
    for (size_t t = 0; t < h; t++) { ev[t] = x[2 * t]; od[t] = x[2 * t + 1]; }
    memcpy(x, ev, h * sizeof(uint64_t));
    memcpy(x + h, od, h * sizeof(uint64_t));
    uint64_t w2 = mulmod(w, w, q);
    dft_rec(x, h, w2, q, scratch);
    dft_rec(x + h, h, w2, q, scratch);
    uint64_t f = 1;
    for (size_t k = 0; k < h; k++) {
        uint64_t e = x[k], o = mulmod(f, x[k + h], q);
        x[k] = addmod(e, o, q);
        x[k + h] = submod(e, o, q);
        f = mulmod(f, w, q);
    }
}

/* a*b mod (X^N+1): with psi a primitive 2N-th root, (a psi^j) and (b psi^j)
 * convolve cyclically to (c psi^j). */
static void polymul_fast(const uint64_t *a, const uint64_t *b, uint64_t *out, int log_n, uint64_t q, uint64_t psi) {
    size_t n = (size_t)1 << log_n;
    uint64_t *x = (uint64_t *)malloc(3 * n * sizeof(uint64_t));
    uint64_t *y = x + n, *s = y + n;
    uint64_t f = 1;
    for (size_t j = 0; j < n; j++) { x[j] = mulmod(a[j], f, q); y[j] = mulmod(b[j], f, q); f = mulmod(f, psi, q); }
    uint64_t w = mulmod(psi, psi, q), w_inv = invmod(w, q);
    dft_rec(x, n, w, q, s);
    dft_rec(y, n, w, q, s);
    for (size_t k = 0; k < n; k++) x[k] = mulmod(x[k], y[k], q);
    dft_rec(x, n, w_inv, q, s);
    uint64_t n_inv = invmod(n % q, q), psi_inv = invmod(psi, q);
    f = n_inv;
    for (size_t j = 0; j < n; j++) { out[j] = mulmod(x[j], f, q); f = mulmod(f, psi_inv, q); }
    free(x);
}

void or_polymul_fast(const uint64_t *a, const uint64_t *b, uint64_t *out, int log_n, uint64_t q) {
    polymul_fast(a, b, out, log_n, q, or_min_root(q, log_n));
}

/* ------------------------------------------------------------------ */
/* RNS parameter context (oracle side, rebuilt per call; cheap)        */
/* ------------------------------------------------------------------ */
typedef struct {
    int log_n, L, K, dnum, alpha;
    size_t n;
    const uint64_t *mod;     /* [L+K]: q_0..q_{L-1}, p_0..p_{K-1} */
    uint64_t *psi;           /* minimal 2N-th root per modulus */
} octx;

static int octx_init(octx *c, int log_n, int L, int K, int dnum, const uint64_t *mod) {
    c->log_n = log_n; c->L = L; c->K = K; c->dnum = dnum;
    c->alpha = (L + dnum - 1) / dnum;
    c->n = (size_t)1 << log_n;
    c->mod = mod;
    c->psi = (uint64_t *)malloc((size_t)(L + K) * sizeof(uint64_t));
    for (int i = 0; i < L + K; i++) { c->psi[i] = or_min_root(mod[i], log_n); if (!c->psi[i]) return -1; }
    return 0;
}
static void octx_free(octx *c) { free(c->psi); }

/* product of two limbs modulo modulus index mi */
static void ring_mul(const octx *c, int mi, const uint64_t *a, const uint64_t *b, uint64_t *out) {
    if (g_schoolbook) or_polymul_schoolbook(a, b, out, c->log_n, c->mod[mi]);
    else polymul_fast(a, b, out, c->log_n, c->mod[mi], c->psi[mi]);
}

/* modulus index of position r in the extended basis B_l = {q_0..q_{l-1}, p_0..p_{K-1}} */
static int ext_index(const octx *c, int l, int r) { return r < l ? r : c->L + (r - l); }

/* ------------------------------------------------------------------ */
/* automorphism sigma_g : a(X) -> a(X^g), g odd                        */
/*   coefficient j moves to g*j mod 2N; X^(N+t) = -X^t                  */
/* ------------------------------------------------------------------ */
void or_automorph(const uint64_t *a, uint64_t *out, int log_n, uint64_t g, uint64_t q) {
    size_t n = (size_t)1 << log_n, two_n = 2 * n;
    for (size_t j = 0; j < n; j++) {
        size_t e = (size_t)(((u128)g * j) % two_n);
        if (e < n) out[e] = a[j];
        else out[e - n] = a[j] ? q - a[j] : 0;
    }
}

/* ------------------------------------------------------------------ */
/* ModUp with the centred fast base conversion                          */
/*   digit j at level l: D_j = {q_i : j*alpha <= i < min((j+1)alpha, l)} */
/*   v_i = [x_i (Q_j/q_i)^-1]_{q_i} lifted to (-q_i/2, q_i/2]           */
/*   y_r = sum_i v_i (Q_j/q_i) mod r  for r outside D_j;  y_r = x_r inside */
/* x: [l][N] coefficient domain.  out: [beta][l+K][N], extended basis B_l */
/* ------------------------------------------------------------------ */
static void modup_digit(const octx *c, int l, int j, const uint64_t *x, uint64_t *y) {
    size_t n = c->n;
    int lo = j * c->alpha, hi = lo + c->alpha; if (hi > l) hi = l;
    int m = l + c->K;
    #pragma omp parallel for schedule(dynamic)
    for (int r = 0; r < m; r++) {
        int mr = ext_index(c, l, r);
        uint64_t qr = c->mod[mr];
        uint64_t *yr = y + (size_t)r * n;
        if (r >= lo && r < hi) { memcpy(yr, x + (size_t)r * n, n * sizeof(uint64_t)); continue; }
        /* constants of the conversion: (Q_j/q_i)^-1 mod q_i and Q_j/q_i mod r */
        uint64_t inv_hat[64], hat_r[64];
        for (int i = lo; i < hi; i++) {
            uint64_t qi = c->mod[i], hi_ = 1, hr = 1;
            for (int t = lo; t < hi; t++) if (t != i) { hi_ = mulmod(hi_, c->mod[t] % qi, qi); hr = mulmod(hr, c->mod[t] % qr, qr); }
            inv_hat[i - lo] = invmod(hi_, qi);
            hat_r[i - lo] = hr;
        }
        for (size_t k = 0; k < n; k++) {
            uint64_t acc = 0;
            for (int i = lo; i < hi; i++) {
                uint64_t qi = c->mod[i];
                uint64_t v = mulmod(x[(size_t)i * n + k], inv_hat[i - lo], qi);
                int64_t vs = (v > (qi - 1) / 2) ? (int64_t)v - (int64_t)qi : (int64_t)v;
                acc = addmod(acc, mulmod(from_signed(vs, qr), hat_r[i - lo], qr), qr);
            }
            yr[k] = acc;
        }
    }
}

void or_modup(const uint64_t *x, int l, int log_n, int L, int K, int dnum, const uint64_t *mod, uint64_t *out) {
    octx c; octx_init(&c, log_n, L, K, dnum, mod);
    int beta = (l + c.alpha - 1) / c.alpha;
    for (int j = 0; j < beta; j++) modup_digit(&c, l, j, x, out + (size_t)j * (l + K) * c.n);
    octx_free(&c);
}

/* ModDown: u over B_l ([l+K][N]) -> (u_q - conv_P->q(u_P)) * P^-1 mod q_i, centred conversion */
static void moddown(const octx *c, int l, const uint64_t *u, uint64_t *out) {
    size_t n = c->n;
    int K = c->K, L = c->L;
    #pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < l; i++) {
        uint64_t qi = c->mod[i];
        uint64_t P_mod_qi = 1;
        for (int k = 0; k < K; k++) P_mod_qi = mulmod(P_mod_qi, c->mod[L + k] % qi, qi);
        uint64_t P_inv = invmod(P_mod_qi, qi);
        /* constants: (P/p_k)^-1 mod p_k and P/p_k mod q_i */
        uint64_t inv_hat[64], hat_i[64];
        for (int k = 0; k < K; k++) {
            uint64_t pk = c->mod[L + k], hk = 1, hq = 1;
            for (int s = 0; s < K; s++) if (s != k) { hk = mulmod(hk, c->mod[L + s] % pk, pk); hq = mulmod(hq, c->mod[L + s] % qi, qi); }
            inv_hat[k] = invmod(hk, pk);
            hat_i[k] = hq;
        }
        for (size_t t = 0; t < n; t++) {
            uint64_t acc = 0;
            for (int k = 0; k < K; k++) {
                uint64_t pk = c->mod[L + k];
                uint64_t v = mulmod(u[(size_t)(l + k) * n + t], inv_hat[k], pk);
                int64_t vs = (v > (pk - 1) / 2) ? (int64_t)v - (int64_t)pk : (int64_t)v;
                acc = addmod(acc, mulmod(from_signed(vs, qi), hat_i[k], qi), qi);
            }
            out[(size_t)i * n + t] = mulmod(submod(u[(size_t)i * n + t], acc, qi), P_inv, qi);
        }
    }
}

void or_moddown(const uint64_t *u, int l, int log_n, int L, int K, int dnum, const uint64_t *mod, uint64_t *out) {
    octx c; octx_init(&c, log_n, L, K, dnum, mod);
    moddown(&c, l, u, out);
    octx_free(&c);
}

/* evk limb for extended position r at level l, from a key stored at full
 * width [dnum][2][L+K][N] (digit j, part 0 = b, part 1 = a) */
static const uint64_t *evk_limb(const octx *c, const uint64_t *evk, int l, int j, int part, int r) {
    int mi = ext_index(c, l, r);
    return evk + (((size_t)j * 2 + part) * (c->L + c->K) + mi) * c->n;
}

/* Key-switch core: d (a [l][N] polynomial under s') -> (u0,u1) [2][l][N]
 * with u0 + u1 s ~ d s' (mod Q_l).  u = sum_j ModUp_j(d) * evk[j], then ModDown. */
static void ks_core(const octx *c, int l, const uint64_t *d, const uint64_t *evk, uint64_t *out) {
    size_t n = c->n;
    int beta = (l + c->alpha - 1) / c->alpha, m = l + c->K;
    uint64_t *y = (uint64_t *)malloc((size_t)m * n * sizeof(uint64_t));
    uint64_t *u = (uint64_t *)calloc((size_t)2 * m * n, sizeof(uint64_t));
    for (int j = 0; j < beta; j++) {
        modup_digit(c, l, j, d, y);
        #pragma omp parallel for schedule(dynamic)
        for (int pr = 0; pr < 2 * m; pr++) {
            int part = pr / m, r = pr % m;
            uint64_t q = c->mod[ext_index(c, l, r)];
            uint64_t *tt = (uint64_t *)malloc(n * sizeof(uint64_t));
            ring_mul(c, ext_index(c, l, r), y + (size_t)r * n, evk_limb(c, evk, l, j, part, r), tt);
            uint64_t *ur = u + ((size_t)part * m + r) * n;
            for (size_t k = 0; k < n; k++) ur[k] = addmod(ur[k], tt[k], q);
            free(tt);
        }
    }
    moddown(c, l, u, out);
    moddown(c, l, u + (size_t)m * n, out + (size_t)l * n);
    free(y); free(u);
}

/* Rotation / automorphism with key switch: ct [2][l][N] -> [2][l][N].
 * (sigma_g(c0) + u0, u1) with (u0,u1) = KS(sigma_g(c1)); evk for g at full width. */
static void rotate(const octx *c, int l, uint64_t g, const uint64_t *ct, const uint64_t *evk, uint64_t *out) {
    size_t n = c->n;
    uint64_t *sc = (uint64_t *)malloc((size_t)2 * l * n * sizeof(uint64_t));
    uint64_t *u = (uint64_t *)malloc((size_t)2 * l * n * sizeof(uint64_t));
    for (int p = 0; p < 2; p++)
        for (int i = 0; i < l; i++)
            or_automorph(ct + ((size_t)p * l + i) * n, sc + ((size_t)p * l + i) * n, c->log_n, g, c->mod[i]);
    ks_core(c, l, sc + (size_t)l * n, evk, u);
    for (int i = 0; i < l; i++) {
        uint64_t q = c->mod[i];
        for (size_t k = 0; k < n; k++) {
            out[(size_t)i * n + k] = addmod(sc[(size_t)i * n + k], u[(size_t)i * n + k], q);
            out[((size_t)l + i) * n + k] = u[((size_t)l + i) * n + k];
        }
    }
    free(sc); free(u);
}

void or_rotate(const uint64_t *ct, int l, uint64_t g, const uint64_t *evk, int log_n, int L, int K, int dnum,
               const uint64_t *mod, uint64_t *out) {
    octx c; octx_init(&c, log_n, L, K, dnum, mod);
    rotate(&c, l, g, ct, evk, out);
    octx_free(&c);
}

/* key-switch core exposed for tests: d [l][N] -> [2][l][N] */
void or_keyswitch(const uint64_t *d, int l, const uint64_t *evk, int log_n, int L, int K, int dnum,
                  const uint64_t *mod, uint64_t *out) {
    octx c; octx_init(&c, log_n, L, K, dnum, mod);
    ks_core(&c, l, d, evk, out);
    octx_free(&c);
}

/* ModUp digit outputs and inner product at a single coefficient position k,
 * for sampled checks at large N: returns u [2][l+K] at coefficient k of
 * sum_j ModUp_j(d) * evk[j]  (before ModDown). */
void or_ks_inner_at(const uint64_t *d, int l, const uint64_t *evk, size_t k, int log_n, int L, int K, int dnum,
                    const uint64_t *mod, uint64_t *out) {
    octx c; octx_init(&c, log_n, L, K, dnum, mod);
    size_t n = c.n;
    int beta = (l + c.alpha - 1) / c.alpha, m = l + K;
    uint64_t *y = (uint64_t *)malloc((size_t)m * n * sizeof(uint64_t));
    for (int r = 0; r < 2 * m; r++) out[r] = 0;
    for (int j = 0; j < beta; j++) {
        modup_digit(&c, l, j, d, y);
        for (int part = 0; part < 2; part++)
            for (int r = 0; r < m; r++) {
                uint64_t q = mod[ext_index(&c, l, r)];
                uint64_t v = or_polymul_at(y + (size_t)r * n, evk_limb(&c, evk, l, j, part, r), k, log_n, q);
                out[part * m + r] = addmod(out[part * m + r], v, q);
            }
    }
    free(y);
    octx_free(&c);
}

/* ModDown of a single coefficient position: u [l+K] -> out [l] */
void or_moddown_at(const uint64_t *u, int l, int log_n, int L, int K, int dnum, const uint64_t *mod, uint64_t *out) {
    (void)log_n;
    octx c; c.log_n = 0; c.L = L; c.K = K; c.dnum = dnum; c.alpha = (L + dnum - 1) / dnum; c.n = 1; c.mod = mod; c.psi = NULL;
    moddown(&c, l, u, out);
}

/* ------------------------------------------------------------------ */
/* rescale: drop q_{l-1} with rounding (centred lift of the top limb)   */
/*   c'_i = (c_i - [c]_{q_{l-1}} centred) * q_{l-1}^-1 mod q_i          */
/* ------------------------------------------------------------------ */
void or_rescale(const uint64_t *ct, int l, int log_n, const uint64_t *mod, uint64_t *out) {
    size_t n = (size_t)1 << log_n;
    uint64_t qt = mod[l - 1];
    for (int p = 0; p < 2; p++) {
        const uint64_t *top = ct + ((size_t)p * l + (l - 1)) * n;
        for (int i = 0; i < l - 1; i++) {
            uint64_t qi = mod[i], inv = invmod(qt % qi, qi);
            const uint64_t *ci = ct + ((size_t)p * l + i) * n;
            uint64_t *oi = out + ((size_t)p * (l - 1) + i) * n;
            for (size_t k = 0; k < n; k++) {
                int64_t v = (top[k] > (qt - 1) / 2) ? (int64_t)top[k] - (int64_t)qt : (int64_t)top[k];
                oi[k] = mulmod(submod(ci[k], from_signed(v, qi), qi), inv, qi);
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* plaintext x ciphertext: (c0*pt, c1*pt), pt [l][N] coefficient domain */
/* ------------------------------------------------------------------ */
void or_mul_pt(const uint64_t *ct, const uint64_t *pt, int l, int log_n, const uint64_t *mod, uint64_t *out) {
    octx c; octx_init(&c, log_n, l, 0, 1, mod);
    size_t n = c.n;
    for (int p = 0; p < 2; p++)
        for (int i = 0; i < l; i++)
            ring_mul(&c, i, ct + ((size_t)p * l + i) * n, pt + (size_t)i * n, out + ((size_t)p * l + i) * n);
    octx_free(&c);
}

/* ------------------------------------------------------------------ */
/* generic baby-step / giant-step linear transform                      */
/*   y_o = sum_k rot_{G_k}( sum_i sum_b pt[o][i][k][b] * rot_{r_b}(x_i) ) */
/* Rotation by r (slots, S = N/2) is the automorphism g = 5^(r mod S) mod 2N; */
/* r = 0 is the identity (no key switch).                               */
/*   x: [n_in][2][l][N]; pt: [n_out][n_in][G][B][l][N] (coefficient domain, */
/*   any level >= l may be passed with row stride pt_l);                 */
/*   keys: galois[n_keys], evk [n_keys][dnum][2][L+K][N]                */
/*   out: [n_out][2][l][N]                                              */
/* Returns 0, or -1 if a needed Galois key is missing.                   */
/* ------------------------------------------------------------------ */
static uint64_t galois_of(int64_t r, int log_n) {
    uint64_t n = (uint64_t)1 << log_n, two_n = 2 * n, slots = n / 2;
    uint64_t e = (uint64_t)(((r % (int64_t)slots) + (int64_t)slots) % (int64_t)slots);
    return powmod(5, e, two_n);
}
uint64_t or_galois_of(int64_t r, int log_n) { return galois_of(r, log_n); }

static const uint64_t *find_key(const octx *c, uint64_t g, const uint32_t *galois, int n_keys, const uint64_t *evk) {
    size_t key_sz = (size_t)c->dnum * 2 * (c->L + c->K) * c->n;
    for (int t = 0; t < n_keys; t++) if (galois[t] == g) return evk + (size_t)t * key_sz;
    return NULL;
}

int or_linear(const uint64_t *x, int n_in, int n_out, int B, const int64_t *rb, int G, const int64_t *gk,
              const uint64_t *pt, int pt_l, int l, const uint32_t *galois, int n_keys, const uint64_t *evk,
              int log_n, int L, int K, int dnum, const uint64_t *mod, uint64_t *out) {
    octx c; octx_init(&c, log_n, L, K, dnum, mod);
    size_t n = c.n, ctsz = (size_t)2 * l * n;
    int rc = 0;
    uint64_t *R = (uint64_t *)malloc((size_t)n_in * B * ctsz * sizeof(uint64_t));
    uint64_t *acc = (uint64_t *)malloc(ctsz * sizeof(uint64_t));
    uint64_t *tmp = (uint64_t *)malloc(ctsz * sizeof(uint64_t));
    /* baby steps */
    for (int i = 0; i < n_in && !rc; i++)
        for (int b = 0; b < B; b++) {
            uint64_t *Rib = R + ((size_t)i * B + b) * ctsz;
            const uint64_t *xi = x + (size_t)i * ctsz;
            uint64_t g = galois_of(rb[b], log_n);
            if (g == 1) { memcpy(Rib, xi, ctsz * sizeof(uint64_t)); continue; }
            const uint64_t *key = find_key(&c, g, galois, n_keys, evk);
            if (!key) { rc = -1; break; }
            rotate(&c, l, g, xi, key, Rib);
        }
    for (int o = 0; o < n_out && !rc; o++) {
        uint64_t *yo = out + (size_t)o * ctsz;
        memset(yo, 0, ctsz * sizeof(uint64_t));
        for (int k = 0; k < G && !rc; k++) {
            memset(acc, 0, ctsz * sizeof(uint64_t));
            #pragma omp parallel for schedule(dynamic)
            for (int pl = 0; pl < 2 * l; pl++) {
                int part = pl / l, li = pl % l;
                uint64_t *pp = (uint64_t *)malloc(n * sizeof(uint64_t));
                uint64_t *a = acc + ((size_t)part * l + li) * n;
                for (int i = 0; i < n_in; i++)
                    for (int b = 0; b < B; b++) {
                        const uint64_t *p = pt + ((((size_t)o * n_in + i) * G + k) * B + b) * (size_t)pt_l * n;
                        const uint64_t *Rib = R + ((size_t)i * B + b) * ctsz;
                        ring_mul(&c, li, Rib + ((size_t)part * l + li) * n, p + (size_t)li * n, pp);
                        for (size_t t = 0; t < n; t++) a[t] = addmod(a[t], pp[t], mod[li]);
                    }
                free(pp);
            }
            uint64_t g = galois_of(gk[k], log_n);
            const uint64_t *src = acc;
            if (g != 1) {
                const uint64_t *key = find_key(&c, g, galois, n_keys, evk);
                if (!key) { rc = -1; break; }
                rotate(&c, l, g, acc, key, tmp);
                src = tmp;
            }
            for (int part = 0; part < 2; part++)
                for (int li = 0; li < l; li++) {
                    uint64_t *a = yo + ((size_t)part * l + li) * n;
                    const uint64_t *s = src + ((size_t)part * l + li) * n;
                    for (size_t t = 0; t < n; t++) a[t] = addmod(a[t], s[t], mod[li]);
                }
        }
    }
    free(R); free(acc); free(tmp);
    octx_free(&c);
    return rc;
}

/* ------------------------------------------------------------------ */
/* baby-step / giant-step transform with hoisted ModDown ("double       */
/* hoisting", Bossuat-Mouchet-Troncoso-Pastoriza-Hubaux, Eurocrypt 2021) */
/* Same layer as or_linear; the key-switch outputs stay in the extended */
/* basis B = {q_0..q_{l-1}, p_0..p_{K-1}} (carrying a factor P):        */
/*   R~_b = (P sigma_b(x0) + u0_b, u1_b),  u_b = sum_j ModUp_j(sigma_b(x1)) evk_b[j] */
/*          (r_b = 0: R~ = (P x0, P x1));                                 */
/*   A~_k = sum_i sum_b pt[o][i][k][b] * R~_b   over B                    */
/*          (pt has residues mod every modulus of B);                     */
/*   Y~ = sum_k T_k with T_k = A~_k when G_k = 0, else                      */
/*        T_k = (sigma_k(A~_k.c0) + v0, v1),                                */
/*        v = sum_j ModUp_j(sigma_k(ModDown(A~_k.c1))) evk_k[j];            */
/*   y = (ModDown(Y~.c0), ModDown(Y~.c1)).                                 */
/* pt layout: [n_out][n_in][G][B][pt_l + K][N]: rows 0..pt_l-1 are mod      */
/* q_0..q_{pt_l-1}, rows pt_l.. are mod p_0..p_{K-1}.                       */
/* ------------------------------------------------------------------ */
/* IP over B (no ModDown): d [l][N] under s(X^g) -> u [2][l+K][N] */
static void ks_inner_ext(const octx *c, int l, const uint64_t *d, const uint64_t *evk, uint64_t *u) {
    size_t n = c->n;
    int beta = (l + c->alpha - 1) / c->alpha, m = l + c->K;
    uint64_t *y = (uint64_t *)malloc((size_t)m * n * sizeof(uint64_t));
    memset(u, 0, (size_t)2 * m * n * sizeof(uint64_t));
    for (int j = 0; j < beta; j++) {
        modup_digit(c, l, j, d, y);
        #pragma omp parallel for schedule(dynamic)
        for (int pr = 0; pr < 2 * m; pr++) {
            int part = pr / m, r = pr % m;
            uint64_t q = c->mod[ext_index(c, l, r)];
            uint64_t *tt = (uint64_t *)malloc(n * sizeof(uint64_t));
            ring_mul(c, ext_index(c, l, r), y + (size_t)r * n, evk_limb(c, evk, l, j, part, r), tt);
            uint64_t *ur = u + ((size_t)part * m + r) * n;
            for (size_t k = 0; k < n; k++) ur[k] = addmod(ur[k], tt[k], q);
            free(tt);
        }
    }
    free(y);
}

/* P mod each modulus of B: q_i -> [P]_{q_i}, p_k -> 0 */
static uint64_t P_mod(const octx *c, int mi) {
    uint64_t q = c->mod[mi], r = 1;
    for (int k = 0; k < c->K; k++) r = mulmod(r, c->mod[c->L + k] % q, q);
    return r;
}

/* (P x) over B for a level-l Q polynomial x [l][N] -> [l+K][N] */
static void lift_P(const octx *c, int l, const uint64_t *x, uint64_t *out) {
    size_t n = c->n;
    for (int r = 0; r < l + c->K; r++) {
        int mi = ext_index(c, l, r);
        uint64_t f = P_mod(c, mi);
        for (size_t k = 0; k < n; k++) out[(size_t)r * n + k] = r < l ? mulmod(x[(size_t)r * n + k], f, c->mod[mi]) : 0;
    }
}

int or_linear_dh(const uint64_t *x, int n_in, int n_out, int B, const int64_t *rb, int G, const int64_t *gk,
                 const uint64_t *pt, int pt_l, int l, const uint32_t *galois, int n_keys, const uint64_t *evk,
                 int log_n, int L, int K, int dnum, const uint64_t *mod, uint64_t *out) {
    octx c; octx_init(&c, log_n, L, K, dnum, mod);
    size_t n = c.n, ctsz = (size_t)2 * l * n;
    int m = l + K;
    size_t ext = (size_t)2 * m * n;
    int rc = 0;
    uint64_t *R = (uint64_t *)malloc((size_t)n_in * B * ext * sizeof(uint64_t));
    uint64_t *A = (uint64_t *)malloc(ext * sizeof(uint64_t));
    uint64_t *Y = (uint64_t *)malloc(ext * sizeof(uint64_t));
    uint64_t *tmp = (uint64_t *)malloc(ext * sizeof(uint64_t));
    uint64_t *sx = (uint64_t *)malloc(ctsz * sizeof(uint64_t));
    uint64_t *c1 = (uint64_t *)malloc((size_t)l * n * sizeof(uint64_t));
    uint64_t *sc1 = (uint64_t *)malloc((size_t)l * n * sizeof(uint64_t));
    /* baby steps in B */
    for (int i = 0; i < n_in && !rc; i++)
        for (int b = 0; b < B; b++) {
            uint64_t *Rib = R + ((size_t)i * B + b) * ext;
            const uint64_t *xi = x + (size_t)i * ctsz;
            uint64_t g = galois_of(rb[b], log_n);
            if (g == 1) {
                lift_P(&c, l, xi, Rib);
                lift_P(&c, l, xi + (size_t)l * n, Rib + (size_t)m * n);
                continue;
            }
            const uint64_t *key = find_key(&c, g, galois, n_keys, evk);
            if (!key) { rc = -1; break; }
            for (int p = 0; p < 2; p++)
                for (int li = 0; li < l; li++)
                    or_automorph(xi + ((size_t)p * l + li) * n, sx + ((size_t)p * l + li) * n, log_n, g, mod[li]);
            ks_inner_ext(&c, l, sx + (size_t)l * n, key, Rib);
            lift_P(&c, l, sx, tmp);
            for (int r = 0; r < m; r++) {
                uint64_t q = mod[ext_index(&c, l, r)];
                for (size_t k = 0; k < n; k++) Rib[(size_t)r * n + k] = addmod(Rib[(size_t)r * n + k], tmp[(size_t)r * n + k], q);
            }
        }
    for (int o = 0; o < n_out && !rc; o++) {
        memset(Y, 0, ext * sizeof(uint64_t));
        for (int k = 0; k < G && !rc; k++) {
            memset(A, 0, ext * sizeof(uint64_t));
            #pragma omp parallel for schedule(dynamic)
            for (int pr = 0; pr < 2 * m; pr++) {
                int part = pr / m, r = pr % m;
                int mi = ext_index(&c, l, r);
                int prow = r < l ? r : pt_l + (r - l);
                uint64_t *pp = (uint64_t *)malloc(n * sizeof(uint64_t));
                uint64_t *a = A + ((size_t)part * m + r) * n;
                for (int i = 0; i < n_in; i++)
                    for (int b = 0; b < B; b++) {
                        const uint64_t *p = pt + ((((size_t)o * n_in + i) * G + k) * B + b) * (size_t)(pt_l + K) * n;
                        const uint64_t *Rib = R + ((size_t)i * B + b) * ext;
                        ring_mul(&c, mi, Rib + ((size_t)part * m + r) * n, p + (size_t)prow * n, pp);
                        for (size_t t = 0; t < n; t++) a[t] = addmod(a[t], pp[t], mod[mi]);
                    }
                free(pp);
            }
            uint64_t g = galois_of(gk[k], log_n);
            const uint64_t *T = A;
            if (g != 1) {
                const uint64_t *key = find_key(&c, g, galois, n_keys, evk);
                if (!key) { rc = -1; break; }
                moddown(&c, l, A + (size_t)m * n, c1);                 /* c1' = ModDown(A~.c1) */
                for (int li = 0; li < l; li++) or_automorph(c1 + (size_t)li * n, sc1 + (size_t)li * n, log_n, g, mod[li]);
                ks_inner_ext(&c, l, sc1, key, tmp);                    /* v over B */
                for (int r = 0; r < m; r++) {                          /* + sigma(A~.c0) on every limb of B */
                    int mi = ext_index(&c, l, r);
                    uint64_t *t0 = (uint64_t *)malloc(n * sizeof(uint64_t));
                    or_automorph(A + (size_t)r * n, t0, log_n, g, mod[mi]);
                    for (size_t t = 0; t < n; t++) tmp[(size_t)r * n + t] = addmod(tmp[(size_t)r * n + t], t0[t], mod[mi]);
                    free(t0);
                }
                T = tmp;
            }
            for (int r = 0; r < 2 * m; r++) {
                uint64_t q = mod[ext_index(&c, l, r % m)];
                for (size_t t = 0; t < n; t++) Y[(size_t)r * n + t] = addmod(Y[(size_t)r * n + t], T[(size_t)r * n + t], q);
            }
        }
        if (rc) break;
        uint64_t *yo = out + (size_t)o * ctsz;
        moddown(&c, l, Y, yo);
        moddown(&c, l, Y + (size_t)m * n, yo + (size_t)l * n);
    }
    free(R); free(A); free(Y); free(tmp); free(sx); free(c1); free(sc1);
    octx_free(&c);
    return rc;
}

/* ------------------------------------------------------------------ */
/* client side (test-input construction and decryption checks only)    */
/* ------------------------------------------------------------------ */

/* m(X) = sum_j s_j X^j with s_j in {-1,0,1} -> limb mod q */
static void ternary_limb(const int8_t *s, size_t n, uint64_t q, uint64_t *out) {
    for (size_t j = 0; j < n; j++) out[j] = s[j] == 0 ? 0 : (s[j] > 0 ? 1 : q - 1);
}

/* Symmetric encryption (paper Sec. 2.1 with (c0,c1) = (b,-a); here c1 = a, c0 = -a s + m + e):
 *   m [l][N] in RNS, s ternary [N], a [l][N] uniform per limb, e [N] small integers. */
void or_encrypt(const uint64_t *m, const int8_t *s, const uint64_t *a, const int64_t *e, int l, int log_n,
                const uint64_t *mod, uint64_t *ct) {
    octx c; octx_init(&c, log_n, l, 0, 1, mod);
    size_t n = c.n;
    uint64_t *sl = (uint64_t *)malloc(n * sizeof(uint64_t)), *as = (uint64_t *)malloc(n * sizeof(uint64_t));
    for (int i = 0; i < l; i++) {
        uint64_t q = mod[i];
        ternary_limb(s, n, q, sl);
        ring_mul(&c, i, a + (size_t)i * n, sl, as);
        for (size_t k = 0; k < n; k++) {
            ct[(size_t)i * n + k] = addmod(submod(m[(size_t)i * n + k], as[k], q), from_signed(e[k], q), q);
            ct[((size_t)l + i) * n + k] = a[(size_t)i * n + k];
        }
    }
    free(sl); free(as);
    octx_free(&c);
}

/* m = c0 + c1 s  (mod q_i), [l][N] */
void or_decrypt(const uint64_t *ct, const int8_t *s, int l, int log_n, const uint64_t *mod, uint64_t *m) {
    octx c; octx_init(&c, log_n, l, 0, 1, mod);
    size_t n = c.n;
    uint64_t *sl = (uint64_t *)malloc(n * sizeof(uint64_t)), *cs = (uint64_t *)malloc(n * sizeof(uint64_t));
    for (int i = 0; i < l; i++) {
        uint64_t q = mod[i];
        ternary_limb(s, n, q, sl);
        ring_mul(&c, i, ct + ((size_t)l + i) * n, sl, cs);
        for (size_t k = 0; k < n; k++) m[(size_t)i * n + k] = addmod(ct[(size_t)i * n + k], cs[k], q);
    }
    free(sl); free(cs);
    octx_free(&c);
}

/* Galois evaluation key for g (key form of Sec. 4.2, hybrid variant):
 *   evk[j] = (b_j, a_j) over all L+K moduli,
 *   b_j = -a_j s + e_j + P * 1_j * s(X^g),  1_j = 1 mod q in D_j, 0 mod the other moduli.
 * a_rand: [dnum][L+K][N] uniform per modulus; e: [dnum][N] small integers.
 * out: [dnum][2][L+K][N]. */
void or_keygen_galois(const int8_t *s, uint64_t g, const uint64_t *a_rand, const int64_t *e, int log_n, int L, int K,
                      int dnum, const uint64_t *mod, uint64_t *out) {
    octx c; octx_init(&c, log_n, L, K, dnum, mod);
    size_t n = c.n;
    int M = L + K;
    uint64_t *sl = (uint64_t *)malloc(n * sizeof(uint64_t)), *sg = (uint64_t *)malloc(n * sizeof(uint64_t));
    uint64_t *as = (uint64_t *)malloc(n * sizeof(uint64_t)), *tmp = (uint64_t *)malloc(n * sizeof(uint64_t));
    for (int j = 0; j < dnum; j++) {
        int lo = j * c.alpha, hi = lo + c.alpha; if (hi > L) hi = L;
        for (int mi = 0; mi < M; mi++) {
            uint64_t q = mod[mi];
            ternary_limb(s, n, q, sl);
            or_automorph(sl, sg, log_n, g, q);
            const uint64_t *a = a_rand + ((size_t)j * M + mi) * n;
            ring_mul(&c, mi, a, sl, as);
            uint64_t P_mod = 1;
            for (int k = 0; k < K; k++) P_mod = mulmod(P_mod, mod[L + k] % q, q);
            int in_digit = (mi >= lo && mi < hi);
            uint64_t *b_out = out + (((size_t)j * 2 + 0) * M + mi) * n;
            uint64_t *a_out = out + (((size_t)j * 2 + 1) * M + mi) * n;
            for (size_t k = 0; k < n; k++) {
                uint64_t v = submod(from_signed(e[(size_t)j * n + k], q), as[k], q);
                if (in_digit) v = addmod(v, mulmod(P_mod, sg[k], q), q);
                b_out[k] = v;
                a_out[k] = a[k];
            }
            (void)tmp;
        }
    }
    free(sl); free(sg); free(as); free(tmp);
    octx_free(&c);
}

/* ------------------------------------------------------------------ */
/* centred CRT lift: [l][N] residues -> centred integer as long double  */
/* Garner mixed radix, then evaluated exactly in a small big integer.   */
/* ------------------------------------------------------------------ */
#define BIG_W 24
typedef struct { uint64_t w[BIG_W]; } big;
static void big_mul_small(big *a, uint64_t m) {
    u128 carry = 0;
    for (int i = 0; i < BIG_W; i++) { u128 t = (u128)a->w[i] * m + carry; a->w[i] = (uint64_t)t; carry = t >> 64; }
}
static void big_add_small(big *a, uint64_t v) {
    u128 carry = v;
    for (int i = 0; i < BIG_W && carry; i++) { u128 t = (u128)a->w[i] + carry; a->w[i] = (uint64_t)t; carry = t >> 64; }
}
static int big_cmp(const big *a, const big *b) {
    for (int i = BIG_W - 1; i >= 0; i--) { if (a->w[i] != b->w[i]) return a->w[i] > b->w[i] ? 1 : -1; }
    return 0;
}
static void big_sub(big *a, const big *b) { /* a -= b, a >= b */
    uint64_t borrow = 0;
    for (int i = 0; i < BIG_W; i++) {
        u128 t = (u128)a->w[i] - b->w[i] - borrow;
        a->w[i] = (uint64_t)t; borrow = (t >> 64) ? 1 : 0;
    }
}
static long double big_to_ld(const big *a) {
    long double r = 0;
    for (int i = BIG_W - 1; i >= 0; i--) r = r * 18446744073709551616.0L + (long double)a->w[i];
    return r;
}

void or_crt_centered(const uint64_t *m, int l, int log_n, const uint64_t *mod, long double *out) {
    size_t n = (size_t)1 << log_n;
    big Q; memset(&Q, 0, sizeof Q); Q.w[0] = 1;
    for (int i = 0; i < l; i++) big_mul_small(&Q, mod[i]);
    big half = Q; /* floor(Q/2): Q is odd */
    { uint64_t carry = 0; for (int i = BIG_W - 1; i >= 0; i--) { uint64_t w = half.w[i]; half.w[i] = (w >> 1) | (carry << 63); carry = w & 1; } }
    uint64_t *v = (uint64_t *)malloc((size_t)l * sizeof(uint64_t));
    for (size_t k = 0; k < n; k++) {
        /* Garner: x = v0 + v1 q0 + v2 q0 q1 + ... */
        for (int i = 0; i < l; i++) {
            uint64_t qi = mod[i], t = m[(size_t)i * n + k] % qi;
            for (int j = 0; j < i; j++) t = mulmod(submod(t, v[j] % qi, qi), invmod(mod[j] % qi, qi), qi);
            v[i] = t;
        }
        big x; memset(&x, 0, sizeof x);
        for (int i = l - 1; i >= 0; i--) { big_mul_small(&x, mod[i]); big_add_small(&x, v[i]); }
        if (big_cmp(&x, &half) > 0) { big y = Q; big_sub(&y, &x); out[k] = -big_to_ld(&y); }
        else out[k] = big_to_ld(&x);
    }
    free(v);
}

/* ------------------------------------------------------------------ */
/* encode / decode by the defining sums (long double, O(N * N/2))       */
/*   zeta = exp(i pi / N); slot j <-> zeta^(5^j mod 2N)                  */
/*   m_k = rint( Delta (2/N) sum_j Re(z_j zeta^(-5^j k)) )  half-to-even   */
/* z given as real parts zr and imaginary parts zi, S = N/2 slots.       */
/* out: integer coefficients (int64).  Exponents are reduced mod 2N in   */
/* integers before any trigonometric call.                               */
/* ------------------------------------------------------------------ */
void or_encode_direct(const double *zr, const double *zi, int log_n, double delta, int64_t *out) {
    size_t n = (size_t)1 << log_n, two_n = 2 * n, slots = n / 2;
    const long double pi = 3.141592653589793238462643383279502884L;
    uint64_t *g = (uint64_t *)malloc(slots * sizeof(uint64_t));
    uint64_t p = 1;
    for (size_t j = 0; j < slots; j++) { g[j] = p; p = p * 5 % two_n; }
    for (size_t k = 0; k < n; k++) {
        long double acc = 0;
        for (size_t j = 0; j < slots; j++) {
            uint64_t e = (two_n - (g[j] * k) % two_n) % two_n; /* -5^j k mod 2N */
            long double ang = pi * (long double)e / (long double)n;
            acc += (long double)zr[j] * cosl(ang) - (long double)zi[j] * sinl(ang);
        }
        long double v = (long double)delta * 2.0L / (long double)n * acc;
        out[k] = (int64_t)rintl(v); /* default rounding mode: to nearest, ties to even */
    }
    free(g);
}

/* z_j = Delta^-1 sum_k m_k zeta^(5^j k), from real coefficients m (centred lift) */
void or_decode_direct(const long double *m, int log_n, double delta, double *zr, double *zi) {
    size_t n = (size_t)1 << log_n, two_n = 2 * n, slots = n / 2;
    const long double pi = 3.141592653589793238462643383279502884L;
    uint64_t p = 1;
    for (size_t j = 0; j < slots; j++) {
        long double ar = 0, ai = 0;
        for (size_t k = 0; k < n; k++) {
            uint64_t e = (p * k) % two_n;
            long double ang = pi * (long double)e / (long double)n;
            ar += m[k] * cosl(ang); ai += m[k] * sinl(ang);
        }
        zr[j] = (double)(ar / (long double)delta);
        zi[j] = (double)(ai / (long double)delta);
        p = p * 5 % two_n;
    }
}
