// linear.hip -- encrypted linear layers: plans, pt x ct multiply-accumulate, and the
// batched evaluation schedule (hot-path rows a5-a9).
//
// A layer is the baby-step / giant-step form
//     y_o = sum_j rot_{G_j}( sum_i sum_b pt[o][i][j][b] * rot_{r_b}(x_i) ),
// which covers the Halevi-Shoup diagonal method for FC layers (baby steps b < n1,
// giant steps n1*j) and multiplexed convolutions (baby = spatial offsets, with the
// low part k1 of the channel offset k = k1 + n1 k2 when the plan splits it; giant =
// the rest of the channel offset).  The baby rotations of each input share one ModUp (hoisting);
// each giant rotation is a full key switch.  The paper's server round (Sec. 4.4)
// folds the unshuffle of the previous round and the shuffle of this round into
// the plaintexts, so they cost nothing here.
//
// Batching: requests are processed in chunks; each kernel of the schedule covers
// every ciphertext of the chunk at its own level (grid.z = entry), so one
// evaluation key or plaintext tile is read once per chunk.
#include <algorithm>

#include "galois.h"
#include "internal.h"
#include "modarith.h"

namespace fl {

constexpr int MAX_BABY = 64;

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int plan_create(Ctx *c, const fhelin_layer_desc *d, Plan **out) {
    FL_CHECK(c && d && out, FHELIN_E_INVALID_ARG, "plan_create: null argument");
    const int S = c->N / 2;
    std::unique_ptr<Plan> p(new Plan());
    p->kind = d->kind;
    p->desc = *d;
    if (d->kind == FHELIN_LAYER_FC) {
        FL_CHECK(pow2(d->fc_n) && S % d->fc_n == 0, FHELIN_E_UNSUPPORTED_PARAM, "fc_n must be a power of two dividing N/2");
        FL_CHECK(d->fc_out >= 1 && d->fc_out <= d->fc_n && d->fc_in >= 1 && d->fc_in <= d->fc_n,
                 FHELIN_E_INVALID_ARG, "fc_out / fc_in must be in [1, fc_n]");
        FL_CHECK(pow2(d->n1) && d->fc_n % d->n1 == 0 && d->n1 <= MAX_BABY, FHELIN_E_UNSUPPORTED_PARAM,
                 "n1 must be a power of two dividing fc_n, at most 64");
        p->n_in = p->n_out = 1;
        for (int b = 0; b < d->n1; ++b) p->rb.push_back(b);
        for (int j = 0; j < d->fc_n / d->n1; ++j) p->gk.push_back(d->n1 * j);
    } else if (d->kind == FHELIN_LAYER_CONV) {
        FL_CHECK(d->k == 1 || d->k == 3, FHELIN_E_UNSUPPORTED_PARAM, "conv kernel must be 1 or 3");
        FL_CHECK(d->c_in >= 1 && d->c_out >= 1 && d->h >= 1 && d->w >= 1, FHELIN_E_INVALID_ARG, "bad conv shape");
        const int hw = d->h * d->w;
        FL_CHECK(S % hw == 0, FHELIN_E_UNSUPPORTED_PARAM, "h*w must divide N/2");
        const int cct = S / hw;
        const int n1 = d->n1 > 1 ? d->n1 : 1;  // channel baby steps
        FL_CHECK(pow2(n1) && cct % n1 == 0 && n1 * d->k * d->k <= MAX_BABY, FHELIN_E_UNSUPPORTED_PARAM,
                 "conv n1 must be a power of two dividing the channels per ciphertext, n1 k^2 <= 64");
        p->n_in = (d->c_in + cct - 1) / cct;
        p->n_out = (d->c_out + cct - 1) / cct;
        FL_CHECK(p->n_in <= MAX_BATCH && p->n_out <= MAX_BATCH, FHELIN_E_UNSUPPORTED_PARAM, "too many ciphertexts per layer");
        for (int k1 = 0; k1 < n1; ++k1) {
            if (d->k == 1) {
                p->rb.push_back(k1 * hw);
            } else {
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) p->rb.push_back(k1 * hw + dy * d->w + dx);
            }
        }
        for (int j = 0; j < cct / n1; ++j) p->gk.push_back(n1 * j * hw);
    } else {
        return set_error(FHELIN_E_INVALID_ARG, "unknown layer kind");
    }
    std::vector<uint32_t> gal;
    for (int r : p->rb)
        if (galois_of_rotation(r, c->log_n) != 1) gal.push_back(galois_of_rotation(r, c->log_n));
    for (int r : p->gk)
        if (galois_of_rotation(r, c->log_n) != 1) gal.push_back(galois_of_rotation(r, c->log_n));
    std::sort(gal.begin(), gal.end());
    gal.erase(std::unique(gal.begin(), gal.end()), gal.end());
    p->galois = gal;
    *out = p.release();
    return FHELIN_OK;
}

// ---------------------------------------------------------------------------
// pt x ct multiply-accumulate: A[e][j] = sum_i sum_b pt[o][i][j][b] * R[i][b]
// grid (N/16, slots, n_out)
// ---------------------------------------------------------------------------
struct MacArgs {
    const uint64_t *x;    // inputs, NTT domain [2][ls] per input entry
    const uint64_t *rb;   // baby rotations [B'][2][ls] per input entry
    const uint64_t *pts;  // [n_pt][pt_level + K][N], Montgomery form
    uint64_t *acc;        // [G][2][ls] per output entry
    int n_in, n_out, B, Bp, G, pt_level;
    int ext;              // 0: Q limbs, ls = L; 1: extended basis, ls = L + K
    int8_t bmap[MAX_BABY];  // baby index -> slot in rb, -1 = identity (use x)
    int32_t order[MAX_BATCH];  // requests by descending level (a slot's active requests: a prefix)
    const uint64_t *zero;      // a zero word: the source of padding loads
    uint32_t b_magic;          // ceil(2^20 / B): t / B = (t b_magic) >> 20 for t < 4096
};

// For one limb (slot s) and coefficient k the multiply-accumulate is a small matrix
// product over the requests: A[r][j] = sum_t pt[o][j][t] * R[r][t] (t = (input i,
// baby b)).  A workgroup takes 16 coefficients, one slot and one output index and runs
// every request: thread (kl, jj) owns coefficient kl and giant step jj mod JT, keeps
// its 16-term plaintext column in registers (read from memory once per workgroup),
// and walks the requests in groups of ET = MY * ES, taking requests jj / JT + m ES of
// each group.  The groups' rotated inputs are staged in LDS, 16 terms at a time
// (zero past the last request), so the inner loop has no branches.  Requests go in
// descending level order, so the requests a q slot exists for are a prefix and
// the rest are skipped.  Operands are in the accumulator's form (28-bit halves
// when every modulus is below 2^55, else plain); every 32 terms (16 with larger
// moduli) end in one Montgomery reduction that seeds the next ones.
constexpr int MAC_K = 16;   // coefficients per workgroup
constexpr int MAC_TB = 16;  // terms per chunk
constexpr int MAC_ET = 8;   // requests per group at most

// MY = requests per thread (a tile choice); ET = requests per group (2, 4 or 8), so
// ES = ET / MY thread rows share a giant step; NC = 16-term chunks of the plaintext
// column kept in registers (terms <= 16 NC), else NC = 1 and the column is reloaded
// per chunk
template <bool SMALL, int MY, int NC, int ET>
__global__ void __launch_bounds__(256) k_mac(MacArgs a, Batch b, const ModConst *__restrict__ mods, int log_n,
                                             int L, int K, int R, int JT) {
    static_assert(ET % MY == 0 && ET <= 8, "bad request group");
    constexpr int ES = ET / MY;
    __shared__ uint64_t Rs[ET][MAC_TB][2][MAC_K];
    const int s = blockIdx.y;  // slot = modulus index (q_s for s < L, p_{s-L} otherwise)
    // a q slot above the plaintexts' level is active for no request (levels <= pt_level)
    if (s < L && s >= a.pt_level) return;
    const int64_t N = (int64_t)1 << log_n;
    const int k0 = blockIdx.x * MAC_K, o = blockIdx.z;
    const int kl = threadIdx.x & 15, jj = threadIdx.x >> 4;
    const int jloc = jj % JT, es = jj / JT;
    const bool computes = es < ES;  // other thread rows only help staging
    const int esc = computes ? es : 0;
    const int ls = a.ext ? L + K : L;
    const int64_t ct = (int64_t)2 * ls * N;
    const int terms = a.n_in * a.B;
    const int prows = a.pt_level + K;
    const int prow = s < L ? s : a.pt_level + (s - L);
    const ModConst mc = mods[s];
    int n_act = R;  // requests this slot exists for
    if (s < L) {
        n_act = 0;
        while (n_act < R && s < b.level[a.order[n_act] * a.n_out + o]) ++n_act;
    }
    // NC = 2 is launched only for terms <= 32
    const bool resident = NC > 1 || terms <= MAC_TB;
    // the request tile of a (group, chunk): thread holds values i < 2 ET, value i at
    // request row i / 2, term row tid / 32 + 8 (i & 1), polynomial (tid / 16) & 1,
    // coefficient tid & 15; the next tile's values are loaded before the current
    // tile's multiply-accumulate so their latency overlaps it
    // every load address below comes from registers and LDS only: an address read
    // from memory would make each load wait for all loads issued before it
    __shared__ int8_t bmap[MAX_BABY];
    __shared__ int32_t order[MAX_BATCH];
    if (threadIdx.x < MAX_BABY) bmap[threadIdx.x] = a.bmap[threadIdx.x];
    if (threadIdx.x < MAX_BATCH) order[threadIdx.x] = a.order[threadIdx.x];
    __syncthreads();
    const int kk = threadIdx.x & 15, pp = (threadIdx.x >> 4) & 1, tr = threadIdx.x >> 5;
    const int64_t lane_off = ((int64_t)pp * ls + s) * N + k0 + kk;
    uint64_t pre[2 * ET];
    auto fetch = [&](int g0, int t0) {
        // the thread's two terms of the chunk: source row of request order 0 and the
        // stride between request entries
        const uint64_t *tb[2];
        int64_t tstride[2];
        bool tv[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int t = t0 + tr + 8 * h;
            tv[h] = t < terms;
            const int ii = (int)(((uint32_t)t * a.b_magic) >> 20), bb = t - ii * a.B;
            const int m = tv[h] ? bmap[bb] : -1;
            tb[h] = (m < 0 ? a.x + (int64_t)ii * ct : a.rb + ((int64_t)ii * a.Bp + m) * ct) + lane_off;
            tstride[h] = (m < 0 ? (int64_t)a.n_in : (int64_t)a.n_in * a.Bp) * ct;
        }
        // the group's request entries, read once (scalar loads issued together)
        int ord[ET];
#pragma unroll
        for (int rr = 0; rr < ET; ++rr) ord[rr] = a.order[g0 + rr < n_act ? g0 + rr : 0];
        // every address first, then the loads: no branch separates them
        const uint64_t *src[2 * ET];
#pragma unroll
        for (int i = 0; i < 2 * ET; ++i) {
            const int h = i & 1, rr = i >> 1;
            const uint64_t *cand = tb[h] + ord[rr] * tstride[h];
            src[i] = tv[h] && g0 + rr < n_act ? cand : a.zero;
        }
#pragma unroll
        for (int i = 0; i < 2 * ET; ++i) pre[i] = *src[i];
    };
    auto stash = [&]() {
#pragma unroll
        for (int i = 0; i < 2 * ET; ++i) Rs[i >> 1][tr + 8 * (i & 1)][pp][kk] = LazyAcc<SMALL>::prep(pre[i]);
    };
    if (n_act > 0) fetch(0, 0);
    for (int jc = 0; jc < a.G; jc += JT) {
        const int j = jc + jloc;
        uint64_t pv[NC][MAC_TB];
        auto load_pv = [&](uint64_t(&col)[MAC_TB], int t0) {
#pragma unroll
            for (int tt = 0; tt < MAC_TB; ++tt) {
                const int t = t0 + tt;
                const uint64_t *src = a.zero;
                if (t < terms && j < a.G) {
                    const int ii = t / a.B, bb = t % a.B;
                    const int64_t pidx = ((int64_t)(o * a.n_in + ii) * a.G + j) * a.B + bb;
                    src = a.pts + (pidx * prows + prow) * N + k0 + kl;
                }
                col[tt] = *src;
            }
#pragma unroll
            for (int tt = 0; tt < MAC_TB; ++tt) col[tt] = LazyAcc<SMALL>::prep(col[tt]);
        };
        if (resident) {
#pragma unroll
            for (int c = 0; c < NC; ++c) load_pv(pv[c], c * MAC_TB);
        }
        for (int g0 = 0; g0 < n_act; g0 += ET) {
            LazyAcc<SMALL> acc[MY][2];
#pragma unroll
            for (int m = 0; m < MY; ++m) {
                acc[m][0].zero();
                acc[m][1].zero();
            }
            for (int t0 = 0; t0 < terms; t0 += MAC_TB) {
                if (!resident) load_pv(pv[0], t0);
                __syncthreads();  // readers of the previous tile are done
                stash();
                __syncthreads();
                // prefetch the next tile: next chunk, next group, or the first of the next
                // giant-step chunk (one call site: one inlined copy of the loads)
                int gn = g0, tn = t0 + MAC_TB;
                bool more = true;
                if (tn >= terms) {
                    tn = 0;
                    gn = g0 + ET;
                    if (gn >= n_act) {
                        gn = 0;
                        more = jc + JT < a.G;
                    }
                }
                if (more) fetch(gn, tn);
                auto compute = [&](const uint64_t(&col)[MAC_TB]) {
#pragma unroll
                    for (int tt = 0; tt < MAC_TB; ++tt) {
#pragma unroll
                        for (int m = 0; m < MY; ++m) {
                            const int rr = esc + m * ES;
                            acc[m][0].mac(Rs[rr][tt][0][kl], col[tt]);
                            acc[m][1].mac(Rs[rr][tt][1][kl], col[tt]);
                        }
                    }
                };
                if constexpr (NC > 1) {
                    if (resident && t0 >= MAC_TB) compute(pv[1]);
                    else compute(pv[0]);
                } else {
                    compute(pv[0]);
                }
                // reduce after every LazyAcc<SMALL>::TERMS products and at the end
                if ((t0 / MAC_TB) % (LazyAcc<SMALL>::TERMS / MAC_TB) == LazyAcc<SMALL>::TERMS / MAC_TB - 1 ||
                    t0 + MAC_TB >= terms) {
#pragma unroll
                    for (int m = 0; m < MY; ++m)
#pragma unroll
                        for (int p = 0; p < 2; ++p) acc[m][p].set(acc[m][p].reduce(mc.q, mc.mont_neg_inv));
                }
            }
            if (computes && j < a.G) {
#pragma unroll
                for (int m = 0; m < MY; ++m) {
                    const int r = g0 + esc + m * ES;
                    if (r < n_act) {
                        const int64_t e = (int64_t)order[r] * a.n_out + o;
                        uint64_t *dst = a.acc + (e * a.G + j) * ct + (int64_t)s * N + k0 + kl;
                        dst[0] = acc[m][0].value();
                        dst[(int64_t)ls * N] = acc[m][1].value();
                    }
                }
            }
        }
    }
}

static int launch_mac(const Ctx *c, const Plan *p, MacArgs &ma, const Batch &bout, hipStream_t s) {
    const int R = bout.n / p->n_out;
    // work: 2 (active limbs) N G B n_in products per output entry; bytes: the rotated
    // inputs (n_in B terms x 2 polys x active limbs per request), the accumulators
    // (G x 2 x active limbs per output entry) and the plaintexts once (slots x n_pt limbs)
    double macs = 0, bytes = 0;
    int lmax = 0;
    const double limb = 8.0 * c->N;
    for (int e = 0; e < bout.n; ++e) {
        lmax = std::max<int>(lmax, bout.level[e]);
        const double act = bout.level[e] + (ma.ext ? c->K : 0);
        macs += 2.0 * act * (double)c->N * ma.G * ma.B * p->n_in;
        bytes += limb * 2 * act * ma.G;
        if (e % p->n_out == 0) bytes += limb * 2 * act * ma.B * p->n_in;
    }
    bytes += limb * (double)p->n_pt() * ((ma.ext ? c->K : 0) + std::min(lmax, ma.pt_level));
    // requests by descending level (stable)
    int idx[MAX_BATCH];
    for (int r = 0; r < R; ++r) idx[r] = r;
    std::stable_sort(idx, idx + R, [&](int x, int y) { return bout.level[x * p->n_out] > bout.level[y * p->n_out]; });
    for (int r = 0; r < R; ++r) ma.order[r] = idx[r];
    ma.zero = c->d_zero;
    ma.b_magic = (uint32_t)(((1u << 20) + ma.B - 1) / ma.B);
    const int JT = std::min(ma.G, 16);
    const int MY = p->tune.mac_my;
    // requests per group: MY times the thread rows per giant step (at most 16 / JT), a power of two <= 8
    int ET = MY;
    while (ET * 2 <= MAC_ET && (ET * 2) / MY <= 16 / JT) ET *= 2;
    const int slots = ma.ext ? c->L + c->K : lmax;
    ProfScope ps(c, s, PK_MAC, macs, bytes);
    dim3 grid(c->N / MAC_K, slots, p->n_out);
    const int terms = p->n_in * ma.B, NC = terms > MAC_TB && terms <= 2 * MAC_TB ? 2 : 1;
#define FL_MAC(SM, Y, C, E) hipLaunchKernelGGL((k_mac<SM, Y, C, E>), grid, dim3(256), 0, s, ma, bout, c->d_mods, \
                                               c->log_n, c->L, c->K, R, JT)
#define FL_MAC_E(SM, Y, C) \
    if (ET == 2) FL_MAC(SM, 2, C, 2); \
    else if (ET == 4 && Y <= 4) FL_MAC(SM, (Y <= 4 ? Y : 4), C, 4); \
    else FL_MAC(SM, Y, C, 8)
#define FL_MAC_Y(SM, C) \
    if (MY == 2) { FL_MAC_E(SM, 2, C); } \
    else if (MY == 4) { FL_MAC_E(SM, 4, C); } \
    else { FL_MAC(SM, 8, C, 8); }
    if (c->small) {
        if (NC == 2) { FL_MAC_Y(true, 2) } else { FL_MAC_Y(true, 1) }
    } else {
        if (NC == 2) { FL_MAC_Y(false, 2) } else { FL_MAC_Y(false, 1) }
    }
#undef FL_MAC_Y
#undef FL_MAC_E
#undef FL_MAC
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

// Baby rotations fused into the multiply-accumulate (double-hoisted schedule, one key
// set for the whole chunk).  The rotated inputs of a tile,
//   R~_b = (P sigma_b(c0) + <sigma_b(D), evk_b>_0, <sigma_b(D), evk_b>_1)
// over the extended basis, are computed into LDS from the hoisted digits D and the key
// rows and multiplied there as in k_mac; they never go to memory (the separate
// rotation launch writes them, 2 (l + K) limbs per rotation and request, and the
// multiply-accumulate reads them back).  Staging thread (tb, kk) computes term t0 + tb
// at coefficient k0 + kk for every request of the group: the digits and c0 are
// gathered at sigma_b(k) -- the 16 coefficients of a 16-aligned group map onto one
// 16-aligned group, one 128-byte line per term and digit -- and the key rows are read
// at k.  The next tile's loads are issued before the current tile is multiplied.  Each
// staged value is the one the rotation launch would have written (exact arithmetic,
// reduced to [0, q)), so the outputs are bit-identical to the unfused path.
struct RotMacArgs {
    const uint64_t *dig;     // hoisted digits [dnum][L+K] per input entry (NTT domain)
    int64_t dig_es;
    const uint64_t *xq;      // inputs [2][L] per input entry (NTT domain): c0 of the addend
    int64_t xq_es;
    const uint64_t *evk;     // the key set of every request of the chunk
    const ModDownTab *mdt;   // P mod q_s (Montgomery form)
    int key_level, alpha;
    uint32_t g[MAX_BABY];    // Galois element of baby b (1: the identity, read from a.x)
    int32_t kidx[MAX_BABY];  // key index of baby b in the set (0 for the identity)
};

constexpr int ROTMAC_MAXB = 4;  // digits per request the fused kernel holds (dnum <= 4)

template <int MY, int NC, int ET>
__global__ void __launch_bounds__(256) k_rot_mac(MacArgs a, RotMacArgs r, Batch b, const ModConst *__restrict__ mods,
                                                 int log_n, int L, int K, int R, int JT) {
    static_assert(ET % MY == 0 && ET <= 8, "bad request group");
    constexpr int ES = ET / MY, MAXB = ROTMAC_MAXB;
    using Acc = LazyAcc<true>;
    __shared__ uint64_t Rs[ET][MAC_TB][2][MAC_K];
    __shared__ int32_t rin[MAX_BATCH];   // first input entry of the request at each position of the order
    __shared__ int32_t rbeta[MAX_BATCH]; // its digit count
    const int s = blockIdx.y;
    if (s < L && s >= a.pt_level) return;
    const int64_t N = (int64_t)1 << log_n;
    const int k0 = blockIdx.x * MAC_K, o = blockIdx.z;
    const int kl = threadIdx.x & 15, jj = threadIdx.x >> 4;
    const int jloc = jj % JT, es = jj / JT;
    const bool computes = es < ES;
    const int esc = computes ? es : 0;
    const int ls = L + K;
    const int64_t ct = (int64_t)2 * ls * N, row = (int64_t)ls * N;
    const int terms = a.n_in * a.B;
    const int prows = a.pt_level + K;
    const int prow = s < L ? s : a.pt_level + (s - L);
    const ModConst mc = mods[s];
    int n_act = R;
    if (s < L) {
        n_act = 0;
        while (n_act < R && s < b.level[a.order[n_act] * a.n_out + o]) ++n_act;
    }
    const bool resident = NC > 1 || terms <= MAC_TB;
    if (threadIdx.x < MAX_BATCH) {
        const int q = threadIdx.x < R ? a.order[threadIdx.x] : 0;
        rin[threadIdx.x] = q * a.n_in;
        rbeta[threadIdx.x] = (b.level[q * a.n_out + o] + r.alpha - 1) / r.alpha;
    }
    __syncthreads();
    // staging role
    const int tb = threadIdx.x >> 4, kk = threadIdx.x & 15, k = k0 + kk;
    const int kbeta = (r.key_level + r.alpha - 1) / r.alpha;
    const int64_t kpart = (int64_t)(r.key_level + K) * N;
    const int64_t krow = (int64_t)(s < L ? s : r.key_level + (s - L)) * N + k;
    const bool has_add = s < L;  // P = 0 mod p_i
    const uint64_t p_mont = r.mdt->p_mont[has_add ? s : 0];
    uint64_t pd[ET][MAXB], pc[ET], pkb[MAXB], pka[MAXB];
    int cnt[ET];
    bool ident = false;
    auto fetch = [&](int g0, int t0) {
        const int t = t0 + tb;
        const bool tv = t < terms;
        const int ii = (int)(((uint32_t)t * a.b_magic) >> 20), bb = t - ii * a.B;
        const int bbc = tv ? bb : 0, iic = tv ? ii : 0;
        const uint32_t g = r.g[bbc];
        ident = g == 1u;
        const int src = ident ? k : auto_index(k, g, log_n);
        // key rows at k (rows past the key's digits repeat its last one, never used)
        const uint64_t *key = r.evk + (int64_t)r.kidx[bbc] * 2 * kbeta * kpart + krow;
#pragma unroll
        for (int j = 0; j < MAXB; ++j) {
            const int jr = j < kbeta ? j : kbeta - 1;
            pkb[j] = key[(2 * jr) * kpart];
            pka[j] = key[(2 * jr + 1) * kpart];
        }
        // every address first, then the loads
        const uint64_t *srcs[ET][MAXB + 1];
#pragma unroll
        for (int rr = 0; rr < ET; ++rr) {
            const int rq = g0 + rr;
            const bool live = tv && rq < n_act;
            const int e_in = rin[live ? rq : 0] + iic;
            // the identity reads both polynomials of a.x (P x on the extended basis), a
            // rotation its digits at sigma_b(k); both are rows ls N apart
            cnt[rr] = !live ? 0 : ident ? 2 : rbeta[rq];
            const uint64_t *base = ident ? a.x + e_in * ct + (int64_t)s * N + k
                                         : r.dig + e_in * r.dig_es + (int64_t)s * N + src;
#pragma unroll
            for (int j = 0; j < MAXB; ++j) srcs[rr][j] = j < cnt[rr] ? base + j * row : a.zero;
            srcs[rr][MAXB] = live && !ident && has_add ? r.xq + e_in * r.xq_es + (int64_t)s * N + src : a.zero;
        }
#pragma unroll
        for (int rr = 0; rr < ET; ++rr) {
#pragma unroll
            for (int j = 0; j < MAXB; ++j) pd[rr][j] = *srcs[rr][j];
            pc[rr] = *srcs[rr][MAXB];
        }
    };
    auto stash = [&]() {
        uint64_t kb[MAXB], ka[MAXB];
#pragma unroll
        for (int j = 0; j < MAXB; ++j) {
            kb[j] = Acc::prep(pkb[j]);
            ka[j] = Acc::prep(pka[j]);
        }
#pragma unroll
        for (int rr = 0; rr < ET; ++rr) {
            uint64_t v0 = pd[rr][0], v1 = pd[rr][1];
            if (!ident) {
                Acc a0, a1;
                a0.zero();
                a1.zero();
                // rows past the request's digits were loaded from the zero word
#pragma unroll
                for (int j = 0; j < MAXB; ++j) {
                    const uint64_t dv = Acc::prep(pd[rr][j]);
                    a0.mac(dv, kb[j]);
                    a1.mac(dv, ka[j]);
                }
                v0 = a0.reduce(mc.q, mc.mont_neg_inv);
                v1 = a1.reduce(mc.q, mc.mont_neg_inv);
                if (has_add) v0 = add_mod(v0, mont_mul(pc[rr], p_mont, mc.q, mc.mont_neg_inv), mc.q);
            }
            if (cnt[rr] == 0) v0 = v1 = 0;
            Rs[rr][tb][0][kk] = Acc::prep(v0);
            Rs[rr][tb][1][kk] = Acc::prep(v1);
        }
    };
    if (n_act > 0) fetch(0, 0);
    for (int jc = 0; jc < a.G; jc += JT) {
        const int j = jc + jloc;
        uint64_t pv[NC][MAC_TB];
        auto load_pv = [&](uint64_t(&col)[MAC_TB], int t0) {
#pragma unroll
            for (int tt = 0; tt < MAC_TB; ++tt) {
                const int t = t0 + tt;
                const uint64_t *src = a.zero;
                if (t < terms && j < a.G) {
                    const int ii = t / a.B, bb = t % a.B;
                    const int64_t pidx = ((int64_t)(o * a.n_in + ii) * a.G + j) * a.B + bb;
                    src = a.pts + (pidx * prows + prow) * N + k0 + kl;
                }
                col[tt] = *src;
            }
#pragma unroll
            for (int tt = 0; tt < MAC_TB; ++tt) col[tt] = Acc::prep(col[tt]);
        };
        if (resident) {
#pragma unroll
            for (int c = 0; c < NC; ++c) load_pv(pv[c], c * MAC_TB);
        }
        for (int g0 = 0; g0 < n_act; g0 += ET) {
            Acc acc[MY][2];
#pragma unroll
            for (int m = 0; m < MY; ++m) {
                acc[m][0].zero();
                acc[m][1].zero();
            }
            for (int t0 = 0; t0 < terms; t0 += MAC_TB) {
                if (!resident) load_pv(pv[0], t0);
                __syncthreads();  // readers of the previous tile are done
                stash();
                __syncthreads();
                int gn = g0, tn = t0 + MAC_TB;
                bool more = true;
                if (tn >= terms) {
                    tn = 0;
                    gn = g0 + ET;
                    if (gn >= n_act) {
                        gn = 0;
                        more = jc + JT < a.G;
                    }
                }
                if (more) fetch(gn, tn);
                auto compute = [&](const uint64_t(&col)[MAC_TB]) {
#pragma unroll
                    for (int tt = 0; tt < MAC_TB; ++tt) {
#pragma unroll
                        for (int m = 0; m < MY; ++m) {
                            const int rr = esc + m * ES;
                            acc[m][0].mac(Rs[rr][tt][0][kl], col[tt]);
                            acc[m][1].mac(Rs[rr][tt][1][kl], col[tt]);
                        }
                    }
                };
                if constexpr (NC > 1) {
                    if (resident && t0 >= MAC_TB) compute(pv[1]);
                    else compute(pv[0]);
                } else {
                    compute(pv[0]);
                }
                if ((t0 / MAC_TB) % (Acc::TERMS / MAC_TB) == Acc::TERMS / MAC_TB - 1 || t0 + MAC_TB >= terms) {
#pragma unroll
                    for (int m = 0; m < MY; ++m)
#pragma unroll
                        for (int p = 0; p < 2; ++p) acc[m][p].set(acc[m][p].reduce(mc.q, mc.mont_neg_inv));
                }
            }
            if (computes && j < a.G) {
#pragma unroll
                for (int m = 0; m < MY; ++m) {
                    const int rq = g0 + esc + m * ES;
                    if (rq < n_act) {
                        const int64_t e = (int64_t)a.order[rq] * a.n_out + o;
                        uint64_t *dst = a.acc + (e * a.G + j) * ct + (int64_t)s * N + k0 + kl;
                        dst[0] = acc[m][0].value();
                        dst[row] = acc[m][1].value();
                    }
                }
            }
        }
    }
}

// The fused launch applies to a chunk whose requests share one key set, holding every
// baby key, with at most ROTMAC_MAXB digits and packed (small-modulus) arithmetic.
static bool rot_mac_applies(const Ctx *c, const Plan *p, const KeySet *const *kss, int Rc) {
    if (!p->tune.fuse_baby || !c->small || (c->L + c->alpha - 1) / c->alpha > ROTMAC_MAXB) return false;
    for (int r = 1; r < Rc; ++r)
        if (kss[r] != kss[0]) return false;
    return kss[0] != nullptr;
}

static int launch_rot_mac(const Ctx *c, const Plan *p, MacArgs &ma, RotMacArgs &ra, const Batch &bout,
                          const Batch &bin, hipStream_t s) {
    const int R = bout.n / p->n_out;
    // work: the multiply-accumulate's products plus the rotations' key products (2 beta
    // per rotation, polynomial pair and active limb); bytes: the digits and c0 once per
    // input entry, the lifted input for the identity, each baby key once, the
    // plaintexts once and the accumulators written
    double units = 0, bytes = 0;
    int lmax = 0;
    const double limb = 8.0 * c->N;
    for (int e = 0; e < bout.n; ++e) {
        lmax = std::max<int>(lmax, bout.level[e]);
        const double l = bout.level[e], act = l + c->K, beta = std::ceil(l / c->alpha);
        units += 2.0 * act * (double)c->N * ma.G * ma.B * p->n_in;
        units += 2.0 * beta * act * (double)c->N * ma.Bp * p->n_in / p->n_out;
        bytes += limb * 2 * act * ma.G;
    }
    for (int e = 0; e < bin.n; ++e) {
        const double l = bin.level[e], act = l + c->K, beta = std::ceil(l / c->alpha);
        bytes += limb * (beta * act + l + (ma.Bp < ma.B ? 2 * l : 0));
    }
    const double kl = ra.key_level;
    bytes += limb * ma.Bp * 2 * std::ceil(kl / c->alpha) * (std::min<double>(kl, lmax) + c->K);
    bytes += limb * (double)p->n_pt() * (c->K + std::min(lmax, ma.pt_level));
    int idx[MAX_BATCH];
    for (int r = 0; r < R; ++r) idx[r] = r;
    std::stable_sort(idx, idx + R, [&](int x, int y) { return bout.level[x * p->n_out] > bout.level[y * p->n_out]; });
    for (int r = 0; r < R; ++r) ma.order[r] = idx[r];
    ma.zero = c->d_zero;
    ma.b_magic = (uint32_t)(((1u << 20) + ma.B - 1) / ma.B);
    const int JT = std::min(ma.G, 16);
    const int MY = p->tune.mac_my;
    int ET = MY;
    while (ET * 2 <= MAC_ET && (ET * 2) / MY <= 16 / JT) ET *= 2;
    ProfScope ps(c, s, PK_ROT_MAC, units, bytes);
    dim3 grid(c->N / MAC_K, c->L + c->K, p->n_out);
    const int terms = p->n_in * ma.B, NC = terms > MAC_TB && terms <= 2 * MAC_TB ? 2 : 1;
#define FL_RM(Y, C, E) hipLaunchKernelGGL((k_rot_mac<Y, C, E>), grid, dim3(256), 0, s, ma, ra, bout, c->d_mods, \
                                          c->log_n, c->L, c->K, R, JT)
#define FL_RM_E(Y, C) \
    if (ET == 2) FL_RM(2, C, 2); \
    else if (ET == 4 && Y <= 4) FL_RM((Y <= 4 ? Y : 4), C, 4); \
    else FL_RM(Y, C, 8)
#define FL_RM_Y(C) \
    if (MY == 2) { FL_RM_E(2, C); } \
    else if (MY == 4) { FL_RM_E(4, C); } \
    else { FL_RM(8, C, 8); }
    if (NC == 2) { FL_RM_Y(2) } else { FL_RM_Y(1) }
#undef FL_RM_Y
#undef FL_RM_E
#undef FL_RM
    FL_TRY_HIP(hipGetLastError());
    return FHELIN_OK;
}

bool tune_valid(const Tune &t) {
    return t.chunk >= 0 && t.chunk <= MAX_BATCH && t.ks_eg >= 1 && t.ks_eg <= MAX_BATCH &&
           (t.mac_my == 2 || t.mac_my == 4 || t.mac_my == 8) &&
           (t.ntt_threads == 128 || t.ntt_threads == 256 || t.ntt_threads == 512) &&
           (t.persistent == 0 || t.persistent == 1) && (t.fuse_baby == 0 || t.fuse_baby == 1);
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
int workspace_get(Ctx *c, hipStream_t s, size_t bytes, uint64_t **out, std::shared_ptr<WsBuf> *hold) {
    Workspace *w;
    {
        std::lock_guard<std::mutex> g(c->mu);
        auto &slot = c->ws[(void *)s];
        if (!slot) slot.reset(new Workspace());
        w = slot.get();
    }
    if (!w->cur || w->cur->bytes < bytes) {
        if (w->cur) {
            // the old buffer is freed here unless a captured graph still holds it
            if (w->cur.use_count() == 1) FL_TRY_HIP(hipStreamSynchronize(s));
            w->cur.reset();
        }
        std::shared_ptr<WsBuf> nb(new WsBuf());
        nb->ctx = c;
        FL_RET(dev_alloc(c, &nb->buf, bytes));
        nb->bytes = bytes;
        w->cur = std::move(nb);
    }
    *out = (uint64_t *)w->cur->buf;
    if (hold) *hold = w->cur;
    return FHELIN_OK;
}

// ---------------------------------------------------------------------------
// helpers building row maps
// ---------------------------------------------------------------------------
static RowMap rows_ct(const Ctx *c, const Batch &b, uint64_t *base, int64_t es, int stride, int poly_lo,
                      int poly_cnt) {
    RowMap m{};
    m.base = base;
    m.ct_stride = es;
    m.kind = ROWS_CT;
    m.n_ct = b.n;
    m.stride = stride;
    m.poly_lo = poly_lo;
    m.poly_cnt = poly_cnt;
    m.L = c->L;
    m.K = c->K;
    m.alpha = c->alpha;
    m.log_n = c->log_n;
    for (int t = 0; t < b.n; ++t) m.level[t] = b.level[t];
    return m;
}

static RowMap rows_kind(const Ctx *c, const Batch &b, uint64_t *base, int64_t es, int kind, int n_part) {
    RowMap m = rows_ct(c, b, base, es, 0, 0, 0);
    m.kind = kind;
    m.n_part = n_part;
    return m;
}

// One full key switch of the batch entries: given c1 (NTT, ct layout) and the
// automorphism/key per entry in `b`, accumulate (sigma_g(c0) + out0, out1) into dst.
struct KsScratch {
    uint64_t *tc;  int64_t tc_es;   // [L] coefficient temp
    uint64_t *dg;  int64_t dg_es;   // [dnum][L+K] digits
    uint64_t *u;   int64_t u_es;    // [2][L+K]
    uint64_t *md;  int64_t md_es;   // [2][L]
    uint32_t *ctl = nullptr;        // control block of the persistent ModUp + NTT launch (null: separate launches)
};

// ModUp of the coefficient-domain limbs at `coef` into digits, then their forward NTT over
// the rows of `rm`: one persistent launch when a control block is given (N >= 2^13),
// else the ModUp kernel and the two NTT passes
static int modup_and_ntt(const Ctx *c, const Batch &b, const uint64_t *coef, int64_t coef_es, const uint64_t *ntt,
                         int64_t ntt_es, uint64_t *dg, int64_t dg_es, const RowMap &rm, uint32_t *ctl, hipStream_t s) {
    if (ctl && c->log_n >= 13) return launch_modup_ntt(c, b, coef, coef_es, ntt, ntt_es, dg, dg_es, rm, ctl, s);
    FL_RET(launch_modup(c, b, coef, coef_es, ntt, ntt_es, dg, dg_es, s));
    return launch_ntt(c, rm, 0, s);
}

// ModUp of the c1 polynomial of ct entries (NTT domain in, digits NTT domain out)
static int modup_ct(const Ctx *c, const Batch &b, const uint64_t *ct, int64_t ct_es, int ct_stride,
                    const KsScratch &w, hipStream_t s) {
    const int64_t N = c->N;
    RowMap src = rows_ct(c, b, (uint64_t *)ct, ct_es, ct_stride, 1, 1);
    RowMap dst = rows_ct(c, b, w.tc, w.tc_es, c->L, 0, 1);
    FL_RET(launch_ntt_from(c, dst, src, 1, s));  // c1 to the coefficient domain, out of place
    return modup_and_ntt(c, b, w.tc, w.tc_es, ct + (int64_t)ct_stride * N, ct_es, w.dg, w.dg_es,
                         rows_kind(c, b, w.dg, w.dg_es, ROWS_MODUP, 0), w.ctl, s);
}

// inner product + ModDown + combine, digits already in w.dg
static int ks_finish(const Ctx *c, const Batch &b, const KsScratch &w, uint64_t *dst, int64_t dst_es, int dst_stride,
                     const uint64_t *c0, int64_t c0_es, int c0_stride, int accumulate, hipStream_t s, int eg = 8) {
    FL_RET(launch_ks_inner(c, b, w.dg, w.dg_es, w.u, w.u_es, s, eg));
    FL_RET(launch_ntt(c, rows_kind(c, b, w.u, w.u_es, ROWS_EXT_P, 2), 1, s));
    FL_RET(launch_moddown_fbc(c, b, w.u, w.u_es, w.md, w.md_es, s));
    FL_RET(launch_ntt(c, rows_ct(c, b, w.md, w.md_es, c->L, 0, 2), 0, s));
    FL_RET(launch_moddown_combine(c, b, w.u, w.u_es, w.md, w.md_es, dst, dst_es, dst_stride, c0, c0_es, c0_stride,
                                  accumulate, s));
    return FHELIN_OK;
}

// entries e of a batch belong to request e / per_req; each gets that request's key for g
static void set_keys(Batch &b, int per_req, const KeySet *const *kss, uint32_t g) {
    for (int e = 0; e < b.n; ++e) {
        const KeySet *ks = kss[e / per_req];
        b.g[e] = g;
        b.key[e] = ks->key_ptr(ks->find(g));
        b.key_level[e] = (uint8_t)ks->level;
    }
}

static int check_batch(const Ctx *c, const fhelin_ct_batch *bt, const char *what) {
    FL_CHECK(bt && bt->data && bt->levels && bt->n_ct >= 0, FHELIN_E_INVALID_ARG, std::string(what) + ": null batch");
    FL_CHECK(bt->stride >= 1 && bt->stride <= c->L, FHELIN_E_INVALID_ARG, std::string(what) + ": stride out of range");
    for (int t = 0; t < bt->n_ct; ++t)
        FL_CHECK(bt->levels[t] >= 1 && bt->levels[t] <= bt->stride, FHELIN_E_LEVEL_MISMATCH,
                 std::string(what) + ": level out of range");
    return FHELIN_OK;
}

// ---------------------------------------------------------------------------
// linear layer over a batch of requests
// ---------------------------------------------------------------------------
static size_t limbs_per_request(const Ctx *c, const Plan *p, int Bp) {
    const size_t L = c->L, K = c->K, D = c->dnum;
    const size_t ni = p->n_in, no = p->n_out, G = p->gk.size();
    const size_t emax = std::max(ni, no);
    return ni * 2 * L             // X
           + ni * D * (L + K)      // hoisted digits
           + ni * Bp * 2 * L       // baby rotations
           + no * G * 2 * L        // accumulators
           + no * 2 * L            // Y
           + emax * L              // coefficient temp
           + emax * D * (L + K)    // giant digits
           + emax * 2 * (L + K)    // u
           + emax * 2 * L;         // md
}

// giant steps other than the identity
static int giant_nonid(const Ctx *c, const Plan *p) {
    int n = 0;
    for (int r : p->gk) n += galois_of_rotation(r, c->log_n) == 1 ? 0 : 1;
    return n;
}

// digit buffers of the giant steps: one per step of a group summed in one launch
// (groups of at most MAX_SUM steps)
static int giant_digit_sets(const Ctx *c, const Plan *p) {
    const int n = giant_nonid(c, p);
    return n < 1 ? 1 : std::min(n, MAX_SUM);
}

static size_t limbs_per_request_dh(const Ctx *c, const Plan *p, int Bp) {
    const size_t L = c->L, K = c->K, D = c->dnum, E = L + K;
    const size_t ni = p->n_in, no = p->n_out, G = p->gk.size();
    const size_t emax = std::max(ni, no), nd = giant_digit_sets(c, p);
    return ni * 2 * L         // X
           + ni * 2 * E        // P * X
           + ni * D * E        // hoisted digits
           + ni * Bp * 2 * E   // baby rotations (extended basis)
           + no * G * 2 * E    // accumulators (extended basis)
           + no * 4 * E        // giant-step sums (extended basis; two, alternating between groups)
           + no * 2 * L        // Y
           + emax * 2 * L      // Q temp for ModDown(c1)
           + emax * L          // coefficient temp
           + emax * D * E * nd // giant digits
           + emax * 2 * L;     // md
}

// requests per chunk: at most MAX_BATCH ciphertexts on either side, the plan's tuned
// chunk if set, and no more than the requests present
static int chunk_of(const Plan *p, int n_requests, int max_chunk) {
    int chunk = std::max(1, std::min(max_chunk, MAX_BATCH / std::max(p->n_in, p->n_out)));
    if (p->tune.chunk > 0) chunk = std::min(chunk, p->tune.chunk);
    return std::min(chunk, std::max(1, n_requests));
}

// the persistent launch's control block, after the chunk's buffers in the workspace
static constexpr size_t CTL_BYTES = ((size_t)PERSIST_CTL_WORDS * 4 + 255) / 256 * 256;

size_t linear_workspace_bytes(const Ctx *c, const Plan *p, int n_requests, int max_chunk, int flags) {
    int Bp = 0;
    for (int r : p->rb) Bp += galois_of_rotation(r, c->log_n) == 1 ? 0 : 1;
    const int chunk = chunk_of(p, n_requests, max_chunk);
    size_t per = (flags & FHELIN_APPLY_HOIST_MODDOWN) ? limbs_per_request_dh(c, p, Bp) : limbs_per_request(c, p, Bp);
    return per * chunk * (size_t)c->N * sizeof(uint64_t) + (p->tune.persistent ? CTL_BYTES : 0);
}

// Export Y (NTT, [2][L] per entry) to the caller's batch, with or without rescale.
static int export_out(Ctx *c, const Batch &bout, uint64_t *Y, const fhelin_ct_batch *out, int64_t first_ct,
                      bool rescale, hipStream_t s) {
    const int64_t N = c->N, ct = 2 * (int64_t)c->L * N;
    RowMap yr = rows_ct(c, bout, Y, ct, c->L, 0, 2);
    FL_RET(launch_ntt(c, yr, 1, s));
    const int64_t out_es = (int64_t)2 * out->stride * N;
    uint64_t *ob = out->data + first_ct * out_es;
    if (rescale) return launch_rescale(c, bout, Y, ct, c->L, ob, out_es, out->stride, s);
    return launch_copy_rows(c, rows_ct(c, bout, ob, out_es, out->stride, 0, 2), yr, s);
}

// Giant step of the double-hoisted schedule: ModDown of A~_j.c1 (extended basis, NTT
// domain, consumed) to the Q basis, then ModUp of the result into the digits dg.  The
// ModDown runs in the coefficient domain (one inverse transform of all l + K limbs,
// conversion and combination in one pass), which is where ModUp needs its input; the
// digits' own limbs are copied there and transformed with the rest.
static int giant_moddown_modup(const Ctx *c, const Batch &b, uint64_t *a1, int64_t a_es, uint64_t *tc,
                               uint64_t *dg, int64_t dg_es, uint32_t *ctl, hipStream_t s) {
    const int64_t LN = (int64_t)c->L * c->N;
    FL_RET(launch_ntt(c, rows_kind(c, b, a1, a_es, ROWS_EXT, 1), 1, s));
    FL_RET(launch_moddown_coef(c, b, a1, a_es, tc, LN, s));
    return modup_and_ntt(c, b, tc, LN, tc, LN, dg, dg_es, rows_kind(c, b, dg, dg_es, ROWS_DIGITS, 0), ctl, s);
}

// One chunk of requests with the double-hoisted schedule (Bossuat et al. 2021): baby
// rotations, the multiply-accumulate and the giant-step sum stay in the extended basis
// (carrying a factor P); each giant step ModDowns only c1 before its ModUp, and one
// ModDown per output ends the layer.
static int apply_chunk_dh(Ctx *c, const Plan *p, const KeySet *const *kss, const PtSet *pts,
                          const fhelin_ct_batch *in, const fhelin_ct_batch *out, bool rescale, hipStream_t s,
                          uint64_t *ws, int r0, int Rc, MacArgs ma, int Bp, uint32_t *ctl) {
    const int64_t N = c->N, L = c->L, K = c->K, E = L + K;
    const int B = (int)p->rb.size(), G = (int)p->gk.size();
    const int64_t ct = 2 * L * N, ext = 2 * E * N, dg = (int64_t)c->dnum * E * N;
    const int Ein = Rc * p->n_in, Eout = Rc * p->n_out, Emax = std::max(Ein, Eout);
    uint64_t *X = ws, *XL = X + Ein * ct, *D = XL + Ein * ext, *RB = D + Ein * dg;
    uint64_t *A = RB + (int64_t)Ein * Bp * ext, *YE = A + (int64_t)Eout * G * ext, *YE2 = YE + Eout * ext;
    uint64_t *Y = YE2 + Eout * ext;
    const int n_dg = giant_digit_sets(c, p);
    uint64_t *TQ = Y + Eout * ct, *TC = TQ + Emax * ct, *DG = TC + Emax * L * N, *MD = DG + Emax * dg * n_dg;
    Batch bin{}, bout{};
    bin.n = Ein;
    bout.n = Eout;
    for (int e = 0; e < Ein; ++e) {
        bin.level[e] = (uint8_t)in->levels[(r0 * p->n_in) + e];
        bin.g[e] = 1;
    }
    for (int e = 0; e < Eout; ++e) {
        bout.level[e] = (uint8_t)in->levels[(r0 + e / p->n_out) * p->n_in];
        bout.g[e] = 1;
    }
    // 1. import
    const int64_t in_es = (int64_t)2 * in->stride * N;
    RowMap src = rows_ct(c, bin, in->data + (int64_t)r0 * p->n_in * in_es, in_es, in->stride, 0, 2);
    RowMap dx = rows_ct(c, bin, X, ct, (int)L, 0, 2);
    FL_RET(launch_ntt_from(c, dx, src, 0, s));
    // 2. P * x for the identity baby step
    bool has_identity = false;
    for (int b = 0; b < B; ++b) has_identity |= ma.bmap[b] < 0;
    if (has_identity) FL_RET(launch_ext_lift_add(c, bin, X, ct, (int)L, 1, 0, XL, ext, s));
    // 3. baby rotations in the extended basis: (P sigma(c0) + u0, u1), either inside the
    // multiply-accumulate (one key set for the chunk) or by their own launch
    const bool fused = Bp > 0 && rot_mac_applies(c, p, kss + r0, Rc);
    ma.x = XL;
    ma.rb = RB;
    ma.pts = pts->data;
    ma.acc = A;
    ma.n_in = p->n_in;
    ma.n_out = p->n_out;
    ma.B = B;
    ma.Bp = Bp;
    ma.G = G;
    ma.pt_level = pts->level;
    ma.ext = 1;
    if (fused) {
        KsScratch wb{TC, L * N, D, dg, nullptr, 0, MD, ct, ctl};
        FL_RET(modup_ct(c, bin, X, ct, (int)L, wb, s));
        const KeySet *ks = kss[r0];
        RotMacArgs ra{};
        ra.dig = D;
        ra.dig_es = dg;
        ra.xq = X;
        ra.xq_es = ct;
        ra.evk = ks->evk;
        ra.mdt = c->d_moddown;
        ra.key_level = ks->level;
        ra.alpha = c->alpha;
        for (int b = 0; b < B; ++b) {
            const uint32_t g = galois_of_rotation(p->rb[b], c->log_n);
            ra.g[b] = g;
            ra.kidx[b] = g == 1 ? 0 : ks->find(g);
        }
        FL_RET(launch_rot_mac(c, p, ma, ra, bout, bin, s));
    } else if (Bp > 0) {
        KsScratch wb{TC, L * N, D, dg, nullptr, 0, MD, ct, ctl};
        FL_RET(modup_ct(c, bin, X, ct, (int)L, wb, s));
        // one launch for every baby rotation when all key sets of the chunk hold the
        // rotations' keys at the same indices (always, for one client)
        KsRot rot{};
        bool same = true;
        for (int b = 0; b < B; ++b) {
            if (ma.bmap[b] < 0) continue;
            const uint32_t g = galois_of_rotation(p->rb[b], c->log_n);
            const int idx = kss[r0]->find(g);
            for (int r = 1; r < Rc; ++r) same = same && kss[r0 + r]->find(g) == idx;
            rot.g[rot.n] = g;
            rot.key[rot.n] = idx;
            rot.out[rot.n] = (int64_t)ma.bmap[b] * ext;
            ++rot.n;
        }
        if (same) {
            for (int e = 0; e < Ein; ++e) {
                const KeySet *ks = kss[r0 + e / p->n_in];
                bin.key[e] = ks->evk;
                bin.key_level[e] = (uint8_t)ks->level;
            }
            FL_RET(launch_ks_inner_rot(c, bin, rot, D, dg, RB, (int64_t)Bp * ext, X, ct, 0, s, p->tune.ks_eg));
        } else {
            for (int b = 0; b < B; ++b) {
                if (ma.bmap[b] < 0) continue;
                set_keys(bin, p->n_in, kss + r0, galois_of_rotation(p->rb[b], c->log_n));
                FL_RET(launch_ks_inner_add(c, bin, D, dg, RB + ma.bmap[b] * ext, (int64_t)Bp * ext, X, ct, 0, 0, s,
                                           p->tune.ks_eg));
            }
        }
        for (int e = 0; e < Ein; ++e) bin.g[e] = 1;
    }
    // 4. multiply-accumulate over the extended basis
    if (!fused) FL_RET(launch_mac(c, p, ma, bout, s));
    // 5. giant steps summed in the extended basis.  When the chunk's key sets hold the
    // giant keys at the same indices, the key switches of a group of up to MAX_SUM
    // steps (each with its own digit buffer) go to one launch that adds them to the
    // running sum (the identity step's accumulator, then the previous group's sum;
    // two sum buffers alternate) and writes it once.  A single output entry takes a
    // group's ModDown/ModUp in one launch per stage, the group's steps as entries.
    const int64_t a_es = (int64_t)G * ext;
    const int nonid = giant_nonid(c, p);
    bool fuse = nonid >= 1;
    for (int j = 0; fuse && j < G; ++j) {
        const uint32_t g = galois_of_rotation(p->gk[j], c->log_n);
        if (g == 1) continue;
        const int idx = kss[r0]->find(g);
        for (int r = 1; r < Rc; ++r) fuse = fuse && kss[r0 + r]->find(g) == idx;
    }
    uint64_t *Ysum = YE;
    if (fuse) {
        const uint64_t *init = nullptr;
        int64_t init_es = a_es;
        for (int j = 0; j < G; ++j)
            if (galois_of_rotation(p->gk[j], c->log_n) == 1) init = A + j * ext;
        Batch bsum = bout;
        for (int e = 0; e < Eout; ++e) {
            const KeySet *ks = kss[r0 + e / p->n_out];
            bsum.key[e] = ks->evk;
            bsum.key_level[e] = ks->level;
            bsum.g[e] = 1;
        }
        uint64_t *bufs[2] = {YE, YE2};
        int which = 0;
        KsSum sum{};
        int jg[MAX_SUM];  // giant index of each term of the group
        for (int j = 0; j < G; ++j) {
            const uint32_t g = galois_of_rotation(p->gk[j], c->log_n);
            if (g != 1) {
                jg[sum.n] = j;
                sum.g[sum.n] = g;
                sum.key[sum.n] = kss[r0]->find(g);
                sum.dig_off[sum.n] = (int64_t)sum.n * Emax * dg;
                sum.add_off[sum.n] = j * ext;
                ++sum.n;
            }
            bool last = true;
            for (int jj = j + 1; jj < G; ++jj) last = last && galois_of_rotation(p->gk[jj], c->log_n) == 1;
            if (sum.n == 0 || (sum.n < MAX_SUM && !last)) continue;
            // the group's ModDown / ModUp into its digit buffers
            if (Eout == 1 && sum.n > 1) {
                // entries = the group's steps: accumulators ext apart when the steps are
                // consecutive (every non-identity step of the group), digits Emax dg apart;
                // their coefficient-domain temporaries go to the baby-rotation buffer, which
                // the multiply-accumulate has consumed
                bool consecutive = true;
                for (int i = 1; i < sum.n; ++i) consecutive = consecutive && jg[i] == jg[0] + i;
                if (consecutive && (int64_t)sum.n * L * N <= (int64_t)Ein * Bp * ext) {
                    Batch bg{};
                    bg.n = sum.n;
                    for (int i = 0; i < sum.n; ++i) {
                        bg.level[i] = bout.level[0];
                        bg.g[i] = 1;
                    }
                    FL_RET(giant_moddown_modup(c, bg, A + jg[0] * ext + E * N, ext, RB, DG, (int64_t)Emax * dg, ctl, s));
                } else {
                    for (int i = 0; i < sum.n; ++i)
                        FL_RET(giant_moddown_modup(c, bout, A + jg[i] * ext + E * N, a_es, TC, DG + sum.dig_off[i], dg,
                                                   ctl, s));
                }
            } else {
                for (int i = 0; i < sum.n; ++i)
                    FL_RET(giant_moddown_modup(c, bout, A + jg[i] * ext + E * N, a_es, TC, DG + sum.dig_off[i], dg, ctl,
                                               s));
            }
            uint64_t *dst = bufs[which];
            FL_RET(launch_ks_sum(c, bsum, sum, DG, dg, A, a_es, init, init_es, dst, ext, s));
            init = dst;
            init_es = ext;
            Ysum = dst;
            which ^= 1;
            sum = KsSum{};
        }
    }
    bool first = true;
    for (int j = 0; !fuse && j < G; ++j) {
        uint32_t g = galois_of_rotation(p->gk[j], c->log_n);
        uint64_t *Aj = A + j * ext;
        if (g == 1) {
            FL_RET(launch_ext_lift_add(c, bout, Aj, a_es, 0, 0, first ? 0 : 1, YE, ext, s));
            first = false;
            continue;
        }
        set_keys(bout, p->n_out, kss + r0, g);
        // ModUp(ModDown(A~_j.c1)) and the inner product, plus sigma(A~_j.c0), summed into YE
        FL_RET(giant_moddown_modup(c, bout, Aj + E * N, a_es, TC, DG, dg, ctl, s));
        FL_RET(launch_ks_inner_add(c, bout, DG, dg, YE, ext, Aj, a_es, 1, first ? 0 : 1, s, p->tune.ks_eg));
        first = false;
    }
    for (int e = 0; e < Eout; ++e) bout.g[e] = 1;
    // 6. final ModDown of both polynomials
    FL_RET(launch_ntt(c, rows_kind(c, bout, Ysum, ext, ROWS_EXT_P, 2), 1, s));
    FL_RET(launch_moddown_fbc(c, bout, Ysum, ext, MD, ct, s, 2));
    FL_RET(launch_ntt(c, rows_ct(c, bout, MD, ct, (int)L, 0, 2), 0, s));
    FL_RET(launch_moddown_combine(c, bout, Ysum, ext, MD, ct, Y, ct, (int)L, nullptr, 0, 0, 0, s, 2));
    // 7. export
    return export_out(c, bout, Y, out, (int64_t)r0 * p->n_out, rescale, s);
}

// fixed_ws / fixed_bytes: a caller-provided scratch buffer instead of the stream's workspace
// (nothing is allocated then; the chunk shrinks until it fits, results do not depend on it)
int linear_apply(Ctx *c, const Plan *p, const KeySet *const *kss, const PtSet *pts, const fhelin_ct_batch *in,
                 const fhelin_ct_batch *out, int flags, hipStream_t s, int max_chunk, uint64_t *fixed_ws,
                 size_t fixed_bytes) {
    FL_CHECK(c && p && pts && in && out, FHELIN_E_INVALID_ARG, "linear_apply: null argument");
    FL_RET(check_batch(c, in, "linear_apply input"));
    FL_RET(check_batch(c, out, "linear_apply output"));
    FL_CHECK(in->n_ct % p->n_in == 0, FHELIN_E_INVALID_ARG, "input count is not a multiple of the plan's n_in");
    const int R = in->n_ct / p->n_in;
    FL_CHECK(out->n_ct == R * p->n_out, FHELIN_E_INVALID_ARG, "output count must be requests * n_out");
    FL_CHECK(pts->n_pt == p->n_pt(), FHELIN_E_INVALID_ARG, "plaintext set does not match the plan");
    const bool rescale = flags & FHELIN_APPLY_RESCALE;
    for (int r = 0; r < R; ++r) {
        int l = in->levels[r * p->n_in];
        for (int i = 1; i < p->n_in; ++i)
            FL_CHECK(in->levels[r * p->n_in + i] == l, FHELIN_E_LEVEL_MISMATCH, "inputs of a request differ in level");
        FL_CHECK(l <= pts->level, FHELIN_E_LEVEL_MISMATCH, "plaintexts encoded below the request level");
        FL_CHECK(!rescale || l >= 2, FHELIN_E_LEVEL_MISMATCH, "rescale needs level >= 2");
        for (int o = 0; o < p->n_out; ++o)
            FL_CHECK(out->levels[r * p->n_out + o] == (rescale ? l - 1 : l), FHELIN_E_LEVEL_MISMATCH,
                     "output levels must equal the input level (minus one when rescaling)");
        if (!p->galois.empty()) {
            const KeySet *ks = kss ? kss[r] : nullptr;
            FL_CHECK(ks != nullptr, FHELIN_E_MISSING_GALOIS_KEY, "layer needs Galois keys");
            FL_CHECK(ks->ctx == c, FHELIN_E_INVALID_ARG, "keyset belongs to another context");
            FL_CHECK(l <= ks->level, FHELIN_E_LEVEL_MISMATCH, "keys loaded below the request level");
            for (uint32_t g : p->galois)
                FL_CHECK(ks->find(g) >= 0, FHELIN_E_MISSING_GALOIS_KEY,
                         "keyset lacks Galois element " + std::to_string(g));
        }
    }
    if (R == 0) return FHELIN_OK;
    // whatever this call enqueues, the key and plaintext sets' release waits for it
    struct NoteUses {
        const KeySet *const *kss;
        const PtSet *pts;
        int R;
        hipStream_t s;
        ~NoteUses() {
            pts->uses.note(s);
            const KeySet *prev = nullptr;
            for (int r = 0; kss && r < R; ++r)
                if (kss[r] && kss[r] != prev) (prev = kss[r])->uses.note(s);
        }
    } note_uses{p->galois.empty() ? nullptr : kss, pts, R, s};
    // the plan's NTT tile for every transform this call launches (restored on return)
    struct NttTile {
        int prev;
        explicit NttTile(int nt) : prev(ntt_threads_set(nt)) {}
        ~NttTile() { ntt_threads_set(prev); }
    } ntt_tile(p->tune.ntt_threads);
    // key and plaintext sets loaded on another stream
    FL_RET(pts->ready.wait(s));
    if (!p->galois.empty()) {
        const KeySet *prev = nullptr;
        for (int r = 0; r < R; ++r)
            if (kss[r] != prev) FL_RET((prev = kss[r])->ready.wait(s));
    }

    const int64_t N = c->N, L = c->L, K = c->K;
    const int B = (int)p->rb.size(), G = (int)p->gk.size();
    MacArgs ma{};
    int Bp = 0;
    for (int b = 0; b < B; ++b) ma.bmap[b] = galois_of_rotation(p->rb[b], c->log_n) == 1 ? -1 : Bp++;
    int chunk = chunk_of(p, R, max_chunk);
    uint64_t *ws;
    const bool dh = flags & FHELIN_APPLY_HOIST_MODDOWN;
    const size_t per_request =
        (dh ? limbs_per_request_dh(c, p, Bp) : limbs_per_request(c, p, Bp)) * (size_t)N * sizeof(uint64_t);
    const size_t ctl_bytes = p->tune.persistent ? CTL_BYTES : 0;
    if (fixed_ws) {
        const size_t fit = fixed_bytes > ctl_bytes ? (fixed_bytes - ctl_bytes) / per_request : 0;
        FL_CHECK(fit >= 1, FHELIN_E_UNSUPPORTED_PARAM,
                 "one request of this layer needs " + std::to_string(per_request + ctl_bytes) + " bytes of scratch; "
                 "the fixed scratch holds " + std::to_string(fixed_bytes));
        chunk = std::min<int>(chunk, (int)std::min<size_t>(fit, MAX_BATCH));
        ws = fixed_ws;
    } else {
        FL_RET(workspace_get(c, s, per_request * chunk + ctl_bytes, &ws));
    }
    uint32_t *ctl = ctl_bytes ? (uint32_t *)((char *)ws + per_request * chunk) : nullptr;

    const int64_t ct = 2 * L * N, dg = (int64_t)c->dnum * (L + K) * N;
    if (dh) {
        for (int r0 = 0; r0 < R; r0 += chunk)
            FL_RET(apply_chunk_dh(c, p, kss, pts, in, out, rescale, s, ws, r0, std::min(chunk, R - r0), ma, Bp, ctl));
        return FHELIN_OK;
    }
    for (int r0 = 0; r0 < R; r0 += chunk) {
        const int Rc = std::min(chunk, R - r0);
        const int Ein = Rc * p->n_in, Eout = Rc * p->n_out, Emax = std::max(Ein, Eout);
        // carve the workspace
        uint64_t *X = ws, *D = X + Ein * ct, *RB = D + Ein * dg, *A = RB + (int64_t)Ein * Bp * ct;
        uint64_t *Y = A + (int64_t)Eout * G * ct, *TC = Y + Eout * ct, *DG = TC + Emax * L * N;
        uint64_t *U = DG + Emax * dg, *MD = U + Emax * 2 * (L + K) * N;
        Batch bin{}, bout{};
        bin.n = Ein;
        bout.n = Eout;
        for (int e = 0; e < Ein; ++e) {
            bin.level[e] = (uint8_t)in->levels[(r0 * p->n_in) + e];
            bin.g[e] = 1;
        }
        for (int e = 0; e < Eout; ++e) {
            bout.level[e] = (uint8_t)in->levels[(r0 + e / p->n_out) * p->n_in];
            bout.g[e] = 1;
        }
        KsScratch w{TC, L * N, DG, dg, U, 2 * (L + K) * N, MD, 2 * L * N, ctl};
        // 1. import inputs to the NTT domain
        const int64_t in_es = (int64_t)2 * in->stride * N;
        RowMap src = rows_ct(c, bin, in->data + (int64_t)r0 * p->n_in * in_es, in_es, in->stride, 0, 2);
        RowMap dx = rows_ct(c, bin, X, ct, (int)L, 0, 2);
        FL_RET(launch_ntt_from(c, dx, src, 0, s));
        // 2-3. hoisted ModUp and baby rotations
        if (Bp > 0) {
            KsScratch wb = w;
            wb.dg = D;
            FL_RET(modup_ct(c, bin, X, ct, (int)L, wb, s));
            for (int b = 0; b < B; ++b) {
                if (ma.bmap[b] < 0) continue;
                set_keys(bin, p->n_in, kss + r0, galois_of_rotation(p->rb[b], c->log_n));
                FL_RET(ks_finish(c, bin, wb, RB + ma.bmap[b] * ct, (int64_t)Bp * ct, (int)L, X, ct, (int)L, 0, s,
                                 p->tune.ks_eg));
            }
            for (int e = 0; e < Ein; ++e) bin.g[e] = 1;
        }
        // 4. multiply-accumulate
        ma.x = X;
        ma.rb = RB;
        ma.pts = pts->data;
        ma.acc = A;
        ma.n_in = p->n_in;
        ma.n_out = p->n_out;
        ma.B = B;
        ma.Bp = Bp;
        ma.G = G;
        ma.pt_level = pts->level;
        ma.ext = 0;
        FL_RET(launch_mac(c, p, ma, bout, s));
        // 5. giant steps, summed into Y
        bool first = true;
        for (int j = 0; j < G; ++j) {
            if (galois_of_rotation(p->gk[j], c->log_n) != 1) continue;
            RowMap ys = rows_ct(c, bout, A + j * ct, (int64_t)G * ct, (int)L, 0, 2);
            RowMap yd = rows_ct(c, bout, Y, ct, (int)L, 0, 2);
            FL_RET(launch_copy_rows(c, yd, ys, s));
            first = false;
            break;
        }
        for (int j = 0; j < G; ++j) {
            uint32_t g = galois_of_rotation(p->gk[j], c->log_n);
            if (g == 1) continue;
            set_keys(bout, p->n_out, kss + r0, g);
            uint64_t *Aj = A + j * ct;
            FL_RET(modup_ct(c, bout, Aj, (int64_t)G * ct, (int)L, w, s));
            FL_RET(ks_finish(c, bout, w, Y, ct, (int)L, Aj, (int64_t)G * ct, (int)L, first ? 0 : 1, s, p->tune.ks_eg));
            first = false;
        }
        for (int e = 0; e < Eout; ++e) bout.g[e] = 1;
        // 6. export (and rescale) in the coefficient domain
        RowMap yr = rows_ct(c, bout, Y, ct, (int)L, 0, 2);
        FL_RET(launch_ntt(c, yr, 1, s));
        const int64_t out_es = (int64_t)2 * out->stride * N;
        uint64_t *ob = out->data + (int64_t)r0 * p->n_out * out_es;
        if (rescale) {
            FL_RET(launch_rescale(c, bout, Y, ct, (int)L, ob, out_es, out->stride, s));
        } else {
            FL_RET(launch_copy_rows(c, rows_ct(c, bout, ob, out_es, out->stride, 0, 2), yr, s));
        }
    }
    return FHELIN_OK;
}

// ---------------------------------------------------------------------------
// autotuner: coordinate descent over the tune fields, timing whole layers
// ---------------------------------------------------------------------------
static int time_apply(Ctx *c, const Plan *p, const KeySet *const *kss, const PtSet *pts, const fhelin_ct_batch *in,
                      const fhelin_ct_batch *out, int flags, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                      double *ms) {
    FL_RET(linear_apply(c, p, kss, pts, in, out, flags, s, MAX_BATCH, nullptr, 0));  // warm (workspace, caches)
    float best = 0;
    for (int rep = 0; rep < 2; ++rep) {
        FL_TRY_HIP(hipEventRecord(e0, s));
        FL_RET(linear_apply(c, p, kss, pts, in, out, flags, s, MAX_BATCH, nullptr, 0));
        FL_TRY_HIP(hipEventRecord(e1, s));
        FL_TRY_HIP(hipEventSynchronize(e1));
        float t = 0;
        FL_TRY_HIP(hipEventElapsedTime(&t, e0, e1));
        if (rep == 0 || t < best) best = t;
    }
    *ms = best;
    return FHELIN_OK;
}

int plan_autotune(Ctx *c, Plan *p, const KeySet *const *kss, const PtSet *pts, const fhelin_ct_batch *in,
                  const fhelin_ct_batch *out, int flags, hipStream_t s, Tune *best_out, double *best_ms) {
    FL_CHECK(c && p && in, FHELIN_E_INVALID_ARG, "autotune: null argument");
    FL_CHECK(in->n_ct % std::max(1, p->n_in) == 0, FHELIN_E_INVALID_ARG, "input count is not a multiple of n_in");
    const int R = in->n_ct / std::max(1, p->n_in);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    FL_TRY_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(FHELIN_E_HIP, "autotune: event creation failed");
    }
    const Tune start = p->tune;
    Tune best = start;
    double best_t = 0;
    int rc = time_apply(c, p, kss, pts, in, out, flags, s, e0, e1, &best_t);
    // one field at a time, in this order; the NTT tile and the persistent ModUp/NTT
    // launch matter only for the two-pass transforms (N >= 2^13), the fused baby
    // rotations only for the double-hoisted schedule with one key set and at most
    // four digits
    struct Field {
        int Tune::*f;
        std::vector<int> vals;
        bool on;
    };
    bool one_set = kss != nullptr && R > 0;
    for (int r = 1; one_set && r < R; ++r) one_set = kss[r] == kss[0];
    const bool fusable = (flags & FHELIN_APPLY_HOIST_MODDOWN) && one_set && c->small &&
                         (c->L + c->alpha - 1) / c->alpha <= ROTMAC_MAXB;
    const Field fields[] = {{&Tune::chunk, {0, 32, 16, 8, 4}, true},
                            {&Tune::ks_eg, {4, 8, 16}, true},
                            {&Tune::mac_my, {2, 4, 8}, true},
                            {&Tune::ntt_threads, {256, 128, 512}, c->log_n > 12},
                            {&Tune::persistent, {0, 1}, c->log_n > 12},
                            {&Tune::fuse_baby, {0, 1}, fusable}};
    for (const Field &fd : fields) {
        if (!fd.on) continue;
        for (size_t i = 0; i < fd.vals.size() && rc == FHELIN_OK; ++i) {
            Tune t = best;
            if (t.*fd.f == fd.vals[i]) continue;
            if (fd.f == &Tune::chunk && fd.vals[i] >= R) continue;  // same as "all" for this batch
            t.*fd.f = fd.vals[i];
            p->tune = t;
            double ms = 0;
            rc = time_apply(c, p, kss, pts, in, out, flags, s, e0, e1, &ms);
            if (rc == FHELIN_OK && ms < best_t) {
                best_t = ms;
                best = t;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != FHELIN_OK) {
        p->tune = start;
        return rc;
    }
    p->tune = best;
    // leave `out` holding the layer computed with the chosen tune
    FL_RET(linear_apply(c, p, kss, pts, in, out, flags, s, MAX_BATCH, nullptr, 0));
    FL_TRY_HIP(hipStreamSynchronize(s));
    if (best_out) *best_out = best;
    if (best_ms) *best_ms = best_t;
    return FHELIN_OK;
}

// ---------------------------------------------------------------------------
// rotation of every ciphertext of a batch (one key switch each)
// ---------------------------------------------------------------------------
int rotate_batch(Ctx *c, const KeySet *ks, const fhelin_ct_batch *in, const int32_t *steps, const fhelin_ct_batch *out,
                 hipStream_t s) {
    FL_CHECK(c && in && out && steps, FHELIN_E_INVALID_ARG, "rotate: null argument");
    FL_RET(check_batch(c, in, "rotate input"));
    FL_RET(check_batch(c, out, "rotate output"));
    FL_CHECK(in->n_ct == out->n_ct, FHELIN_E_INVALID_ARG, "rotate: batch sizes differ");
    for (int t = 0; t < in->n_ct; ++t) {
        FL_CHECK(in->levels[t] == out->levels[t], FHELIN_E_LEVEL_MISMATCH, "rotate: levels differ");
        uint32_t g = galois_of_rotation(steps[t], c->log_n);
        if (g == 1) continue;
        FL_CHECK(ks != nullptr && ks->find(g) >= 0, FHELIN_E_MISSING_GALOIS_KEY,
                 "keyset lacks Galois element " + std::to_string(g));
        FL_CHECK(in->levels[t] <= ks->level, FHELIN_E_LEVEL_MISMATCH, "keys loaded below the ciphertext level");
    }
    if (ks) FL_RET(ks->ready.wait(s));
    struct NoteUse {
        const KeySet *ks;
        hipStream_t s;
        ~NoteUse() {
            if (ks) ks->uses.note(s);
        }
    } note_use{ks, s};
    const int64_t N = c->N, L = c->L, K = c->K;
    const int64_t ct = 2 * L * N, dg = (int64_t)c->dnum * (L + K) * N;
    const int64_t per = ct * 2 + L * N + dg + 2 * (L + K) * N + 2 * L * N;
    const int chunk = std::min(in->n_ct, MAX_BATCH);
    if (chunk == 0) return FHELIN_OK;
    uint64_t *ws;
    FL_RET(workspace_get(c, s, (size_t)per * chunk * sizeof(uint64_t), &ws));
    const int64_t in_es = (int64_t)2 * in->stride * N, out_es = (int64_t)2 * out->stride * N;
    for (int t0 = 0; t0 < in->n_ct; t0 += chunk) {
        const int n = std::min(chunk, in->n_ct - t0);
        uint64_t *X = ws, *Y = X + n * ct, *TC = Y + n * ct, *DG = TC + n * L * N, *U = DG + n * dg;
        uint64_t *MD = U + n * 2 * (L + K) * N;
        // entries that really rotate
        Batch b{};
        std::vector<int> idx;
        for (int t = 0; t < n; ++t) {
            uint32_t g = galois_of_rotation(steps[t0 + t], c->log_n);
            if (g == 1) {  // identity: plain copy
                Batch one{};
                one.n = 1;
                one.level[0] = (uint8_t)in->levels[t0 + t];
                FL_RET(launch_copy_rows(c, rows_ct(c, one, out->data + (t0 + t) * out_es, out_es, out->stride, 0, 2),
                                        rows_ct(c, one, in->data + (t0 + t) * in_es, in_es, in->stride, 0, 2), s));
                continue;
            }
            b.level[b.n] = (uint8_t)in->levels[t0 + t];
            b.g[b.n] = g;
            b.key[b.n] = ks->key_ptr(ks->find(g));
            b.key_level[b.n] = (uint8_t)ks->level;
            idx.push_back(t0 + t);
            ++b.n;
        }
        if (b.n == 0) continue;
        // gather inputs (entries may be non-contiguous after skipping identities)
        for (int e = 0; e < b.n; ++e) {
            Batch one{};
            one.n = 1;
            one.level[0] = b.level[e];
            FL_RET(launch_copy_rows(c, rows_ct(c, one, X + e * ct, ct, (int)L, 0, 2),
                                    rows_ct(c, one, in->data + idx[e] * in_es, in_es, in->stride, 0, 2), s));
        }
        FL_RET(launch_ntt(c, rows_ct(c, b, X, ct, (int)L, 0, 2), 0, s));
        KsScratch w{TC, L * N, DG, dg, U, 2 * (L + K) * N, MD, 2 * L * N};
        FL_RET(modup_ct(c, b, X, ct, (int)L, w, s));
        FL_RET(ks_finish(c, b, w, Y, ct, (int)L, X, ct, (int)L, 0, s));
        FL_RET(launch_ntt(c, rows_ct(c, b, Y, ct, (int)L, 0, 2), 1, s));
        for (int e = 0; e < b.n; ++e) {
            Batch one{};
            one.n = 1;
            one.level[0] = b.level[e];
            FL_RET(launch_copy_rows(c, rows_ct(c, one, out->data + idx[e] * out_es, out_es, out->stride, 0, 2),
                                    rows_ct(c, one, Y + e * ct, ct, (int)L, 0, 2), s));
        }
    }
    return FHELIN_OK;
}

// ---------------------------------------------------------------------------
// standalone rescale of a coefficient-domain batch
// ---------------------------------------------------------------------------
int rescale_batch(Ctx *c, const fhelin_ct_batch *in, const fhelin_ct_batch *out, hipStream_t s) {
    FL_CHECK(c && in && out, FHELIN_E_INVALID_ARG, "rescale: null argument");
    FL_RET(check_batch(c, in, "rescale input"));
    FL_RET(check_batch(c, out, "rescale output"));
    FL_CHECK(in->n_ct == out->n_ct, FHELIN_E_INVALID_ARG, "rescale: batch sizes differ");
    if (in->data == out->data)
        FL_CHECK(in->stride == out->stride, FHELIN_E_INVALID_ARG, "rescale: in-place needs equal strides");
    for (int t = 0; t < in->n_ct; ++t) {
        FL_CHECK(in->levels[t] >= 2, FHELIN_E_LEVEL_MISMATCH, "rescale needs level >= 2");
        FL_CHECK(out->levels[t] == in->levels[t] - 1, FHELIN_E_LEVEL_MISMATCH, "rescale: output level must be input - 1");
    }
    const int64_t N = c->N;
    const int64_t in_es = (int64_t)2 * in->stride * N, out_es = (int64_t)2 * out->stride * N;
    for (int t0 = 0; t0 < in->n_ct; t0 += MAX_BATCH) {
        Batch b{};
        b.n = std::min(MAX_BATCH, in->n_ct - t0);
        for (int e = 0; e < b.n; ++e) b.level[e] = (uint8_t)in->levels[t0 + e];
        // in place is safe: limb i < l-1 of entry t reads limb i and limb l-1 of the same
        // entry; limb l-1 is never written.
        FL_RET(launch_rescale(c, b, in->data + t0 * in_es, in_es, in->stride, out->data + t0 * out_es, out_es,
                              out->stride, s));
    }
    return FHELIN_OK;
}

}  // namespace fl
