// api.hip -- the extern "C" boundary: argument checks, handle ownership, stream plumbing,
// and evaluation-key loading (hot-path row a2).
#include <algorithm>
#include <set>

#include "internal.h"
#include "native.h"

namespace fl {
int primes_generate(int log_n, int bits, int count, uint64_t *out);
const char *last_error();
int plan_create(Ctx *c, const fhelin_layer_desc *d, Plan **out);
int linear_apply(Ctx *c, const Plan *p, const KeySet *const *kss, const PtSet *pts, const fhelin_ct_batch *in,
                 const fhelin_ct_batch *out, int flags, hipStream_t s, int max_chunk, uint64_t *fixed_ws = nullptr,
                 size_t fixed_bytes = 0);
size_t linear_workspace_bytes(const Ctx *c, const Plan *p, int n_requests, int max_chunk, int flags);
int plan_autotune(Ctx *c, Plan *p, const KeySet *const *kss, const PtSet *pts, const fhelin_ct_batch *in,
                  const fhelin_ct_batch *out, int flags, hipStream_t s, Tune *best_out, double *best_ms);

// A captured linear-layer schedule: the kernels of one fhelin_linear_apply with fixed
// buffers, replayed with hipGraphLaunch.
struct Graph {
    Ctx *ctx = nullptr;
    const KeySet *ks = nullptr;  // the key and plaintext sets the captured kernels read
    const PtSet *pts = nullptr;
    std::shared_ptr<WsBuf> ws;  // the workspace the captured kernels use
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~Graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

static int graph_capture_linear(Ctx *c, const Plan *p, const KeySet *ks, const PtSet *pts, const fhelin_ct_batch *in,
                                const fhelin_ct_batch *out, int flags, hipStream_t s, Graph **g) {
    FL_CHECK(p && in && g, FHELIN_E_INVALID_ARG, "graph_capture: null argument");
    FL_CHECK(s != nullptr, FHELIN_E_INVALID_ARG, "graph capture needs a non-null stream");
    // size the stream's workspace before capture (no allocation may happen inside it)
    uint64_t *ws;
    std::unique_ptr<Graph> gr(new Graph());
    gr->ctx = c;
    gr->ks = ks;
    gr->pts = pts;
    FL_RET(workspace_get(c, s, linear_workspace_bytes(c, p, in->n_ct / std::max(1, p->n_in), MAX_BATCH, flags), &ws,
                         &gr->ws));
    const int R = in->n_ct / std::max(1, p->n_in);
    std::vector<const KeySet *> kss((size_t)std::max(1, R), ks);
    // loads still in flight on other streams finish before the capture (no cross-capture waits)
    if (ks) FL_RET(ks->ready.host_wait());
    if (pts) FL_RET(pts->ready.host_wait());
    FL_TRY_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = linear_apply(c, p, kss.data(), pts, in, out, flags, s, MAX_BATCH);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc != FHELIN_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return set_error(FHELIN_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    gr->graph = graph;
    FL_TRY_HIP(hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0));
    *g = gr.release();
    return FHELIN_OK;
}
int rotate_batch(Ctx *c, const KeySet *ks, const fhelin_ct_batch *in, const int32_t *steps, const fhelin_ct_batch *out,
                 hipStream_t s);
int rescale_batch(Ctx *c, const fhelin_ct_batch *in, const fhelin_ct_batch *out, hipStream_t s);
int ptset_new(Ctx *c, int n_pt, int level, PtSet **out);
void ptset_free(PtSet *p);
int pt_import(Ctx *c, const uint64_t *src, int n_pt, int level, int on_device, hipStream_t s, PtSet **out);
int pt_export(Ctx *c, const PtSet *p, int level, uint64_t *dst, hipStream_t s);
int pt_encode(Ctx *c, const double *slots, int n_pt, int level, double scale, hipStream_t s, PtSet **out);
int plan_encode_weights(Ctx *c, const Plan *pl, const double *W, const int32_t *perm_out, const int32_t *perm_in,
                        int level, double scale, hipStream_t s, PtSet **out);

// device set of the context for the duration of a call
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(const Ctx *c) : DeviceGuard(c->device) {}
    explicit DeviceGuard(int device) {
        if (hipGetDevice(&prev) == hipSuccess && prev != device) (void)hipSetDevice(device);
    }
    ~DeviceGuard() {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

static int keyset_load(Ctx *c, const uint32_t *galois, int n_keys, int level, const uint64_t *evk, int on_device,
                       hipStream_t s, KeySet **out) {
    FL_CHECK(galois && evk && out && n_keys >= 1, FHELIN_E_INVALID_ARG, "keyset_load: null argument or no keys");
    FL_CHECK(level >= 1 && level <= c->L, FHELIN_E_LEVEL_MISMATCH, "keyset_load: level out of range");
    const uint32_t two_n = 2u * (uint32_t)c->N;
    for (int i = 0; i < n_keys; ++i) {
        FL_CHECK(galois[i] % 2 == 1 && galois[i] < two_n, FHELIN_E_INVALID_ARG, "Galois elements must be odd and < 2N");
        for (int j = 0; j < i; ++j) FL_CHECK(galois[j] != galois[i], FHELIN_E_INVALID_ARG, "duplicate Galois element");
    }
    std::unique_ptr<KeySet> k(new KeySet());
    k->ctx = c;
    k->level = level;
    k->beta = (level + c->alpha - 1) / c->alpha;
    k->n_keys = n_keys;
    k->galois.assign(galois, galois + n_keys);
    k->bytes = (size_t)n_keys * k->key_stride() * sizeof(uint64_t);
    FL_RET(dev_alloc(c, (void **)&k->evk, k->bytes));
    // a host source is copied in first; a device source is read by the NTT's first pass
    if (!on_device) {
        hipError_t e = hipMemcpyAsync(k->evk, evk, k->bytes, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            dev_free(c, k->evk, k->bytes);
            return set_error(FHELIN_E_HIP, std::string("keyset_load copy: ") + hipGetErrorString(e));
        }
    }
    // every row: NTT then Montgomery form; rows grouped per (key, digit, part)
    RowMap m{};
    m.kind = ROWS_KEY;
    m.log_n = c->log_n;
    m.L = c->L;
    m.K = c->K;
    m.alpha = c->alpha;
    const int parts = n_keys * k->beta * 2;
    const int per = 64;  // parts per launch (rows = per * (level + K))
    int rc = FHELIN_OK;
    for (int p0 = 0; p0 < parts && rc == FHELIN_OK; p0 += per) {
        RowMap e2 = m;
        e2.base = k->evk + (int64_t)p0 * (level + c->K) * c->N;
        e2.n_ct = 1;
        e2.n_part = std::min(per, parts - p0);
        e2.level[0] = (uint8_t)level;
        RowMap src{};
        if (on_device) {
            src = e2;
            src.base = const_cast<uint64_t *>(evk) + (int64_t)p0 * (level + c->K) * c->N;
        }
        rc = launch_ntt_from(c, e2, src, 0, s, true);
    }
    if (rc == FHELIN_OK) rc = k->ready.record(s);
    if (rc) {
        dev_free(c, k->evk, k->bytes);
        return rc;
    }
    *out = k.release();
    return FHELIN_OK;
}

static void keyset_free(KeySet *k) {
    if (!k) return;
    dev_free(k->ctx, k->evk, k->bytes);
    delete k;
}

static int ntt_rows(Ctx *c, uint64_t *rows, const int32_t *mods, int n_rows, int inverse, hipStream_t s) {
    FL_CHECK(rows && mods && n_rows >= 0, FHELIN_E_INVALID_ARG, "ntt: null argument");
    for (int i = 0; i < n_rows; ++i)
        FL_CHECK(mods[i] >= 0 && mods[i] < c->L + c->K, FHELIN_E_INVALID_ARG, "ntt: modulus index out of range");
    if (n_rows == 0) return FHELIN_OK;
    const int per = 4096;
    int32_t *d_mods = nullptr;
    FL_RET(dev_alloc(c, (void **)&d_mods, (size_t)n_rows * sizeof(int32_t)));
    hipError_t e = hipMemcpyAsync(d_mods, mods, (size_t)n_rows * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    int rc = e == hipSuccess ? FHELIN_OK : set_error(FHELIN_E_HIP, "ntt: module list upload failed");
    for (int r0 = 0; r0 < n_rows && rc == FHELIN_OK; r0 += per) {
        RowMap m{};
        m.base = rows + (int64_t)r0 * c->N;
        m.list = d_mods + r0;
        m.kind = ROWS_LIST;
        m.n_ct = 1;
        m.n_list = std::min(per, n_rows - r0);
        m.log_n = c->log_n;
        m.L = c->L;
        m.K = c->K;
        m.alpha = c->alpha;
        rc = launch_ntt(c, m, inverse, s);
    }
    (void)hipStreamSynchronize(s);
    dev_free(c, d_mods, (size_t)n_rows * sizeof(int32_t));
    return rc;
}

// ---------------------------------------------------------------------------
// live handles: every handle the library hands out is registered until its
// destroy/release call, so a null, foreign or already destroyed handle passed to
// a destroy/release or layer call is rejected (FHELIN_E_INVALID_ARG) instead of
// being dereferenced
// ---------------------------------------------------------------------------
enum HandleKind : int { H_CTX = 0, H_KEYSET, H_PTSET, H_PLAN, H_GRAPH, H_NATIVE, H_KINDS };
static std::mutex live_mu;
static std::set<const void *> live_set[H_KINDS];
static void live_add(int kind, const void *h) {
    std::lock_guard<std::mutex> g(live_mu);
    live_set[kind].insert(h);
}
static bool live_has(int kind, const void *h) {
    std::lock_guard<std::mutex> g(live_mu);
    return h && live_set[kind].count(h) > 0;
}
static bool live_remove(int kind, const void *h) {
    std::lock_guard<std::mutex> g(live_mu);
    return h && live_set[kind].erase(h) > 0;
}
static const char *const HANDLE_NAMES[H_KINDS] = {"context", "key set", "plaintext set", "plan", "graph",
                                                   "native pipeline"};
#define FL_LIVE(kind, h)                                                                                    \
    FL_CHECK(live_has((kind), (h)), FHELIN_E_INVALID_ARG,                                                   \
             std::string("null, unknown or destroyed ") + HANDLE_NAMES[(kind)] + " handle")

// handles of a layer call: context and plan live, key set (if given) and plaintext set live
static int check_layer_handles(const void *ctx, const void *plan, const void *ks, const void *pts) {
    FL_LIVE(H_CTX, ctx);
    FL_LIVE(H_PLAN, plan);
    if (ks) FL_LIVE(H_KEYSET, ks);
    FL_LIVE(H_PTSET, pts);
    return FHELIN_OK;
}

// ---------------------------------------------------------------------------
// fixed device scratch of the allocation-free layer call
// ---------------------------------------------------------------------------
// One array per GPU, held until the process ends.  Host code never uses the array's
// name as an address (on the host it is only a stand-in for the symbol): the device
// address of each GPU's copy comes from hipGetSymbolAddress with that GPU current,
// once per device, and is kept in scratch_ptr.
constexpr size_t SCRATCH_BYTES = (size_t)256 << 20;
constexpr int SCRATCH_MAX_DEVICES = 64;
static __device__ __align__(256) uint64_t scratch[SCRATCH_BYTES / sizeof(uint64_t)];
static std::mutex scratch_mu;
static uint64_t *scratch_ptr[SCRATCH_MAX_DEVICES];

// With `device` current: look up (once) the device address of its scratch array.
static int scratch_init(int device) {
    FL_CHECK(device >= 0 && device < SCRATCH_MAX_DEVICES, FHELIN_E_UNSUPPORTED_PARAM, "device index out of range");
    std::lock_guard<std::mutex> g(scratch_mu);
    if (scratch_ptr[device]) return FHELIN_OK;
    void *ptr = nullptr;
    FL_TRY_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    FL_CHECK(ptr != nullptr, FHELIN_E_HIP, "hipGetSymbolAddress returned a null scratch address");
    scratch_ptr[device] = (uint64_t *)ptr;
    return FHELIN_OK;
}

static int linear_apply_noalloc(Ctx *c, const Plan *p, const KeySet *ks, const PtSet *pts, const fhelin_ct_batch *in,
                                const fhelin_ct_batch *out, int flags, hipStream_t s) {
    FL_CHECK(p && in && out, FHELIN_E_INVALID_ARG, "linear_apply_noalloc: null argument");
    FL_CHECK(p->n_in >= 1 && in->n_ct % p->n_in == 0, FHELIN_E_INVALID_ARG,
             "input count is not a multiple of the plan's n_in");
    const int R = in->n_ct / p->n_in;
    FL_CHECK(out->n_ct == R * p->n_out, FHELIN_E_INVALID_ARG, "output count must be requests * n_out");
    uint64_t *ws;
    {
        std::lock_guard<std::mutex> g(scratch_mu);
        ws = scratch_ptr[c->device];
    }
    FL_CHECK(ws != nullptr, FHELIN_E_HIP, "fixed scratch of the device not initialised");
    // requests in groups of at most MAX_BATCH (one key-set pointer each, on the stack)
    const KeySet *kss[MAX_BATCH];
    for (int r = 0; r < MAX_BATCH; ++r) kss[r] = ks;
    const int64_t in_es = (int64_t)2 * in->stride * c->N, out_es = (int64_t)2 * out->stride * c->N;
    for (int r0 = 0; r0 < R || r0 == 0; r0 += MAX_BATCH) {
        const int n = std::min(MAX_BATCH, R - r0);
        fhelin_ct_batch bi{in->data + (int64_t)r0 * p->n_in * in_es, n * p->n_in, in->stride,
                           in->levels + (int64_t)r0 * p->n_in};
        fhelin_ct_batch bo{out->data + (int64_t)r0 * p->n_out * out_es, n * p->n_out, out->stride,
                           out->levels + (int64_t)r0 * p->n_out};
        FL_RET(linear_apply(c, p, kss, pts, &bi, &bo, flags, s, MAX_BATCH, ws, SCRATCH_BYTES));
        if (R == 0) break;
    }
    return FHELIN_OK;
}

}  // namespace fl

using namespace fl;

#define API_BEGIN try {
#define API_END                                                         \
    }                                                                   \
    catch (const std::bad_alloc &) {                                    \
        return set_error(FHELIN_E_OOM, "host allocation failed");       \
    }                                                                   \
    catch (...) {                                                       \
        return set_error(FHELIN_E_INVALID_ARG, "unexpected exception"); \
    }

#define FHELIN_EXPORT __attribute__((visibility("default")))

extern "C" {

FHELIN_EXPORT int fhelin_primes_generate(int32_t log_n, int32_t bits, int32_t count, uint64_t *out) {
    API_BEGIN return primes_generate(log_n, bits, count, out);
    API_END
}

FHELIN_EXPORT int fhelin_ctx_create(const fhelin_params *prm, fhelin_ctx **out) {
    API_BEGIN Ctx *c = nullptr;
    int rc = ctx_create(prm, &c);
    if (rc != FHELIN_OK) return rc;
    // the context's device is current here: find its fixed scratch (allocation-free calls)
    rc = scratch_init(c->device);
    if (rc != FHELIN_OK) {
        ctx_destroy(c);
        return rc;
    }
    *out = (fhelin_ctx *)c;
    live_add(H_CTX, c);
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_ctx_destroy(fhelin_ctx *ctx) {
    API_BEGIN FL_CHECK(live_remove(H_CTX, ctx), FHELIN_E_INVALID_ARG,
                       "ctx_destroy: null, unknown or destroyed context handle");
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    (void)hipDeviceSynchronize();
    ctx_destroy(c);
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_ctx_set_budget(fhelin_ctx *ctx, uint64_t bytes) {
    API_BEGIN FL_CHECK(ctx, FHELIN_E_INVALID_ARG, "null context");
    Ctx *c = (Ctx *)ctx;
    std::lock_guard<std::mutex> g(c->mu);
    c->budget = bytes;
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_ctx_memory(const fhelin_ctx *ctx, uint64_t *used) {
    API_BEGIN FL_CHECK(ctx && used, FHELIN_E_INVALID_ARG, "null argument");
    Ctx *c = (Ctx *)ctx;
    std::lock_guard<std::mutex> g(c->mu);
    *used = c->used;
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_ctx_trim(fhelin_ctx *ctx) {
    API_BEGIN FL_CHECK(ctx, FHELIN_E_INVALID_ARG, "null context");
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    FL_TRY_HIP(hipDeviceSynchronize());
    std::map<void *, std::unique_ptr<Workspace>> old;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        old.swap(c->ws);
    }
    old.clear();
    cache_flush(c);
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_ctx_root(const fhelin_ctx *ctx, int32_t mod_index, uint64_t *psi) {
    API_BEGIN FL_CHECK(ctx && psi, FHELIN_E_INVALID_ARG, "null argument");
    const Ctx *c = (const Ctx *)ctx;
    FL_CHECK(mod_index >= 0 && mod_index < c->L + c->K, FHELIN_E_INVALID_ARG, "modulus index out of range");
    *psi = c->psi[mod_index];
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_keyset_load(fhelin_ctx *ctx, const uint32_t *galois, int32_t n_keys, int32_t level,
                                     const uint64_t *evk, int32_t src_on_device, void *stream, fhelin_keyset **out) {
    API_BEGIN FL_CHECK(ctx, FHELIN_E_INVALID_ARG, "null context");
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    KeySet *k = nullptr;
    int rc = keyset_load(c, galois, n_keys, level, evk, src_on_device, (hipStream_t)stream, &k);
    if (rc == FHELIN_OK) {
        *out = (fhelin_keyset *)k;
        live_add(H_KEYSET, k);
    }
    return rc;
    API_END
}

FHELIN_EXPORT int fhelin_keyset_release(fhelin_keyset *ks) {
    API_BEGIN FL_CHECK(live_remove(H_KEYSET, ks), FHELIN_E_INVALID_ARG,
                       "keyset_release: null, unknown or released key set handle");
    KeySet *k = (KeySet *)ks;
    DeviceGuard g(k->ctx);
    // wait for the load and for the uses enqueued since, on their own streams only
    (void)k->ready.host_wait();
    k->uses.host_wait();
    keyset_free(k);
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_pt_import(fhelin_ctx *ctx, const uint64_t *pt, int32_t n_pt, int32_t level,
                                   int32_t src_on_device, void *stream, fhelin_ptset **out) {
    API_BEGIN FL_CHECK(ctx && out, FHELIN_E_INVALID_ARG, "null argument");
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    PtSet *p = nullptr;
    int rc = pt_import(c, pt, n_pt, level, src_on_device, (hipStream_t)stream, &p);
    if (rc == FHELIN_OK) {
        *out = (fhelin_ptset *)p;
        live_add(H_PTSET, p);
    }
    return rc;
    API_END
}

FHELIN_EXPORT int fhelin_pt_encode(fhelin_ctx *ctx, const double *slots, int32_t n_pt, int32_t level, double scale,
                                   void *stream, fhelin_ptset **out) {
    API_BEGIN FL_CHECK(ctx && out, FHELIN_E_INVALID_ARG, "null argument");
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    PtSet *p = nullptr;
    int rc = pt_encode(c, slots, n_pt, level, scale, (hipStream_t)stream, &p);
    if (rc == FHELIN_OK) {
        *out = (fhelin_ptset *)p;
        live_add(H_PTSET, p);
    }
    return rc;
    API_END
}

FHELIN_EXPORT int fhelin_pt_export(fhelin_ctx *ctx, const fhelin_ptset *pts, int32_t level, uint64_t *out,
                                   void *stream) {
    API_BEGIN FL_CHECK(ctx && pts, FHELIN_E_INVALID_ARG, "null argument");
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    const int rc = pt_export(c, (const PtSet *)pts, level, out, (hipStream_t)stream);
    ((const PtSet *)pts)->uses.note((hipStream_t)stream);
    return rc;
    API_END
}

FHELIN_EXPORT int fhelin_ptset_info(const fhelin_ptset *pts, int32_t *n_pt, int32_t *level) {
    API_BEGIN FL_CHECK(pts, FHELIN_E_INVALID_ARG, "null plaintext set");
    const PtSet *p = (const PtSet *)pts;
    if (n_pt) *n_pt = p->n_pt;
    if (level) *level = p->level;
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_ptset_release(fhelin_ptset *pts) {
    API_BEGIN FL_CHECK(live_remove(H_PTSET, pts), FHELIN_E_INVALID_ARG,
                       "ptset_release: null, unknown or released plaintext set handle");
    PtSet *p = (PtSet *)pts;
    DeviceGuard g(p->ctx);
    (void)p->ready.host_wait();
    p->uses.host_wait();
    ptset_free(p);
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_plan_create(fhelin_ctx *ctx, const fhelin_layer_desc *desc, fhelin_plan **out) {
    API_BEGIN FL_CHECK(ctx && out, FHELIN_E_INVALID_ARG, "null argument");
    Plan *p = nullptr;
    int rc = plan_create((Ctx *)ctx, desc, &p);
    if (rc == FHELIN_OK) {
        *out = (fhelin_plan *)p;
        live_add(H_PLAN, p);
    }
    return rc;
    API_END
}

FHELIN_EXPORT int fhelin_plan_destroy(fhelin_plan *plan) {
    API_BEGIN FL_CHECK(live_remove(H_PLAN, plan), FHELIN_E_INVALID_ARG,
                       "plan_destroy: null, unknown or destroyed plan handle");
    delete (Plan *)plan;
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_plan_info(const fhelin_plan *plan, int32_t *n_in, int32_t *n_out, int32_t *n_baby,
                                   int32_t *n_giant, int32_t *n_pt) {
    API_BEGIN FL_CHECK(plan, FHELIN_E_INVALID_ARG, "null plan");
    const Plan *p = (const Plan *)plan;
    if (n_in) *n_in = p->n_in;
    if (n_out) *n_out = p->n_out;
    if (n_baby) *n_baby = (int32_t)p->rb.size();
    if (n_giant) *n_giant = (int32_t)p->gk.size();
    if (n_pt) *n_pt = p->n_pt();
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_plan_rotations(const fhelin_plan *plan, int32_t *baby, int32_t *giant) {
    API_BEGIN FL_CHECK(plan, FHELIN_E_INVALID_ARG, "null plan");
    const Plan *p = (const Plan *)plan;
    if (baby) std::copy(p->rb.begin(), p->rb.end(), baby);
    if (giant) std::copy(p->gk.begin(), p->gk.end(), giant);
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_plan_galois(const fhelin_plan *plan, uint32_t *out, int32_t cap, int32_t *n) {
    API_BEGIN FL_CHECK(plan && n, FHELIN_E_INVALID_ARG, "null argument");
    const Plan *p = (const Plan *)plan;
    *n = (int32_t)p->galois.size();
    if (out)
        for (int i = 0; i < cap && i < *n; ++i) out[i] = p->galois[i];
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_plan_encode_weights(fhelin_ctx *ctx, const fhelin_plan *plan, const double *weights,
                                             const int32_t *perm_out, const int32_t *perm_in, int32_t level,
                                             double scale, void *stream, fhelin_ptset **out) {
    API_BEGIN FL_CHECK(ctx && plan && out, FHELIN_E_INVALID_ARG, "null argument");
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    PtSet *p = nullptr;
    int rc = plan_encode_weights(c, (const Plan *)plan, weights, perm_out, perm_in, level, scale, (hipStream_t)stream, &p);
    if (rc == FHELIN_OK) {
        *out = (fhelin_ptset *)p;
        live_add(H_PTSET, p);
    }
    return rc;
    API_END
}

FHELIN_EXPORT int fhelin_linear_apply(fhelin_ctx *ctx, const fhelin_plan *plan, const fhelin_keyset *ks,
                                      const fhelin_ptset *pts, const fhelin_ct_batch *in, const fhelin_ct_batch *out,
                                      int32_t flags, void *stream) {
    API_BEGIN FL_RET(check_layer_handles(ctx, plan, ks, pts));
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    FL_CHECK(plan && in, FHELIN_E_INVALID_ARG, "null argument");
    const Plan *p = (const Plan *)plan;
    const int R = in->n_ct / std::max(1, p->n_in);
    std::vector<const KeySet *> kss((size_t)std::max(1, R), (const KeySet *)ks);
    return linear_apply(c, p, kss.data(), (const PtSet *)pts, in, out, flags, (hipStream_t)stream, MAX_BATCH);
    API_END
}

FHELIN_EXPORT int fhelin_plan_workspace_bytes(fhelin_ctx *ctx, const fhelin_plan *plan, int32_t n_requests,
                                              int32_t flags, uint64_t *bytes) {
    API_BEGIN FL_CHECK(ctx && plan && bytes && n_requests >= 0, FHELIN_E_INVALID_ARG, "null argument");
    *bytes = linear_workspace_bytes((Ctx *)ctx, (const Plan *)plan, n_requests, MAX_BATCH, flags);
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_plan_reserve_workspace(fhelin_ctx *ctx, const fhelin_plan *plan, int32_t n_requests,
                                                int32_t flags, void *stream) {
    API_BEGIN FL_CHECK(ctx && plan && n_requests >= 0, FHELIN_E_INVALID_ARG, "null argument");
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    uint64_t *ws = nullptr;
    return workspace_get(c, (hipStream_t)stream,
                         linear_workspace_bytes(c, (const Plan *)plan, n_requests, MAX_BATCH, flags), &ws);
    API_END
}

FHELIN_EXPORT int fhelin_plan_get_tune(const fhelin_plan *plan, fhelin_tune *out) {
    API_BEGIN FL_CHECK(plan && out, FHELIN_E_INVALID_ARG, "null argument");
    const Tune &t = ((const Plan *)plan)->tune;
    out->chunk = t.chunk;
    out->ks_eg = t.ks_eg;
    out->mac_my = t.mac_my;
    out->ntt_threads = t.ntt_threads;
    out->persistent = t.persistent;
    out->fuse_baby = t.fuse_baby;
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_plan_set_tune(fhelin_plan *plan, const fhelin_tune *tune) {
    API_BEGIN FL_CHECK(plan && tune, FHELIN_E_INVALID_ARG, "null argument");
    Tune t;
    t.chunk = tune->chunk;
    t.ks_eg = tune->ks_eg;
    t.mac_my = tune->mac_my;
    t.ntt_threads = tune->ntt_threads;
    t.persistent = tune->persistent;
    t.fuse_baby = tune->fuse_baby;
    FL_CHECK(tune_valid(t), FHELIN_E_INVALID_ARG,
             "tune out of range (chunk 0..64, ks_eg 1..64, mac_my 2, 4 or 8, ntt_threads 128, 256 or 512, "
             "persistent 0 or 1, fuse_baby 0 or 1)");
    ((Plan *)plan)->tune = t;
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_plan_autotune(fhelin_ctx *ctx, fhelin_plan *plan, const fhelin_keyset *const *ks_per_request,
                                       const fhelin_ptset *pts, const fhelin_ct_batch *in,
                                       const fhelin_ct_batch *out, int32_t flags, void *stream, fhelin_tune *best,
                                       double *best_ms) {
    API_BEGIN FL_CHECK(ctx && plan, FHELIN_E_INVALID_ARG, "null argument");
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    Tune t;
    double ms = 0;
    FL_RET(plan_autotune(c, (Plan *)plan, (const KeySet *const *)ks_per_request, (const PtSet *)pts, in, out, flags,
                         (hipStream_t)stream, &t, &ms));
    if (best) {
        best->chunk = t.chunk;
        best->ks_eg = t.ks_eg;
        best->mac_my = t.mac_my;
        best->ntt_threads = t.ntt_threads;
        best->persistent = t.persistent;
        best->fuse_baby = t.fuse_baby;
    }
    if (best_ms) *best_ms = ms;
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_linear_apply_noalloc(fhelin_ctx *ctx, const fhelin_plan *plan, const fhelin_keyset *ks,
                                              const fhelin_ptset *pts, const fhelin_ct_batch *in,
                                              const fhelin_ct_batch *out, int32_t flags, void *stream) {
    API_BEGIN FL_RET(check_layer_handles(ctx, plan, ks, pts));
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    return linear_apply_noalloc(c, (const Plan *)plan, (const KeySet *)ks, (const PtSet *)pts, in, out, flags,
                                (hipStream_t)stream);
    API_END
}

FHELIN_EXPORT int fhelin_linear_apply_multi(fhelin_ctx *ctx, const fhelin_plan *plan,
                                            const fhelin_keyset *const *ks_per_request, const fhelin_ptset *pts,
                                            const fhelin_ct_batch *in, const fhelin_ct_batch *out, int32_t flags,
                                            void *stream) {
    API_BEGIN FL_CHECK(ks_per_request, FHELIN_E_INVALID_ARG, "null argument");
    FL_RET(check_layer_handles(ctx, plan, nullptr, pts));
    if (in)
        for (int r = 0; r < in->n_ct / std::max(1, ((const Plan *)plan)->n_in); ++r)
            if (ks_per_request[r]) FL_LIVE(H_KEYSET, ks_per_request[r]);
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    return linear_apply(c, (const Plan *)plan, (const KeySet *const *)ks_per_request, (const PtSet *)pts, in, out,
                        flags, (hipStream_t)stream, MAX_BATCH);
    API_END
}

FHELIN_EXPORT int fhelin_rescale(fhelin_ctx *ctx, const fhelin_ct_batch *in, const fhelin_ct_batch *out,
                                 void *stream) {
    API_BEGIN FL_CHECK(ctx, FHELIN_E_INVALID_ARG, "null context");
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    return rescale_batch(c, in, out, (hipStream_t)stream);
    API_END
}

FHELIN_EXPORT int fhelin_rotate(fhelin_ctx *ctx, const fhelin_keyset *ks, const fhelin_ct_batch *in,
                                const int32_t *steps, const fhelin_ct_batch *out, void *stream) {
    API_BEGIN FL_LIVE(H_CTX, ctx);
    FL_LIVE(H_KEYSET, ks);
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    return rotate_batch(c, (const KeySet *)ks, in, steps, out, (hipStream_t)stream);
    API_END
}

FHELIN_EXPORT int fhelin_ntt(fhelin_ctx *ctx, uint64_t *rows, const int32_t *mod_index, int32_t n_rows,
                             int32_t inverse, void *stream) {
    API_BEGIN FL_CHECK(ctx, FHELIN_E_INVALID_ARG, "null context");
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    return ntt_rows(c, rows, mod_index, n_rows, inverse ? 1 : 0, (hipStream_t)stream);
    API_END
}

FHELIN_EXPORT int fhelin_graph_capture_linear(fhelin_ctx *ctx, const fhelin_plan *plan, const fhelin_keyset *ks,
                                              const fhelin_ptset *pts, const fhelin_ct_batch *in,
                                              const fhelin_ct_batch *out, int32_t flags, void *stream,
                                              fhelin_graph **graph) {
    API_BEGIN FL_CHECK(graph, FHELIN_E_INVALID_ARG, "null argument");
    FL_RET(check_layer_handles(ctx, plan, ks, pts));
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    Graph *gr = nullptr;
    int rc = graph_capture_linear(c, (const Plan *)plan, (const KeySet *)ks, (const PtSet *)pts, in, out, flags,
                                  (hipStream_t)stream, &gr);
    if (rc == FHELIN_OK) {
        *graph = (fhelin_graph *)gr;
        live_add(H_GRAPH, gr);
    }
    return rc;
    API_END
}

FHELIN_EXPORT int fhelin_graph_launch(fhelin_graph *graph, void *stream) {
    API_BEGIN FL_LIVE(H_GRAPH, graph);
    Graph *gr = (Graph *)graph;
    DeviceGuard g(gr->ctx);
    FL_TRY_HIP(hipGraphLaunch(gr->exec, (hipStream_t)stream));
    // a release of the sets waits for this replay (the graph must not outlive them)
    if (gr->ks && live_has(H_KEYSET, gr->ks)) gr->ks->uses.note((hipStream_t)stream);
    if (gr->pts && live_has(H_PTSET, gr->pts)) gr->pts->uses.note((hipStream_t)stream);
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_graph_destroy(fhelin_graph *graph) {
    API_BEGIN FL_CHECK(live_remove(H_GRAPH, graph), FHELIN_E_INVALID_ARG,
                       "graph_destroy: null, unknown or destroyed graph handle");
    Graph *gr = (Graph *)graph;
    DeviceGuard g(gr->ctx);
    (void)hipDeviceSynchronize();
    delete gr;
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_profile_enable(fhelin_ctx *ctx, int32_t enable) {
    API_BEGIN FL_CHECK(ctx, FHELIN_E_INVALID_ARG, "null context");
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    Profiler *p = c->prof.get();
    FL_TRY_HIP(hipDeviceSynchronize());
    std::lock_guard<std::mutex> lk(p->mu);
    for (auto &r : p->recs) {
        p->pool.push_back(r.a);
        p->pool.push_back(r.b);
    }
    p->recs.clear();
    p->on = enable != 0;
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_diag_alu_rate(int32_t op, int32_t waves_per_simd, int32_t iters, double *ghz,
                                       double *clk_per_op, double *ops_per_s) {
    API_BEGIN return diag_alu_rate(op, waves_per_simd, iters, ghz, clk_per_op, ops_per_s);
    API_END
}

// ---- the paper's own pipeline (native.hip) -------------------------------------
FHELIN_EXPORT int fhelin_native_create(const fhelin_native_params *prm, fhelin_native **out) {
    API_BEGIN FL_CHECK(out, FHELIN_E_INVALID_ARG, "null argument");
    Native *n = nullptr;
    FL_RET(native_create(prm, &n));
    *out = (fhelin_native *)n;
    live_add(H_NATIVE, n);
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_native_destroy(fhelin_native *nt) {
    API_BEGIN FL_CHECK(live_remove(H_NATIVE, nt), FHELIN_E_INVALID_ARG, "null, unknown or destroyed native handle");
    native_destroy((Native *)nt);
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_native_keys_load(fhelin_native *nt, const uint64_t *ksk, void *stream) {
    API_BEGIN FL_LIVE(H_NATIVE, nt);
    Native *n = (Native *)nt;
    DeviceGuard g(n->device);
    return native_keys_load(n, ksk, (hipStream_t)stream);
    API_END
}

FHELIN_EXPORT int fhelin_native_extract(fhelin_native *nt, const uint64_t *chunks, int32_t n_chunks, uint64_t *rows,
                                        void *stream) {
    API_BEGIN FL_LIVE(H_NATIVE, nt);
    Native *n = (Native *)nt;
    DeviceGuard g(n->device);
    return native_extract(n, chunks, n_chunks, rows, (hipStream_t)stream);
    API_END
}

FHELIN_EXPORT int fhelin_native_linear(fhelin_native *nt, const int32_t *row_ptr, const int32_t *col, const int32_t *val,
                                       int32_t n_out, const uint64_t *rows, uint64_t *out, void *stream) {
    API_BEGIN FL_LIVE(H_NATIVE, nt);
    Native *n = (Native *)nt;
    DeviceGuard g(n->device);
    return native_linear(n, row_ptr, col, val, n_out, rows, out, (hipStream_t)stream);
    API_END
}

FHELIN_EXPORT int fhelin_native_conv(fhelin_native *nt, int32_t c_in, int32_t c_out, int32_t h, int32_t w, int32_t k,
                                     int32_t stride, const int32_t *weights, const int32_t *out_row,
                                     const uint64_t *rows, uint64_t *out, void *stream) {
    API_BEGIN FL_LIVE(H_NATIVE, nt);
    Native *n = (Native *)nt;
    DeviceGuard g(n->device);
    return native_conv(n, c_in, c_out, h, w, k, stride, weights, out_row, rows, out, (hipStream_t)stream);
    API_END
}

FHELIN_EXPORT int fhelin_native_pack(fhelin_native *nt, const uint64_t *rows, int32_t n_rows, uint64_t *packed,
                                     void *stream) {
    API_BEGIN FL_LIVE(H_NATIVE, nt);
    Native *n = (Native *)nt;
    DeviceGuard g(n->device);
    return native_pack(n, rows, n_rows, packed, (hipStream_t)stream);
    API_END
}

FHELIN_EXPORT int fhelin_native_profile_enable(fhelin_native *nt, int32_t enable) {
    API_BEGIN FL_LIVE(H_NATIVE, nt);
    Native *n = (Native *)nt;
    DeviceGuard g(n->device);
    return native_profile_enable(n, enable != 0);
    API_END
}

FHELIN_EXPORT int fhelin_native_profile_read(fhelin_native *nt, const char *kernel, int64_t *launches, double *ms,
                                             double *units, double *bytes) {
    API_BEGIN FL_LIVE(H_NATIVE, nt);
    Native *n = (Native *)nt;
    DeviceGuard g(n->device);
    return native_profile_read(n, kernel, launches, ms, units, bytes);
    API_END
}

FHELIN_EXPORT int fhelin_native_pack_workspace(const fhelin_native *nt, int32_t n_rows, uint64_t *bytes) {
    API_BEGIN FL_LIVE(H_NATIVE, nt);
    FL_CHECK(bytes && n_rows >= 0, FHELIN_E_INVALID_ARG, "null argument or negative row count");
    *bytes = native_pack_workspace((const Native *)nt, n_rows);
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_ctx_faults(fhelin_ctx *ctx, uint32_t *faults) {
    API_BEGIN FL_LIVE(H_CTX, ctx);
    FL_CHECK(faults, FHELIN_E_INVALID_ARG, "null argument");
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    FL_TRY_HIP(hipDeviceSynchronize());
    uint32_t v = 0;
    FL_TRY_HIP(hipMemcpy(&v, c->d_fault, sizeof(v), hipMemcpyDeviceToHost));
    if (v) {
        const uint32_t zero = 0;
        FL_TRY_HIP(hipMemcpy(c->d_fault, &zero, sizeof(zero), hipMemcpyHostToDevice));
    }
    *faults = v;
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT int fhelin_profile_read(fhelin_ctx *ctx, const char *kernel, int64_t *launches, double *total_ms,
                                      double *units, double *bytes) {
    API_BEGIN FL_CHECK(ctx && kernel, FHELIN_E_INVALID_ARG, "null argument");
    Ctx *c = (Ctx *)ctx;
    DeviceGuard g(c);
    int kind = -1;
    for (int k = 0; k < PK_COUNT; ++k)
        if (std::string(PROF_NAMES[k]) == kernel) kind = k;
    FL_CHECK(kind >= 0, FHELIN_E_INVALID_ARG, std::string("unknown kernel class ") + kernel);
    Profiler *p = c->prof.get();
    std::lock_guard<std::mutex> lk(p->mu);
    int64_t n = 0;
    double ms = 0, u = 0, by = 0;
    for (auto &r : p->recs) {
        if (r.kind != kind) continue;
        FL_TRY_HIP(hipEventSynchronize(r.b));
        float t = 0;
        FL_TRY_HIP(hipEventElapsedTime(&t, r.a, r.b));
        ++n;
        ms += t;
        u += r.units;
        by += r.bytes;
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms;
    if (units) *units = u;
    if (bytes) *bytes = by;
    return FHELIN_OK;
    API_END
}

FHELIN_EXPORT const char *fhelin_last_error(void) { return last_error(); }

FHELIN_EXPORT const char *fhelin_status_string(int status) { return status_string(status); }

}  // extern "C"
