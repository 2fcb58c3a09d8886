/*
 * fhelin.h -- C ABI of the MI355X encrypted linear-layer library.
 *
 * The library evaluates the server side of hybrid FHE inference (arxiv
 * 2509.01253, Sec. 3-4): the linear layers of a network run on encrypted
 * inputs, the client decrypts and applies the activations between layers.
 * Ciphertexts are RNS-CKKS: a ciphertext at level l is a pair (c0, c1) of
 * polynomials in Z_Q[X]/(X^N+1), Q = q_0 ... q_{l-1}, decrypting as c0 + c1*s.
 * The library never sees a secret key: it loads evaluation keys, encodes the
 * server's plaintext weights, applies linear layers and rescales.
 *
 * Conventions shared by every entry point
 *   - Status: 0 on success, a negative FHELIN_E_* code otherwise; nothing is
 *     thrown across the ABI.  fhelin_last_error() gives a message for the
 *     calling thread's last failure.
 *   - Device pointers are plain HIP device addresses (e.g. a torch tensor's
 *     data_ptr()); they stay owned by the caller and are never freed by the
 *     library.  Handles (ctx, keyset, ptset, plan) are owned by the library and
 *     released with their destroy/release call.
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *     stream).  Work is enqueued on it and ordered by it; a call returns once
 *     the work is enqueued.  Inputs must stay valid until the stream reaches
 *     the work.  Calls on different streams that share a handle may run
 *     concurrently: each stream gets its own workspace.  A key set or
 *     plaintext set may be used on a stream other than the one that loaded
 *     it: the using call waits for the load to finish.
 *   - Ciphertext and plaintext data cross the ABI in the COEFFICIENT domain:
 *     uint64 residues in [0, q_i), limb-major, N values per limb.
 *   - The modulus list of a context is q_0..q_{L-1} followed by p_0..p_{K-1}
 *     (K special primes of the hybrid key switch).
 */
#ifndef FHELIN_H
#define FHELIN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define FHELIN_OK 0
#define FHELIN_E_INVALID_ARG (-1)       /* null handle/pointer, bad size or layout */
#define FHELIN_E_UNSUPPORTED_PARAM (-2) /* parameters outside what the kernels support */
#define FHELIN_E_LEVEL_MISMATCH (-3)    /* levels inconsistent between operands */
#define FHELIN_E_MISSING_GALOIS_KEY (-4)/* a rotation needs a key the keyset lacks */
#define FHELIN_E_OOM (-5)               /* device allocation failed */
#define FHELIN_E_BUDGET (-6)            /* the context's HBM budget would be exceeded */
#define FHELIN_E_HIP (-7)               /* a HIP runtime call failed */
#define FHELIN_E_UNIMPLEMENTED (-8)

typedef struct fhelin_ctx fhelin_ctx;
typedef struct fhelin_keyset fhelin_keyset;
typedef struct fhelin_ptset fhelin_ptset;
typedef struct fhelin_plan fhelin_plan;
typedef struct fhelin_graph fhelin_graph;

/* ---- parameters and context ------------------------------------------ */

/* RNS-CKKS parameter set.  N = 2^log_n with 10 <= log_n <= 16; every modulus
 * is a distinct prime below 2^60 with q = 1 (mod 2N); 1 <= n_q <= 32,
 * 1 <= n_p <= 8, 1 <= dnum <= n_q.  Digits of the hybrid key switch hold
 * alpha = ceil(n_q/dnum) consecutive q's; the product of the p's must exceed
 * every digit's product (checked).  Arrays are host memory, copied. */
typedef struct {
    int32_t log_n;
    int32_t n_q;        /* L */
    int32_t n_p;        /* K */
    int32_t dnum;
    const uint64_t *q;  /* [n_q] */
    const uint64_t *p;  /* [n_p] */
} fhelin_params;

/* Helper for choosing moduli: the first `count` primes q = 1 (mod 2N) below
 * 2^bits, scanning downwards, written to host array out[count] in descending
 * order.  A common choice takes the first n_p as special primes and the next
 * n_q as q_0 > q_1 > ... .  Returns FHELIN_E_UNSUPPORTED_PARAM if the range
 * runs out. */
int fhelin_primes_generate(int32_t log_n, int32_t bits, int32_t count, uint64_t *out);

/* Context setup on the current HIP device: the ring Z[X]/(X^N + 1) and the RNS
 * modulus chain of the server's evaluation parameters (the RLWE parameters of
 * paper Sec. 2.1 -- ring degree and ciphertext modulus -- fixed once at setup,
 * paper Sec. 4.2; here in the full-RNS CKKS form of Cheon-Han-Kim-Kim-Song 2018
 * with the hybrid key-switching digits of Han-Ki 2020).  Builds the minimal
 * primitive 2N-th roots, NTT twiddles with their Shoup companions and every
 * base-conversion constant.  The parameters are checked on the host before any
 * device work: bad values return FHELIN_E_INVALID_ARG (null pointers) or
 * FHELIN_E_UNSUPPORTED_PARAM (log_n, counts, dnum, moduli not prime, not 1 mod
 * 2N, not below 2^60, not distinct, P not above every digit modulus) with a
 * message and create nothing.  The encoding scale is not a context parameter:
 * every encode call takes its own (scales change with rescales).  The context
 * owns its device tables; destroy it after every handle created from it. */
int fhelin_ctx_create(const fhelin_params *prm, fhelin_ctx **out);
/* Handles are registered while alive: destroy/release calls (and the layer
 * calls) reject a null, unknown or already destroyed handle with
 * FHELIN_E_INVALID_ARG instead of freeing it twice. */
int fhelin_ctx_destroy(fhelin_ctx *ctx);

/* HBM budget (bytes) for everything the context allocates: keys, plaintexts
 * and per-stream workspaces.  0 = unlimited (the default).  Allocations that
 * would exceed it fail with FHELIN_E_BUDGET. */
int fhelin_ctx_set_budget(fhelin_ctx *ctx, uint64_t bytes);
/* Bytes currently allocated by the context (keys + plaintexts + workspaces).
 * Released blocks (at most 32 GiB) are kept for reuse by a later allocation of
 * the same size instead of being returned to HIP; they are not counted here.
 * A release waits for the device to be idle, as hipFree does. */
int fhelin_ctx_memory(const fhelin_ctx *ctx, uint64_t *used_bytes);
/* Release the per-stream workspaces (they are re-created on demand) and return
 * the kept released blocks to HIP. */
int fhelin_ctx_trim(fhelin_ctx *ctx);

/* The minimal primitive 2N-th root of unity the context uses for modulus
 * index mod_index (0..n_q+n_p-1); the forward NTT of fhelin_ntt evaluates at
 * its odd powers. */
int fhelin_ctx_root(const fhelin_ctx *ctx, int32_t mod_index, uint64_t *psi);

/* ---- evaluation keys (paper Sec. 4.2: uploaded once at setup) --------- */

/* Load Galois evaluation keys.  galois[n_keys] are odd elements g of
 * (Z/2N)^*, rotation of slots left by r <=> g = 5^r mod 2N.  Keys are stored
 * up to Q-level `level` (1..n_q) and serve every level <= level.
 * evk layout, coefficient domain:
 *   [n_keys][beta][2][level + n_p][N],  beta = ceil(level / alpha),
 * digit j < beta, part 0 = b_j, part 1 = a_j, limbs q_0..q_{level-1} then
 * p_0..p_{n_p-1}; the key for digit j satisfies
 *   b_j + a_j s = e_j + P * [j-th digit CRT indicator] * s(X^g)  (mod QP).
 * src_on_device selects whether evk is a device or host pointer; it is copied,
 * transformed to the NTT domain and kept resident.  Charged to the budget. */
int fhelin_keyset_load(fhelin_ctx *ctx, const uint32_t *galois, int32_t n_keys, int32_t level,
                       const uint64_t *evk, int32_t src_on_device, void *stream, fhelin_keyset **out);
/* Release waits on the host for the load and for every use of the key set enqueued
 * so far (layer calls, rotations, graph replays), each on its own stream, then
 * frees it; other streams keep running. */
int fhelin_keyset_release(fhelin_keyset *ks);

/* ---- plaintexts -------------------------------------------------------- */

/* Import integer plaintexts [n_pt][level + n_p][N] (coefficient domain,
 * residues mod q_0..q_{level-1} then p_0..p_{n_p-1}; the special-prime rows
 * serve the double-hoisted schedule); host or device source. */
int fhelin_pt_import(fhelin_ctx *ctx, const uint64_t *pt, int32_t n_pt, int32_t level, int32_t src_on_device,
                     void *stream, fhelin_ptset **out);

/* CKKS encode (canonical embedding, slot j at zeta^(5^j), zeta = exp(i pi/N);
 * Cheon-Kim-Kim-Song 2017): real slot vectors slots[n_pt][N/2] (device, FP64)
 * -> m_k = round(scale * (2/N) * sum_j z_j Re(zeta^(-5^j k))), ties to even,
 * reduced mod q_0..q_{level-1} and p_0..p_{n_p-1}.  |m_k| must stay below 2^62. */
int fhelin_pt_encode(fhelin_ctx *ctx, const double *slots, int32_t n_pt, int32_t level, double scale, void *stream,
                     fhelin_ptset **out);

/* Write a plaintext set back in the coefficient domain: out[n_pt][level + n_p][N]
 * (device; q rows 0..level-1 then the special rows), level <= the set's level. */
int fhelin_pt_export(fhelin_ctx *ctx, const fhelin_ptset *pts, int32_t level, uint64_t *out, void *stream);
int fhelin_ptset_info(const fhelin_ptset *pts, int32_t *n_pt, int32_t *level);
/* Like fhelin_keyset_release: waits for the set's own uses, not the device. */
int fhelin_ptset_release(fhelin_ptset *pts);

/* ---- linear-layer plans ------------------------------------------------ */

#define FHELIN_LAYER_FC 1
#define FHELIN_LAYER_CONV 2

/* Layer description.
 *  FC (Halevi-Shoup diagonal method, baby-step giant-step):
 *    fc_n: padded square size, a power of two dividing N/2; the weight is
 *    fc_out x fc_in (<= fc_n each) and is zero-padded.  The input ciphertext
 *    holds x (length fc_n, zero-padded) replicated N/(2 fc_n) times.  n1 is
 *    the number of baby steps (a power of two dividing fc_n); n1 = fc_n is the
 *    plain method with a single giant step.
 *  CONV (multiplexed, channel-major packing): c_in, c_out channels, h x w
 *    spatial, kernel k in {1, 3}, stride 1, zero padding k/2 ("same").  Slot
 *    s = c*h*w + y*w + x with c_ct = N/(2hw) channels per ciphertext, so a
 *    layer maps ceil(c_in/c_ct) input ciphertexts to ceil(c_out/c_ct) outputs.
 *    The channel offsets k < c_ct split as k = k1 + n1*k2 (n1 a power of two
 *    dividing c_ct with n1*k*k <= 64; n1 = 0 or 1: no split).  Baby steps are
 *    (k1, (dy, dx)), k1-major then the k*k spatial offsets row-major, rotation
 *    k1*h*w + dy*w + dx; giant steps are k2 < c_ct/n1, rotation n1*k2*h*w.
 * Every layer is evaluated as
 *    y_o = sum_j rot_{G_j}( sum_i sum_b pt[o][i][j][b] * rot_{r_b}(x_i) )
 * (rot_0 = identity, no key switch), with plaintext index
 *    ((o*n_in + i)*n_giant + j)*n_baby + b. */
typedef struct {
    int32_t kind;
    int32_t fc_n, fc_out, fc_in, n1;
    int32_t c_in, c_out, h, w, k;
} fhelin_layer_desc;

int fhelin_plan_create(fhelin_ctx *ctx, const fhelin_layer_desc *desc, fhelin_plan **out);
int fhelin_plan_destroy(fhelin_plan *plan);
/* Shape of a plan: ciphertexts in/out per request, baby and giant step counts,
 * number of plaintexts (n_out*n_in*n_giant*n_baby). */
int fhelin_plan_info(const fhelin_plan *plan, int32_t *n_in, int32_t *n_out, int32_t *n_baby, int32_t *n_giant,
                     int32_t *n_pt);
/* Rotation amounts (slots, left): baby[n_baby], giant[n_giant]; either may be NULL. */
int fhelin_plan_rotations(const fhelin_plan *plan, int32_t *baby, int32_t *giant);
/* Distinct Galois elements the plan needs (ascending), up to cap; *n gets the count. */
int fhelin_plan_galois(const fhelin_plan *plan, uint32_t *out, int32_t cap, int32_t *n);

/* Encode a layer's weights for a plan (paper Sec. 4.4: the previous round's
 * unshuffle and this round's shuffle are folded into the weights):
 *   W'[t][u] = W[perm_out[t]][perm_in[u]]       (FC, W is fc_out x fc_in)
 *   W'[t][u][.][.] = W[perm_out[t]][perm_in[u]][.][.]   (conv channels,
 *                                                   W is c_out x c_in x k x k)
 * weights, perm_out, perm_in are device pointers (perms may be NULL =
 * identity).  The diagonals / multiplexed slot vectors of the plan are formed
 * on the device and encoded like fhelin_pt_encode. */
int fhelin_plan_encode_weights(fhelin_ctx *ctx, const fhelin_plan *plan, const double *weights,
                               const int32_t *perm_out, const int32_t *perm_in, int32_t level, double scale,
                               void *stream, fhelin_ptset **out);

/* ---- ciphertext batches and evaluation -------------------------------- */

/* A batch of ciphertexts in device memory, coefficient domain:
 *   data[n_ct][2][stride][N]; ciphertext t uses limbs 0..levels[t]-1 of each
 *   polynomial (levels is a host array).  stride >= max level. */
typedef struct {
    uint64_t *data;
    int32_t n_ct;
    int32_t stride;
    const int32_t *levels;
} fhelin_ct_batch;

#define FHELIN_APPLY_RESCALE 1
/* Double-hoisted schedule (Bossuat-Mouchet-Troncoso-Pastoriza-Hubaux, Eurocrypt
 * 2021): baby rotations, the plaintext multiply-accumulate and the giant-step
 * sum are kept in the extended basis Q*P; each giant step ModDowns only c1
 * before its ModUp and one ModDown per output ends the layer:
 *   R~_b = (P sigma_b(x0) + u0_b, u1_b) (r_b = 0: P x),  A~_j = sum pt (.) R~_b,
 *   Y~ = sum_j [A~_j if G_j = 0 else (sigma_j(A~_j.c0) + v0, v1)],
 *   v = KS_j(ModDown(A~_j.c1)),  y = ModDown(Y~).
 * The result decrypts to the same layer with different rounding than the
 * default per-rotation schedule; both are exact functions of their inputs. */
#define FHELIN_APPLY_HOIST_MODDOWN 2

/* Apply a linear layer to a batch of requests.  in->n_ct = R * n_in (request
 * r owns input ciphertexts r*n_in .. r*n_in+n_in-1, all at the same level);
 * out->n_ct = R * n_out.  Without flags the outputs are at the input level;
 * with FHELIN_APPLY_RESCALE they are rescaled by the top prime (level - 1).
 * out->levels is read and must hold the resulting levels.  The plaintext set
 * must be encoded for this plan at a level >= every request level; the keyset
 * must cover the plan's Galois elements at a level >= every request level.
 * Results are bit-identical whatever the batch composition. */
int fhelin_linear_apply(fhelin_ctx *ctx, const fhelin_plan *plan, const fhelin_keyset *ks, const fhelin_ptset *pts,
                        const fhelin_ct_batch *in, const fhelin_ct_batch *out, int32_t flags, void *stream);

/* Workspace (bytes of device memory) that fhelin_linear_apply needs on a
 * stream for n_requests requests of this plan with these flags; the stream's
 * workspace grows to it on first use and is charged to the budget.  Lets a
 * scheduler admit work by memory before launching it. */
int fhelin_plan_workspace_bytes(fhelin_ctx *ctx, const fhelin_plan *plan, int32_t n_requests, int32_t flags,
                                uint64_t *bytes);

/* Grow the stream's workspace now to what fhelin_linear_apply needs for
 * n_requests requests of this plan with these flags (never shrinks it), so that
 * later calls on the stream allocate nothing.  A grow synchronises the stream
 * first; the memory is charged to the budget (FHELIN_E_BUDGET / FHELIN_E_OOM if it
 * does not fit) and released by fhelin_ctx_trim or fhelin_ctx_destroy.  For
 * schedulers that size memory up front instead of on the first large batch. */
int fhelin_plan_reserve_workspace(fhelin_ctx *ctx, const fhelin_plan *plan, int32_t n_requests, int32_t flags,
                                  void *stream);

/* fhelin_linear_apply with one key set per request (ks_per_request[R], host
 * array; requests from different clients batched in one call).  Every key set
 * must belong to ctx and cover the plan's Galois elements at the request's
 * level.  Results equal per-request fhelin_linear_apply calls bit for bit. */
int fhelin_linear_apply_multi(fhelin_ctx *ctx, const fhelin_plan *plan, const fhelin_keyset *const *ks_per_request,
                              const fhelin_ptset *pts, const fhelin_ct_batch *in, const fhelin_ct_batch *out,
                              int32_t flags, void *stream);

/* Allocation-free fhelin_linear_apply, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, checks and results as fhelin_linear_apply
 * (bit for bit), but the layer's intermediate buffers live in a fixed scratch
 * array of 256 MiB per GPU inside the library (reserved when the library's code
 * is loaded on the device, held until the process ends) instead of the stream's
 * workspace: the call performs no hipMalloc, hipFree or other device allocation.
 * Requests are processed in chunks that fit the scratch; a layer of which one
 * request needs more than 256 MiB (fhelin_plan_workspace_bytes with n_requests
 * 1) is rejected with FHELIN_E_UNSUPPORTED_PARAM before any kernel is launched --
 * at N = 2^16 that is every layer, at N = 2^15 a multiplexed conv at level 8
 * fits.  Every call on a GPU shares that GPU's scratch and leaves its contents
 * behind: calls that may overlap in time on one GPU (other streams, other
 * threads, other contexts) race and must be serialised by the caller.  With
 * profiling enabled (fhelin_profile_enable) the call records HIP events. */
int fhelin_linear_apply_noalloc(fhelin_ctx *ctx, const fhelin_plan *plan, const fhelin_keyset *ks,
                                const fhelin_ptset *pts, const fhelin_ct_batch *in, const fhelin_ct_batch *out,
                                int32_t flags, void *stream);

/* Tile and chunk choices of a plan's schedule.  They change speed only: every
 * choice gives bit-identical results.
 *   chunk   requests per chunk, 0 = as many as 64 ciphertexts allow (a smaller
 *           chunk keeps the working set of a chunk in the GPU's caches)
 *   ks_eg   batch entries per workgroup of the key-switch inner product (each
 *           workgroup reuses an evaluation-key tile across its entries), 1..64
 *   mac_my  requests per thread in the plaintext multiply-accumulate: 2, 4, 8
 *   ntt_threads  workgroup size of the two-pass NTT kernels (N >= 2^13): 128,
 *           256 or 512 threads of 16 elements, i.e. column tiles of 8, 16 or 32
 *           columns (2^16) in the first pass and 8, 16 or 32 blocks of 256 in the
 *           second (LDS 17, 35 or 68 KiB per workgroup)
 *   persistent  1: each key switch's ModUp and forward NTT run as one persistent
 *           launch (N >= 2^13): workgroups claim ModUp chunks, then column tiles,
 *           then row tiles in ticket order, each tile waiting (bounded) on device
 *           counters for the tiles it reads; 0: three launches
 *   fuse_baby  1: in the double-hoisted schedule, the baby rotations of a chunk
 *           whose requests share one key set are computed inside the plaintext
 *           multiply-accumulate (never written to memory) when the context has
 *           at most 4 digits and moduli below 2^55; 0: a rotation launch writes
 *           them and the multiply-accumulate reads them back
 * A new plan starts at chunk 0, ks_eg 16, mac_my 2, ntt_threads 256, persistent 0,
 * fuse_baby 0. */
typedef struct fhelin_tune {
    int32_t chunk;
    int32_t ks_eg;
    int32_t mac_my;
    int32_t ntt_threads;
    int32_t persistent;
    int32_t fuse_baby;
} fhelin_tune;

int fhelin_plan_get_tune(const fhelin_plan *plan, fhelin_tune *out);
/* FHELIN_E_INVALID_ARG if a field is out of range; the plan is unchanged then. */
int fhelin_plan_set_tune(fhelin_plan *plan, const fhelin_tune *tune);

/* Autotuner: times the plan's schedule on the caller's batch (the arguments of
 * fhelin_linear_apply_multi) for candidate tunes, one field at a time starting
 * from the plan's current tune (chunk in {all, 32, 16, 8, 4} up to the request
 * count, ks_eg in {4, 8, 16}, mac_my in {2, 4, 8}, and when N >= 2^13 ntt_threads
 * in {256, 128, 512} and persistent in {0, 1}; fuse_baby in {0, 1} for the
 * double-hoisted schedule when every request uses one key set), with HIP events on
 * `stream`, and keeps the fastest in the plan.  Every timed run computes the
 * layer, so `out` holds the layer's result on return.  Synchronises `stream`.
 * best (optional) receives the chosen tune, best_ms (optional) its time in ms. */
int fhelin_plan_autotune(fhelin_ctx *ctx, fhelin_plan *plan, const fhelin_keyset *const *ks_per_request,
                         const fhelin_ptset *pts, const fhelin_ct_batch *in, const fhelin_ct_batch *out,
                         int32_t flags, void *stream, fhelin_tune *best, double *best_ms);

/* Capture the kernels of one fhelin_linear_apply call (same arguments) into a
 * HIP graph and instantiate it; nothing runs at capture time.  The device
 * buffers, levels, keys and plaintexts are baked in: each fhelin_graph_launch
 * reads the current contents of in->data and overwrites out->data with the
 * same result an eager call would produce.  `stream` must be non-NULL; the
 * graph uses that stream's workspace, so replays of one graph, and eager calls
 * on the capture stream, must not overlap in time.  The handles and buffers
 * must outlive the graph.  The schedule holds kernels only (no memset or
 * copy nodes). */
int fhelin_graph_capture_linear(fhelin_ctx *ctx, const fhelin_plan *plan, const fhelin_keyset *ks,
                                const fhelin_ptset *pts, const fhelin_ct_batch *in, const fhelin_ct_batch *out,
                                int32_t flags, void *stream, fhelin_graph **graph);
int fhelin_graph_launch(fhelin_graph *graph, void *stream);
int fhelin_graph_destroy(fhelin_graph *graph);

/* Rescale (full-RNS CKKS): drop the top prime q_{l-1} with rounding,
 * c'_i = (c_i - [c]_{q_{l-1}}) * q_{l-1}^{-1} mod q_i with the centred
 * representative of the top limb.  out levels = in levels - 1 (each >= 1).
 * out may alias in only if the strides match. */
int fhelin_rescale(fhelin_ctx *ctx, const fhelin_ct_batch *in, const fhelin_ct_batch *out, void *stream);

/* Rotate every ciphertext of a batch left by steps[t] slots (host array):
 * automorphism g = 5^steps mod 2N followed by a hybrid key switch. */
int fhelin_rotate(fhelin_ctx *ctx, const fhelin_keyset *ks, const fhelin_ct_batch *in, const int32_t *steps,
                  const fhelin_ct_batch *out, void *stream);

/* Batched negacyclic NTT (inverse = 0) or INTT (inverse = 1) in place on
 * rows[n_rows][N] (device), row t reduced modulo modulus mod_index[t] (host
 * array).  Forward output: A[k] = sum_j a_j psi^(j(2 brv(k) + 1)) (bit-
 * reversed order, psi = fhelin_ctx_root); the inverse undoes it exactly. */
int fhelin_ntt(fhelin_ctx *ctx, uint64_t *rows, const int32_t *mod_index, int32_t n_rows, int32_t inverse,
               void *stream);

/* ---- diagnostics ------------------------------------------------------- */

/* Per-kernel timing: when enabled, each kernel launch of the context is
 * bracketed by two HIP events recorded on its launching stream (not while the
 * stream is being captured into a graph).  enable != 0 also discards earlier
 * records.  Kernel classes: ntt_fwd_cols, ntt_fwd_rows, ntt_inv_rows,
 * ntt_inv_cols, ntt_fwd_1, ntt_inv_1, mac, ks_inner (one rotation per
 * entry), ks_rot (a list of rotations for every entry: hoisted baby steps),
 * ks_sum (a sum of key switches per entry: giant steps), modup, moddown_fbc,
 * combine, rescale, copy, mont, encode, modup_ntt (the persistent ModUp + forward
 * NTT launch). */
int fhelin_profile_enable(fhelin_ctx *ctx, int32_t enable);
/* Totals of one kernel class since enabling: launches, summed event time (ms),
 * summed algorithmic work units (butterflies for NTT passes, 64-bit
 * multiply-adds for mac / ks_inner / ks_rot / ks_sum, output elements otherwise) and summed
 * algorithmic HBM bytes (every input and output stream of the launch counted
 * once; distinct evaluation keys once per launch; 0 for classes without a byte
 * model).  Waits for the recorded events.  Output pointers may be NULL. */
int fhelin_profile_read(fhelin_ctx *ctx, const char *kernel, int64_t *launches, double *total_ms, double *units,
                        double *bytes);

/* Issue-rate probe of the GPU's integer ALUs (measures the "alu" rooflines): runs
 * `iters` rounds (a multiple of 32, at most 2^24) of one operation on 8 independent
 * register chains per lane, in 256-thread workgroups, waves_per_simd (1..8)
 * workgroups per compute unit, on the current device (allocates and frees two small
 * buffers, synchronises the device).  op: 0 v_add_u32, 1 v_mul_lo_u32,
 * 2 v_mul_hi_u32, 3 v_mad_u64_u32, 4 v_fma_f64 (single instructions), 5 the NTT's
 * lazy forward butterfly with 53-bit twiddle companions (16 per round, operands in
 * registers), 6 v_lshl_add_u64, 7 v_lshrrev_b64, 8 one product of the packed 28-bit
 * multiply-accumulate (four v_mad_u64_u32; one Montgomery reduction per 32
 * products, operands in registers), 9 v_mfma_i32_16x16x64_i8 (the int8 matrix-core
 * product of the native key-switch engine) on 16 independent accumulators per wave.
 * Outputs (each may be NULL): ghz = core clock measured in the
 * kernel (clock counter over the constant-rate wall clock); clk_per_op = clocks per
 * wave-level operation on one SIMD (4 for a wave64 instruction issued at the full
 * rate; for op 9 one matrix instruction); ops_per_s = lane-level operations per
 * second over the whole GPU (op 9: int8 operations, a multiply-add counting two). */
int fhelin_diag_alu_rate(int32_t op, int32_t waves_per_simd, int32_t iters, double *ghz, double *clk_per_op,
                         double *ops_per_s);

/* Faults of bounded device-side waits since the last call: the persistent ModUp/NTT
 * launch gives up a wait after a fixed number of polls instead of hanging, sets
 * this context's fault word and finishes (its results are then wrong).  Waits for
 * the device to be idle, returns the word in *faults (0 = none) and clears it. */
int fhelin_ctx_faults(fhelin_ctx *ctx, uint32_t *faults);

/* ---- the paper's own pipeline: RLWE over Z_{2^64}[X]/Phi_M ----------------------
 *
 * The scheme of Sec. 2.1: M = t^alpha (t an odd prime), N = phi(M), ciphertexts
 * (a, b) of two polynomials of N coefficients (power basis, uint64: the discrete
 * torus with q = 2^64), b - s a = mu + e, a message m mod p = 2^log_p carried as
 * m 2^64 / p.  The server round of Sec. 4.4 runs in three calls: partial trace
 * extraction of the client's chunks (the lemma on partial trace extraction),
 * an integer-weight layer on the extracted rows (convolution / FC with the
 * round's shuffle folded into the weights' rows), and fast packing of the
 * outputs back into RLWE ciphertexts (Sec. 2.3-2.4), whose automorphisms are
 * key-switched with the gadget keys of Sec. 4.2.  A ciphertext is [2][N]
 * (a then b); batches are contiguous.  All buffers are device memory owned by
 * the caller; the handle owns its key matrices and workspace.  Work goes to
 * `stream` (NULL = null stream). */
typedef struct fhelin_native fhelin_native;

typedef struct fhelin_native_params {
    int32_t t, alpha;   /* M = t^alpha <= 8192, t an odd prime, alpha >= 2 */
    int32_t gamma;      /* partial trace extraction level, 1 or 2 (Sec. 4.4) */
    int32_t beta;       /* packing level gamma..alpha-1: phi(t^beta) outputs per packed
                           ciphertext, output o at coefficient o M / t^beta */
    int32_t log_d, l;   /* gadget base D = 2^log_d (1..16) and depth l (1..8), log_d l < 64 */
    int32_t log_p;      /* message modulus p = 2^log_p (1..31) */
    int32_t engine;     /* key-switch products: 0 = int8 matrix cores (digits split into
                           two balanced int8 pieces for D <= 512, three up to D = 2^16,
                           times balanced key bytes, exact i32 sums; l M <= 2^19),
                           1 = 64-bit integer ALU products */
    int32_t base;       /* 0: gadget base D = 2^log_d; otherwise D itself (the paper's
                           16-bit set takes 310): even, 4..65536, D^l < 2^63, log_d
                           ignored.  The keys then encrypt s(X^g) round(2^64 / D^i)
                           and a mask a is decomposed as round(a D^l / 2^64) written
                           in balanced base D, the carry out of the top digit dropped */
} fhelin_native_params;

/* FHELIN_E_UNSUPPORTED_PARAM for parameters outside the ranges above (checked on
 * the host).  The handle lives on the current device.  Both engines give the same
 * bits. */
int fhelin_native_create(const fhelin_native_params *prm, fhelin_native **out);
int fhelin_native_destroy(fhelin_native *nt);

/* Key-switching keys of the packing (Sec. 4.2): for each tower level
 * i = gamma..alpha-1 the Galois element 1 + t^i mod M and its l gadget
 * encryptions RLWE_s(s(X^(1+t^i)) 2^64 / D^k), k = 1..l: device
 * [alpha-gamma][l][2][N] uint64, read during the call's stream work only.  The
 * handle keeps, per key polynomial, its N x N product matrix modulo Phi_M
 * (about (alpha-gamma) 2 N l N 8 bytes of device memory, as 64-bit words or as
 * eight signed byte planes); FHELIN_E_OOM if that fails. */
int fhelin_native_keys_load(fhelin_native *nt, const uint64_t *ksk, void *stream);

/* Partial trace extraction (Sec. 4.4 and its lemma): chunks
 * [n_chunks][phi(t^gamma)][2][N], the client's encryptions of m(X^d) for
 * d = 1..t-1 (gamma = 1) or d = k (j t + 1) mod M, k = 1..t-1, j = 0..t-1
 * (gamma = 2), in that order.  Writes rows [n_chunks N][2][N]: row c N + i is
 * u sum_d ct_d (X^(d (M - i)) - X^(d (M/t - r))), r = i mod M/t,
 * u = M^-1 mod p taken in (-p/2, p/2], whose trace down to K_gamma decrypts to
 * coefficient i of chunk c.  n_chunks <= 65535. */
int fhelin_native_extract(fhelin_native *nt, const uint64_t *chunks, int32_t n_chunks, uint64_t *rows,
                          void *stream);

/* Integer layer on rows (Sec. 4.4 "Convolution", "Shuffle"): out[o] =
 * sum_k val[k] rows[col[k]] modulo 2^64 for k in [row_ptr[o], row_ptr[o+1]) (CSR,
 * int32 device arrays; the shuffle is the order of the CSR rows).  rows
 * [n_rows][2][N], out [n_out][2][N]; column indices must be < the rows given
 * (not checked on the device).  n_out <= 65535. */
int fhelin_native_linear(fhelin_native *nt, const int32_t *row_ptr, const int32_t *col, const int32_t *val,
                         int32_t n_out, const uint64_t *rows, uint64_t *out, void *stream);

/* The same layer for a convolution (Sec. 4.4 "Convolution": the server reshapes the
 * rows to H x W x C_in and convolves with the rows' coefficients as the batch):
 * rows [c_in h w][2][N] in channels-last order (row (y w + x) c_in + ci), weights
 * [c_out][c_in][k][k] int32 device array, k odd, zero padding k / 2, the given
 * stride; output (position p = y' w' + x', channel co), w' = (w - 1) / stride + 1,
 * goes to out row out_row[p c_out + co] (the shuffle; a permutation of
 * [0, c_out h' w')).  An FC layer is the case h = w = k = 1.  Indices are not
 * checked on the device.  The handle keeps a transposed copy of the weights
 * (c_in k k 16 ceil(c_out / 16) int32; a regrow synchronises the stream), so
 * calls that share the handle must not overlap in time. */
int fhelin_native_conv(fhelin_native *nt, int32_t c_in, int32_t c_out, int32_t h, int32_t w, int32_t k,
                       int32_t stride, const int32_t *weights, const int32_t *out_row, const uint64_t *rows,
                       uint64_t *out, void *stream);

/* Fast packing (Sec. 2.4, 4.4): rows [n_rows][2][N], each with trace down to
 * K_gamma decrypting to a scalar y_o, into packed [ceil(n_rows / phi(t^beta))][2][N]
 * encrypting sum_o y_o X^(o M / t^beta) (rows past n_rows count as zero).  Uses
 * t^(beta-gamma) - 1 + (alpha-beta)(t-1) key switches per packed ciphertext.
 * FHELIN_E_MISSING_GALOIS_KEY before fhelin_native_keys_load.  The handle's
 * workspace grows to fhelin_native_pack_workspace bytes (a regrow synchronises
 * the stream); calls that share the handle must not overlap in time. */
int fhelin_native_pack(fhelin_native *nt, const uint64_t *rows, int32_t n_rows, uint64_t *packed, void *stream);
int fhelin_native_pack_workspace(const fhelin_native *nt, int32_t n_rows, uint64_t *bytes);

/* Per-kernel-class timing of the native pipeline (HIP events around every launch on
 * its stream while enabled; enabling or disabling clears the sums).  Classes:
 * "extract", "linear", "leaves", "merge", "aut_decomp", "ksprod" (the key-switch
 * products, units = 64-bit products), "kmat" (key load).  read waits for the
 * recorded launches and returns launches, total ms, work units and the byte model
 * of each class (any output pointer may be NULL).  While enabled, a linear call
 * reads its nonzero count back from the device (a host synchronisation). */
int fhelin_native_profile_enable(fhelin_native *nt, int32_t enable);
int fhelin_native_profile_read(fhelin_native *nt, const char *kernel, int64_t *launches, double *ms, double *units,
                               double *bytes);

const char *fhelin_last_error(void);
const char *fhelin_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* FHELIN_H */
