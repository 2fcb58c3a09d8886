// native.h -- the paper's own pipeline over Z_{2^64}[X]/Phi_M (native.hip).
#pragma once
#include <vector>

#include "internal.h"

namespace fl {

constexpr int NAT_MAX_M = 8192;  // M = t^alpha
constexpr int NAT_MAX_POW = 64;  // powers m(X^d) per chunk: phi(t^gamma)

// kernel classes of the native pipeline's profiler
enum NatKind : int { NK_EXTRACT = 0, NK_LINEAR, NK_LEAVES, NK_MERGE, NK_AUT_DECOMP, NK_KSPROD, NK_KMAT, NK_COUNT };
extern const char *const NAT_KIND_NAMES[NK_COUNT];

// the gadget of the key switching: base D (2^log_d when log_d > 0), depth l, D^l
struct NatGadget {
    int log_d = 0, l = 0;
    uint64_t D = 0, Dl = 0;
};

struct Native {
    fhelin_native_params prm{};
    int M = 0, N = 0, Mt = 0;
    int n_pack = 0;  // phi(t^beta): coefficients per packed ciphertext
    int T = 0;       // t^(beta - gamma): leaves per packed ciphertext
    int phig = 0;    // phi(t^gamma): rows per leaf, powers per chunk
    uint64_t u = 0;  // M^-1 mod p (balanced), as a 64-bit two's-complement integer
    std::vector<int> powers;       // d of the client's powers m(X^d)
    std::vector<int> tau, tau_inv; // Galois elements 1 + t^i (i = gamma .. alpha-1) and inverses mod M
    NatGadget gad;
    int device = 0;
    int cus = 0;               // compute units of the device
    int lds_max = 0;           // shared memory per workgroup (bytes)
    int KDp = 0;               // l N rounded up to a multiple of 64 (int8 engine)
    uint64_t *kmat = nullptr;  // [alpha-gamma][2][N][l N] key product matrices (64-bit engine)
    int8_t *kmat8 = nullptr;   // [alpha-gamma][2][8][N][KDp] their balanced bytes (int8 engine)
    uint64_t *kcorr = nullptr; // [alpha-gamma][2][N] (D/2) row sums of kmat
    bool keys = false;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    int32_t *wt = nullptr;  // a convolution's transposed weights
    size_t wt_bytes = 0;
    // profiler: HIP events around every launch while enabled (not under graph capture)
    struct Rec {
        int kind;
        hipEvent_t a, b;
        double units, bytes;
    };
    bool prof = false;
    std::vector<Rec> pending;
    double sum_ms[NK_COUNT] = {}, sum_units[NK_COUNT] = {}, sum_bytes[NK_COUNT] = {};
    int64_t launches[NK_COUNT] = {};
};

// brackets one launch with events while the handle's profiler is on
struct NatProf {
    Native *n;
    hipStream_t s;
    int kind;
    double units, bytes;
    hipEvent_t a{};
    bool on = false;
    NatProf(Native *n_, hipStream_t s_, int k, double u, double by);
    ~NatProf();
};
int native_profile_enable(Native *n, bool on);
int native_profile_read(Native *n, const char *kind, int64_t *launches, double *ms, double *units, double *bytes);

int native_create(const fhelin_native_params *prm, Native **out);
void native_destroy(Native *n);
int native_keys_load(Native *n, const uint64_t *ksk, hipStream_t s);
int native_extract(Native *n, const uint64_t *pows, int n_chunks, uint64_t *rows, hipStream_t s);
int native_linear(Native *n, const int32_t *row_ptr, const int32_t *col, const int32_t *val, int n_out,
                  const uint64_t *rows, uint64_t *out, hipStream_t s);
int native_conv(Native *n, int c_in, int c_out, int h, int w, int k, int stride, const int32_t *wts,
                const int32_t *out_row, const uint64_t *rows, uint64_t *out, hipStream_t s);
size_t native_pack_workspace(const Native *n, int n_rows);
int native_pack(Native *n, const uint64_t *rows, int n_rows, uint64_t *packed, hipStream_t s);

}  // namespace fl
