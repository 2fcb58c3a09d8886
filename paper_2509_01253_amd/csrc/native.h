// native.h -- the paper's own pipeline over Z_{2^64}[X]/Phi_M (native.hip).
#pragma once
#include <vector>

#include "internal.h"

namespace fl {

constexpr int NAT_MAX_M = 8192;  // M = t^alpha
constexpr int NAT_MAX_POW = 64;  // powers m(X^d) per chunk: phi(t^gamma)

struct Native {
    fhelin_native_params prm{};
    int M = 0, N = 0, Mt = 0;
    int n_pack = 0;  // phi(t^beta): coefficients per packed ciphertext
    int T = 0;       // t^(beta - gamma): leaves per packed ciphertext
    int phig = 0;    // phi(t^gamma): rows per leaf, powers per chunk
    uint64_t u = 0;  // M^-1 mod p (balanced), as a 64-bit two's-complement integer
    std::vector<int> powers;       // d of the client's powers m(X^d)
    std::vector<int> tau, tau_inv; // Galois elements 1 + t^i (i = gamma .. alpha-1) and inverses mod M
    int device = 0;
    uint64_t *kmat = nullptr;  // [alpha-gamma][2][N][l N] key product matrices
    uint64_t *kcorr = nullptr; // [alpha-gamma][2][N] (D/2) row sums of kmat
    bool keys = false;
    void *ws = nullptr;
    size_t ws_bytes = 0;
};

int native_create(const fhelin_native_params *prm, Native **out);
void native_destroy(Native *n);
int native_keys_load(Native *n, const uint64_t *ksk, hipStream_t s);
int native_extract(Native *n, const uint64_t *pows, int n_chunks, uint64_t *rows, hipStream_t s);
int native_linear(Native *n, const int32_t *row_ptr, const int32_t *col, const int32_t *val, int n_out,
                  const uint64_t *rows, uint64_t *out, hipStream_t s);
size_t native_pack_workspace(const Native *n, int n_rows);
int native_pack(Native *n, const uint64_t *rows, int n_rows, uint64_t *packed, hipStream_t s);

}  // namespace fl
