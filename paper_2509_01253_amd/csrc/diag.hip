// diag.hip -- issue-rate probes of the integer ALU work the kernels are built from
// (diagnostics: they price the "alu" rooflines from measurement instead of assumption).
//
// Each probe runs `iters` rounds of one operation on CHAINS independent register
// chains per lane, in 256-thread workgroups, waves_per_simd workgroups per compute
// unit, so every SIMD holds that many waves.  Per wave the kernel records the core
// clock counter (s_memtime) and the constant-rate wall clock (s_memrealtime) around
// its loop; the host takes the core clock frequency from their ratio and the
// throughput from HIP events around the launch:
//   clocks per wave-level operation per SIMD = elapsed * f / (wave-ops per SIMD).
// A wave64 instruction that issues at the full rate on a 16-lane SIMD takes 4 clocks.
// The single-instruction probes are written as inline assembly so each loop body is
// exactly the instruction named (no other VALU work besides the loop counter).
#include <algorithm>
#include <vector>

#include "internal.h"
#include "modarith.h"

namespace fl {

constexpr int DIAG_CHAINS = 8;

enum DiagOp : int {
    DIAG_ADD_U32 = 0,
    DIAG_MUL_LO_U32 = 1,
    DIAG_MUL_HI_U32 = 2,
    DIAG_MAD_U64_U32 = 3,
    DIAG_FMA_F64 = 4,
    DIAG_NTT_BFLY = 5,
    DIAG_LSHL_ADD_U64 = 6,
    DIAG_LSHRREV_B64 = 7,
    DIAG_MAC28 = 8,
    DIAG_MFMA_I8 = 9,
};

__device__ __forceinline__ void diag_stamp(uint64_t *stamps, uint64_t c0, uint64_t r0) {
    const uint64_t c1 = clock64(), r1 = wall_clock64();
    if ((threadIdx.x & 63) == 0) {
        const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
        stamps[2 * wave] = c1 - c0;
        stamps[2 * wave + 1] = r1 - r0;
    }
}

template <int OP>
__global__ void __launch_bounds__(256) k_diag_op(uint64_t *__restrict__ sink, uint64_t *__restrict__ stamps,
                                                 int iters, uint32_t k) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t x[DIAG_CHAINS];
    uint64_t y[DIAG_CHAINS];
    double d[DIAG_CHAINS];
#pragma unroll
    for (int c = 0; c < DIAG_CHAINS; ++c) {
        x[c] = tid * 2654435761u + c;
        y[c] = ((uint64_t)x[c] << 20) | c;
        d[c] = 1.0 + 1e-9 * c;
    }
    const uint64_t c0 = clock64(), r0 = wall_clock64();
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < DIAG_CHAINS; ++c) {
            if constexpr (OP == DIAG_ADD_U32) {
                asm volatile("v_add_u32 %0, %1, %2" : "=v"(x[c]) : "v"(x[c]), "v"(k));
            } else if constexpr (OP == DIAG_MUL_LO_U32) {
                asm volatile("v_mul_lo_u32 %0, %1, %2" : "=v"(x[c]) : "v"(x[c]), "v"(k));
            } else if constexpr (OP == DIAG_MUL_HI_U32) {
                asm volatile("v_mul_hi_u32 %0, %1, %2" : "=v"(x[c]) : "v"(x[c]), "v"(k));
            } else if constexpr (OP == DIAG_MAD_U64_U32) {
                uint64_t cc;
                asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %4"
                             : "=v"(y[c]), "=s"(cc)
                             : "v"((uint32_t)y[c]), "v"(k), "v"(y[c]));
            } else if constexpr (OP == DIAG_FMA_F64) {
                asm volatile("v_fma_f64 %0, %1, %2, %3" : "=v"(d[c]) : "v"(d[c]), "v"(d[c]), "v"(d[c]));
            } else if constexpr (OP == DIAG_LSHL_ADD_U64) {
                asm volatile("v_lshl_add_u64 %0, %1, 3, %2" : "=v"(y[c]) : "v"(y[c]), "v"(y[c]));
            } else if constexpr (OP == DIAG_LSHRREV_B64) {
                asm volatile("v_lshrrev_b64 %0, 1, %1" : "=v"(y[c]) : "v"(y[c]));
            }
        }
    }
    diag_stamp(stamps, c0, r0);
    uint64_t acc = 0;
#pragma unroll
    for (int c = 0; c < DIAG_CHAINS; ++c) acc ^= x[c] ^ y[c] ^ (uint64_t)__double_as_longlong(d[c]);
    sink[tid] = acc;
}

// The multiply-accumulate's product: four 32x32->64 multiply-adds into the three sums
// of the packed 28-bit accumulator (inline assembly, so the compiler cannot merge
// products of a shared operand), one Montgomery reduction of each chain's sums every
// 32 products as the multiply-accumulate kernel does.  4 chains, 32 distinct second
// operands in registers.
constexpr int MAC_CHAINS = 4;
__device__ __forceinline__ void mad_acc(uint64_t &acc, uint32_t x, uint32_t y) {
    uint64_t cc;
    asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(acc), "=s"(cc) : "v"(x), "v"(y), "v"(acc));
}
__global__ void __launch_bounds__(256) k_diag_mac28(uint64_t *__restrict__ sink, uint64_t *__restrict__ stamps,
                                                    int iters, uint64_t q, uint64_t ninv) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    LazyAcc<true> acc[MAC_CHAINS];
    uint64_t a[MAC_CHAINS], b[32];
#pragma unroll
    for (int c = 0; c < MAC_CHAINS; ++c) {
        acc[c].zero();
        a[c] = pack28((tid * 0x9E3779B97F4A7C15ull + c) & ((1ull << 49) - 1));
    }
#pragma unroll
    for (int j = 0; j < 32; ++j) b[j] = pack28((tid * 0xBF58476D1CE4E5B9ull + 7 * j) & ((1ull << 49) - 1));
    const uint64_t c0 = clock64(), r0 = wall_clock64();
    for (int it = 0; it < iters; it += 32) {
#pragma unroll
        for (int j = 0; j < 32; ++j) {
#pragma unroll
            for (int c = 0; c < MAC_CHAINS; ++c) {
                const uint32_t a0 = (uint32_t)a[c], a1 = (uint32_t)(a[c] >> 32);
                const uint32_t b0 = (uint32_t)b[j], b1 = (uint32_t)(b[j] >> 32);
                mad_acc(acc[c].a.s0, a0, b0);
                mad_acc(acc[c].a.s1, a0, b1);
                mad_acc(acc[c].a.s1, a1, b0);
                mad_acc(acc[c].a.s2, a1, b1);
            }
        }
#pragma unroll
        for (int c = 0; c < MAC_CHAINS; ++c) {
            const uint64_t v = acc[c].reduce(q, ninv);
            acc[c].set(v);
        }
    }
    diag_stamp(stamps, c0, r0);
    uint64_t s = 0;
#pragma unroll
    for (int c = 0; c < MAC_CHAINS; ++c) s ^= acc[c].value();
    sink[tid] = s;
}

// The int8 matrix-core product of the key-switch engine: v_mfma_i32_16x16x64_i8 on
// MFMA_ACCS independent accumulators per wave (the product kernel keeps 16), operands in
// registers, 16 instructions per round.
constexpr int MFMA_ACCS = 16;
typedef int diag_v4i __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_diag_mfma_i8(uint64_t *__restrict__ sink, uint64_t *__restrict__ stamps,
                                                      int iters) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    diag_v4i a[2], b[2], acc[MFMA_ACCS];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        a[i] = diag_v4i{(int)(tid * 2654435761u + i), (int)tid, i, 3};
        b[i] = diag_v4i{(int)(tid ^ 0x5bd1e995u), i, (int)tid + 7, 1};
    }
#pragma unroll
    for (int i = 0; i < MFMA_ACCS; ++i) acc[i] = diag_v4i{0, 0, 0, 0};
    const uint64_t c0 = clock64(), r0 = wall_clock64();
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < MFMA_ACCS; ++i)
            acc[i] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i & 1], b[(i >> 1) & 1], acc[i], 0, 0, 0);
    }
    diag_stamp(stamps, c0, r0);
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < MFMA_ACCS; ++i) s ^= (uint64_t)(uint32_t)(acc[i][0] ^ acc[i][1] ^ acc[i][2] ^ acc[i][3]) << (i & 31);
    sink[tid] = s;
}

int diag_alu_rate(int op, int waves_per_simd, int iters, double *ghz, double *clk_per_op, double *ops_per_s) {
    FL_CHECK(op >= DIAG_ADD_U32 && op <= DIAG_MFMA_I8, FHELIN_E_INVALID_ARG, "diag: unknown probe");
    FL_CHECK(waves_per_simd >= 1 && waves_per_simd <= 8, FHELIN_E_INVALID_ARG, "diag: waves_per_simd in 1..8");
    FL_CHECK(iters >= 32 && iters <= (1 << 24) && iters % 32 == 0, FHELIN_E_INVALID_ARG,
             "diag: iters must be a multiple of 32 in [32, 2^24]");
    int dev = 0, cus = 0, wall_khz = 0;
    FL_TRY_HIP(hipGetDevice(&dev));
    FL_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    FL_TRY_HIP(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev));
    FL_CHECK(cus > 0 && wall_khz > 0, FHELIN_E_HIP, "diag: device attributes unavailable");
    const int blocks = cus * waves_per_simd, threads = blocks * 256, waves = threads / 64;
    uint64_t *sink = nullptr, *stamps = nullptr;
    FL_TRY_HIP(hipMalloc(&sink, (size_t)threads * sizeof(uint64_t)));
    if (hipMalloc(&stamps, (size_t)waves * 2 * sizeof(uint64_t)) != hipSuccess) {
        (void)hipFree(sink);
        return set_error(FHELIN_E_OOM, "diag: allocation failed");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = FHELIN_OK;
    float ms = 0;
    std::vector<uint64_t> st((size_t)waves * 2);
    // a prime q = 1 mod 2^17 below 2^50 and a twiddle of the probe butterfly
    uint64_t q = 0;
    if (primes_generate(16, 50, 1, &q) != FHELIN_OK) q = 1125899906826241ull;
    const uint64_t w = q / 3 + 12345, wp = h_shoup53(w, q), ninv = h_neg_inv64(q);
    auto launch = [&]() {
        switch (op) {
        case DIAG_ADD_U32: hipLaunchKernelGGL(k_diag_op<DIAG_ADD_U32>, dim3(blocks), dim3(256), 0, 0, sink, stamps, iters, 7u); break;
        case DIAG_MUL_LO_U32: hipLaunchKernelGGL(k_diag_op<DIAG_MUL_LO_U32>, dim3(blocks), dim3(256), 0, 0, sink, stamps, iters, 2654435761u); break;
        case DIAG_MUL_HI_U32: hipLaunchKernelGGL(k_diag_op<DIAG_MUL_HI_U32>, dim3(blocks), dim3(256), 0, 0, sink, stamps, iters, 2654435761u); break;
        case DIAG_MAD_U64_U32: hipLaunchKernelGGL(k_diag_op<DIAG_MAD_U64_U32>, dim3(blocks), dim3(256), 0, 0, sink, stamps, iters, 2654435761u); break;
        case DIAG_FMA_F64: hipLaunchKernelGGL(k_diag_op<DIAG_FMA_F64>, dim3(blocks), dim3(256), 0, 0, sink, stamps, iters, 1u); break;
        case DIAG_NTT_BFLY: launch_diag_bfly(blocks, sink, stamps, iters, q, w, wp); break;
        case DIAG_LSHL_ADD_U64: hipLaunchKernelGGL(k_diag_op<DIAG_LSHL_ADD_U64>, dim3(blocks), dim3(256), 0, 0, sink, stamps, iters, 1u); break;
        case DIAG_LSHRREV_B64: hipLaunchKernelGGL(k_diag_op<DIAG_LSHRREV_B64>, dim3(blocks), dim3(256), 0, 0, sink, stamps, iters, 1u); break;
        case DIAG_MAC28: hipLaunchKernelGGL(k_diag_mac28, dim3(blocks), dim3(256), 0, 0, sink, stamps, iters, q, ninv); break;
        case DIAG_MFMA_I8: hipLaunchKernelGGL(k_diag_mfma_i8, dim3(blocks), dim3(256), 0, 0, sink, stamps, iters); break;
        }
    };
    do {
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            rc = set_error(FHELIN_E_HIP, "diag: event creation failed");
            break;
        }
        launch();  // warm-up (code load, clocks up)
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
            rc = set_error(FHELIN_E_HIP, "diag: probe launch failed");
            break;
        }
        (void)hipEventRecord(e0, 0);
        launch();
        (void)hipEventRecord(e1, 0);
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
            hipMemcpy(st.data(), stamps, st.size() * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess) {
            rc = set_error(FHELIN_E_HIP, "diag: timing failed");
            break;
        }
    } while (0);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    (void)hipFree(stamps);
    if (rc != FHELIN_OK) return rc;
    // core clock: the median over waves of core cycles per wall-clock second
    std::vector<double> fr;
    for (int i = 0; i < waves; ++i)
        if (st[2 * i + 1] > 0) fr.push_back((double)st[2 * i] / ((double)st[2 * i + 1] / (wall_khz * 1e3)));
    double f = 0;  // Hz
    if (!fr.empty()) {
        std::nth_element(fr.begin(), fr.begin() + fr.size() / 2, fr.end());
        f = fr[fr.size() / 2];
    }
    // operations per lane: single instructions count CHAINS per round; the butterfly
    // probe runs 16 butterflies per round, the multiply-accumulate probe MAC_CHAINS
    // products per round; the matrix-core probe MFMA_ACCS wave-level instructions per
    // round, each 16 x 16 x 64 multiply-adds (2 int8 operations each)
    const double per_lane = (op == DIAG_NTT_BFLY ? 16.0
                             : op == DIAG_MAC28  ? (double)MAC_CHAINS
                             : op == DIAG_MFMA_I8 ? (double)MFMA_ACCS
                                                  : (double)DIAG_CHAINS) *
                            iters;
    const double wave_ops_per_simd = per_lane * waves / (4.0 * cus);
    if (ghz) *ghz = f / 1e9;
    if (clk_per_op) *clk_per_op = ms > 0 ? (ms * 1e-3 * f) / wave_ops_per_simd : 0;
    if (ops_per_s)
        *ops_per_s = ms <= 0                ? 0
                     : op == DIAG_MFMA_I8 ? per_lane * waves * (16.0 * 16 * 64 * 2) / (ms * 1e-3)
                                          : per_lane * threads / (ms * 1e-3);
    return FHELIN_OK;
}

}  // namespace fl
