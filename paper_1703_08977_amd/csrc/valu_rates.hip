// valu_rates -- issue cost of each class of VALU instruction on this GPU, for the
// class-weighted issue roofline of the walker step.
//
// Each kernel runs 16 independent dependency chains per lane (enough to hide
// every class's latency: the 8-chain forms are no faster) over 2048
// iterations on 8192 blocks of 256 threads, and the chains' results are
// written out so that nothing is removed.  A class measured "with fmac" runs
// one vector-operand binary32 fused multiply-add chain step beside each step
// of the class, the mix of the walker step, where the class's incremental
// cost is the pair's cost less the multiply-add's.  Helper instructions a
// chain step needs (the add after a 32x32->64 multiply, the xor after a
// convert) are listed with each kernel.
//
// The program prints each kernel's duration; the SIMD-cycles per wave
// instruction come from the GPU's own counters (GRBM_GUI_ACTIVE over
// SQ_INSTS_VALU per SIMD) in a rocprofv3 --pmc run of this program.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>

#define CK(x)                                                                                      \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) {                                                                    \
            std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);    \
            std::exit(1);                                                                          \
        }                                                                                          \
    } while (0)

namespace {

constexpr int kChains = 16, kBlock = 256, kGrid = 8192, kIters = 2048;

enum Kind {
    F32_FMA,         // v_fmac_f32
    F32_ADD,         // v_add_f32
    F32_MUL,         // v_mul_f32
    I32_XOR,         // v_xor_b32
    SEL,             // v_cndmask_b32 with a lane mask
    CVT_F32_U32,     // v_cvt_f32_u32 + v_xor_b32
    MAD_U64_U32,     // v_mad_u64_u32 + v_add_u32
    TRANS_F32,       // v_rsq_f32
    F64_FMA,         // v_fma_f64
    SEED_F64,        // v_rsq_f64
    MIX_TRANS_F32,   // fmac + v_rsq_f32
    MIX_MAD_U64_U32, // fmac + v_mad_u64_u32 + v_add_u32
    MIX_F64_FMA,     // fmac + v_fma_f64
    MIX_SEL,         // fmac + v_cndmask_b32
    MIX_CVT_F32_U32, // fmac + v_cvt_f32_u32 + v_xor_b32
    MIX_SEED_F64,    // fmac + v_rsq_f64
    CVT_F64,         // v_cvt_f64_f32 + v_add_f64 + v_cvt_f32_f64
    MIX_CVT_F64,     // fmac + the same three
    F32_FMA_AB,      // v_fma_f32 with the chain value as the multiplicand and two shared operands
    N_KINDS
};

const char* const kNames[N_KINDS] = {
    "f32 fma",          "f32 add",          "f32 mul",        "i32 xor",        "select",
    "cvt f32 u32 + xor", "mad u64 u32 + add", "f32 rsq",        "f64 fma",        "f64 rsq",
    "fmac + f32 rsq",   "fmac + mad + add", "fmac + f64 fma", "fmac + select",  "fmac + cvt + xor",
    "fmac + f64 rsq",   "cvt f64 f32 + f64 add + cvt f32 f64", "fmac + the same three", "f32 fma, shared operands"};
// VALU instructions per chain step of each kernel
const int kInsts[N_KINDS] = {1, 1, 1, 1, 1, 2, 2, 1, 1, 1, 2, 3, 2, 2, 3, 2, 3, 4, 1};

template <int K>
__global__ __launch_bounds__(kBlock) void rate_kernel(int iters, double* __restrict__ out)
{
    const int tid = blockIdx.x * kBlock + threadIdx.x;
    // lane-dependent operands, so that every operand is a vector register
    const float fa = 0.9999f + 1e-9f * (float)(tid & 1023), fb = 1e-7f * (float)(tid & 7);
    const double da = 0.9999 + 1e-12 * (double)(tid & 1023), db = 1e-9 * (double)(tid & 7);
    const uint32_t ua = 0x9E3779B9u ^ (uint32_t)tid, ub = 0xD2511F53u + (uint32_t)(tid & 15);
    float x[kChains], z[kChains];
    double y[kChains];
    uint32_t u[kChains];
    bool msk[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
        x[k] = 1.0f + 1e-3f * k + 1e-9f * tid;
        z[k] = 2.0f + 1e-3f * k + 1e-9f * tid;
        y[k] = 1.0 + 1e-3 * k + 1e-12 * tid;
        u[k] = (uint32_t)tid * 7u + (uint32_t)k;
        msk[k] = ((tid >> (k & 7)) & 1) != 0;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) {
            const bool mix = K >= MIX_TRANS_F32 && K != CVT_F64 && K != F32_FMA_AB;
            if (K == F32_FMA || mix) z[k] = __builtin_fmaf(fa, fb + (float)k, z[k]);
            if (K == F32_FMA_AB) x[k] = __builtin_fmaf(x[k], fa, fb);
            if (K == F32_ADD) x[k] = x[k] + fb;
            if (K == F32_MUL) x[k] = x[k] * fa;
            if (K == I32_XOR) u[k] = u[k] ^ (ua + (uint32_t)k);
            if (K == SEL || K == MIX_SEL) x[k] = msk[k] ? x[k] : z[(k + 5) % kChains];
            if (K == CVT_F32_U32 || K == MIX_CVT_F32_U32) u[k] = __float_as_uint((float)u[k]) ^ ua;
            if (K == MAD_U64_U32 || K == MIX_MAD_U64_U32) {
                const uint64_t p = (uint64_t)u[k] * (uint64_t)ub;
                u[k] = (uint32_t)(p >> 32) + (uint32_t)p;
            }
            if (K == TRANS_F32 || K == MIX_TRANS_F32) x[k] = __builtin_amdgcn_rsqf(x[k]);
            if (K == F64_FMA || K == MIX_F64_FMA) y[k] = __builtin_fma(y[k], da, db);
            if (K == SEED_F64 || K == MIX_SEED_F64) y[k] = __builtin_amdgcn_rsq(y[k]);
            if (K == CVT_F64 || K == MIX_CVT_F64) x[k] = (float)((double)x[k] + db);
        }
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += (double)x[k] + (double)z[k] + y[k] + (double)(u[k] & 0xffu);
    out[tid] = s;
}

template <int K>
void run(double* out, hipEvent_t e0, hipEvent_t e1)
{
    rate_kernel<K><<<kGrid, kBlock>>>(kIters, out);  // warm-up
    CK(hipGetLastError());
    float best = 1e30f;
    for (int r = 0; r < 3; ++r) {
        CK(hipEventRecord(e0, 0));
        rate_kernel<K><<<kGrid, kBlock>>>(kIters, out);
        CK(hipEventRecord(e1, 0));
        CK(hipEventSynchronize(e1));
        float ms;
        CK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) best = ms;
    }
    const double wave_insts = (double)kGrid * (kBlock / 64) * kIters * kChains * kInsts[K];
    std::printf("rate_kernel<%d> %-18s %d VALU per chain step  %8.3f ms  %.3f ms per 2^30 wave instructions\n", K,
                kNames[K], kInsts[K], best, best * 1073741824.0 / wave_insts);
    std::fflush(stdout);
}

template <int K>
void run_all(double* out, hipEvent_t e0, hipEvent_t e1)
{
    if constexpr (K < N_KINDS) {
        run<K>(out, e0, e1);
        run_all<K + 1>(out, e0, e1);
    }
}

}  // namespace

int main()
{
    double* out;
    CK(hipMalloc(&out, (size_t)kGrid * kBlock * sizeof(double)));
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    run_all<0>(out, e0, e1);
    CK(hipFree(out));
    std::printf("valu_rates done\n");
    return 0;
}
