// gemm_f8.hip -- FP8-E4M3 GEMM with per-128x128-tile power-of-two scales on
// the gfx950 matrix cores (v_mfma_scale_f32_32x32x64_f8f6f4).
//
// A tile scale is 2^E with E in [-127, 127], so it is passed to the MFMA as
// its E8M0 block-scale code E + 127 and applied in hardware:
//   acc += (2^Ea * qA) (2^Eb * qB)  over each 64-deep K chunk.
// A 64-deep chunk never straddles a 128-wide K tile and a 32-row / 32-column
// output block never straddles a 128 tile, so one scale per operand applies
// to the whole instruction.  Accumulation order: K chunks 0, 64, 128, ...
#include "device.h"
#include "internal.h"

namespace mfg {

// E8M0 code of a power-of-two FP32 scale 2^E (E in [-127, 127]): the biased
// exponent field; 2^-127 is the FP32 subnormal with field 0, code 0.
__device__ __forceinline__ int e8m0_code(float s) {
    return (int)((__builtin_bit_cast(uint32_t, s) >> 23) & 0xFFu);
}

__device__ __forceinline__ void store_out_f8(float* C, int64_t off, float v, float alpha, float beta) {
    C[off] = (beta == 0.0f) ? alpha * v : __builtin_fmaf(alpha, v, beta * C[off]);
}

// One wavefront per 32x32 output tile; operands from global memory.  Lane
// (r, g) supplies the 32 codes k = k0 + 32 g + 0..31 of A row r and of B
// column r.
__global__ __launch_bounds__(64) void gemmf8_simple(GemmF8Args p, int vecA) {
    const int lane = threadIdx.x;
    const int r = lane & 31, g = lane >> 5;
    const int64_t m0 = (int64_t)blockIdx.y * 32, n0 = (int64_t)blockIdx.x * 32;
    const int64_t am = m0 + r, bn = n0 + r;
    const int64_t ktiles = cdiv(p.K, MFG_FP8_TILE), ntiles = cdiv(p.N, MFG_FP8_TILE);
    const int64_t mt = m0 / MFG_FP8_TILE, nt = n0 / MFG_FP8_TILE;
    f32x16 acc = {};
    for (int64_t k0 = 0; k0 < p.K; k0 += 64) {
        const int64_t kb = k0 + g * 32;
        const int64_t kt = k0 / MFG_FP8_TILE;
        union {
            i32x8 v;
            uint8_t b[32];
            u32x4 q[2];
        } a, b;
        if (am < p.M && vecA && kb + 32 <= p.K) {
            a.q[0] = *reinterpret_cast<const u32x4*>(p.A + am * p.lda + kb);
            a.q[1] = *reinterpret_cast<const u32x4*>(p.A + am * p.lda + kb + 16);
        } else {
#pragma unroll
            for (int j = 0; j < 32; ++j) a.b[j] = (am < p.M && kb + j < p.K) ? p.A[am * p.lda + kb + j] : (uint8_t)0;
        }
#pragma unroll
        for (int j = 0; j < 32; ++j) b.b[j] = (bn < p.N && kb + j < p.K) ? p.B[(kb + j) * p.ldb + bn] : (uint8_t)0;
        const int sa = e8m0_code(p.sa[mt * ktiles + kt]);
        const int sb = e8m0_code(p.sb[kt * ntiles + nt]);
        acc = mma_32x32x64_e4m3(a.v, b.v, acc, sa, sb);
    }
    if (bn < p.N) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int64_t row = m0 + mfma_out_row(i, lane);
            if (row < p.M) store_out_f8(p.C, row * p.ldc + bn, acc[i], p.alpha, p.beta);
        }
    }
}

int num_configs_f8() { return 1; }
const char* config_f8_name(int cfg) { return cfg == 0 ? "simple32" : nullptr; }
int pick_config_f8(int64_t, int64_t, int64_t, bool) { return 0; }

int launch_gemm_f8(int cfg, const GemmF8Args& a, bool vec_ok, hipStream_t s) {
    if (cfg != 0) return MFG_ERR_INVALID_ARG;
    dim3 grid((unsigned)cdiv(a.N, 32), (unsigned)cdiv(a.M, 32), 1);
    hipLaunchKernelGGL(gemmf8_simple, grid, dim3(64), 0, s, a, vec_ok ? 1 : 0);
    MFG_LAUNCH_CHECK();
    return MFG_OK;
}

}  // namespace mfg
