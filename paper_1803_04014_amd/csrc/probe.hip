// probe.hip -- the matrix-core ceiling of the chip as the GEMM kernels see
// it: a register-only loop of MFMA instructions with no memory traffic, on
// random or all-zero operand values.  Measurement aid for the roofline of
// the FP16 and FP8 GEMMs (the dense-peak figure assumes the top clock; the clock the
// chip holds under a sustained MFMA load depends on power, and so on the
// operand bit patterns).
#include "device.h"
#include "internal.h"
#include "runtime.h"

namespace mfg {

// Each wavefront keeps CHAINS independent accumulators and issues
// iters * CHAINS MFMAs on operands loaded once from `src` (4096 dwords:
// 16-bit values, or E4M3 codes for SHAPE 2).  The accumulators are summed into out[wave] so the loop
// is not removed.
template <int SHAPE, int CHAINS>
__global__ __launch_bounds__(256) void mfma_probe_kernel(const uint32_t* __restrict__ src, float* __restrict__ out,
                                                         int64_t iters) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (tid >> 6);
    const int o = (int)((wave * 64 + lane) * 8 % 4096);
    u32x4 a = *reinterpret_cast<const u32x4*>(src + o);
    u32x4 b = *reinterpret_cast<const u32x4*>(src + ((o + 2048) % 4096));
    float s = 0.0f;
    if constexpr (SHAPE == 0) {  // v_mfma_f32_32x32x16_f16
        f32x16 acc[CHAINS];
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = f32x16{};
        for (int64_t i = 0; i < iters; ++i)
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) acc[c] = mma_32x32x16<false>(a, b, acc[c]);
#pragma unroll
        for (int c = 0; c < CHAINS; ++c)
#pragma unroll
            for (int e = 0; e < 16; ++e) s += acc[c][e];
    } else if constexpr (SHAPE == 2) {  // v_mfma_scale_f32_32x32x64_f8f6f4, E4M3 codes, unit scales
        const int o8 = (int)((wave * 64 + lane) * 8 % 4096);  // 32 bytes per lane
        const i32x8 a8 = *reinterpret_cast<const i32x8*>(src + o8);
        const i32x8 b8 = *reinterpret_cast<const i32x8*>(src + ((o8 + 2048) % 4096));
        f32x16 acc[CHAINS];
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = f32x16{};
        for (int64_t i = 0; i < iters; ++i)
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) acc[c] = mma_32x32x64_e4m3(a8, b8, acc[c], 127, 127);
#pragma unroll
        for (int c = 0; c < CHAINS; ++c)
#pragma unroll
            for (int e = 0; e < 16; ++e) s += acc[c][e];
        (void)a, (void)b;
    } else {  // v_mfma_f32_16x16x32_f16
        f32x4 acc[CHAINS];
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = f32x4{};
        for (int64_t i = 0; i < iters; ++i)
#pragma unroll
            for (int c = 0; c < CHAINS; ++c)
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                                __builtin_bit_cast(f16x8, b), acc[c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < CHAINS; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) s += acc[c][e];
    }
    out[wave * 64 + lane] = s;
}

}  // namespace mfg

using namespace mfg;

extern "C" int mfg_probe_mfma(int shape, const void* operands, int64_t workgroups, int64_t iters, float* out,
                              double* flops, void* stream) {
    if (shape < 0 || shape > 2 || !operands || !out || workgroups < 1 || workgroups > (1 << 20) || iters < 1)
        return MFG_ERR_INVALID_ARG;
    constexpr int kChains = 8;
    const double per = shape == 0 ? 2.0 * 32 * 32 * 16 : shape == 1 ? 2.0 * 16 * 16 * 32 : 2.0 * 32 * 32 * 64;
    if (flops) *flops = per * kChains * (double)iters * (double)workgroups * 4.0;  // 4 wavefronts per workgroup
    hipStream_t s = (hipStream_t)stream;
    if (shape == 0)
        hipLaunchKernelGGL((mfma_probe_kernel<0, kChains>), dim3((unsigned)workgroups), dim3(256), 0, s,
                           static_cast<const uint32_t*>(operands), out, iters);
    else if (shape == 1)
        hipLaunchKernelGGL((mfma_probe_kernel<1, kChains>), dim3((unsigned)workgroups), dim3(256), 0, s,
                           static_cast<const uint32_t*>(operands), out, iters);
    else
        hipLaunchKernelGGL((mfma_probe_kernel<2, kChains>), dim3((unsigned)workgroups), dim3(256), 0, s,
                           static_cast<const uint32_t*>(operands), out, iters);
    MFG_LAUNCH_CHECK();
    return MFG_OK;
}
