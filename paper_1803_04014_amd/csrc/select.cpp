// select.cpp -- default tile configuration of each mode when the caller
// asks for none and the tuned table has no entry: thresholds on the number
// of output tiles, from measured sweeps on MI355X.  Host code only; kept
// apart from the kernels so that the policy can change without touching
// them.  Configuration indices refer to the menus in gemm16.hip,
// gemm_f8.hip and gemm_f32.hip.
#include <cstdint>

#include "internal.h"

namespace mfg {

// Default configuration per kind, from measured sweeps on MI355X (square
// N = 1024 .. 8192, random operands): the pipelined 64-wide kernels once the
// grid fills the chip, the 64 x 64 tiled kernel below that, the simple
// kernel when rows are not 16-byte aligned.
int pick_config16(int kind, int64_t M, int64_t N, int64_t K, bool vec_ok) {
    if (!vec_ok) return 0;
    const bool fast = K % 64 == 0 && N % 8 == 0 && N >= 8;
    const int64_t t256 = cdiv(M, 256) * cdiv(N, 256);
    const int64_t t128 = cdiv(M, 128) * cdiv(N, 128);
    const bool big = M >= 64 && N >= 64;
    if (kind == K_F16 || kind == K_BF16) {
        if (fast && t256 >= 256) return 29;  // q256x256k64s2w2x2g8e
        if (fast && t128 >= 64) return 28;   // q128x128k64s3w2x2g8
        return big ? 6 : 0;                  // t64x64k64w2x2g8
    }
    if (kind == K_SPLIT4) {
        if (fast && t128 >= 256) return 5;   // q128x128k64s2w2x2g8e
        if (fast && t128 >= 64) return 3;    // f128x128k32w2x2g8dma
        return big ? 2 : 0;                  // t64x64k32w2x2g8
    }
    // 192 x 128: two 64-deep stages fill the 160 KB of LDS and each MFMA
    // needs 17% fewer operand bytes than on 128 x 128 (N = 8192: SPLIT3
    // 2.74 vs 2.96 ms, BF16_SPLIT3 2.63 vs 2.87, REFINE_A 2.16 vs 2.27); at
    // N = 4096 the partial last wave of 192-row tiles makes it a tie
    if (fast && cdiv(M, 192) * cdiv(N, 128) >= 1024) return 9;  // q192x128k64s2w2x2g8e
    if (fast && t128 >= 256) return 7;       // q128x128k64s2w2x2g8
    if (fast && t128 >= 64) return 6;        // f128x128k64w2x2g8dma
    return big ? 3 : 0;                      // t64x64k32w2x2g8
}

// Default: the tiled kernels once the grid fills the chip (measured sweeps,
// square N = 1024 .. 8192), else the simple kernel.
int pick_config_f8(int64_t M, int64_t N, int64_t K, bool vec_ok) {
    if (!vec_ok || K % 128 != 0 || M < 1 || N < 1) return 0;
    if (cdiv(M, 256) * cdiv(N, 256) >= 256) return 4;  // p256x256k128s2w2x2g8e (4096^2: 1.78 vs 1.58 PF for p256x128)
    if (cdiv(M, 256) * cdiv(N, 128) >= 256) return 3;  // p256x128
    if (cdiv(M, 128) * cdiv(N, 128) >= 64) return 2;   // p128x128
    return 0;
}

// FP32: the 128 x 128 tiled kernel from 128 x 128 up (two wavefronts per
// SIMD; alternating timings against 256 x 128 at N = 4096 / 8192 / 16384:
// 122.6 / 125.1 / 126.1 against 120.8 / 122.0 / 121.7 TFLOP/s), the simple
// kernel otherwise (or for unaligned rows).
int pick_config_f32(int64_t M, int64_t N, int64_t K, bool vec_ok) {
    (void)K;
    if (!vec_ok) return 0;
    if (M >= 128 && N >= 128) return 1;
    return 0;
}

}  // namespace mfg
