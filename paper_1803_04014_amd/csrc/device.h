// device.h -- gfx950 device helpers: vector types, MFMA wrappers, LDS swizzles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mfg {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Residual scale s = 2^11 and its inverse (exact).
constexpr float kResidInv = 1.0f / 2048.0f;

// v_mfma_f32_32x32x16_{f16,bf16}: D(32x32) += A(32x16) * B(16x32).
// Lane l supplies A row (l % 32), eight K values of group (l / 32), and B
// column (l % 32) for the same eight K values.  Lane l receives D column
// (l % 32), rows 8*(i/4) + 4*(l/32) + (i%4) in element i.
template <bool BF>
__device__ __forceinline__ f32x16 mma_32x32x16(u32x4 a, u32x4 b, f32x16 c) {
    if constexpr (BF) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    } else {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    }
}

// v_mfma_f32_32x32x2_f32: lane l supplies A[row l%32][k l/32], B[k l/32][col l%32].
__device__ __forceinline__ f32x16 mma_32x32x2_f32(float a, float b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// v_mfma_scale_f32_32x32x64_f8f6f4 with E4M3 operands (format code 0) and
// E8M0 block scales: D += (A * 2^(sa-127)) * (B * 2^(sb-127)).  Lane l
// supplies 32 codes of A row (l % 32) and of B column (l % 32).
__device__ __forceinline__ f32x16 mma_32x32x64_e4m3(i32x8 a, i32x8 b, f32x16 c, int sa, int sb) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, sa, 0, sb);
}

// Row of the 32x32 MFMA output held in element i of lane l.
__device__ __forceinline__ int mfma_out_row(int i, int lane) {
    return 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
}

// Epilogue of one row of FN 32x32 accumulator blocks of a wavefront: block
// fn covers rows rbase + mfma_out_row(i, lane) and column cbase + 32 fn +
// lane % 32, value val(fn, i).  C = alpha * v when beta == 0 (C is not
// read), else fma(alpha, v, beta * C).  Every C read of the row of blocks is
// issued before any of its writes (reads go to clamped, always valid
// addresses), so the row costs one memory latency rather than one per
// element: stores and loads to C could otherwise not be reordered.  C may
// be a generic or a global (address space 1) pointer.
template <int FN, class Val, class CPtr>
__device__ __forceinline__ void store_blocks(CPtr C, int64_t ldc, int64_t M, int64_t N, int64_t rbase,
                                             int64_t cbase, int lane, float alpha, float beta, Val val) {
    const int64_t col0 = cbase + (lane & 31);
    if (beta == 0.0f) {
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
            const int64_t col = col0 + fn * 32;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int64_t row = rbase + mfma_out_row(i, lane);
                if (row < M && col < N) C[row * ldc + col] = alpha * val(fn, i);
            }
        }
        return;
    }
    float c[FN][16];
#pragma unroll
    for (int fn = 0; fn < FN; ++fn) {
        const int64_t col = col0 + fn * 32;
        const int64_t cc = col < N ? col : N - 1;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int64_t row = rbase + mfma_out_row(i, lane);
            c[fn][i] = C[(row < M ? row : M - 1) * ldc + cc];
        }
    }
#pragma unroll
    for (int fn = 0; fn < FN; ++fn) {
        const int64_t col = col0 + fn * 32;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int64_t row = rbase + mfma_out_row(i, lane);
            if (row < M && col < N) C[row * ldc + col] = __builtin_fmaf(alpha, val(fn, i), beta * c[fn][i]);
        }
    }
}

// XOR swizzle of 16-byte chunks inside an LDS row.  Rows of 8 chunks
// (128 B): chunk c of row r lives at c ^ ((r ^ (r >> 3)) & 7), so eight
// consecutive rows read at the same logical chunk hit eight different
// 16-byte bank groups, and so do rows r and r + 8.  Rows of 4 chunks (64 B,
// two rows per 128 B): c ^ (((r >> 1) ^ (r >> 3)) & 3).
template <int CPR>
__device__ __forceinline__ int swz(int row) {
    if constexpr (CPR == 8) return (row ^ (row >> 3)) & 7;
    else if constexpr (CPR == 4) return ((row >> 1) ^ (row >> 3)) & 3;
    else return 0;
}

// Transpose an 8x8 block of 16-bit values held as 8 rows of 16 bytes:
// out[j] holds element j of in[0..7] (i.e. column j), packed low-to-high.
__device__ __forceinline__ void transpose8x8_b16(const u32x4 in[8], u32x4 out[8]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int w = j >> 1;          // 32-bit word holding element j
        const bool hi = (j & 1) != 0;  // upper half of that word
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            uint32_t lo_src = in[2 * p][w];
            uint32_t hi_src = in[2 * p + 1][w];
            // v_perm_b32 selector: bytes 0-1 from lo_src's chosen half,
            // bytes 2-3 from hi_src's chosen half.  __builtin_amdgcn_perm(a, b, sel)
            // indexes bytes of {a, b} with b as bytes 0-3 and a as bytes 4-7.
            uint32_t sel = hi ? 0x07060302u : 0x05040100u;
            out[j][p] = __builtin_amdgcn_perm(hi_src, lo_src, sel);
        }
    }
}

__device__ __forceinline__ u32x4 zero4() { return u32x4{0u, 0u, 0u, 0u}; }

}  // namespace mfg
