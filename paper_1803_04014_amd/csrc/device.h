// device.h -- gfx950 device helpers: vector types, MFMA wrappers, LDS swizzles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

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

// A value the caller knows to be the same in every lane, made visibly so
// (scalar registers) for the compiler.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Buffer resource for raw (untyped) accesses to `bytes` bytes from `base`:
// loads at or beyond the end return 0 and stores there are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}

// Row of the 32x32 MFMA output held in element i of lane l.
__device__ __forceinline__ int mfma_out_row(int i, int lane) {
    return 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
}

// Epilogue of one row of FN 32x32 accumulator blocks of a wavefront, any
// leading dimension: block fn covers rows rbase + mfma_out_row(i, lane) and
// column cbase + 32 fn + lane % 32, value val(fn, i).  C = alpha * v when
// beta == 0 (C is not read), else fma(alpha, v, beta * C).  Every C read of
// the row of blocks is issued before any of its writes (reads go to
// clamped, always valid addresses), so the row costs one memory latency
// rather than one per element.
template <int FN, class Val, class CPtr>
__device__ __forceinline__ void store_blocks_wide(CPtr C, int64_t ldc, int64_t M, int64_t N, int64_t rbase,
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

// Addressing of one row of FN 32x32 blocks for buffer instructions:
// resource, per-element offsets (out of range outside C) and the row pitch.
template <int FN>
struct BlockAddr {
    __amdgpu_buffer_rsrc_t rs;
    int off[FN][16];
    int l4;
};

template <int FN, class CPtr>
__device__ __forceinline__ BlockAddr<FN> block_addr(CPtr C, int64_t ldc, int64_t M, int64_t N, int64_t rbase,
                                                    int64_t cbase, int lane) {
    const int64_t rb = uniform64(rbase), cb = uniform64(cbase);
    BlockAddr<FN> a;
    a.rs = buffer_rsrc((float*)C + rb * ldc + cb, (uint32_t)((31 * ldc + 32 * FN) * 4));
    a.l4 = (int)ldc * 4;
    int vo[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) vo[j] = (4 * (lane >> 5) + j) * a.l4 + (lane & 31) * 4;
    if (rb + 32 <= M && cb + 32 * FN <= N) {
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
#pragma unroll
            for (int i = 0; i < 16; ++i) a.off[fn][i] = vo[i & 3] + fn * 128;
    } else {
        constexpr int kOut = INT32_MIN;  // 2^31 as an unsigned offset: beyond any resource here
        const int64_t rows = M - rb, cols = N - cb;
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                a.off[fn][i] = (mfma_out_row(i, lane) < rows && (lane & 31) + 32 * fn < cols) ? vo[i & 3] + fn * 128
                                                                                               : kOut;
    }
    return a;
}

// C values of the blocks (0 outside C).
template <int FN>
__device__ __forceinline__ void block_load(const BlockAddr<FN>& a, float (&c)[FN][16]) {
#pragma unroll
    for (int fn = 0; fn < FN; ++fn)
#pragma unroll
        for (int i = 0; i < 16; ++i)
            c[fn][i] = __builtin_bit_cast(
                float, __builtin_amdgcn_raw_buffer_load_b32(a.rs, a.off[fn][i], 8 * (i >> 2) * a.l4, 0));
}

// C = v(fn, i) for the elements inside C.
template <int FN, class V>
__device__ __forceinline__ void block_store(const BlockAddr<FN>& a, V v) {
#pragma unroll
    for (int fn = 0; fn < FN; ++fn)
#pragma unroll
        for (int i = 0; i < 16; ++i)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v(fn, i)), a.rs, a.off[fn][i],
                                                  8 * (i >> 2) * a.l4, 0);
}

// The epilogue with buffer instructions (ldc < kBufferLdcLimit, the bound of
// 32-bit offsets over a 32-row block).  rbase and cbase are the same in
// every lane.  One buffer resource covers the row of blocks; element i of a
// lane sits at a per-lane byte offset (four of them, one per i % 4) plus a
// scalar offset of 8 (i / 4) rows, so each value costs one memory
// instruction and no address arithmetic.  Blocks that cross the edge of C
// give the elements outside it an offset beyond the resource's range: the
// hardware drops those stores and returns 0 for those loads, so there are
// no branches.  All loads of the row are issued before its stores.
template <int FN, class Val, class CPtr>
__device__ __forceinline__ void store_blocks_buf(CPtr C, int64_t ldc, int64_t M, int64_t N, int64_t rbase,
                                                 int64_t cbase, int lane, float alpha, float beta, Val val) {
    const BlockAddr<FN> a = block_addr<FN>(C, ldc, M, N, rbase, cbase, lane);
    if (beta == 0.0f) {
        block_store<FN>(a, [&](int fn, int i) { return alpha * val(fn, i); });
        return;
    }
    float c[FN][16];
    block_load<FN>(a, c);
    block_store<FN>(a, [&](int fn, int i) { return __builtin_fmaf(alpha, val(fn, i), beta * c[fn][i]); });
}

// store_blocks_buf, or for single blocks with ldc >= kBufferLdcLimit the
// 64-bit path.
template <int FN, class Val, class CPtr>
__device__ __forceinline__ void store_blocks(CPtr C, int64_t ldc, int64_t M, int64_t N, int64_t rbase,
                                             int64_t cbase, int lane, float alpha, float beta, Val val) {
    if constexpr (FN == 1) {
        if (ldc >= kBufferLdcLimit) {
            store_blocks_wide<1>(C, ldc, M, N, rbase, cbase, lane, alpha, beta, val);
            return;
        }
    }
    store_blocks_buf<FN>(C, ldc, M, N, rbase, cbase, lane, alpha, beta, val);
}

// Epilogue of a wavefront's FM x FN accumulator blocks: rows rbase + 32 fm,
// columns cbase + 32 fn, value val(fm, fn, i).  When beta != 0 and the
// whole FM x FN tile lies inside C, the C reads of block row fm + 1 are
// issued before the writes of row fm (two rows of C values in registers),
// so the tile exposes one read latency instead of one per row; otherwise
// it is store_blocks row by row.
template <int FM, int FN, class Val, class CPtr>
__device__ __forceinline__ void store_tile(CPtr C, int64_t ldc, int64_t M, int64_t N, int64_t rbase, int64_t cbase,
                                           int lane, float alpha, float beta, Val val) {
    const int64_t rb = uniform64(rbase), cb = uniform64(cbase);
    if (FM == 1 || beta == 0.0f || ldc >= kBufferLdcLimit || rb + 32 * FM > M || cb + 32 * FN > N) {
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
            store_blocks<FN>(C, ldc, M, N, rb + 32 * fm, cb, lane, alpha, beta,
                             [&](int fn, int i) { return val(fm, fn, i); });
        return;
    }
    const int l4 = (int)ldc * 4;
    const uint32_t extent = (uint32_t)((31 * ldc + 32 * FN) * 4);
    int vo[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) vo[j] = (4 * (lane >> 5) + j) * l4 + (lane & 31) * 4;
    float c[2][FN][16];
    auto load = [&](int fm, float (&d)[FN][16]) {
        const __amdgpu_buffer_rsrc_t rs = buffer_rsrc((float*)C + (rb + 32 * fm) * ldc + cb, extent);
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                d[fn][i] = __builtin_bit_cast(
                    float, __builtin_amdgcn_raw_buffer_load_b32(rs, vo[i & 3] + fn * 128, 8 * (i >> 2) * l4, 0));
    };
    load(0, c[0]);
#pragma unroll
    for (int fm = 0; fm < FM; ++fm) {
        if (fm + 1 < FM) load(fm + 1, c[(fm + 1) & 1]);
        const __amdgpu_buffer_rsrc_t rs = buffer_rsrc((float*)C + (rb + 32 * fm) * ldc + cb, extent);
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                __builtin_amdgcn_raw_buffer_store_b32(
                    __builtin_bit_cast(uint32_t, __builtin_fmaf(alpha, val(fm, fn, i), beta * c[fm & 1][fn][i])), rs,
                    vo[i & 3] + fn * 128, 8 * (i >> 2) * l4, 0);
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
