// gemm16.hip -- GEMM on 16-bit operand planes with FP32 accumulation on the
// gfx950 matrix cores (v_mfma_f32_32x32x16_{f16,bf16}).
//
// Paper Sec. IV: C = alpha*A*B + beta*C on matrix units, FP16 inputs and FP32
// accumulation.  Paper Sec. V, Eq. 1 and Eq. 2: the refined products
//   REFINE_A : A_h B_h + (R_A B_h) / s
//   SPLIT3   : A_h B_h + (A_h R_B + R_A B_h) / s
//   SPLIT4   : SPLIT3 + (R_A R_B) / s^2
// fused into one K loop.  A_h B_h accumulates in `hi`, the residual products
// in `lo` (and R_A R_B in `rr`), each in FP32; the epilogue folds them with
// the exact scale 2^-11.  One launch replaces the paper's chain of four GEMM
// calls, so C is written once.
//
// Every kernel here accumulates an output element over K in the same order
// (16-wide chunks k0 = 0, 16, 32, ...; within a chunk, products in the
// order fixed above) and applies the same epilogue, so all tile
// configurations of a kind give bitwise-identical results.
#include "fast16.h"
#include "pipe16.h"
#include "runtime.h"
#include "tile16.h"

namespace mfg {

// ---------------------------------------------------------------------------
// Configuration tables and launch.
// ---------------------------------------------------------------------------
struct Cfg16 {
    const char* name;
    int bm, bn;  // 0, 0 = simple kernel
    int group_m;
    int fast;    // 0: tile16 kernel; 1: fast kernel, loads via VGPRs; 2: fast kernel, loads straight to LDS;
                 // 3: pipelined kernel, 4 stages; 5: fast kernel with BK = 32, loads straight to LDS;
                 // 6: as 5 with a register budget for 2 (or 4) wavefronts per SIMD;
                 // 7: pipelined kernel with 64-wide LDS stages (2 or 3); 8: the
                 //    same with the LDS reads spread evenly over the MFMAs
    int wm, wn;  // wavefront grid of the fast kernel
};

template <int KIND, int BM, int BN, int WM, int WN, bool DMA, int BK = 64, int OCC = 1>
static int launch_fast(const Gemm16Args& a, int64_t batch, int group_m, hipStream_t s) {
    using G = FastCfg<KIND, BM, BN, WM, WN, DMA, BK>;
    auto kern = gemm16_fast<KIND, BM, BN, WM, WN, DMA, BK, OCC>;
    static bool attr_set = false;
    if (!attr_set) {
        MFG_HIP_CHECK(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          G::LDS_BYTES));
        attr_set = true;
    }
    const int tiles_m = (int)cdiv(a.M, BM), tiles_n = (int)cdiv(a.N, BN);
    dim3 grid(tiles_m * tiles_n, (unsigned)batch, 1);
    hipLaunchKernelGGL(kern, grid, dim3(G::NT), G::LDS_BYTES, s, a, tiles_m, tiles_n, group_m);
    MFG_LAUNCH_CHECK();
    return MFG_OK;
}

template <int KIND, int BM, int BN, int WM, int WN, int S>
static int launch_pipe(const Gemm16Args& a, int64_t batch, int group_m, hipStream_t s) {
    using G = PipeCfg<KIND, BM, BN, WM, WN, S>;
    const int tiles_m = (int)cdiv(a.M, BM), tiles_n = (int)cdiv(a.N, BN);
    dim3 grid(tiles_m * tiles_n, (unsigned)batch, 1);
    hipLaunchKernelGGL((gemm16_pipe<KIND, BM, BN, WM, WN, S>), grid, dim3(G::NT), 0, s, a, tiles_m, tiles_n, group_m);
    MFG_LAUNCH_CHECK();
    return MFG_OK;
}

template <int KIND, int BM, int BN, int WM, int WN, int S, int KK = 2, bool EVEN = false>
static int launch_pipe64(const Gemm16Args& a, int64_t batch, int group_m, hipStream_t s) {
    using G = Pipe64Cfg<KIND, BM, BN, WM, WN, S, KK>;
    const int tiles_m = (int)cdiv(a.M, BM), tiles_n = (int)cdiv(a.N, BN);
    dim3 grid(tiles_m * tiles_n, (unsigned)batch, 1);
    hipLaunchKernelGGL((gemm16_pipe64<KIND, BM, BN, WM, WN, S, KK, EVEN>), grid, dim3(G::NT), 0, s, a, tiles_m,
                       tiles_n, group_m);
    MFG_LAUNCH_CHECK();
    return MFG_OK;
}

// The fast kernel needs K % 64 == 0, 16-byte aligned rows and N % 8 == 0, N >= 8.
static bool fast_ok(const Gemm16Args& a, bool vec_ok) {
    return vec_ok && a.K % 64 == 0 && a.N % 8 == 0 && a.N >= 8 && a.M >= 1;
}

template <int KIND, int BM, int BN, int BK, int WM, int WN>
static int launch_tiled(const Gemm16Args& a, int64_t batch, int group_m, hipStream_t s) {
    using G = TileCfg<KIND, BM, BN, BK, WM, WN>;
    auto kern = gemm16_tiled<KIND, BM, BN, BK, WM, WN>;
    static bool attr_set = false;  // benign race: the attribute call is idempotent
    if (!attr_set) {
        MFG_HIP_CHECK(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          G::LDS_BYTES));
        attr_set = true;
    }
    const int tiles_m = (int)cdiv(a.M, BM), tiles_n = (int)cdiv(a.N, BN);
    dim3 grid(tiles_m * tiles_n, (unsigned)batch, 1);
    hipLaunchKernelGGL(kern, grid, dim3(G::NT), G::LDS_BYTES, s, a, tiles_m, tiles_n, group_m);
    MFG_LAUNCH_CHECK();
    return MFG_OK;
}

template <int KIND>
static int launch_simple(const Gemm16Args& a, int64_t batch, bool vec_ok, hipStream_t s) {
    dim3 grid((unsigned)cdiv(a.N, 32), (unsigned)cdiv(a.M, 32), (unsigned)batch);
    hipLaunchKernelGGL(gemm16_simple<KIND>, grid, dim3(64), 0, s, a, vec_ok ? 1 : 0);
    MFG_LAUNCH_CHECK();
    return MFG_OK;
}

// Tile menus per kind.  Index 0 is the simple kernel.
static const Cfg16 kCfgPlain[] = {
    {"simple32", 0, 0, 0, 0, 0, 0},
    {"t256x256k64w2x2g8", 256, 256, 8, 0, 0, 0},
    {"t256x256k64w2x2g4", 256, 256, 4, 0, 0, 0},
    {"t128x128k64w2x2g8", 128, 128, 8, 0, 0, 0},
    {"t256x128k64w2x2g8", 256, 128, 8, 0, 0, 0},
    {"t128x256k64w2x2g8", 128, 256, 8, 0, 0, 0},
    {"t64x64k64w2x2g8", 64, 64, 8, 0, 0, 0},
    {"f256x256k64w2x2g8dma", 256, 256, 8, 2, 2, 2},
    {"f256x256k64w2x2g8reg", 256, 256, 8, 1, 2, 2},
    {"f256x256k64w2x4g8dma", 256, 256, 8, 2, 2, 4},
    {"f256x128k64w2x2g8dma", 256, 128, 8, 2, 2, 2},
    {"f128x128k64w2x2g8dma", 128, 128, 8, 2, 2, 2},
    {"f128x128k32w2x2g8dma", 128, 128, 8, 5, 2, 2},
    {"f256x128k32w2x2g8dma", 256, 128, 8, 5, 2, 2},
    {"f128x256k32w2x2g8dma", 128, 256, 8, 5, 2, 2},
    {"f256x128k32w2x2g8o2", 256, 128, 8, 6, 2, 2},
    {"f128x256k32w2x2g8o2", 128, 256, 8, 6, 2, 2},
    {"f128x128k32w2x2g8o4", 128, 128, 8, 6, 2, 2},
    {"f256x256k32w2x4g8dma", 256, 256, 8, 5, 2, 4},
    {"f256x256k32w2x2g8dma", 256, 256, 8, 5, 2, 2},
    {"p256x256k32s4w2x2g8", 256, 256, 8, 3, 2, 2},
    {"p256x128k32s4w2x2g8", 256, 128, 8, 3, 2, 2},
    {"p256x256k32s4w2x2g4", 256, 256, 4, 3, 2, 2},
    {"p256x256k32s4w2x2g16", 256, 256, 16, 3, 2, 2},
    {"q256x256k64s2w2x2g8", 256, 256, 8, 7, 2, 2},
    {"q256x256k64s2w2x4g8", 256, 256, 8, 7, 2, 4},
    {"q128x256k64s3w2x2g8", 128, 256, 8, 7, 2, 2},
    {"q256x128k64s3w2x2g8", 256, 128, 8, 7, 2, 2},
    {"q128x128k64s3w2x2g8", 128, 128, 8, 7, 2, 2},
    {"q256x256k64s2w2x2g8e", 256, 256, 8, 8, 2, 2},
    {"q256x128k64s3w2x2g8e", 256, 128, 8, 8, 2, 2},
};
static const Cfg16 kCfgSplit[] = {
    {"simple32", 0, 0, 0},
    {"t256x128k32w2x2g8", 256, 128, 8},
    {"t128x128k32w2x2g8", 128, 128, 8},
    {"t64x64k32w2x2g8", 64, 64, 8},
    {"f128x128k32w2x2g8dma", 128, 128, 8, 5, 2, 2},
    {"f256x128k32w2x2g8dma", 256, 128, 8, 5, 2, 2},
    {"f128x128k64w2x2g8dma", 128, 128, 8, 2, 2, 2},
    {"q128x128k64s2w2x2g8", 128, 128, 8, 7, 2, 2},
    {"q128x128k64s2w2x2g8e", 128, 128, 8, 8, 2, 2},
    {"q192x128k64s2w2x2g8e", 192, 128, 8, 8, 2, 2},
};
static const Cfg16 kCfgSplit4[] = {
    {"simple32", 0, 0, 0},
    {"t128x128k32w2x2g8", 128, 128, 8},
    {"t64x64k32w2x2g8", 64, 64, 8},
    {"f128x128k32w2x2g8dma", 128, 128, 8, 5, 2, 2},
    {"q128x128k64s2w2x2g8", 128, 128, 8, 7, 2, 2},
    {"q128x128k64s2w2x2g8e", 128, 128, 8, 8, 2, 2},
};

static const Cfg16* menu(int kind, int* n) {
    if (kind == K_F16 || kind == K_BF16) {
        *n = (int)(sizeof(kCfgPlain) / sizeof(kCfgPlain[0]));
        return kCfgPlain;
    }
    if (kind == K_SPLIT4) {
        *n = (int)(sizeof(kCfgSplit4) / sizeof(kCfgSplit4[0]));
        return kCfgSplit4;
    }
    *n = (int)(sizeof(kCfgSplit) / sizeof(kCfgSplit[0]));
    return kCfgSplit;
}

int num_configs16(int kind) {
    int n;
    menu(kind, &n);
    return n;
}

const char* config16_name(int kind, int cfg) {
    int n;
    const Cfg16* m = menu(kind, &n);
    return (cfg >= 0 && cfg < n) ? m[cfg].name : nullptr;
}

// Whether configuration `cfg` of `kind` serves this problem (launch_kind would
// not return MFG_ERR_UNSUPPORTED): the simple kernel serves every problem;
// the others need 16-byte aligned rows and ldc < kBufferLdcLimit, and the
// fast and pipelined kernels also K % 64 == 0, N % 8 == 0, N >= 8.
bool config16_ok(int kind, int cfg, int64_t M, int64_t N, int64_t K, int64_t ldc, bool vec_ok) {
    int n;
    const Cfg16* m = menu(kind, &n);
    if (cfg < 0 || cfg >= n) return false;
    if (cfg == 0) return true;
    if (!vec_ok || !buffer_ldc_ok(ldc)) return false;
    if (m[cfg].fast == 0) return true;
    return K % 64 == 0 && N % 8 == 0 && N >= 8 && M >= 1;
}

template <int KIND>
static int launch_kind(int cfg, const Gemm16Args& a, int64_t batch, bool vec_ok, hipStream_t s) {
    int n;
    const Cfg16* m = menu(KIND, &n);
    if (cfg < 0 || cfg >= n) return MFG_ERR_INVALID_ARG;
    if (cfg != 0 && (!vec_ok || !buffer_ldc_ok(a.ldc))) return MFG_ERR_UNSUPPORTED;
    const Cfg16& c = m[cfg];
    if (c.bm == 0) return launch_simple<KIND>(a, batch, vec_ok, s);
    if (c.fast == 6) {  // BK = 32 with a higher occupancy target
        if (!fast_ok(a, vec_ok)) return MFG_ERR_UNSUPPORTED;
        if constexpr (KIND == K_F16 || KIND == K_BF16) {
            if (c.bm == 256 && c.bn == 128) return launch_fast<KIND, 256, 128, 2, 2, true, 32, 2>(a, batch, c.group_m, s);
            if (c.bm == 128 && c.bn == 256) return launch_fast<KIND, 128, 256, 2, 2, true, 32, 2>(a, batch, c.group_m, s);
            if (c.bm == 128 && c.bn == 128) return launch_fast<KIND, 128, 128, 2, 2, true, 32, 4>(a, batch, c.group_m, s);
        }
        return MFG_ERR_INTERNAL;
    }
    if (c.fast == 5) {
        if (!fast_ok(a, vec_ok)) return MFG_ERR_UNSUPPORTED;
        if constexpr (KIND == K_F16 || KIND == K_BF16) {
            if (c.bm == 128 && c.bn == 128) return launch_fast<KIND, 128, 128, 2, 2, true, 32>(a, batch, c.group_m, s);
            if (c.bm == 256 && c.bn == 128) return launch_fast<KIND, 256, 128, 2, 2, true, 32>(a, batch, c.group_m, s);
            if (c.bm == 128 && c.bn == 256) return launch_fast<KIND, 128, 256, 2, 2, true, 32>(a, batch, c.group_m, s);
            if (c.bm == 256 && c.bn == 256 && c.wn == 4)
                return launch_fast<KIND, 256, 256, 2, 4, true, 32>(a, batch, c.group_m, s);
            if (c.bm == 256 && c.bn == 256) return launch_fast<KIND, 256, 256, 2, 2, true, 32>(a, batch, c.group_m, s);
        } else {
            if (c.bm == 128 && c.bn == 128) return launch_fast<KIND, 128, 128, 2, 2, true, 32>(a, batch, c.group_m, s);
            if constexpr (KIND != K_SPLIT4)
                if (c.bm == 256 && c.bn == 128) return launch_fast<KIND, 256, 128, 2, 2, true, 32>(a, batch, c.group_m, s);
        }
        return MFG_ERR_INTERNAL;
    }
    if (c.fast == 8) {  // even read interleave
        if (!fast_ok(a, vec_ok)) return MFG_ERR_UNSUPPORTED;
        if constexpr (KIND == K_F16 || KIND == K_BF16) {
            if (c.bm == 256 && c.bn == 256) return launch_pipe64<KIND, 256, 256, 2, 2, 2, 2, true>(a, batch, c.group_m, s);
            if (c.bm == 256 && c.bn == 128) return launch_pipe64<KIND, 256, 128, 2, 2, 3, 2, true>(a, batch, c.group_m, s);
        } else {
            if (c.bm == 128 && c.bn == 128) return launch_pipe64<KIND, 128, 128, 2, 2, 2, 2, true>(a, batch, c.group_m, s);
            if constexpr (KIND != K_SPLIT4)
                if (c.bm == 192 && c.bn == 128) return launch_pipe64<KIND, 192, 128, 2, 2, 2, 2, true>(a, batch, c.group_m, s);
        }
        return MFG_ERR_INTERNAL;
    }
    if (c.fast == 7) {
        if (!fast_ok(a, vec_ok)) return MFG_ERR_UNSUPPORTED;
        if constexpr (KIND == K_F16 || KIND == K_BF16) {
            if (c.bm == 256 && c.bn == 256 && c.wn == 4) return launch_pipe64<KIND, 256, 256, 2, 4, 2>(a, batch, c.group_m, s);
            if (c.bm == 256 && c.bn == 256) return launch_pipe64<KIND, 256, 256, 2, 2, 2>(a, batch, c.group_m, s);
            if (c.bm == 128 && c.bn == 256) return launch_pipe64<KIND, 128, 256, 2, 2, 3>(a, batch, c.group_m, s);
            if (c.bm == 256 && c.bn == 128) return launch_pipe64<KIND, 256, 128, 2, 2, 3>(a, batch, c.group_m, s);
            if (c.bm == 128 && c.bn == 128) return launch_pipe64<KIND, 128, 128, 2, 2, 3>(a, batch, c.group_m, s);
        } else {
            if (c.bm == 128 && c.bn == 128) return launch_pipe64<KIND, 128, 128, 2, 2, 2>(a, batch, c.group_m, s);
        }
        return MFG_ERR_INTERNAL;
    }
    if (c.fast == 3) {
        if (!fast_ok(a, vec_ok)) return MFG_ERR_UNSUPPORTED;  // K % 64 == 0 implies K % 32 == 0
        if constexpr (KIND == K_F16 || KIND == K_BF16) {
            if (c.bm == 256 && c.bn == 256) return launch_pipe<KIND, 256, 256, 2, 2, 4>(a, batch, c.group_m, s);
            if (c.bm == 256 && c.bn == 128) return launch_pipe<KIND, 256, 128, 2, 2, 4>(a, batch, c.group_m, s);
        }
        return MFG_ERR_INTERNAL;
    }
    if (c.fast) {
        if (!fast_ok(a, vec_ok)) return MFG_ERR_UNSUPPORTED;
        if constexpr (KIND == K_F16 || KIND == K_BF16) {
            if (c.bm == 256 && c.bn == 256 && c.wn == 2)
                return c.fast == 2 ? launch_fast<KIND, 256, 256, 2, 2, true>(a, batch, c.group_m, s)
                                   : launch_fast<KIND, 256, 256, 2, 2, false>(a, batch, c.group_m, s);
            if (c.bm == 256 && c.bn == 256 && c.wn == 4) return launch_fast<KIND, 256, 256, 2, 4, true>(a, batch, c.group_m, s);
            if (c.bm == 256 && c.bn == 128) return launch_fast<KIND, 256, 128, 2, 2, true>(a, batch, c.group_m, s);
            if (c.bm == 128 && c.bn == 128) return launch_fast<KIND, 128, 128, 2, 2, true>(a, batch, c.group_m, s);
        } else if constexpr (KIND != K_SPLIT4) {
            if (c.bm == 128 && c.bn == 128) return launch_fast<KIND, 128, 128, 2, 2, true>(a, batch, c.group_m, s);
        }
        return MFG_ERR_INTERNAL;
    }
    if constexpr (KIND == K_F16 || KIND == K_BF16) {
        if (c.bm == 256 && c.bn == 256) return launch_tiled<KIND, 256, 256, 64, 2, 2>(a, batch, c.group_m, s);
        if (c.bm == 128 && c.bn == 128) return launch_tiled<KIND, 128, 128, 64, 2, 2>(a, batch, c.group_m, s);
        if (c.bm == 256 && c.bn == 128) return launch_tiled<KIND, 256, 128, 64, 2, 2>(a, batch, c.group_m, s);
        if (c.bm == 128 && c.bn == 256) return launch_tiled<KIND, 128, 256, 64, 2, 2>(a, batch, c.group_m, s);
        if (c.bm == 64 && c.bn == 64) return launch_tiled<KIND, 64, 64, 64, 2, 2>(a, batch, c.group_m, s);
    } else if constexpr (KIND == K_SPLIT4) {
        if (c.bm == 128 && c.bn == 128) return launch_tiled<KIND, 128, 128, 32, 2, 2>(a, batch, c.group_m, s);
        if (c.bm == 64 && c.bn == 64) return launch_tiled<KIND, 64, 64, 32, 2, 2>(a, batch, c.group_m, s);
    } else {
        if (c.bm == 256 && c.bn == 128) return launch_tiled<KIND, 256, 128, 32, 2, 2>(a, batch, c.group_m, s);
        if (c.bm == 128 && c.bn == 128) return launch_tiled<KIND, 128, 128, 32, 2, 2>(a, batch, c.group_m, s);
        if (c.bm == 64 && c.bn == 64) return launch_tiled<KIND, 64, 64, 32, 2, 2>(a, batch, c.group_m, s);
    }
    return MFG_ERR_INTERNAL;
}

int launch_gemm16(int kind, int cfg, const Gemm16Args& a, int64_t batch, bool vec_ok, hipStream_t s) {
    if (fault_hit(kFaultLaunch)) return hip_fail(hipErrorLaunchFailure);  // injected (tests)
    switch (kind) {
        case K_F16: return launch_kind<K_F16>(cfg, a, batch, vec_ok, s);
        case K_BF16: return launch_kind<K_BF16>(cfg, a, batch, vec_ok, s);
        case K_REFINE_A: return launch_kind<K_REFINE_A>(cfg, a, batch, vec_ok, s);
        case K_SPLIT3: return launch_kind<K_SPLIT3>(cfg, a, batch, vec_ok, s);
        case K_SPLIT4: return launch_kind<K_SPLIT4>(cfg, a, batch, vec_ok, s);
        case K_BF16_SPLIT3: return launch_kind<K_BF16_SPLIT3>(cfg, a, batch, vec_ok, s);
        default: return MFG_ERR_INVALID_ARG;
    }
}

}  // namespace mfg
