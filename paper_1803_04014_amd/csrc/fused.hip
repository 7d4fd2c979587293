// fused.hip -- the refined GEMMs (paper Sec. V, Eq. 1 and Eq. 2) straight
// from FP32 operands: the split of Eq. R happens while a tile is staged into
// LDS, so no head or residual plane is ever written to HBM and the call
// needs no workspace.
//
// Each workgroup computes a BM x BN tile over K steps of 64 with two LDS
// stages, in the LDS layout of fast16.h (head and residual planes of A and
// B, swizzled 16-byte chunks), and runs eight wavefronts, two per SIMD:
//   - four matrix wavefronts (a 2 x 2 grid over the tile) read the operand
//     fragments of step t from its stage and issue the MFMAs;
//   - four conversion wavefronts issue the global loads of the FP32 sources
//     of step t+2 into one set of staging registers, convert step t+1
//     (loaded one step earlier into the other set) into head and residual
//     chunks and write them into the other stage;
//   - one barrier per step, after each wavefront's own LDS traffic is done.
// The SIMD interleaves its two wavefronts, so the conversion's VALU work
// runs beside the MFMAs (the paper's closing suggestion of vector units
// working next to the matrix units, Sec. VIII), and the loads have a whole
// K step to arrive.
//
// The element conversions are cvt.h's formulas, the chunk layout and the
// fragment reads those of the two-pass kernels, and the MFMAs the same
// mma_step in the same order, so every output is bitwise the two-pass result
// (split pass, then the GEMM on the planes) for operands without NaN.
// Requirements: K % 64 == 0, N % 4 == 0 and N >= 4 (a lane's four columns
// are wholly inside or wholly outside B), A and B 16-byte aligned with
// lda % 4 == 0 and ldb % 4 == 0, lda and ldb below 2^22 (the per-lane
// offsets stay in 31 bits), ldc < 2^24.
#include "cvt.h"
#include "fast16.h"
#include "runtime.h"

namespace mfg {

namespace {

constexpr int kFusedBK = 64;

// Global-memory view of the FP32 sources (global_load, counted by vmcnt only;
// a generic pointer would give flat loads, which the LDS counter waits of the
// K loop would also wait for).
typedef __attribute__((address_space(1))) const f32x4 g_f32x4;

// FP32 sources of one K step held by one lane of a conversion wavefront:
// 4 consecutive values of each of PIECES rows of A and of B.
template <class F>
struct FusedRegs {
    static constexpr int PIECES = 8;
    f32x4 a[PIECES];
    f32x4 b[PIECES];
};

// The loads of a conversion wavefront (index cid of NW) and where their
// values go in LDS.  Every load instruction reads 1 KB of contiguous row
// segments: A (BM x 64 FP32, 256 bytes a row) 4 rows at a time, lane l at
// row 4 i + l / 16, columns 4 (l % 16) .. +3; B (64 x BN FP32, 512 bytes a
// row for BN = 128) 2 rows at a time, lane l at row 2 i + l / 32, columns
// 4 (l % 32) .. +3.  The 4 converted values of a lane are one 8-byte half of
// a 16-byte chunk of the 16-bit tile, placed by the chunk swizzles of
// fast16.h.  Global addressing is split as in P64Loader: per-lane byte
// offsets from the tile corner fixed for the K loop, a per-step K offset in
// scalar registers.  Rows past M repeat row M - 1 and columns past N repeat
// the last four (N % 4 == 0): they feed only outputs that are not stored.
template <class F>
struct FusedLoader {
    static constexpr int P = FusedRegs<F>::PIECES;
    static_assert(F::BK == 64 && F::A_PLANE == 128 * 64 && F::B_PLANE == 64 * 128 && F::NW == 4, "the 128 x 128 x 64 tile");
    const char* a;  // A + m0 * lda (uniform)
    const char* b;  // B + n0 (uniform)
    int64_t ldb4;   // B row pitch in bytes
    int32_t offa[P], offb[P];  // bytes from the corner
    int32_t lda_[P], ldb_[P];  // LDS destinations (16-bit elements from the stage start)

    __device__ __forceinline__ void init(const float* A, const float* B, int64_t lda, int64_t ldb, int64_t M,
                                         int64_t N, int64_t m0, int64_t n0, int cid, int lane) {
        a = (const char*)uniform64((int64_t)(A + m0 * lda));
        b = (const char*)uniform64((int64_t)(B + n0));
        ldb4 = uniform64(ldb * 4);
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int r = cid * 32 + i * 4 + (lane >> 4), k = (lane & 15) * 4;
            const int64_t gm = m0 + r < M ? m0 + r : M - 1;
            offa[i] = (int32_t)(((gm - m0) * lda + k) * 4);
            lda_[i] = r * 64 + (((k >> 3) ^ swz<8>(r)) << 3) + (k & 7);
        }
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int kr = cid * 16 + i * 2 + (lane >> 5), n = (lane & 31) * 4;
            const int64_t gn = n0 + n + 4 <= N ? n0 + n : N - 4;
            offb[i] = (int32_t)((kr * ldb + (gn - n0)) * 4);
            ldb_[i] = F::NPA * F::A_PLANE + kr * 128 + (((n >> 3) ^ swzB(kr)) << 3) + (n & 7);
        }
    }

    __device__ __forceinline__ void load(int64_t k0, FusedRegs<F>& r) const {
        const int64_t ka = uniform64(k0 * 4), kb = uniform64(k0 * ldb4);
#pragma unroll
        for (int i = 0; i < P; ++i) r.a[i] = *(const g_f32x4*)(a + ka + offa[i]);
#pragma unroll
        for (int i = 0; i < P; ++i) r.b[i] = *(const g_f32x4*)(b + kb + offb[i]);
    }
};

// Four FP32 values -> four 16-bit heads and, with SPLIT, four residuals,
// as the split (and rounding) passes compute each finite element: head =
// RNE(x), residual = RNE((x - head) * 2^11) for FP16, RNE(x - head) for
// BF16, the difference exact in FP32.  Pairs go through gfx950's packed
// conversions (v_cvt_pk_f16_f32 / v_cvt_pk_bf16_f32, round to nearest even),
// which write the MFMA operand's packed layout directly.  (A NaN input gives
// a NaN head whose payload may differ from the passes' sign-keeping quiet
// NaN; every product with it is NaN either way.)
template <bool BF, bool SPLIT>
__device__ __forceinline__ void split4(const f32x4& v, u32x2& h, u32x2& r) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    uint32_t hw[2], rw[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const f2 x = {v[2 * j], v[2 * j + 1]};
        if constexpr (BF) {
            const b2 hh = __builtin_convertvector(x, b2);
            hw[j] = __builtin_bit_cast(uint32_t, hh);
            if constexpr (SPLIT) rw[j] = __builtin_bit_cast(uint32_t, __builtin_convertvector(x - __builtin_convertvector(hh, f2), b2));
        } else {
            const h2 hh = __builtin_convertvector(x, h2);
            hw[j] = __builtin_bit_cast(uint32_t, hh);
            if constexpr (SPLIT)
                rw[j] = __builtin_bit_cast(uint32_t, __builtin_convertvector((x - __builtin_convertvector(hh, f2)) * 2048.0f, h2));
        }
        if constexpr (!SPLIT) rw[j] = 0u;
    }
    h = u32x2{hw[0], hw[1]};
    r = u32x2{rw[0], rw[1]};
}

// Convert the staged sources of one K step and write them into LDS stage
// `st` (head plane, then residual plane where the kind splits the operand).
template <int KIND, class F>
__device__ __forceinline__ void fused_store(uint16_t* st, const FusedLoader<F>& ld, const FusedRegs<F>& r) {
    using T = KT<KIND>;
#pragma unroll
    for (int i = 0; i < FusedRegs<F>::PIECES; ++i) {
        u32x2 h, q;
        split4<T::BF, (T::NPA == 2)>(r.a[i], h, q);
        *reinterpret_cast<u32x2*>(st + ld.lda_[i]) = h;
        if constexpr (T::NPA == 2) *reinterpret_cast<u32x2*>(st + ld.lda_[i] + F::A_PLANE) = q;
    }
#pragma unroll
    for (int i = 0; i < FusedRegs<F>::PIECES; ++i) {
        u32x2 h, q;
        split4<T::BF, (T::NPB == 2)>(r.b[i], h, q);
        *reinterpret_cast<u32x2*>(st + ld.ldb_[i]) = h;
        if constexpr (T::NPB == 2) *reinterpret_cast<u32x2*>(st + ld.ldb_[i] + F::B_PLANE) = q;
    }
}

__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this wavefront's LDS reads and writes done
    __builtin_amdgcn_s_barrier();
}

template <int KIND, int BM, int BN, int WM, int WN>
struct Fused {
    using T = KT<KIND>;
    using F = FastCfg<KIND, BM, BN, WM, WN, false, kFusedBK>;
    static constexpr int FM = F::FM, FN = F::FN, KK = kFusedBK / 16, NW = WM * WN;

    // Operand fragments of one 16-deep chunk kk of the stage at `cur`.
    static __device__ __forceinline__ void read(const uint16_t* cur, int kk, int wm, int wn, int lane,
                                                u32x4 (&af)[FM][2], u32x4 (&bf)[FN][2]) {
        const int c = kk * 2 + (lane >> 5);
#pragma unroll
        for (int fm = 0; fm < FM; ++fm) {
            const int row = wm * F::TMW + fm * 32 + (lane & 31);
#pragma unroll
            for (int q = 0; q < 2; ++q)
                af[fm][q] = (q < T::NPA) ? *reinterpret_cast<const u32x4*>(cur + q * F::A_PLANE + row * kFusedBK +
                                                                           ((c ^ swz<F::CPR>(row)) * 8))
                                         : zero4();
        }
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
#pragma unroll
            for (int q = 0; q < 2; ++q)
                bf[fn][q] = (q < T::NPB) ? read_b_tr<BN>(cur, T::NPA * F::A_PLANE + q * F::B_PLANE, kk * 16,
                                                         wn * F::TNW + fn * 32, lane)
                                         : zero4();
    }

    // Matrix wavefront, one K step: the MFMAs of the stage at `cur`, one
    // 16-deep chunk at a time, the fragments of chunk kk+1 read while those
    // of chunk kk are in use.
    static __device__ __forceinline__ void mma(const uint16_t* cur, int wm, int wn, int lane, f32x16 (&hi)[FM][FN],
                                               f32x16 (&lo)[FM][FN], f32x16 (&rr)[FM][FN]) {
        u32x4 af[2][FM][2], bf[2][FN][2];
        read(cur, 0, wm, wn, lane, af[0], bf[0]);
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
            if (kk + 1 < KK) read(cur, kk + 1, wm, wn, lane, af[(kk + 1) & 1], bf[(kk + 1) & 1]);
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < FN; ++fn)
                    mma_step<KIND>(af[kk & 1][fm], bf[kk & 1][fn], hi[fm][fn], lo[fm][fn], rr[fm][fn]);
        }
        lds_barrier();
    }

    // Conversion wavefront, one K step: issue the loads of step t+2 into
    // `rfree` (load), convert step t+1 from `rnext` into the other stage
    // (store).  The conditions are the same in every lane.
    static __device__ __forceinline__ void convert(int64_t t, uint16_t* lds, const FusedLoader<F>& ld,
                                                   FusedRegs<F>& rnext, FusedRegs<F>& rfree, bool load, bool store) {
        if (load) ld.load((t + 2) * kFusedBK, rfree);
        if (store) fused_store<KIND, F>(lds + ((t + 1) & 1) * F::STAGE, ld, rnext);
        lds_barrier();
    }
};

// Two wavefronts per SIMD with different roles: wavefronts 0 .. NW-1 (the
// WM x WN grid over the tile) only read operand fragments and issue MFMAs;
// wavefronts NW .. 2 NW-1 only load FP32 sources, split them and write the
// LDS stages.  The SIMD interleaves the two instruction streams, so the
// conversion's VALU work runs while the matrix core is busy with the other
// wavefront's MFMAs (with one wavefront per SIMD doing both, the in-order
// issue serialises them).  Both roles pass the same barriers: one after the
// first stage is written, then one per K step.
template <int KIND, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(128 * WM * WN, 1) void gemm_fused_split(FusedArgs p, int tiles_m, int tiles_n,
                                                                     int group_m) {
    using S = Fused<KIND, BM, BN, WM, WN>;
    using F = typename S::F;
    using T = KT<KIND>;
    constexpr int FM = S::FM, FN = S::FN, NW = S::NW;
    extern __shared__ __attribute__((aligned(16))) uint16_t lds[];
    int tm, tn;
    raster(xcd_remap(blockIdx.x, gridDim.x), tiles_m, tiles_n, group_m, tm, tn);
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t KTN = uniform64(p.K / kFusedBK);

    if (wid < NW) {
        const int wm = wid / WN, wn = wid % WN;
        f32x16 hi[FM][FN], lo[FM][FN], rr[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                hi[i][j] = f32x16{};
                if constexpr (T::LO) lo[i][j] = f32x16{};
                if constexpr (T::RR) rr[i][j] = f32x16{};
            }
        lds_barrier();  // the first stage is written
        for (int64_t t = 0; t < KTN; ++t) S::mma(lds + (t & 1) * F::STAGE, wm, wn, lane, hi, lo, rr);
        store_tile<FM, FN>(p.C, p.ldc, p.M, p.N, m0 + wm * F::TMW, n0 + wn * F::TNW, lane, p.alpha, p.beta,
                           [&](int fm, int fn, int i) { return combine_at<KIND>(hi[fm][fn], lo[fm][fn], rr[fm][fn], i); });
        return;
    }

    const int cid = wid - NW;
    FusedLoader<F> ld;
    ld.init(p.A, p.B, p.lda, p.ldb, p.M, p.N, m0, n0, cid, lane);
    FusedRegs<F> r0, r1;  // set t % 2 holds step t
    ld.load(0, r0);
    if (KTN > 1) ld.load(kFusedBK, r1);
    fused_store<KIND, F>(lds, ld, r0);
    lds_barrier();
    for (int64_t t = 0; t < KTN; t += 2) {
        S::convert(t, lds, ld, r1, r0, t + 2 < KTN, t + 1 < KTN);
        if (t + 1 < KTN) S::convert(t + 1, lds, ld, r0, r1, t + 3 < KTN, t + 2 < KTN);
    }
}

template <int KIND>
int launch_fused_kind(const FusedArgs& a, int group_m, hipStream_t s) {
    constexpr int BM = 128, BN = 128, WM = 2, WN = 2;
    using F = FastCfg<KIND, BM, BN, WM, WN, false, kFusedBK>;
    auto kern = gemm_fused_split<KIND, BM, BN, WM, WN>;
    static bool attr_set = false;  // benign race: the attribute call is idempotent
    if (!attr_set) {
        MFG_HIP_CHECK(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          2 * F::STAGE * 2));
        attr_set = true;
    }
    const int tiles_m = (int)cdiv(a.M, BM), tiles_n = (int)cdiv(a.N, BN);
    hipLaunchKernelGGL(kern, dim3(tiles_m * tiles_n), dim3(128 * WM * WN), 2 * F::STAGE * 2, s, a, tiles_m, tiles_n,
                       group_m);
    MFG_LAUNCH_CHECK();
    return MFG_OK;
}

const char* const kFusedNames[] = {"fused128x128k64w2x2c4g8"};

}  // namespace

// SPLIT4 keeps a third accumulator block, which leaves no registers for two
// staging sets: it runs two-pass only.
int num_configs_fused(int kind) {
    return (kind == K_REFINE_A || kind == K_SPLIT3 || kind == K_BF16_SPLIT3) ? 1 : 0;
}

const char* config_fused_name(int kind, int cfg) {
    return (cfg >= 0 && cfg < num_configs_fused(kind)) ? kFusedNames[cfg] : nullptr;
}

bool fused_ok(int kind, int cfg, const FusedArgs& a) {
    if (cfg < 0 || cfg >= num_configs_fused(kind)) return false;
    const bool al = ((uintptr_t)a.A & 15u) == 0 && ((uintptr_t)a.B & 15u) == 0;
    return al && a.M >= 1 && a.K % kFusedBK == 0 && a.K > 0 && a.N % 4 == 0 && a.N >= 4 && a.lda % 4 == 0 &&
           a.ldb % 4 == 0 && a.lda < ((int64_t)1 << 22) && a.ldb < ((int64_t)1 << 22) && buffer_ldc_ok(a.ldc) &&
           a.M <= ((int64_t)1 << 30) && a.N <= ((int64_t)1 << 30) && cdiv(a.M, 128) * cdiv(a.N, 128) <= INT32_MAX;
}

int launch_gemm_fused(int kind, int cfg, const FusedArgs& a, hipStream_t s) {
    if (!fused_ok(kind, cfg, a)) return MFG_ERR_UNSUPPORTED;
    if (fault_hit(kFaultLaunch)) return hip_fail(hipErrorLaunchFailure);  // injected (tests)
    switch (kind) {
        case K_REFINE_A: return launch_fused_kind<K_REFINE_A>(a, 8, s);
        case K_SPLIT3: return launch_fused_kind<K_SPLIT3>(a, 8, s);
        case K_BF16_SPLIT3: return launch_fused_kind<K_BF16_SPLIT3>(a, 8, s);
        default: return MFG_ERR_UNSUPPORTED;
    }
}

}  // namespace mfg
