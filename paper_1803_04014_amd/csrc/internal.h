// internal.h -- private declarations shared by libmfgemm's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include <cstddef>
#include <cstdint>

#include "mfgemm.h"

namespace mfg {

// Records a failed HIP call for mfg_last_hip_error() (per thread) and
// returns MFG_ERR_HIP.
int hip_fail(hipError_t e);

#define MFG_HIP_CHECK(call)                                    \
    do {                                                       \
        hipError_t mfg_e_ = (call);                            \
        if (mfg_e_ != hipSuccess) return ::mfg::hip_fail(mfg_e_); \
    } while (0)

// After a kernel launch: report a launch error.
#define MFG_LAUNCH_CHECK() MFG_HIP_CHECK(hipGetLastError())

// Per-(device, stream) workspace.  Returns a device pointer holding at least
// `bytes`, or nullptr with *status set.  The region stays valid until the
// next workspace() call on the same stream; growing it synchronises the
// stream before freeing the old region.
void* workspace(hipStream_t s, size_t bytes, int* status);
// A second, independent per-stream region for reduction partials.
void* partials_ws(hipStream_t s, size_t bytes, int* status);
// Number of compute units of the current device (cached).
int device_cu_count();

// -------------------------------------------------------------- arguments
// One GEMM (or a strided batch of them) on 16-bit planes.  A[p] / B[p] are
// the head (p = 0) and scaled-residual (p = 1) planes.
struct Gemm16Args {
    int64_t M, N, K;
    const uint16_t* A[2];
    const uint16_t* B[2];
    float* C;
    int64_t lda, ldb, ldc;
    int64_t sA, sB, sC;  // batch strides (elements)
    float alpha, beta;
};

struct GemmF32Args {
    int64_t M, N, K;
    const float* A;
    const float* B;
    float* C;
    int64_t lda, ldb, ldc;
    int64_t sA, sB, sC;
    float alpha, beta;
};

struct GemmF8Args {
    int64_t M, N, K;
    const uint8_t* A;    // codes
    const uint8_t* B;
    const uint8_t* Bt;   // B's codes transposed (N x K, ld ldbt), for the tiled kernels
    int64_t ldbt;
    const float* sa;     // ceil(M/128) x ceil(K/128)
    const float* sb;     // ceil(K/128) x ceil(N/128)
    float* C;
    int64_t lda, ldb, ldc;
    float alpha, beta;
};

// Kernel families.  `kind` selects the operand format and products:
// K_BF16_SPLIT3: Eq. 2 without R_A R_B on BF16 head and unscaled BF16 residual planes.
enum Kind16 { K_F16 = 0, K_BF16 = 1, K_REFINE_A = 2, K_SPLIT3 = 3, K_SPLIT4 = 4, K_BF16_SPLIT3 = 5 };

// Tile configurations (index 0 is always the simple one-wave-per-32x32 kernel).
int num_configs16(int kind);
const char* config16_name(int kind, int cfg);
int pick_config16(int kind, int64_t M, int64_t N, int64_t K, bool vec_ok);
int launch_gemm16(int kind, int cfg, const Gemm16Args& a, int64_t batch, bool vec_ok, hipStream_t s);
// Whether a configuration serves a problem (its launch would not return
// MFG_ERR_UNSUPPORTED); a tuned choice that does not is replaced by the
// default.  vec_ok: 16-byte aligned rows of A and B (FP8: of A's codes).
bool config16_ok(int kind, int cfg, int64_t M, int64_t N, int64_t K, int64_t ldc, bool vec_ok);
bool config_f32_ok(int cfg, int64_t ldc, bool vec_ok);

// Refined GEMMs straight from FP32 operands, split while staged (fused.hip).
// Their configurations follow the plane kernels' in a kind's menu.
struct FusedArgs {
    int64_t M, N, K;
    const float* A;
    const float* B;
    float* C;
    int64_t lda, ldb, ldc;
    float alpha, beta;
};
int num_configs_fused(int kind);
const char* config_fused_name(int kind, int cfg);
bool fused_ok(int kind, int cfg, const FusedArgs& a);
int launch_gemm_fused(int kind, int cfg, const FusedArgs& a, hipStream_t s);
bool config_f8_ok(int cfg, int64_t M, int64_t N, int64_t K, int64_t ldc, bool vec_ok);

int num_configs_f32();
const char* config_f32_name(int cfg);
int pick_config_f32(int64_t M, int64_t N, int64_t K, bool vec_ok);
int launch_gemm_f32(int cfg, const GemmF32Args& a, int64_t batch, bool vec_ok, hipStream_t s);

int num_configs_f8();
const char* config_f8_name(int cfg);
int pick_config_f8(int64_t M, int64_t N, int64_t K, bool vec_ok);
int launch_gemm_f8(int cfg, const GemmF8Args& a, bool vec_ok, hipStream_t s);
bool f8_config_needs_bt(int cfg);
int launch_transpose_b8(int64_t rows, int64_t cols, const uint8_t* src, int64_t lds, uint8_t* dst, int64_t ldd,
                        hipStream_t s);

// Conversions (convert.hip).
int launch_round_f16(int64_t rows, int64_t cols, const float* X, int64_t ldx, uint16_t* out,
                     int64_t ldo, hipStream_t s);
int launch_round_bf16(int64_t rows, int64_t cols, const float* X, int64_t ldx, uint16_t* out,
                      int64_t ldo, hipStream_t s);
int launch_split_f16(int64_t rows, int64_t cols, const float* X, int64_t ldx, uint16_t* head,
                     uint16_t* resid, int64_t ldo, double* norms, hipStream_t s);
int launch_split_bf16(int64_t rows, int64_t cols, const float* X, int64_t ldx, uint16_t* head,
                      uint16_t* resid, int64_t ldo, double* norms, hipStream_t s);
int launch_split6_bf16(int64_t rows, int64_t cols, const float* X, int64_t ldx, uint16_t* out, int64_t ldo,
                       int64_t kp, bool side_b, hipStream_t s);
int launch_quantize_fp8(int64_t rows, int64_t cols, const float* X, int64_t ldx, uint8_t* codes,
                        int64_t ldo, float* scales, hipStream_t s);
// The same codes written transposed (code of X[r][c] at codes_t[c * ldt + r]),
// scales in the untransposed tile order.
int launch_quantize_fp8_t(int64_t rows, int64_t cols, const float* X, int64_t ldx, uint8_t* codes_t, int64_t ldt,
                          float* scales, hipStream_t s);
// Conversion job lists (grouped plans over FP32 operands): job = one matrix,
// rows x cols FP32 at src (ld lds) into 16-bit dst (ld ldo); kind 0 rne16,
// 1 rnebf16, 2 FP16 split (head at dst, scaled residual at dst + plane),
// 3 BF16 split (unscaled residual).  Task =
// rpt rows of one job (one workgroup): about kJobChunks four-element pieces.
constexpr int kJobChunks = 512;
struct ConvJob {
    const float* src;
    uint16_t* dst;
    int64_t lds, ldo, rows, cols, plane;
    int32_t kind, vec;  // vec: src rows 16-byte aligned (whole four-float loads)
    int32_t rpt, pad;   // rows per task
};
inline int32_t conv_rows_per_task(int64_t rows, int64_t cols) {
    const int64_t cpr = (cols + 3) / 4, r = kJobChunks / (cpr > 0 ? cpr : 1);
    return (int32_t)(r < 1 ? 1 : (r < rows ? r : rows));
}
struct ConvTask {
    int32_t job, row0;
};
int launch_convert_jobs(const ConvJob* jobs, const ConvTask* tasks, int64_t ntasks, hipStream_t s);
int launch_error_norms(int64_t M, int64_t N, const float* C, int64_t ldc, const double* R,
                       int64_t ldr, double* out4, hipStream_t s);
int launch_count_mismatch(int64_t M, int64_t N, const float* C, int64_t ldc, const float* R,
                          int64_t ldr, unsigned long long* out, hipStream_t s);
int launch_scale_c(int64_t M, int64_t N, float* C, int64_t ldc, float beta, int64_t batch,
                   int64_t sC, hipStream_t s);

// Batched and grouped launches (batched.hip).
struct GroupedDesc {  // one problem (host side; the kernel reads GroupedWork)
    int64_t M, N, K, lda, ldb, ldc;
    const uint16_t* A;
    const uint16_t* B;
    float* C;
    int32_t vec;  // 1: 16-byte aligned rows and ld a multiple of 8 (whole 16-byte loads)
    int32_t pad;
    int64_t pa, pb;  // refined kinds: element offsets of the residual planes of A and B (else 0)
};
// Tiled kernels address C with 32-bit buffer offsets within a 32-row block:
// ldc must stay below this bound for them; larger ldc uses the simple
// kernels (single 32 x 32 blocks, 64-bit addressing).
constexpr int64_t kBufferLdcLimit = int64_t(1) << 24;
inline bool buffer_ldc_ok(int64_t ldc) { return ldc < kBufferLdcLimit; }
// The 64-wide pipelined kernels address a tile's operand rows with 32-bit
// byte offsets from its corner (at most 256 rows of A, 64 of B): lda and
// ldb must stay below this bound for the tiled 16-bit kernels; larger ones
// use the simple kernels.
constexpr int64_t kOperandLdLimit = int64_t(1) << 22;
inline bool operand_ld_ok(int64_t lda, int64_t ldb) { return lda < kOperandLdLimit && ldb < kOperandLdLimit; }
// Likewise for the FP8 tiled kernel's code rows (A and transposed B, bytes;
// up to 256 rows per tile).
constexpr int64_t kF8LdLimit = int64_t(1) << 24;

// Output tile classes of the grouped kernel (one workgroup per tile): 128 or
// 64 a side.  Without a tuned entry a problem takes its kind's default.
constexpr int kGroupedTile = 128;        // default for F16, BF16
constexpr int kGroupedTileRefined = 64;  // default for REFINE_A, SPLIT3, SPLIT4, BF16_SPLIT3 (two planes in LDS)
inline int grouped_tile(int kind) { return kind >= K_REFINE_A ? kGroupedTileRefined : kGroupedTile; }
bool grouped_tile_ok(int kind, int tile);
// The classes of a kind, its default first; returns their number (<= 2).
int grouped_tiles(int kind, int* tiles);
// Tuned-table entries of grouped tile classes use mode kGroupedTuneBase + mode
// (config = tile side).
constexpr int kGroupedTuneBase = 32;
// One tile x tile output tile with everything its workgroup
// reads (16 dwords, so that 16 lanes fetch one record with one load each).
struct GroupedWork {
    const uint16_t* A;  // row m0 of the problem's A
    const uint16_t* B;  // column n0 of its B
    float* C;           // element (m0, n0) of its C
    int64_t lda, ldb, ldc;
    int32_t rows, cols;  // of the tile inside the problem: min(tile, M - m0), min(tile, N - n0)
    int32_t K, vec;
};
static_assert(sizeof(GroupedWork) == 64, "a work record is 16 dwords");
int launch_batched_small(int kind, const Gemm16Args& a, int64_t count, bool vec_ok, int num_cu,
                         hipStream_t s);
// Work list of a grouped launch, split into one contiguous range per XCD
// (workgroup b runs on XCD b % kXcds): each problem's tiles stay on one XCD,
// so its operands are fetched into one L2.
constexpr int kXcds = 8;
struct GroupedSplit {
    int64_t off[2][kXcds + 1];  // list 0: aligned rows (vec), ldc < kBufferLdcLimit, lda and ldb < kOperandLdLimit; list 1: the rest
};
// `planes` (if not null) receives two int64 per work item, in work order:
// the problem's residual-plane offsets pa, pb.
// `tile`: the output tile side of the kind that will run the list (grouped_tile).
void build_grouped_work(const GroupedDesc* descs, int64_t n, std::vector<GroupedWork>& work, GroupedSplit& split,
                        std::vector<int64_t>* planes = nullptr, int tile = kGroupedTile);
// One launch per non-empty list (the grid of each from grouped_grid) of the
// tile class `tile` (the one the list was built for).  The refined kinds need
// `planes` in device memory, as build_grouped_work wrote it; F16 / BF16
// ignore it (may be null).
int grouped_launch(int kind, int tile, const GroupedWork* work, const int64_t* planes, const GroupedSplit& split,
                   float alpha, float beta, hipStream_t s);
// Workgroups of a list's launch (a multiple of kXcds).
int grouped_grid(const GroupedSplit& split, int list, int kind, int tile);

// Validation (validate.cpp; pure host code).
int validate_gemm(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B,
                  int64_t ldb, const void* C, int64_t ldc, int mode);
int validate_matrix(int64_t rows, int64_t cols, const void* X, int64_t ld);

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace mfg
