/*
 * mfgemm.h -- C ABI of libmfgemm, a mixed-precision GEMM library for AMD
 * Instinct MI355X (gfx950).
 *
 * The library computes the BLAS GEMM that matrix units express,
 *     C = alpha * A * B + beta * C                      (paper Sec. IV)
 * with half-precision (FP16 / BF16) or FP8 operands and FP32 accumulation on
 * the MFMA units, its batched forms (paper Sec. IV.B), and the residual-based
 * precision refinement of paper Sec. V (Eq. R, Eq. 1, Eq. 2).
 *
 * Conventions shared by every call
 *   - Matrices are row-major.  A is M x K with leading dimension lda >= K,
 *     B is K x N with ldb >= N, C is M x N FP32 with ldc >= N.  Leading
 *     dimensions count elements of the stored type.
 *   - Data pointers are device pointers (HIP device memory) unless a
 *     parameter says "host".  The caller owns every buffer it passes and must
 *     keep it alive until the stream has passed the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls are asynchronous: they validate, enqueue and return.
 *   - Every call returns an int status (MFG_OK or a negative MFG_ERR_*).
 *     Arguments are validated before anything is enqueued; on error nothing
 *     is launched and no output is touched.  No C++ exception crosses this
 *     ABI and the library never aborts the process.  After MFG_ERR_HIP the
 *     HIP error code is available from mfg_last_hip_error() (per thread).
 *   - Edge cases follow BLAS: M == 0 or N == 0 is a no-op; K == 0 or
 *     alpha == 0 gives C = beta * C; when beta == 0, C is never read (NaN or
 *     Inf already in C do not propagate).  C must not overlap A or B.
 *   - Calls are thread-safe.  The library keeps one workspace per
 *     (device, stream) for the operands it converts, grown on demand with
 *     hipMalloc and released at process exit.
 */
#ifndef MFGEMM_H
#define MFGEMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
enum {
    MFG_OK = 0,
    MFG_PENDING = 1,              /* mfg_poll: request not finished yet        */
    MFG_ERR_INVALID_ARG = -1,     /* bad size, leading dimension, pointer, mode */
    MFG_ERR_UNSUPPORTED = -2,     /* valid request the library does not serve   */
    MFG_ERR_NO_MEMORY = -3,       /* workspace or descriptor allocation failed  */
    MFG_ERR_OVER_BUDGET = -4,     /* serving: request larger than the budget    */
    MFG_ERR_HIP = -5,             /* a HIP runtime call failed                  */
    MFG_ERR_UNKNOWN_TICKET = -6,  /* serving: ticket never issued or released   */
    MFG_ERR_INTERNAL = -7
};

/* -------------------------------------------------------------------- modes
 * A mode names the operand format fed to the matrix units.  Unless the flag
 * MFG_IN_PRECONVERTED is or-ed in, A and B are FP32 and the library rounds,
 * splits or quantises them itself into its workspace (counted in the call).
 *
 *   MFG_F32           FP32 operands, FP32 MFMA (the single-precision comparator).
 *   MFG_F16           rne16(A) rne16(B), FP32 accumulate (paper Sec. V: FP32
 *                     rounded to half before the matrix-unit GEMM, Sec. VI).
 *   MFG_BF16          the same with bfloat16 operands.
 *   MFG_F16_REFINE_A  one-sided refinement, paper Eq. 1:
 *                     A_h B_h + (R_A B_h) / s, with R_A = rne16(s (A - A_h)).
 *   MFG_F16_SPLIT3    two-sided refinement, paper Eq. 2 without R_A R_B:
 *                     A_h B_h + (A_h R_B + R_A B_h) / s.
 *   MFG_F16_SPLIT4    paper Eq. 2 in full: SPLIT3 + R_A R_B / s^2.
 *   MFG_BF16_SPLIT3   Eq. 2 without R_A R_B on bfloat16 planes: head
 *                     A_h = rnebf16(A), residual R_A = rnebf16(A - A_h),
 *                     unscaled (bfloat16 keeps FP32's exponent range):
 *                     A_h B_h + A_h R_B + R_A B_h.  About 16 significant
 *                     bits per operand over FP32's whole range.
 *   MFG_FP8_E4M3      OCP E4M3 codes with one power-of-two FP32 scale per
 *                     128 x 128 tile of A (M x K) and of B (K x N).
 *   MFG_BF16_SPLIT6   the paper's Eq. R applied twice on bfloat16 planes:
 *                     h = rnebf16(A), r1 = rnebf16(A - h), r2 =
 *                     rnebf16(A - h - r1) (h + r1 + r2 == A for FP32 A
 *                     away from the subnormal range), likewise for B, and
 *                     the six products of combined order <= 2:
 *                     r2 h + r1 r1 + h r2 + r1 h + h r1 + h h, summed in one
 *                     FP32 accumulator in that order per K chunk (the
 *                     dropped r1 r2 + r2 r1 + r2 r2 is below 2^-23 |A||B|).
 *                     FP32 operands only (no preconverted form); not served
 *                     by the batched and grouped launches.
 * The residual scale is s = 2^11 (MFG_RESID_SCALE_LOG2).
 *
 * Preconverted storage forms (MFG_IN_PRECONVERTED), as written by
 * mfg_convert():
 *   F16 / BF16        16-bit matrix, ld in elements.
 *   REFINE_A          A: head plane then residual plane at A + rows*lda
 *                     elements; B: FP16 head plane only.
 *   SPLIT3 / SPLIT4   A and B: head plane then residual plane.
 *   BF16_SPLIT3       likewise, bfloat16 planes.
 *   FP8_E4M3          byte codes (ld in bytes) followed, at byte offset
 *                     mfg_fp8_scale_offset(rows, ld), by ceil(rows/128) x
 *                     ceil(cols/128) FP32 tile scales, row-major.
 *   F32               ignores the flag.
 */
enum {
    MFG_F32 = 0,
    MFG_F16 = 1,
    MFG_BF16 = 2,
    MFG_F16_REFINE_A = 3,
    MFG_F16_SPLIT3 = 4,
    MFG_F16_SPLIT4 = 5,
    MFG_FP8_E4M3 = 6,
    MFG_BF16_SPLIT3 = 7,
    MFG_BF16_SPLIT6 = 8,
    MFG_NUM_MODES = 9
};
#define MFG_IN_PRECONVERTED 0x100
/* mfg_grouped_plan_create only: A and B are FP32 (see "grouped GEMM"). */
#define MFG_IN_FP32 0x200
#define MFG_MODE_MASK 0xFF
#define MFG_RESID_SCALE_LOG2 11
#define MFG_FP8_TILE 128

/* Byte offset of the FP8 tile-scale array behind `rows x ld` code bytes. */
int64_t mfg_fp8_scale_offset(int64_t rows, int64_t ld);

/* ---------------------------------------------------------------- the GEMM
 * mfg_gemm -- C = alpha * op(A) * op(B) + beta * C in the given mode
 * (paper Sec. IV; refinement modes paper Sec. V Eq. 1 / Eq. 2).
 *   M, N, K    problem sizes (>= 0).
 *   A, lda     M x K operand, FP32 or the mode's preconverted form.
 *   B, ldb     K x N operand, likewise.
 *   C, ldc     M x N FP32, read (beta != 0) and written in place.
 *   mode       MFG_* mode, optionally | MFG_IN_PRECONVERTED.
 * Errors: MFG_ERR_INVALID_ARG for negative sizes, lda < max(1,K),
 * ldb < max(1,N), ldc < max(1,N), a NULL pointer with nonzero extent, or an
 * unknown mode; MFG_ERR_NO_MEMORY if the workspace cannot grow; MFG_ERR_HIP.
 */
int mfg_gemm(int64_t M, int64_t N, int64_t K,
             const void* A, int64_t lda,
             const void* B, int64_t ldb,
             float* C, int64_t ldc,
             float alpha, float beta, int mode, void* stream);

/* mfg_gemm_config -- mfg_gemm with an explicit tile configuration index
 * (0 <= config < mfg_num_configs(mode)), or -1 for the tuned choice.  Every
 * configuration of a mode produces bitwise-identical results: they differ
 * only in how output tiles are assigned to workgroups, never in the order in
 * which an output element accumulates its products.  Used by the autotuner.
 * For MFG_F16_REFINE_A, MFG_F16_SPLIT3 and MFG_BF16_SPLIT3 the last
 * configuration is the fused kernel: it reads the FP32 operands and splits
 * them while staging its tiles (paper Sec. V, Eq. R), so it converts nothing
 * into a workspace; it needs FP32 operands (with MFG_IN_PRECONVERTED:
 * MFG_ERR_UNSUPPORTED), K % 64 == 0, N % 4 == 0, N >= 4, 16-byte aligned A
 * and B with lda and ldb multiples of 4 below 2^22, ldc < 2^24, and reports
 * MFG_ERR_UNSUPPORTED otherwise.  Its results equal the other
 * configurations' bitwise for operands without NaN. */
int mfg_gemm_config(int64_t M, int64_t N, int64_t K,
                    const void* A, int64_t lda,
                    const void* B, int64_t ldb,
                    float* C, int64_t ldc,
                    float alpha, float beta, int mode, int config, void* stream);

/* mfg_gemm_noalloc -- mfg_gemm for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments and results (bitwise) as mfg_gemm.  The
 * operands the call converts (the FP32 inputs of the 16-bit, refined and
 * FP8 modes) go into a fixed per-device array of MFG_NOALLOC_SCRATCH_BYTES
 * that the library holds on every device it runs on until the process
 * ends, instead of the per-stream workspace: the call makes no hipMalloc,
 * hipFree or other allocating call.  A call whose converted operands need
 * more than that (e.g. FP16 from FP32 beyond about M*K + K*N = 32 Mi
 * elements, the two-plane modes beyond half that) returns
 * MFG_ERR_UNSUPPORTED before anything is enqueued -- except that REFINE_A,
 * SPLIT3 and BF16_SPLIT3 then run the fused kernel (see mfg_gemm_config)
 * when the shape allows it, which needs no array.  Every call on one device
 * shares that device's array and leaves its contents behind: calls that
 * overlap on one GPU (other streams, other threads) race, so the caller
 * orders them.  The first call on a device looks up the array's address
 * there (no allocation). */
#define MFG_NOALLOC_SCRATCH_BYTES (64ull << 20)
int mfg_gemm_noalloc(int64_t M, int64_t N, int64_t K,
                     const void* A, int64_t lda,
                     const void* B, int64_t ldb,
                     float* C, int64_t ldc,
                     float alpha, float beta, int mode, void* stream);

/* Number of tile configurations of a mode and a short text description of
 * one of them (written to `buf`, host, at most `n` bytes incl. the NUL). */
int mfg_num_configs(int mode);
int mfg_config_name(int mode, int config, char* buf, int n);

/* --------------------------------------------------------- batched GEMM
 * mfg_gemm_batched -- for b in [0, count):
 *     C_b = alpha * A_b * B_b + beta * C_b,
 * A_b = A + b*strideA, B_b = B + b*strideB, C_b = C + b*strideC (strides in
 * elements of the stored type), all problems M x N x K (paper Sec. IV.B:
 * many small GEMMs in one launch).  Modes F16, BF16 and F32 take their
 * operands directly (F16/BF16 as 16-bit data; the flag MFG_IN_PRECONVERTED
 * is implied and may be given); the refinement modes take FP32 operands and
 * split them into the workspace, or with MFG_IN_PRECONVERTED each entry in
 * the mode's preconverted storage form (head plane at A + b*strideA, its
 * residual plane at A + b*strideA + M*lda; likewise B for the two-sided
 * splits).  Any other flag is MFG_ERR_INVALID_ARG.  FP8 is not served
 * batched (MFG_ERR_UNSUPPORTED).
 */
int mfg_gemm_batched(int64_t count, int64_t M, int64_t N, int64_t K,
                     const void* A, int64_t lda, int64_t strideA,
                     const void* B, int64_t ldb, int64_t strideB,
                     float* C, int64_t ldc, int64_t strideC,
                     float alpha, float beta, int mode, void* stream);

/* --------------------------------------------------------- grouped GEMM
 * Thousands of GEMMs of different shapes in one persistent launch (paper
 * Sec. IV.B, batched GEMM, generalised to uneven shapes).  Modes MFG_F16,
 * MFG_BF16 and the refined modes (paper Sec. V, Eq. 1 and Eq. 2:
 * MFG_F16_REFINE_A, MFG_F16_SPLIT3, MFG_F16_SPLIT4); MFG_F32 and
 * MFG_FP8_E4M3 are MFG_ERR_UNSUPPORTED.  Operands are either
 *   - in the mode's preconverted storage form (the default; the flag
 *     MFG_IN_PRECONVERTED is implied): 16-bit matrices, and for the refined
 *     modes head plane then residual plane, at A + M*lda and (two-sided
 *     splits) B + K*ldb elements; or
 *   - FP32 (mode | MFG_IN_FP32): the plan owns converted copies (ld rounded
 *     up to 8) and every run first converts all problems' A and B in one
 *     launch (the paper's rounding, or the Eq. R split), then runs the
 *     grouped kernel; a graph replay holds both launches.
 * Each problem's result is bitwise that of mfg_gemm on the problem alone in
 * the same mode (preconverted, or from FP32 respectively).  The descriptor array is host memory; the plan copies it
 * to the device, so it may be freed after mfg_grouped_plan_create.
 * The grouped GEMM is a plan, not one call taking the problem list and a
 * plan in/out argument: mfg_grouped_plan_create validates the list and
 * builds the work list once, and mfg_grouped_run (or mfg_grouped_graph_launch, a
 * captured replay) executes it with a given alpha, beta as often as needed.
 */
typedef struct mfg_problem {
    int64_t M, N, K;
    int64_t lda, ldb, ldc;
    const void* A;
    const void* B;
    float* C;
} mfg_problem;

typedef struct mfg_grouped_plan mfg_grouped_plan;

/* Build a plan: validates every problem (M, N <= 2^24, K < 2^31), splits it
 * into square output tiles of its tile class (work items, one workgroup
 * each), orders each class's items by decreasing K, and uploads the work
 * list: one self-contained record per item (device memory owned by the
 * plan).  Tile classes (mfg_grouped_tile_classes): 128 and 64 for F16 /
 * BF16 / REFINE_A / SPLIT3 / BF16_SPLIT3, 64 for SPLIT4.  A problem takes
 * the class the tuned table names for its mode and size bucket (entries of
 * mode 32 + mode, config = tile side, written by mfg_grouped_autotune or
 * loaded with mfg_tune_load), else the default: 128 for F16 / BF16, 64 for
 * the refined modes.  A run launches the grouped kernel once per class
 * present; a class that would carry under a quarter of the plan's flops
 * runs in the other class instead (each launch adds its own tail).  Rows of A and B that are 16-byte
 * aligned with ld a multiple of 8 (and lda, ldb < 2^22, ldc < 2^24; other
 * problems are read element by element in a second launch of their class)
 * are read in whole 16-byte pieces, which may
 * touch up to 14 bytes past a row's last element (inside the same aligned 16
 * bytes, never another page); those bytes never reach a result.
 * `out` receives the plan (host). */
int mfg_grouped_plan_create(int64_t count, const mfg_problem* problems, int mode,
                            mfg_grouped_plan** out);
/* Run the plan once on `stream` (one persistent kernel launch). */
int mfg_grouped_run(mfg_grouped_plan* plan, float alpha, float beta, void* stream);
/* Run the plan through a HIP graph: captured on first use for (alpha, beta,
 * stream), replayed afterwards.  The graph holds the plan's launch only. */
int mfg_grouped_graph_launch(mfg_grouped_plan* plan, float alpha, float beta, void* stream);
/* Total useful flops 2*sum(M*N*K) and algorithmic bytes of one run: the
 * operands read by the grouped kernel (both planes of the refined modes) and
 * C written, plus with MFG_IN_FP32 the conversion pass (FP32 read, 16-bit
 * planes written). */
int mfg_grouped_plan_info(const mfg_grouped_plan* plan, double* flops, double* bytes,
                          int64_t* work_items);
int mfg_grouped_plan_destroy(mfg_grouped_plan* plan);
/* The grouped kernel's tile classes for `mode` (tile sides, the default
 * first) into `tiles` (host, `max` entries); returns their number. */
int mfg_grouped_tile_classes(int mode, int* tiles, int max);
/* The classes a plan launches (tile sides) and their work items, into
 * `tiles` and `items` (host, `max` entries each); returns their number. */
int mfg_grouped_plan_classes(const mfg_grouped_plan* plan, int* tiles, int64_t* items, int max);
/* Autotune the grouped tile class on the caller's problems (mode as for
 * mfg_grouped_plan_create): each class is forced on all of them and timed
 * over `reps` runs with HIP events after one warm-up run (alpha = 1,
 * beta = 0: every C is overwritten); a class counts only if every output is
 * bitwise that of the first class.  The fastest is stored in the tuned table
 * for every size bucket among the problems (tune one bucket's problems to
 * decide that bucket, or a workload's mix to decide all of its buckets) and
 * in *best_tile (host), its mean time per run in *best_ms (host). */
int mfg_grouped_autotune(int64_t count, const mfg_problem* problems, int mode, int reps, int* best_tile,
                         float* best_ms, void* stream);

/* ------------------------------------------- linear solve (a GEMM consumer)
 * Mixed-precision iterative refinement for A X = B, the technique the paper
 * sets its precision refinement beside (Sec. V): an LU factorisation whose
 * O(n^3) trailing updates run through mfg_gemm in a chosen mode (the
 * factorisation's precision), corrections solved in FP32 from FP64
 * residuals, the solution accumulated in FP64.  Row-major throughout.
 *
 * mfg_lu_factor -- in-place LU with partial pivoting of the n x n FP32
 * matrix A (device, lda >= max(1, n)): P A = L U with L unit lower (below
 * the diagonal) and U upper (on and above it), right-looking by panels of
 * 64 columns; each trailing update A22 -= L21 U12 is one mfg_gemm call with
 * `mode` (any MFG_* mode without flags: MFG_F32 for an FP32 factorisation,
 * MFG_F16 for the paper's half-precision products, a refined mode for
 * FP32-level accuracy at matrix-core speed).  ipiv (device, n int32):
 * row i was swapped with row ipiv[i] (0-based, in order i = 0 .. n-1).
 * info (host, may be NULL): 0, or the 1-based index of the first exactly
 * zero pivot (the factorisation is then complete but U is singular).  The
 * call allocates (and frees) a status word and two min(n, 8192) x 8 FP32
 * copies of 8-column sub-panels (they alternate), and synchronises `stream`
 * before it returns.
 * Errors: MFG_ERR_INVALID_ARG (n < 0, lda < max(1, n), NULL pointers with
 * n > 0, a mode with flags); MFG_ERR_NO_MEMORY if those allocations fail;
 * MFG_ERR_UNSUPPORTED for n > 2^31 - 1; those of mfg_gemm. */
int mfg_lu_factor(int64_t n, float* A, int64_t lda, int32_t* ipiv, int64_t* info, int mode, void* stream);
/* mfg_lu_solve -- B = (L U)^-1 P B in place for the n x nrhs FP32 B (device,
 * ldb >= max(1, nrhs)) with the factors and pivots of mfg_lu_factor: the
 * permutation, then forward and backward substitution by 64-row blocks
 * (each block's solve and the update of the rows still to be solved in one
 * launch; beyond 65535 right-hand sides, the updates by FP32 mfg_gemm).
 * Allocates an n x nrhs FP32 work array and the permutation; B's contents
 * are unspecified after an error.  Synchronises `stream`. */
int mfg_lu_solve(int64_t n, int64_t nrhs, const float* LU, int64_t ldlu, const int32_t* ipiv, float* B, int64_t ldb,
                 void* stream);
/* mfg_solve_ir -- X (n x nrhs FP64, device, ldx >= max(1, nrhs)) solving
 * A X = B for the FP64 n x n A and n x nrhs B (device): an FP32 copy of A
 * is factored by mfg_lu_factor(mode); x0 = the FP32 solve of B; then while
 * the normwise backward error max_j |b_j - A x_j|_inf / (|A|_inf |x_j|_inf
 * + |b_j|_inf), residuals in FP64, exceeds `tol` and fewer than `max_iter`
 * corrections were made: d = the FP32 solve of the residual, x += d in
 * FP64.  iters (host, may be NULL): corrections made; berr (host, may be
 * NULL): the final backward error; info (host, may be NULL): as for
 * mfg_lu_factor (when nonzero nothing is solved and X is unchanged).
 * Device workspace (n^2 FP32 + O(n nrhs)) is allocated and freed inside
 * the call, which synchronises `stream`.
 * Errors: as mfg_lu_factor, plus MFG_ERR_INVALID_ARG for nrhs < 0,
 * ldb, ldx < max(1, nrhs), max_iter < 0, tol < 0 or NaN; MFG_ERR_NO_MEMORY. */
int mfg_solve_ir(int64_t n, int64_t nrhs, const double* A, int64_t lda, const double* B, int64_t ldb, double* X,
                 int64_t ldx, int mode, int max_iter, double tol, int* iters, double* berr, int64_t* info,
                 void* stream);

/* ----------------------------------------------------- operand conversion
 * The paper rounds FP32 inputs to half precision before the matrix-unit
 * GEMM and leaves that step out of its timings (Sec. VI).  These calls do
 * that step explicitly.  X is rows x cols FP32 with leading dimension ldx.
 */
/* out = rne16(X): IEEE round-to-nearest-even, overflow to +-Inf, gradual
 * underflow (paper Sec. V, "Limited range"). ldo in 16-bit elements. */
int mfg_round_f16(int64_t rows, int64_t cols, const float* X, int64_t ldx,
                  void* out, int64_t ldo, void* stream);
/* out = rnebf16(X), NaN kept quiet. */
int mfg_round_bf16(int64_t rows, int64_t cols, const float* X, int64_t ldx,
                   void* out, int64_t ldo, void* stream);
/* Residual split (paper Sec. V, Eq. R, scaled): head = rne16(X),
 * resid = rne16(2^11 * (X - head)).  If norms != NULL (device, 4 doubles)
 * it receives, in FP64: sum X^2, max|X|, sum r^2, max|r| with r = X - head. */
int mfg_split_f16(int64_t rows, int64_t cols, const float* X, int64_t ldx,
                  void* head, void* resid, int64_t ldo, double* norms, void* stream);
/* FP8-E4M3 with one scale per 128 x 128 tile: scale = 2^E with E the
 * smallest integer such that 448 * 2^E >= max|tile| (E = 0 for an all-zero
 * tile, clamped to [-127, 127]); codes = sat_rne_e4m3(X / scale).
 * codes: rows x ldo bytes; scales: ceil(rows/128) x ceil(cols/128) FP32. */
int mfg_quantize_fp8(int64_t rows, int64_t cols, const float* X, int64_t ldx,
                     void* codes, int64_t ldo, float* scales, void* stream);
/* Write X in `mode`'s preconverted storage form (see "modes" above); `out`
 * must hold mfg_convert_bytes(rows, ldo, mode) bytes. */
int mfg_convert(int64_t rows, int64_t cols, const float* X, int64_t ldx,
                void* out, int64_t ldo, int mode, void* stream);
int64_t mfg_convert_bytes(int64_t rows, int64_t cols, int64_t ldo, int mode);

/* ----------------------------------------------------- FP64 error norms
 * Error of a result against an FP64 reference (paper Sec. VI: the max norm
 * of e = C - C_ref), computed on the GPU in FP64 with a deterministic
 * two-stage reduction.  out4 (device, 4 doubles) receives
 *   max|C - Cref|,  ||C - Cref||_F,  ||Cref||_F,  max|Cref|.
 */
int mfg_error_norms(int64_t M, int64_t N, const float* C, int64_t ldc,
                    const double* Cref, int64_t ldr, double* out4, void* stream);

/* ------------------------------------------------------------- autotuner
 * Time every tile configuration of `mode` on the caller's operands with HIP
 * events (`reps` timed runs after one warm-up each), keep the fastest whose
 * output is bitwise equal to configuration 0's, and record it in the tuned
 * table for the size bucket of (M, N, K).  best_config / best_ms (host) may
 * be NULL.  C is overwritten. */
int mfg_autotune(int64_t M, int64_t N, int64_t K,
                 const void* A, int64_t lda, const void* B, int64_t ldb,
                 float* C, int64_t ldc, int mode, int reps,
                 int* best_config, float* best_ms, void* stream);
/* Save / load the tuned table as text lines "mode mbucket nbucket kbucket config". */
int mfg_tune_save(const char* path);
int mfg_tune_load(const char* path);
int mfg_tune_clear(void);
/* Configuration mfg_gemm would use for this problem (tuned or heuristic). */
int mfg_tune_lookup(int64_t M, int64_t N, int64_t K, int mode);

/* ---------------------------------------------------------------- serving
 * A request loop with continuous batching and HBM admission.  Requests are
 * GEMMs over caller-owned FP32 A/B and FP32 C device buffers; the server
 * owns the converted operands (paper Sec. V-VI: FP32 data rounded, split
 * or quantised before the matrix-unit GEMM).  A request is admitted, first
 * come first served, when its converted-operand footprint fits in
 * hbm_budget_bytes next to those already admitted (a request that does not
 * fit waits, and so do the ones behind it).  When a slot (one HIP stream) is
 * free, the oldest admitted request takes up to max_group admitted requests
 * of its mode, alpha and beta into one group: operands are converted on the
 * slot's stream, small FP16 / BF16 / refined problems (M*N < 512*512, at
 * most 256 output tiles of the grouped kernel: 128 x 128, or 64 x 64 for
 * REFINE_A / SPLIT3 / SPLIT4) run as one persistent grouped launch, the
 * others one by one; one completion event per group.  Footprint: the mode's converted A (ld = K
 * rounded up to 8, or to 16 for FP8) and B (ld = N rounded likewise), each
 * rounded up to 256 bytes; 0 for MFG_F32 and for empty problems, and 0 for
 * MFG_BF16_SPLIT6, which runs through mfg_gemm and its per-stream workspace
 * (12 bytes per element of A and B, outside the budget).  The fixed
 * per-slot descriptor staging is not counted.  Results are bitwise those of
 * mfg_gemm on the same FP32 operands, whatever a request is grouped with.
 * Config limits: 1 <= slots <= 64, 1 <= max_group <= 4096, reserved = 0.
 * Request limits: mode without flags, reserved = 0, mfg_gemm's validation.
 * Caller's A, B, C must stay valid until mfg_poll returns a final status.
 */
typedef struct mfg_server mfg_server;

typedef struct mfg_server_config {
    uint64_t hbm_budget_bytes;  /* bytes of converted operands in flight     */
    int32_t slots;              /* concurrent launches (streams), >= 1        */
    int32_t device;             /* HIP device ordinal; -1 = dry run: requests
                                   are validated, admitted, grouped and
                                   accounted, but no HIP call is made, nothing
                                   is computed and A, B, C are never touched
                                   (a group "runs" for flops / 1e14 s); for
                                   testing the scheduler without a GPU        */
    int32_t max_group;          /* requests per grouped launch, >= 1          */
    int32_t reserved;
} mfg_server_config;

typedef struct mfg_request {
    int64_t M, N, K;
    int64_t lda, ldb, ldc;
    const float* A;   /* FP32, device */
    const float* B;   /* FP32, device */
    float* C;         /* FP32, device */
    float alpha, beta;
    int32_t mode;     /* MFG_F16, MFG_BF16, MFG_F16_SPLIT3, ... (no flag) */
    int32_t reserved;
} mfg_request;

typedef struct mfg_result {
    int32_t status;        /* MFG_OK, MFG_PENDING or an error              */
    int32_t slot;          /* slot (stream) index that ran it, -1 if none  */
    int64_t t_submit_ns;   /* steady-clock timestamps                      */
    int64_t t_admit_ns;
    int64_t t_start_ns;    /* launch enqueued                              */
    int64_t t_end_ns;      /* completion observed                          */
    int64_t group_size;    /* requests in the launch that carried it       */
    double flops;          /* 2*M*N*K                                      */
} mfg_result;

typedef struct mfg_server_stats {
    int64_t submitted, completed, failed, launches;
    uint64_t bytes_in_use, peak_bytes_in_use;
    int64_t max_concurrent_slots;
} mfg_server_stats;

int mfg_server_create(const mfg_server_config* cfg, mfg_server** out);
/* Submit (host copies *req).  MFG_ERR_OVER_BUDGET if the request alone
 * exceeds the budget; `ticket` (host) receives the request's id. */
int mfg_submit(mfg_server* s, const mfg_request* req, uint64_t* ticket);
/* MFG_PENDING while running; the final status once done (the result is
 * copied to *out, host, may be NULL), after which the ticket is released. */
int mfg_poll(mfg_server* s, uint64_t ticket, mfg_result* out);
/* Block until every submitted request has finished. */
int mfg_server_drain(mfg_server* s);
int mfg_server_get_stats(mfg_server* s, mfg_server_stats* out);
int mfg_server_destroy(mfg_server* s);

/* ------------------------------------------------------------------ misc */
const char* mfg_status_string(int status);
int mfg_last_hip_error(void);
const char* mfg_version(void);
/* Validation only (host, no HIP call): the status mfg_gemm would return for
 * these arguments before enqueueing anything. */
int mfg_validate_gemm(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda,
                      const void* B, int64_t ldb, const float* C, int64_t ldc, int mode);
/* Matrix-core ceiling probe (measurement aid for the roofline of the GEMM
 * kernels, not part of the GEMM path): `workgroups` workgroups of four
 * wavefronts each issue iters x 8 independent MFMAs from registers, with no
 * memory traffic.  shape 0: v_mfma_f32_32x32x16_f16, 1: 16x16x32_f16,
 * 2: v_mfma_scale_f32_32x32x64_f8f6f4 on E4M3 codes with unit scales (the
 * FP8 GEMM's instruction).  operands (device): 4096 dwords of 16-bit values
 * (shapes 0, 1) or E4M3 codes (shape 2) that every wavefront loads once
 * (random values or zeros: the sustained clock depends on them).  out
 * (device): workgroups * 256 floats (the accumulators' sums).  flops (host,
 * may be NULL) receives the matrix flops of the launch.  Time it with
 * events on `stream`. */
int mfg_probe_mfma(int shape, const void* operands, int64_t workgroups, int64_t iters, float* out,
                   double* flops, void* stream);
/* Fault injection, for tests of failure handling: after this call the
 * launch_n-th GEMM kernel launch (mfg_gemm, batched, grouped; conversions
 * are not counted) fails with MFG_ERR_HIP (hipErrorLaunchFailure) without
 * launching, and the alloc_n-th device allocation (a workspace growing, a
 * served request's operand storage) fails with MFG_ERR_NO_MEMORY, each once;
 * 0 disarms.  Process-wide.  The environment variable
 * MFG_FAULT=launch:<n>,alloc:<n> arms the same at the library's first call
 * and at every mfg_server_create.  The dry-run server (device = -1) meets
 * the same hooks: one allocation per request with a nonzero footprint, one
 * launch per request run alone or per grouped launch.  Negative counts are
 * MFG_ERR_INVALID_ARG. */
int mfg_fault_inject(int64_t launch_n, int64_t alloc_n);

#ifdef __cplusplus
}
#endif
#endif /* MFGEMM_H */
