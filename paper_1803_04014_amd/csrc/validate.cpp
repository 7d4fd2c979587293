// validate.cpp -- argument checks of the C ABI.  Pure host code (no HIP
// call), so the rules are unit-tested without a GPU.
#include <cstdint>

#include "mfgemm.h"

namespace mfg {

static bool mode_ok(int mode) {
    const int m = mode & MFG_MODE_MASK;
    const int flags = mode & ~MFG_MODE_MASK;
    return m >= 0 && m < MFG_NUM_MODES && (flags & ~MFG_IN_PRECONVERTED) == 0;
}

int validate_matrix(int64_t rows, int64_t cols, const void* X, int64_t ld) {
    if (rows < 0 || cols < 0) return MFG_ERR_INVALID_ARG;
    if (ld < (cols > 1 ? cols : 1)) return MFG_ERR_INVALID_ARG;
    if (rows > 0 && cols > 0 && X == nullptr) return MFG_ERR_INVALID_ARG;
    return MFG_OK;
}

int validate_gemm(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B, int64_t ldb,
                  const void* C, int64_t ldc, int mode) {
    if (!mode_ok(mode)) return MFG_ERR_INVALID_ARG;
    if (M < 0 || N < 0 || K < 0) return MFG_ERR_INVALID_ARG;
    if (lda < (K > 1 ? K : 1) || ldb < (N > 1 ? N : 1) || ldc < (N > 1 ? N : 1)) return MFG_ERR_INVALID_ARG;
    if (M > 0 && K > 0 && A == nullptr) return MFG_ERR_INVALID_ARG;
    if (K > 0 && N > 0 && B == nullptr) return MFG_ERR_INVALID_ARG;
    if (M > 0 && N > 0 && C == nullptr) return MFG_ERR_INVALID_ARG;
    // Sizes beyond int32 tile indices are not served.
    if (M > (int64_t)1 << 30 || N > (int64_t)1 << 30 || K > (int64_t)1 << 40) return MFG_ERR_UNSUPPORTED;
    return MFG_OK;
}

}  // namespace mfg

extern "C" int mfg_validate_gemm(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B,
                                 int64_t ldb, const float* C, int64_t ldc, int mode) {
    return mfg::validate_gemm(M, N, K, A, lda, B, ldb, C, ldc, mode);
}

extern "C" const char* mfg_status_string(int status) {
    switch (status) {
        case MFG_OK: return "MFG_OK";
        case MFG_PENDING: return "MFG_PENDING";
        case MFG_ERR_INVALID_ARG: return "MFG_ERR_INVALID_ARG";
        case MFG_ERR_UNSUPPORTED: return "MFG_ERR_UNSUPPORTED";
        case MFG_ERR_NO_MEMORY: return "MFG_ERR_NO_MEMORY";
        case MFG_ERR_OVER_BUDGET: return "MFG_ERR_OVER_BUDGET";
        case MFG_ERR_HIP: return "MFG_ERR_HIP";
        case MFG_ERR_UNKNOWN_TICKET: return "MFG_ERR_UNKNOWN_TICKET";
        case MFG_ERR_INTERNAL: return "MFG_ERR_INTERNAL";
        default: return "MFG_ERR_UNKNOWN_STATUS";
    }
}

extern "C" const char* mfg_version(void) { return "libmfgemm 0.1 (gfx950)"; }

extern "C" int64_t mfg_fp8_scale_offset(int64_t rows, int64_t ld) {
    const int64_t b = rows * ld;
    return (b + 255) / 256 * 256;
}

extern "C" int64_t mfg_convert_bytes(int64_t rows, int64_t cols, int64_t ldo, int mode) {
    if (rows < 0 || cols < 0 || ldo < (cols > 1 ? cols : 1)) return -1;
    switch (mode & MFG_MODE_MASK) {
        case MFG_F32: return rows * ldo * 4;
        case MFG_F16:
        case MFG_BF16: return rows * ldo * 2;
        case MFG_F16_REFINE_A:
        case MFG_F16_SPLIT3:
        case MFG_F16_SPLIT4:
        case MFG_BF16_SPLIT3: return 2 * rows * ldo * 2;
        case MFG_FP8_E4M3: {
            const int64_t tr = (rows + MFG_FP8_TILE - 1) / MFG_FP8_TILE;
            const int64_t tc = (cols + MFG_FP8_TILE - 1) / MFG_FP8_TILE;
            return mfg_fp8_scale_offset(rows, ldo) + tr * tc * 4;
        }
        default: return -1;
    }
}
