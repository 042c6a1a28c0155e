// Internal plan object shared by the host (fit, serialisation) and device
// (upload, launches) halves of libsaq.so.  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/saq.h"

namespace saq {

// Device plan layout (one caller-owned buffer, every region 256-byte aligned):
//   M_split 16-byte chunks [n_pad/128][k_pad/16][3][2][128]: M (rows = kept
//           dims in plan order) zero padded to [n_pad x k_pad] and written as
//           three bf16 terms per entry (m = m0 + m1 + m2, each the RNE bf16 of
//           what the previous terms leave), chunk (tile, step, term, half, row)
//           holding entries k = 16 step + 8 half .. + 7 of row 128 tile + row,
//           the order the split-operand GEMM stages them in LDS
//   c_pad   float [k_pad]
//   segtab  int32 [n_kept x 4]      column start, width, bits, code byte offset
//   S       float [sum_s W_s^2]     per kept segment, row-major W x W blocks
//                                   sqrt(sigma_i^2) R_s^T (one float if absent)
constexpr int kGemmTileN = 128;   // GEMM tile along the kept dims
constexpr int kGemmTileK = 32;    // k_pad granularity: the GEMM's k-steps of 16 run in
                                  // pairs (32-wide k-tiles for FP64 totals)
constexpr int kSplitK = 16;       // k-step of the split-operand GEMM
constexpr int kSplitChunks = 3 * 2 * kGemmTileN;   // 16-byte chunks per tile and k-step

struct SegEntry {
    int32_t col;      // first kept column
    int32_t width;    // W
    int32_t bits;     // B (> 0)
    int32_t code_off; // byte offset of the segment's first plane in a record
};

struct DeviceLayout {
    int32_t n_pad = 0, k_pad = 0;
    int64_t off_Ms = 0, off_c = 0, off_seg = 0, off_S = 0, bytes = 0;
};

}  // namespace saq

struct saq_plan {
    int32_t D = 0;
    std::vector<int32_t> widths, bits;   // all segments, plan order
    std::vector<float> M;                // D_kept x D
    std::vector<float> c;                // D
    std::vector<double> var;             // D (variances sorted descending), zeros if unknown
    // Per kept segment s (plan order) a W x W block, row-major:
    // S_s[i][j] = sqrt(lambda_i) R_s[j][i], R_s the segment's rotation and
    // lambda_i the variance of the PCA axis behind kept dim i.  For a query's
    // projection q'_s = R_s P_s (q - c), (S_s q'_s)_i = sqrt(lambda_i) P_i (q - c),
    // so ||S_s q'_s||^2 is the variance over the data of <o_s, q_s>
    // (Section 4.3).  Empty when the variances are unknown.
    std::vector<float> S;
    saq_plan_params params{};
    double model_error = 0.0, min_error = 0.0;
    int64_t quota = 0, used = 0;

    // derived
    int32_t D_kept = 0, n_kept = 0, max_kept_w = 0, max_kept_b = 0;
    bool acc64 = false;                  // projection accumulates k-tiles into FP64
    int64_t code_bytes = 0;
    std::vector<saq::SegEntry> kept;

    // device copy
    saq::DeviceLayout layout;
    std::vector<unsigned char> staging;  // host image of the device buffer
    void* dev = nullptr;                 // last upload target (caller-owned)
    int dev_id = -1;

    void derive();                       // fills the derived fields
};

namespace saq {
void set_error(const std::string& msg);
saq_status fail(saq_status st, const std::string& msg);
DeviceLayout device_layout(const saq_plan& p);
void build_staging(saq_plan& p);
// Eigen-decomposition of the covariance C [D x D] (row-major, symmetric),
// then the plan search and projection of the fit (Sections 4.1-4.2).
saq_status plan_from_moments(int32_t D, const std::vector<double>& mean, std::vector<double> C,
                             const saq_plan_params& P, saq_plan** out);
}  // namespace saq
