// Device half of libsaq.so (gfx950): the SAQ encode hot path and the
// estimate scan, plus their C-ABI entry points.
//
//   project_kernel   o = M (x - c) as a matrix-core GEMM: each FP32 product
//                    formed from operands split exactly into bf16 terms
//                    (v_mfma_f32_32x32x16_bf16), accumulated in FP32 or in
//                    FP64 totals of 32-wide k-tiles; centering fused into
//                    the A-tile staging, exact FP64 ||x - c||^2 on the side.
//   quantize_kernel  per (vector, kept segment): v_max, the grid code of
//                    Eq. (find_nearest_code), the code adjustment of
//                    Algorithm 1 with FP64 decisions, the factor and the
//                    bit-plane record.  One lane per vector, 64 vectors per
//                    wave, all lanes on the same segment in lock step.
//   estimate_kernel  Section 3.2 estimator over packed records, as an FP32
//                    matrix-core contraction of scaled codes with queries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>

#include "plan.hpp"

using saq::SegEntry;

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int TN = saq::kGemmTileN;   // 128 kept dims per tile
constexpr int NXCD = 8;               // MI355X: 8 XCDs, workgroups dealt round-robin

enum { LAYOUT_ROWS = 0, LAYOUT_DIMS = 1, LAYOUT_TILES = 2 };

// ---------------------------------------------------------------------------
// Projection GEMM.  Workgroup = 256 threads (4 waves) computes a (64 BI) x 128
// tile of O (vectors x kept dims); each wave a (32 BI) x 64 part as BI x 2
// 32x32 MFMA blocks.  BI = 2 with FP32 accumulation; BI = 1 with FP64 k-tile
// totals (64 doubles per 32 x 32 block and lane pair).
//
// Tile order is XCD-aware: workgroup b runs on XCD b % 8; XCD x walks row
// tiles x, x+8, ... and, inside each, all column tiles back to back, so the
// X tile is fetched from HBM once per XCD and re-read from that XCD's L2.
// When the pre-split M is larger than one L2 but half of it fits, each half
// of the XCDs takes half of the column tiles instead (the projection kernel's
// `halves` order): every workgroup streams its column tile's M, and M then
// stays in L2 (the fetch per launch at 1M x 960 drops from 26-28 GB to 16 GB
// at the same speed).
// ---------------------------------------------------------------------------
template <int BI> constexpr int gemm_rows() { return 64 * BI; }

// Per-record reference vectors (Section 3.1's c; the IVF centroid of each
// record's list in the paper's experiments): record i is centered on row
// ids[i] of refs [K x D] (all records on row 0 when ids is null) instead of
// the plan's c.  A record whose id is outside [0, K) is centered on row 0 and
// gets a NaN norm, so its factors show it.
struct RefRows {
    const float* refs;   // null: the plan's c
    const int32_t* ids;
    int32_t K;
};

// Stores rows row .. row+3 of column col of O in the output layout.
template <int LAYOUT>
__device__ __forceinline__ void store_quad(float* __restrict__ O, int64_t ld, int64_t n, int64_t row,
                                           int col, float v0, float v1, float v2, float v3) {
    if (LAYOUT == LAYOUT_TILES) {
        // whole 64-row tiles: rows of the last tile past n (copies of row
        // n-1) are stored too
        if (row < ((n + 63) & ~int64_t(63))) {
            float* dst = O + ((row >> 6) * ld + col) * 64 + (row & 63);
            *reinterpret_cast<float4*>(dst) = make_float4(v0, v1, v2, v3);
        }
    } else if (LAYOUT == LAYOUT_DIMS) {
        float* dst = O + int64_t(col) * ld + row;
        if (row + 3 < n) {
            *reinterpret_cast<float4*>(dst) = make_float4(v0, v1, v2, v3);
        } else {
            if (row + 0 < n) dst[0] = v0;
            if (row + 1 < n) dst[1] = v1;
            if (row + 2 < n) dst[2] = v2;
            if (row + 3 < n) dst[3] = v3;
        }
    } else {
        if (row + 0 < n) O[(row + 0) * ld + col] = v0;
        if (row + 1 < n) O[(row + 1) * ld + col] = v1;
        if (row + 2 < n) O[(row + 2) * ld + col] = v2;
        if (row + 3 < n) O[(row + 3) * ld + col] = v3;
    }
}

// ---------------------------------------------------------------------------
// Split-operand projection.  Every FP32 operand a is written exactly as
// a0 + a1 + a2 in bf16 (RNE to 8 significant bits, then RNE of the exact
// remainder, twice), and a b as the six products a_i b_j with i + j <= 2, the
// bf16x6 scheme of Henry, Tang and Heinecke (2019).  Since |a1| <= 2^-8 |a|
// and |a2| <= 2^-16 |a|, the three dropped products (a1 b2, a2 b1, a2 b2) are
// below (2^-23 + 2^-32) |a b| together, about two FP32 unit roundoffs, and
// the MFMAs (v_mfma_f32_32x32x16_bf16) accumulate in FP32, so o keeps FP32
// accuracy; the bf16 matrix rate is 16x the FP32 one, so the six products
// take 3/8 of the FP32 MFMA time.  With ACC64 each 32-wide k-tile (two
// k-steps) is accumulated in FP32 from zero and then added into FP64 totals,
// so the FP32 rounding error grows with the tile length (32) rather than
// with D.
//
// Tile (64 BI) x 128, k-step 16, four waves of (32 BI) x 64 (BI x 2 blocks of
// 32 x 32); BI = 2 for FP32 accumulation, 1 for FP64 totals and in grouped
// launches that also carry FP64-total datasets.  Every output element sees
// the same MFMA sequence over k in both shapes, so they give identical
// results.
//
// Per buffer, LDS holds both operands as 16-byte chunks [A|B][term][k half]
// [row]: a lane's MFMA operand (8 bf16 of one row, k half = lane / 32) is one
// chunk, and a wave reads two contiguous 512-byte runs.  The X rows are split
// as they are staged, thread t taking row t % (64 BI) and k half t / (64 BI),
// so a wave writes 64 consecutive chunks; M comes pre-split from the plan in
// the same chunk order, one 16-byte copy per chunk.
//
// A k-step has only 24 MFMAs per wave (768 cycles), too short to cover a
// global load, so X and the B chunks are loaded two k-steps ahead into
// alternating register sets.  The bulk of the k-steps runs in a loop whose
// loads are all full-width and unconditional: behind the ragged-tail branch
// the compiler can no longer count the loads in flight, and its wait before
// each A-tile store then also covered the loads issued two steps ahead.
//
// For BI = 2, 48 KB of LDS and at most 168 VGPRs give three workgroups per
// compute unit (two with per-row references, whose extra c registers would
// spill at three); FP64 totals run two.
// ---------------------------------------------------------------------------
constexpr int SK = saq::kSplitK;              // input dims per k-step
constexpr int SCB = saq::kSplitChunks;        // B chunks per buffer
template <int BI> constexpr int split_lds_floats() { return 2 * (6 * 64 * BI + SCB) * 4; }

__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
    const bf16x2 v = {static_cast<__bf16>(a), static_cast<__bf16>(b)};
    return __builtin_bit_cast(uint32_t, v);
}
// (a, b) -> three packed bf16 pairs, a = a0 + a1 + a2 exactly (normal a)
__device__ __forceinline__ void split3(float a, float b, uint32_t& h0, uint32_t& h1, uint32_t& h2) {
    h0 = pack_bf16x2(a, b);
    const float ra = a - __uint_as_float(h0 << 16), rb = b - __uint_as_float(h0 & 0xffff0000u);
    h1 = pack_bf16x2(ra, rb);
    h2 = pack_bf16x2(ra - __uint_as_float(h1 << 16), rb - __uint_as_float(h1 & 0xffff0000u));
}
__device__ __forceinline__ floatx16 mfma_bf16(u32x4 a, u32x4 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// lds: split_lds_floats<BI>() floats, free on entry; on return free except
// after a NORM tile (the norm hand-off leaves a barrier-protected write).
template <int LAYOUT, bool NORM, int BI, bool FULLB, bool REF, bool ACC64>
__device__ __forceinline__ void gemm_split_tile_impl(
    bool vec, const float* __restrict__ X, int64_t n, int D, const u32x4* __restrict__ Ms,
    int k_pad, const float* __restrict__ cp, int dk, float* __restrict__ O, int64_t ld,
    float* __restrict__ norm2, int tile_m, int tile_n, float* __restrict__ lds, RefRows R) {
    static_assert(BI == 1 || BI == 2, "tile shapes: 64 x 128 or 128 x 128");
    constexpr int RM = 64 * BI;                 // vectors per tile
    constexpr int SCA = 6 * RM;                 // A chunks per buffer
    constexpr int SCH = SCA + SCB;              // chunks per buffer
    u32x4* L = reinterpret_cast<u32x4*>(lds);
    const int64_t m0 = int64_t(tile_m) * RM;
    const int n0 = tile_n * TN;
    const int ksteps = k_pad / SK;

    const int t = threadIdx.x;
    const bool stager = t < 2 * RM;     // threads that stage A
    const int lr = t % RM;              // A row staged by this thread
    // its k half of the step, the same for the whole wave: the plan's c is
    // read with scalar loads
    const int kh = __builtin_amdgcn_readfirstlane((t / RM) & 1);
    const int64_t arow = m0 + lr;
    const bool arow_ok = arow < n;
    // rows past n read row n-1 (always valid memory); their outputs and
    // norms are never stored
    const float* xrow = X + (arow_ok ? arow : n - 1) * int64_t(D);
    // this thread copies B chunks t, t + 256, t + 512 of every k-step
    const u32x4* msrc = Ms + int64_t(tile_n) * ksteps * SCB + t;
    const float* crow = cp;
    // the plan's c as constant memory: scalar loads also when the pointer
    // comes from a grouped launch's argument struct
    typedef const __attribute__((address_space(4))) float cfloat;
    cfloat* ccp = (cfloat*)(cp);
    bool ref_bad = false;
    if (REF) {
        const int32_t id = R.ids != nullptr ? R.ids[arow_ok ? arow : n - 1] : 0;
        ref_bad = id < 0 || id >= R.K;
        crow = R.refs + int64_t(ref_bad ? 0 : id) * D;
    }
    double nacc = 0.0;

    // raw global values, loaded two k-steps ahead into alternating register
    // sets: X (and, with per-row references, c) and the B chunks
    struct Stage { float x[8]; float c[8]; u32x4 b[3]; };
    Stage sA, sB;
    const int kfull = vec ? (D / SK) : 0;
    auto load_stage = [&](int kt, Stage& g, auto fast) {
        if (stager) {
            const int kb = kt * SK + 8 * kh;
            if (decltype(fast)::value || kt < kfull) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const float4 x4 = *reinterpret_cast<const float4*>(xrow + kb + 4 * q);
                    g.x[4 * q + 0] = x4.x; g.x[4 * q + 1] = x4.y; g.x[4 * q + 2] = x4.z; g.x[4 * q + 3] = x4.w;
                    if (REF) {
                        const float4 c4 = *reinterpret_cast<const float4*>(crow + kb + 4 * q);
                        g.c[4 * q + 0] = c4.x; g.c[4 * q + 1] = c4.y;
                        g.c[4 * q + 2] = c4.z; g.c[4 * q + 3] = c4.w;
                    }
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    g.x[e] = (kb + e < D) ? xrow[kb + e] : 0.f;
                    if (REF) g.c[e] = (kb + e < D) ? crow[kb + e] : 0.f;
                }
            }
        }
#pragma unroll
        for (int p = 0; p < 3; ++p) g.b[p] = msrc[int64_t(kt) * SCB + 256 * p];
    };
    auto store_step = [&](int kt, int buf, const Stage& g) {
        if (stager) {
            const int kb = kt * SK + 8 * kh;
            float ra[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                // the plan's c is zero padded to k_pad: one uniform address,
                // read as constant memory (scalar loads)
                const float c = REF ? g.c[e] : ccp[kb + e];
                ra[e] = g.x[e] - c;
                if (NORM) {
                    // exact (x - c)^2 in FP64; padding entries are 0 - 0
                    const double d = double(g.x[e]) - double(c);
                    nacc = fma(d, d, nacc);
                }
            }
            uint32_t a0[4], a1[4], a2[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) split3(ra[2 * q], ra[2 * q + 1], a0[q], a1[q], a2[q]);
            u32x4* A = L + buf * SCH + kh * RM + lr;
            A[0] = u32x4{a0[0], a0[1], a0[2], a0[3]};
            A[2 * RM] = u32x4{a1[0], a1[1], a1[2], a1[3]};
            A[4 * RM] = u32x4{a2[0], a2[1], a2[2], a2[3]};
        }
        u32x4* B = L + buf * SCH + SCA + t;
#pragma unroll
        for (int p = 0; p < 3; ++p) B[256 * p] = g.b[p];
    };

    const int wave = t >> 6, lane = t & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int li = lane & 31, lh = lane >> 5;
    floatx16 acc[BI][2];
    double tot[BI][2][ACC64 ? 16 : 1];
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
#pragma unroll
            for (int r = 0; r < (ACC64 ? 16 : 1); ++r) tot[i][j][r] = 0.0;
        }

    // fast: steps kt + 1 and kt + 2 exist and are full (16-byte X loads)
    auto kstep = [&](int kt, const Stage& cur, Stage& nxt, auto fast) {
        constexpr bool F = decltype(fast)::value;
        const int buf = kt & 1;
        if (F || kt + 2 < ksteps) load_stage(kt + 2, nxt, fast);
        const u32x4* Ar = L + buf * SCH + lh * RM + wm * (32 * BI) + li;
        const u32x4* Br = L + buf * SCH + SCA + lh * TN + wn * 64 + li;
        u32x4 a[BI][3], b[2][3];
#pragma unroll
        for (int p = 0; p < 3; ++p) {
#pragma unroll
            for (int i = 0; i < BI; ++i) a[i][p] = Ar[2 * RM * p + 32 * i];
            b[0][p] = Br[2 * TN * p];
            if (FULLB) b[1][p] = Br[2 * TN * p + 32];
        }
        // the six products, smallest terms first
        constexpr int TA[6] = {2, 1, 0, 1, 0, 0};
        constexpr int TB[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
        for (int u = 0; u < 6; ++u)
#pragma unroll
            for (int i = 0; i < BI; ++i) {
                acc[i][0] = mfma_bf16(a[i][TA[u]], b[0][TB[u]], acc[i][0]);
                if (FULLB) acc[i][1] = mfma_bf16(a[i][TA[u]], b[1][TB[u]], acc[i][1]);
            }
        if (ACC64 && (kt & 1)) {
            // end of a 32-wide k-tile: into the FP64 totals
#pragma unroll
            for (int i = 0; i < BI; ++i)
#pragma unroll
                for (int j = 0; j < (FULLB ? 2 : 1); ++j)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        tot[i][j][r & (ACC64 ? 15 : 0)] += double(acc[i][j][r]);
                        acc[i][j][r] = 0.f;
                    }
        }
        if (F || kt + 1 < ksteps) store_step(kt + 1, buf ^ 1, cur);
        __syncthreads();
    };
    load_stage(0, sA, std::false_type{});
    store_step(0, 0, sA);
    load_stage(1, sB, std::false_type{});   // k_pad is a multiple of 32: ksteps >= 2, even
    __syncthreads();
    // the bulk of the steps with branch-free loads, so the compiler's wait
    // before each store covers only the loads that store needs
    int kt = 0;
    for (; kt + 3 < kfull; kt += 2) {
        kstep(kt, sB, sA, std::true_type{});
        kstep(kt + 1, sA, sB, std::true_type{});
    }
    for (; kt < ksteps; kt += 2) {
        kstep(kt, sB, sA, std::false_type{});
        kstep(kt + 1, sA, sB, std::false_type{});
    }

    if (NORM) {
        // the row's second half-sum comes from thread t + RM through LDS
        // (free after the last k-step's barrier)
        double* hand = reinterpret_cast<double*>(lds);
        if (stager && kh == 1) hand[lr] = nacc;
        __syncthreads();
        if (stager && kh == 0 && arow_ok)
            norm2[arow] = ref_bad ? __builtin_nanf("") : float(nacc + hand[lr]);
    }
    // epilogue: lane holds column n0 + wn*64 + 32*bj + li and, for register
    // r, row m0 + wm*32*BI + 32*bi + 8*(r/4) + 4*lh + r%4
#pragma unroll
    for (int bi = 0; bi < BI; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            const int col = n0 + wn * 64 + bj * 32 + li;
            if (col >= dk) continue;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int64_t row = m0 + wm * (32 * BI) + bi * 32 + 8 * g + 4 * lh;
                if (ACC64)
                    store_quad<LAYOUT>(O, ld, n, row, col,
                                       float(tot[bi][bj][(4 * g + 0) & (ACC64 ? 15 : 0)]),
                                       float(tot[bi][bj][(4 * g + 1) & (ACC64 ? 15 : 0)]),
                                       float(tot[bi][bj][(4 * g + 2) & (ACC64 ? 15 : 0)]),
                                       float(tot[bi][bj][(4 * g + 3) & (ACC64 ? 15 : 0)]));
                else
                    store_quad<LAYOUT>(O, ld, n, row, col, acc[bi][bj][4 * g + 0],
                                       acc[bi][bj][4 * g + 1], acc[bi][bj][4 * g + 2],
                                       acc[bi][bj][4 * g + 3]);
            }
        }
}

// One output tile.  ||x - c||^2 is produced by the first column tile only;
// the k-loop is specialised so the other tiles carry none of its work.
template <int LAYOUT, bool ACC64, int BI, bool REF = false>
__device__ __forceinline__ void gemm_tile(
    bool vec, const float* __restrict__ X, int64_t n, int D, const u32x4* __restrict__ Ms,
    int k_pad, const float* __restrict__ cp, int dk, float* __restrict__ O, int64_t ld,
    float* __restrict__ norm2, int tile_m, int tile_n, float* __restrict__ lds, RefRows R) {
    // the wave's second 32-column block (wave w covers columns
    // 64 (w % 2) .. 64 (w % 2) + 63 of the tile) holds kept dims
    const bool fullb = tile_n * TN + 64 * int((threadIdx.x >> 6) & 1) + 32 < dk;
    if (norm2 != nullptr && tile_n == 0)
        gemm_split_tile_impl<LAYOUT, true, BI, true, REF, ACC64>(vec, X, n, D, Ms, k_pad, cp, dk,
                                                                 O, ld, norm2, tile_m, tile_n, lds, R);
    else if (fullb)
        gemm_split_tile_impl<LAYOUT, false, BI, true, REF, ACC64>(vec, X, n, D, Ms, k_pad, cp, dk,
                                                                  O, ld, norm2, tile_m, tile_n, lds, R);
    else
        gemm_split_tile_impl<LAYOUT, false, BI, false, REF, ACC64>(vec, X, n, D, Ms, k_pad, cp, dk,
                                                                   O, ld, norm2, tile_m, tile_n, lds,
                                                                   R);
}

// FP32 accumulation runs the 128 x 128 tile, FP64 k-tile totals the 64 x 128
template <bool ACC64> constexpr int gemm_bi() { return ACC64 ? 1 : 2; }
template <bool ACC64> constexpr int gemm_lds_size() { return split_lds_floats<gemm_bi<ACC64>()>(); }

template <bool VEC, int LAYOUT, bool ACC64, bool REF>
__global__ __launch_bounds__(256, (ACC64 || REF) ? 2 : 3) void project_kernel(
    const float* __restrict__ X, int64_t n, int D, const u32x4* __restrict__ Ms, int k_pad, const float* __restrict__ cp, int dk,
    float* __restrict__ O, int64_t ld, float* __restrict__ norm2, int tiles_m, int tiles_n,
    RefRows R, int halves) {
    constexpr int BI = gemm_bi<ACC64>();
    __shared__ __attribute__((aligned(16))) float lds[gemm_lds_size<ACC64>()];
    const int bid = blockIdx.x;
    const int xcd = bid % NXCD, local = bid / NXCD;
    int tile_n, tile_m;
    if (!halves) {
        tile_n = local % tiles_n;
        tile_m = (local / tiles_n) * NXCD + xcd;
    } else {
        // each half of the XCDs takes half of the column tiles (the middle one
        // of an odd count split by row tiles), so each XCD's L2 holds half of
        // the pre-split M; inside a half, XCD xi walks row tiles xi, xi+4, ...
        // with the half's column tiles back to back, then its share of the
        // middle column tile
        const int g = xcd / (NXCD / 2), xi = xcd % (NXCD / 2);
        const int cm = tiles_n / 2, odd = tiles_n & 1, hm = (tiles_m + 1) / 2;
        const int c0 = g == 0 ? 0 : cm + odd, nc = g == 0 ? cm : tiles_n - cm - odd;
        const int rows = (tiles_m - xi + NXCD / 2 - 1) / (NXCD / 2);   // row tiles xi, xi+4, ...
        if (local < nc * rows) {
            tile_n = c0 + local % nc;
            tile_m = (local / nc) * (NXCD / 2) + xi;
        } else {
            if (!odd) return;
            const int r0 = g == 0 ? 0 : hm, r1 = g == 0 ? hm : tiles_m;
            tile_n = cm;
            tile_m = r0 + (local - nc * rows) * (NXCD / 2) + xi;
            if (tile_m >= r1) return;
        }
    }
    if (tile_m >= tiles_m) return;
    gemm_tile<LAYOUT, ACC64, BI, REF>(VEC, X, n, D, Ms, k_pad, cp, dk, O, ld, norm2, tile_m, tile_n,
                                      lds, R);
}

// ---------------------------------------------------------------------------
// Quantize + adjust + factor + pack.  One wave (64 lanes) per 64 vectors, one
// vector per lane; the wave's 64 codes of the current segment live in LDS as
// [dim][lane] (conflict-free), the projected values stream from O in chunks
// of QCH dims, the next chunk in flight while the current one is used.
//
// Adjustment decision (Algorithm 1, "L(x') > L(x)"), exact reformulation:
// with u = code - (2^B-1)/2, ip = <u,o>, n = ||u||^2 and a move u_i += s,
// L' > L  <=>  ip'^2 n > ip^2 n'  (given ip' > 0, which holds for every move
// that passes this test because each term u_j o_j >= 0), i.e.
//   s = +1:  n o (2 ip + o) > ip^2 (2u + 1)   <=>  A + Bv > 0
//   s = -1:  n o (o - 2 ip) > ip^2 (1 - 2u)   <=>  A - Bv > 0
// with A = n o^2 - ip^2 and Bv = 2 ip n o - 2u ip^2, evaluated in FP64 (o is
// FP32, so both are within a few ulps of exact).  An all-zero segment has
// o = 0 and ip = 0, so A = Bv = 0 and nothing is ever accepted.
// +1 is tried first; after an accepted +1 the reverting -1 can never pass.
// A round that accepts nothing leaves the state unchanged, so once no lane
// of the wave accepted anything the remaining rounds are skipped.
// ---------------------------------------------------------------------------
constexpr int QCH = 32;   // dims per prefetch chunk in the quantize kernel

// Where one lane's projected values sit.  Tiled layout: the 64 vectors of a
// wave are one tile, dim j of the tile 64 contiguous floats, so a chunk is
// QCH loads at immediate offsets from one wave-uniform base.
template <int LAYOUT>
struct LaneView {
    const float* p;   // kept dim 0 of this lane's vector
    int64_t sd;       // elements between consecutive dims (row and dims layouts)

    __device__ __forceinline__ int64_t stride() const { return LAYOUT == LAYOUT_TILES ? 64 : sd; }

    // dims j0 .. j0+QCH-1, all inside the segment
    __device__ __forceinline__ void load_full(float (&dst)[QCH], int col, int j0) const {
        const float* q = p + int64_t(col + j0) * stride();
#pragma unroll
        for (int t = 0; t < QCH; ++t) dst[t] = q[int64_t(t) * stride()];
    }
    // dims j0 .. j0+QCH-1 of the segment starting at kept dim col; dims past
    // its width W are clamped to its last dim (loaded, never used)
    __device__ __forceinline__ void load(float (&dst)[QCH], int col, int j0, int W) const {
        const float* q = p + int64_t(col + j0) * stride();
        if (j0 + QCH <= W) {
#pragma unroll
            for (int t = 0; t < QCH; ++t) dst[t] = q[int64_t(t) * stride()];
        } else {
            const int last = W - 1 - j0;
#pragma unroll
            for (int t = 0; t < QCH; ++t) dst[t] = q[int64_t(min(t, last)) * stride()];
        }
    }
};

// One in-order pass over the W dims of a segment: body(x, i0, full) for every
// chunk, full = std::true_type when all QCH dims of the chunk are inside the
// segment.  On entry a holds chunk 0; on return a holds chunk 0 again,
// loaded during the last chunk for the pass that follows.
template <int LAYOUT, class Body>
__device__ __forceinline__ void sweep(const LaneView<LAYOUT>& lv, int col, int W,
                                      float (&a)[QCH], float (&b)[QCH], Body&& body) {
    auto run = [&](const float (&x)[QCH], int i0) {
        if (i0 + QCH <= W) body(x, i0, std::true_type{});
        else body(x, i0, std::false_type{});
    };
    int i0 = 0;
    // steady state, two chunks per trip: every chunk used and every chunk
    // loaded is whole, so the loads are unconditional and the compiler's
    // wait before a chunk's use covers only that chunk's loads (behind the
    // whole/ragged branch it also waited for most of the next chunk's)
    while (i0 + 3 * QCH <= W) {
        lv.load_full(b, col, i0 + QCH);
        body(a, i0, std::true_type{});
        lv.load_full(a, col, i0 + 2 * QCH);
        body(b, i0 + QCH, std::true_type{});
        i0 += 2 * QCH;
    }
    for (;;) {
        const bool more = i0 + QCH < W;
        lv.load(b, col, more ? i0 + QCH : 0, W);
        run(a, i0);
        i0 += QCH;
        if (!more) {
#pragma unroll
            for (int t = 0; t < QCH; ++t) a[t] = b[t];
            return;
        }
        const bool more2 = i0 + QCH < W;
        lv.load(a, col, more2 ? i0 + QCH : 0, W);
        run(b, i0);
        i0 += QCH;
        if (!more2) return;
    }
}

// Bit planes of one segment, most significant first; dim i -> byte i/8,
// bit i%8 of the plane.  The wave's 64 records are packed in its LDS code
// buffer and then stored record by record, consecutive lanes writing
// consecutive bytes of a record (coalesced), rather than each lane writing
// its own record at a stride of code_bytes.
//
// Packing, 32 dims at a time: block j's codes are read into registers, its
// B plane words are formed, and word (block j, plane q from the most
// significant) of lane L goes to 32-bit slot
//   (j B + q) 64 + (L ^ ((j B + q) mod 64))
// of the buffer.  Those slots end at byte (j + 1) B 256 <= (j + 1) 32 64
// sizeof(CT), the end of block j's codes (B <= 8 sizeof(CT)), so packing
// overwrites only codes already read (the buffer is rounded up to whole
// 32-dim blocks for a ragged last block).  The XOR spreads one record's
// words over the banks for the read-back, and keeps each store of 64 lanes
// a permutation of one 64-slot row.
template <typename CT, int B>
__device__ __forceinline__ void stage_planes(CT* __restrict__ lc, int W, int lane) {
    uint32_t* st = reinterpret_cast<uint32_t*>(lc);
    for (int j0 = 0, j = 0; j0 < W; j0 += 32, ++j) {
        uint32_t word[B];
#pragma unroll
        for (int p = 0; p < B; ++p) word[p] = 0u;
        if (j0 + 32 <= W) {
#pragma unroll
            for (int t = 0; t < 32; ++t) {
                const uint32_t c = uint32_t(lc[(j0 + t) * 64 + lane]);
#pragma unroll
                for (int p = 0; p < B; ++p) word[p] |= ((c >> p) & 1u) << t;
            }
        } else {
            for (int t = 0; j0 + t < W; ++t) {
                const uint32_t c = uint32_t(lc[(j0 + t) * 64 + lane]);
#pragma unroll
                for (int p = 0; p < B; ++p) word[p] |= ((c >> p) & 1u) << t;
            }
        }
        // codes and words are different types: keep the compiler from moving
        // any word store above this block's code loads
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
        for (int p = 0; p < B; ++p) {
            const int slot = j * B + (B - 1 - p);
            st[slot * 64 + (lane ^ (slot & 63))] = word[p];
        }
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <typename CT>
__device__ __forceinline__ void stage_segment(CT* __restrict__ lc, int W, int B, int lane) {
    switch (B) {
#define SAQ_PACK_CASE(K) \
    case K: stage_planes<CT, K>(lc, W, lane); break;
        SAQ_PACK_CASE(1) SAQ_PACK_CASE(2) SAQ_PACK_CASE(3) SAQ_PACK_CASE(4)
        SAQ_PACK_CASE(5) SAQ_PACK_CASE(6) SAQ_PACK_CASE(7) SAQ_PACK_CASE(8)
        default:
            if constexpr (sizeof(CT) > 1) {
                switch (B) {
                    SAQ_PACK_CASE(9) SAQ_PACK_CASE(10) SAQ_PACK_CASE(11) SAQ_PACK_CASE(12)
                    SAQ_PACK_CASE(13) SAQ_PACK_CASE(14) SAQ_PACK_CASE(15) SAQ_PACK_CASE(16)
                    default: break;
                }
            }
            break;
#undef SAQ_PACK_CASE
    }
}

// Stores the staged segment: record r (vector v0 + r, r < 64, v0 + r < n)
// gets its B pb bytes at codes + (v0 + r) code_bytes + code_off, U bytes per
// lane and store.  With at most 64 units per record each store covers
// 64 / units records, consecutive lanes on consecutive units; otherwise it
// covers 64 consecutive units of one record.
template <int U>
__device__ __forceinline__ void store_staged(const uint32_t* __restrict__ st, int B, int pb,
                                             int lane, uint8_t* __restrict__ codes,
                                             int64_t code_bytes, int code_off, int64_t v0,
                                             int64_t n) {
    const int upr = B * pb / U;                      // units per record
    const int live = int(min<int64_t>(64, n - v0));  // records of this wave
    auto unit = [&](int r, int e, int slot, int bo) {
        const uint32_t w = st[slot * 64 + (r ^ (slot & 63))] >> (8 * bo);
        uint8_t* dst = codes + (v0 + r) * code_bytes + code_off + e;
        if (U == 4) *reinterpret_cast<uint32_t*>(dst) = w;
        else if (U == 2) *reinterpret_cast<uint16_t*>(dst) = uint16_t(w);
        else *dst = uint8_t(w);
    };
    if (upr <= 64) {
        const int rpi = 64 / upr;                    // records per store
        const int rr = lane / upr, e = (lane - rr * upr) * U;
        const int q = e / pb, t = e - q * pb;
        const int slot = (t >> 2) * B + q, bo = t & 3;
        if (rr < rpi)
            for (int r = rr; r < live; r += rpi) unit(r, e, slot, bo);
    } else {
        for (int k = lane; k < upr; k += 64) {
            const int e = k * U, q = e / pb, t = e - q * pb;
            const int slot = (t >> 2) * B + q, bo = t & 3;
            for (int r = 0; r < live; ++r) unit(r, e, slot, bo);
        }
    }
}
// One wave quantizes vectors v0 .. v0+63 (one per lane; v0 % 64 == 0).
// lc: this wave's code buffer, [max kept width][64] entries of LDS.
template <typename CT, int LAYOUT>
__device__ __forceinline__ void quantize_wave(
    const float* __restrict__ O, int64_t ld, int64_t n, int64_t v0, int lane,
    const SegEntry* __restrict__ segs, int n_kept, const float* __restrict__ norm2, int rounds,
    uint8_t* __restrict__ codes, int64_t code_bytes, int codes_align,
    float* __restrict__ factors, CT* __restrict__ lc) {
    const int64_t v = v0 + lane;
    const bool live = v < n;
    const int64_t vv = live ? v : n - 1;
    LaneView<LAYOUT> lv;
    if (LAYOUT == LAYOUT_TILES) {
        // lanes past n read their own slots of the last tile (never used)
        lv.p = O + (v0 >> 6) * ld * 64 + lane;
        lv.sd = 64;
    } else {
        lv.p = O + (LAYOUT == LAYOUT_DIMS ? vv : vv * ld);
        lv.sd = LAYOUT == LAYOUT_DIMS ? ld : 1;
    }
    double kept_norm = 0.0;
    float a[QCH], b[QCH];

    for (int s = 0; s < n_kept; ++s) {
        const SegEntry e = segs[s];
        const int W = e.width, B = e.bits, col = e.col;
        const int cmax = (1 << B) - 1;
        lv.load(a, col, 0, W);

        // v_max = max |o_i| (exact in FP32)
        float vmax = 0.f;
        sweep(lv, col, W, a, b, [&](const float (&x)[QCH], int i0, auto full) {
#pragma unroll
            for (int t = 0; t < QCH; ++t)
                if (decltype(full)::value || i0 + t < W) vmax = fmaxf(vmax, fabsf(x[t]));
        });
        const bool zero = !(vmax > 0.f);

        // initial code c = floor((o + v) / Delta), Delta = 2 v / 2^B, clamped to
        // 2^B - 1.  a = o + v is exact in FP64 up to one rounding the CPU
        // evaluation shares; q = floor(a / Delta) is taken from a * (1/Delta)
        // and corrected by the exact remainder r = a - q Delta (exact in FP64
        // for q >= 1, and r = a for q = 0).  An all-zero segment takes the
        // middle code 2^(B-1) through v = 2^(B-1), Delta = 1.
        const double vd = zero ? ldexp(1.0, B - 1) : double(vmax);
        const double delta = zero ? 1.0 : ldexp(2.0 * vd, -B);
        const double inv = zero ? 1.0 : ldexp(0.5 / vd, B);
        const double half = 0.5 * double(cmax);
        double ip = 0.0, nn = 0.0, oo = 0.0;
        sweep(lv, col, W, a, b, [&](const float (&x)[QCH], int i0, auto full) {
#pragma unroll
            for (int t = 0; t < QCH; ++t) {
                if (!(decltype(full)::value || i0 + t < W)) continue;
                const double o = double(x[t]);
                const double av = o + vd;
                const double q = floor(av * inv);
                const double r = fma(-q, delta, av);
                int c = int(q) + (r >= delta ? 1 : 0) - (r < 0.0 ? 1 : 0);
                c = min(max(c, 0), cmax);
                lc[(i0 + t) * 64 + lane] = CT(c);
                const double u = double(c) - half;
                ip = fma(u, o, ip);
                nn = fma(u, u, nn);
                oo = fma(o, o, oo);
            }
        });
        kept_norm += oo;

        // code adjustment (Algorithm 1)
        if (B >= 2 && rounds > 0) {
            const double cmd = double(cmax);
            double P = 2.0 * ip, nS = -(ip * ip);
            for (int rd = 0; rd < rounds; ++rd) {
                int moved = 0;
                sweep(lv, col, W, a, b, [&](const float (&x)[QCH], int i0, auto full) {
                    constexpr bool F = decltype(full)::value;
                    int cc[QCH];
#pragma unroll
                    for (int t = 0; t < QCH; ++t)
                        cc[t] = int(lc[(F ? i0 + t : min(i0 + t, W - 1)) * 64 + lane]);
#pragma unroll
                    for (int t = 0; t < QCH; ++t) {
                        if (!(F || i0 + t < W)) continue;
                        const double o = double(x[t]);
                        const int c = cc[t];
                        const double w = fma(2.0, double(c), -cmd);     // 2u, exact
                        // A = n o^2 - ip^2, Bv = 2 ip n o - ip^2 (2u):
                        //   +1 passes iff A + Bv > 0, -1 iff A - Bv > 0
                        const double no = nn * o;
                        const double A = fma(no, o, nS);
                        const double Bv = fma(no, P, nS * w);
                        const bool up = c < cmax && Bv > -A;
                        const bool dn = c > 0 && A > Bv;   // taken only when up fails
                        if (up || dn) {
                            const double sg = up ? 1.0 : -1.0;
                            nn = nn + fma(sg, w, 1.0);      // (u + s)^2 = u^2 + 2su + 1
                            ip = fma(sg, o, ip);
                            P = 2.0 * ip;
                            nS = -(ip * ip);
                            lc[(i0 + t) * 64 + lane] = CT(c + (up ? 1 : -1));
                            moved = 1;
                        }
                    }
                });
                if (!__any(moved && live)) break;
            }
        }

        // factor f_s = ||o_s||^2 / <u_s, o_s>
        if (live) factors[v * (n_kept + 1) + s] = zero ? 0.f : float(oo / ip);

        const int pb = (W + 7) >> 3;
        const int al = pb | e.code_off | int(code_bytes) | codes_align;
        stage_segment<CT>(lc, W, B, lane);
        const uint32_t* st = reinterpret_cast<const uint32_t*>(lc);
        if ((al & 3) == 0)
            store_staged<4>(st, B, pb, lane, codes, code_bytes, e.code_off, v0, n);
        else if ((al & 1) == 0)
            store_staged<2>(st, B, pb, lane, codes, code_bytes, e.code_off, v0, n);
        else
            store_staged<1>(st, B, pb, lane, codes, code_bytes, e.code_off, v0, n);
        // the next segment's codes overwrite the staged words
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
    if (live) factors[v * (n_kept + 1) + n_kept] = norm2 ? norm2[v] : float(kept_norm);
}

template <typename CT, int LAYOUT>
__global__ __launch_bounds__(64) void quantize_kernel(
    const float* __restrict__ O, int64_t ld, int64_t n, const SegEntry* __restrict__ segs,
    int n_kept, const float* __restrict__ norm2, int rounds, uint8_t* __restrict__ codes,
    int64_t code_bytes, int codes_align, float* __restrict__ factors) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    quantize_wave<CT, LAYOUT>(O, ld, n, int64_t(blockIdx.x) * 64, threadIdx.x, segs, n_kept,
                              norm2, rounds, codes, code_bytes, codes_align, factors,
                              reinterpret_cast<CT*>(smem));
}

// ---------------------------------------------------------------------------
// Batched encode: up to BATCH_MAX datasets, each with its own plan (uneven
// segment widths and bits), in two grouped launches for the whole batch:
// one runs every dataset's projection tiles, the next every dataset's
// quantize/adjust/pack blocks.  A workgroup finds its dataset from the block
// ranges in the launch arguments; no workgroup ever waits for another.
// ---------------------------------------------------------------------------
constexpr int BATCH_MAX = 16;

struct GemmSet {
    const float* X; int64_t n; int D; int vec; int acc64;
    const u32x4* Ms; int k_pad; const float* cp; int dk; int tiles_m; int tiles_n;
    float* O; int64_t ld; float* norm2;
    int64_t first_block;
};
struct GemmArgs { GemmSet set[BATCH_MAX]; int count; int xcd_order; };

template <bool ACC64>
__global__ __launch_bounds__(256, ACC64 ? 2 : 3) void grouped_gemm_kernel(const GemmArgs args) {
    constexpr int BI = gemm_bi<ACC64>();
    __shared__ __attribute__((aligned(16))) float lds[gemm_lds_size<ACC64>()];
    const int64_t b = blockIdx.x;
    int d = 0;
    while (d + 1 < args.count && b >= args.set[d + 1].first_block) ++d;
    const GemmSet& S = args.set[d];
    const int64_t lb = b - S.first_block;
    int tile_m, tile_n;
    if (args.xcd_order) {
        // every dataset's block range starts at a multiple of 8, so lb % 8 is
        // the XCD this workgroup runs on
        const int xcd = int(lb % NXCD);
        const int64_t local = lb / NXCD;
        tile_n = int(local % S.tiles_n);
        tile_m = int(local / S.tiles_n) * NXCD + xcd;
    } else {
        tile_m = int(lb / S.tiles_n);
        tile_n = int(lb % S.tiles_n);
    }
    if (tile_m >= S.tiles_m) return;
    // one tile shape per launch: in a launch with FP64 totals, datasets
    // without them accumulate in FP32 on the same tile
    if (S.acc64)
        gemm_tile<LAYOUT_TILES, ACC64, BI>(S.vec != 0, S.X, S.n, S.D, S.Ms, S.k_pad, S.cp, S.dk,
                                          S.O, S.ld, S.norm2, tile_m, tile_n, lds,
                                          RefRows{nullptr, nullptr, 0});
    else
        gemm_tile<LAYOUT_TILES, false, BI>(S.vec != 0, S.X, S.n, S.D, S.Ms, S.k_pad, S.cp, S.dk,
                                          S.O, S.ld, S.norm2, tile_m, tile_n, lds,
                                          RefRows{nullptr, nullptr, 0});
}

struct QuantSet {
    const float* O; int64_t ld; int64_t n;
    const SegEntry* segs; int n_kept; const float* norm2;
    uint8_t* codes; int64_t code_bytes; int codes_align; float* factors;
    int64_t first_block;
};
struct QuantArgs { QuantSet set[BATCH_MAX]; int count; int rounds; int wmax; };

template <typename CT>
__global__ __launch_bounds__(256) void grouped_quantize_kernel(const QuantArgs args) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int64_t b = blockIdx.x;
    int d = 0;
    while (d + 1 < args.count && b >= args.set[d + 1].first_block) ++d;
    const QuantSet& S = args.set[d];
    const int waves = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t v0 = (b - S.first_block) * 64 * waves + int64_t(wave) * 64;
    if (v0 >= S.n) return;
    CT* lc = reinterpret_cast<CT*>(smem) + int64_t(wave) * args.wmax * 64;
    quantize_wave<CT, LAYOUT_TILES>(S.O, S.ld, S.n, v0, lane, S.segs, S.n_kept, S.norm2,
                                   args.rounds, S.codes, S.code_bytes, S.codes_align,
                                   S.factors, lc);
}

// ---------------------------------------------------------------------------
// Batched encode in one persistent launch.  The work items are blocks of
// 64 Q rows of every dataset (Q quantize waves, as many as the LDS code
// buffers allow, up to 4; a whole number of projection row tiles), numbered
// dataset by dataset.  A workgroup takes the next item from one atomic
// ticket, projects the item's rows against every column tile of its dataset
// into the dataset's tiled O (the same tile functions and MFMA sequence as
// the plain projection, so the same values), and then quantizes, adjusts
// and packs those rows with its first Q waves, 64 vectors each.  The rows it quantizes are the rows it projected, so no
// workgroup ever waits for another: every item is finished by the workgroup
// that took its ticket, and each workgroup leaves once the ticket passes the
// item count.  While one workgroup of a compute unit runs its quantize phase
// (VALU) others run projection tiles (matrix cores).  The ticket is cleared
// by clear_ticket_kernel, launched before on the same stream.
// ---------------------------------------------------------------------------
struct FusedSet {
    const float* X; const u32x4* Ms; const float* cp; float* O; float* norm2;
    const SegEntry* segs; uint8_t* codes; float* factors;
    int64_t n; int64_t ld; int64_t code_bytes; int64_t first_item;
    int D; int vec; int acc64; int k_pad; int dk; int tiles_m; int tiles_n; int n_kept;
    int codes_align;
};
struct FusedArgs {
    FusedSet set[BATCH_MAX];
    unsigned long long* ticket;
    int64_t items;
    int count; int rounds; int wmax;
    int qwaves;               // quantize waves per item: the item is 64 qwaves rows
};

__global__ void clear_ticket_kernel(unsigned long long* ticket) {
    if (threadIdx.x == 0) *ticket = 0ull;
}

// Two workgroups per compute unit: the projection phase alone fits three
// in 168 VGPRs, but with the quantize phase and the item loop in the same
// kernel it would spill there.
template <int BI, bool ANY64, typename CT>
__global__ __launch_bounds__(256, 2) void fused_encode_kernel(const FusedArgs args) {
    static_assert(!ANY64 || BI == 1, "FP64 k-tile totals run the 64 x 128 tile");
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __shared__ long long item_s;
    float* lds = reinterpret_cast<float*>(smem);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (;;) {
        if (threadIdx.x == 0) item_s = static_cast<long long>(atomicAdd(args.ticket, 1ull));
        __syncthreads();
        const int64_t it = item_s;
        if (it >= args.items) return;         // the same value in every thread
        int d = 0;
        while (d + 1 < args.count && it >= args.set[d + 1].first_item) ++d;
        const FusedSet& S = args.set[d];
        const int64_t row0 = (it - S.first_item) * 64 * args.qwaves;
        const int tm0 = int(row0 / (64 * BI));
        const int tm1 = min(S.tiles_m, int((row0 + 64 * args.qwaves) / (64 * BI)));
        for (int tile_m = tm0; tile_m < tm1; ++tile_m)
            for (int tn = 0; tn < S.tiles_n; ++tn) {
                if (ANY64 && S.acc64)
                    gemm_tile<LAYOUT_TILES, ANY64, BI>(S.vec != 0, S.X, S.n, S.D, S.Ms, S.k_pad,
                                                       S.cp, S.dk, S.O, S.ld, S.norm2, tile_m, tn,
                                                       lds, RefRows{nullptr, nullptr, 0});
                else
                    gemm_tile<LAYOUT_TILES, false, BI>(S.vec != 0, S.X, S.n, S.D, S.Ms, S.k_pad,
                                                       S.cp, S.dk, S.O, S.ld, S.norm2, tile_m, tn,
                                                       lds, RefRows{nullptr, nullptr, 0});
                // the tile's LDS (and the norm hand-off) is free for the next
                // one; its O and norm stores are visible to every wave
                __syncthreads();
            }
        if (wave < args.qwaves) {
            const int64_t v0 = row0 + int64_t(64) * wave;
            if (v0 < S.n)
                quantize_wave<CT, LAYOUT_TILES>(S.O, S.ld, S.n, v0, lane, S.segs, S.n_kept,
                                                S.norm2, args.rounds, S.codes, S.code_bytes,
                                                S.codes_align, S.factors,
                                                reinterpret_cast<CT*>(smem) +
                                                    int64_t(wave) * args.wmax * 64);
        }
        __syncthreads();                      // LDS is reused by the next item
    }
}

// ---------------------------------------------------------------------------
// Estimate scan (Section 3.2) as a matrix-core contraction:
//   dist2[q][i] = ||o_i||^2 + ||q - c||^2 - 2 sum_s f_s <u_s(i), q'_s>
// is a GEMM between the records' scaled codes a_i = (f_s u_s), one row of
// D_kept values per record, and the projected queries q'.  A workgroup takes
// 128 records x 64 queries; a k-step covers 32 kept dims of one segment.
// Each k-step's raw inputs (16 dims of every bit plane of one record per
// lane, 8 query dims per thread as three bf16 terms, the record's f_s) are
// fetched one k-step ahead.  After the current k-step's MFMAs each lane
// unpacks its 16 dims as FP32 f_s (c - (2^B - 1)/2), splits them exactly
// into three bf16 terms straight into its own A operand registers (wave w
// holds records 32w .. 32w + 31), and the query terms go to LDS, the only
// operand the four waves share.  Each FP32 product is then formed as the
// projection forms it, from the six products a_i q_j with i + j <= 2 of
// the exact splits, accumulated in FP32: per 16-dim half and 32-query block
// six v_mfma_f32_32x32x16_bf16 (24 per wave and k-step with two blocks).
// That is the form of the multi-stage scan and of packed k-steps.  Plain
// scans stepping segment by segment (TR) transpose the product instead:
// the query terms are the A operand and each lane's own record the B
// operand, so all 16 accumulators of a lane belong to the record it
// unpacks.  The lane then applies f_s to its accumulators, rescaling them
// from the previous segment's factor where a segment starts, and its
// operand is c - (2^B - 1)/2 itself, exact as one bf16 term up to 8 bits
// (two above): three products per 16 dims and 32-query block (five above 8
// bits), the exact products of the query's split with the code, and no
// FP32 scaling or split of the record's values.
// The queries are split once per scan (split_query_kernel) when a
// segment's first kept column is a multiple of 8, else while staging.  A
// segment whose width is not a multiple of 32 pads its last k-step with
// zeros on the record side.  Segments of at most 8 bits unpack a plane
// byte (8 dims) with one lookup in a 256-entry table that spreads its bits
// to one bit per byte.  With prefix b > 0 a segment reads only its
// first min(b, B) bit planes, the b-bit prefix floor(c / 2^(B-b)) of every
// code, and scales its factor by 2^(B-b) (progressive approximation).
//
// Multi-stage mode (MS, Section 4.3, prefix 0): the k-steps already run
// segment by segment in plan order, so when a segment starts the
// accumulators hold the terms of the segments before it.  There every lane
// bounds its 32 (query, record) pairs from below,
//   LB_s = ||o||^2 - 2 acc + lbq[q][s],  lbq[q][s] = ||q - c||^2 - 2 m sum_{t>=s} sigma_t,
// and a pair with LB_s > tau[q] is closed: it gets LB_s and stage s.  Pairs
// still open after the last segment get the full estimate and stage k.
// Once no pair of the workgroup is open, the workgroup stops reading codes.
//
// Sparse finish: the matrix cores pay for every pair of the tile while most
// are closed after the first segments (at D = 3072, m = 4 and a 10-nearest
// threshold, about 3 % of the pairs are open after two segments), so once at
// most EMS_CAP pairs of the tile are open at a segment start, the tile
// leaves the MFMA loop.  Its open pairs, with their partial sums, go to a
// list in LDS; one lane per pair then reads that pair's codes and query
// values for the next segment, adds f_s (c - h) q' over its dims in FP32,
// bounds the pair before the segment after it, and either closes it or
// appends it to the next list.  Every segment thus costs only its still-open
// pairs, and the waves stay full because the list is rebuilt per segment.
// The terms and the bound are the MFMA path's; only the summation order
// inside a segment differs (FP32 either way).
// ---------------------------------------------------------------------------
constexpr int ER = 128;                 // records per estimate tile
constexpr int EQ = 64;                  // queries per estimate tile
constexpr int EK = 32;                  // kept dims per k-step
// the query slices in LDS: per buffer, bf16 terms 0..2 of each query's 32
// dims, rows of EROW bf16 (80 bytes: 16 lanes' 16-byte reads of 16
// consecutive rows hit distinct banks)
constexpr int EROW = EK + 8;
constexpr int EST_LDS_FLOATS = 2 * 3 * EQ * EROW / 2;  // 30,720 bytes
// open pairs at which a multi-stage tile leaves the matrix cores; two lists
// of this many (key, partial sum) entries reuse the query-slice LDS
constexpr int EMS_CAP = 256;
constexpr int EMS_LANES = 8;    // lanes per open pair in the sparse finish
static_assert(2 * EMS_CAP * 2 <= EST_LDS_FLOATS, "pair lists must fit the query-slice LDS");

// One open pair's sum over one segment for the multi-stage sparse finish,
// this lane's share: S = sum of c_j q'_j over the dims of chunks c0, c0 + cs,
// c0 + 2 cs, ... of 32 dims (the caller turns S into the segment's term
// f_s (S - h sum_j q'_j), h = (2^B - 1)/2).  rec: the record's bit planes of
// the segment (plane p at rec + p pb, dim j at byte j/8, bit j%8, most
// significant plane first); qs: the query's projected values of the
// segment.  A whole chunk reads 4 bytes per plane unconditionally (they lie
// inside the plane), a ragged last chunk only the plane's bytes, with zero
// query values past W.
template <int B>
__device__ __forceinline__ float pair_segment(const uint8_t* __restrict__ rec, int W,
                                              const float* __restrict__ qs, bool qvec,
                                              const uint64_t* __restrict__ spread, int c0, int cs) {
    const int pb = (W + 7) >> 3;
    struct Chunk { uint32_t w[B]; float q[32]; };
    auto load_full = [&](Chunk& c, int j0) {
        const uint8_t* src = rec + (j0 >> 3);
#pragma unroll
        for (int p = 0; p < B; ++p) __builtin_memcpy(&c.w[p], src + int64_t(p) * pb, 4);
        if (qvec) {
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const float4 x = reinterpret_cast<const float4*>(qs + j0)[v];
                c.q[4 * v] = x.x; c.q[4 * v + 1] = x.y; c.q[4 * v + 2] = x.z; c.q[4 * v + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int d = 0; d < 32; ++d) c.q[d] = qs[j0 + d];
        }
    };
    auto load_tail = [&](Chunk& c, int j0) {
        const int b0 = j0 >> 3;
#pragma unroll
        for (int p = 0; p < B; ++p) {
            uint32_t v = 0u;
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (b0 + b < pb) v |= uint32_t(rec[int64_t(p) * pb + b0 + b]) << (8 * b);
            c.w[p] = v;
        }
#pragma unroll
        for (int d = 0; d < 32; ++d) c.q[d] = j0 + d < W ? qs[j0 + d] : 0.f;
    };
    // 8 dims per table lookup and plane: the last 8 planes build the low
    // byte of each code, the planes before them (B > 8) the high byte
    float acc = 0.f, acc2 = 0.f;
    auto use = [&](const Chunk& c) {
#pragma unroll
        for (int by = 0; by < 4; ++by) {
            uint64_t lo = 0, hi = 0;
#pragma unroll
            for (int p = 0; p < B; ++p) {
                const uint64_t sp = spread[(c.w[p] >> (8 * by)) & 0xffu];
                if (p < B - 8) hi = (hi << 1) | sp;
                else lo = (lo << 1) | sp;
            }
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                float code = float(uint32_t(lo >> (8 * d)) & 0xffu);
                if (B > 8) code = fmaf(float(uint32_t(hi >> (8 * d)) & 0xffu), 256.f, code);
                if (by & 1) acc2 = fmaf(code, c.q[8 * by + d], acc2);
                else acc = fmaf(code, c.q[8 * by + d], acc);
            }
        }
    };
    Chunk x;
    int j0 = 32 * c0;
    for (; j0 + 32 <= W; j0 += 32 * cs) {
        load_full(x, j0);
        use(x);
    }
    if (j0 < W) {
        load_tail(x, j0);
        use(x);
    }
    return acc + acc2;
}

__device__ __forceinline__ float pair_segment_any(int B, const uint8_t* __restrict__ rec, int W,
                                                  const float* __restrict__ qs, bool qvec,
                                                  const uint64_t* __restrict__ spread, int c0,
                                                  int cs) {
    switch (B) {
#define SAQ_PAIR_CASE(K) \
    case K: return pair_segment<K>(rec, W, qs, qvec, spread, c0, cs);
        SAQ_PAIR_CASE(1) SAQ_PAIR_CASE(2) SAQ_PAIR_CASE(3) SAQ_PAIR_CASE(4)
        SAQ_PAIR_CASE(5) SAQ_PAIR_CASE(6) SAQ_PAIR_CASE(7) SAQ_PAIR_CASE(8)
        SAQ_PAIR_CASE(9) SAQ_PAIR_CASE(10) SAQ_PAIR_CASE(11) SAQ_PAIR_CASE(12)
        SAQ_PAIR_CASE(13) SAQ_PAIR_CASE(14) SAQ_PAIR_CASE(15) SAQ_PAIR_CASE(16)
#undef SAQ_PAIR_CASE
        default: return 0.f;
    }
}

// Occupancy: the plain scan fits 4 waves per SIMD (about 127 VGPRs), the
// multi-stage variant 3 (its bound state and lists need up to 168).
// QB: 32-query MFMA blocks per tile, 2, or 1 when at most 32 queries are
// scanned (the second block would be all padding).  FL: lanes per open pair
// in the multi-stage sparse finish, EMS_LANES, or 1 for plans whose kept
// segments are all at most 32 dims (one chunk: the other lanes of a group
// would idle).  A separate instantiation, so plans with wider segments keep
// their code and registers unchanged.  PK: packed k-steps for plain scans of
// plans whose kept widths are all multiples of 16 and whose segments would
// leave many steps half empty (see fetch_packed).  TR: plain scans
// stepping segment by segment take the records as the B operand, so each
// lane's accumulators belong to the one record it unpacks; the operand is
// then c - h itself (exact in one bf16 term up to 8 bits, two up to 16) and
// the segment factor is applied by rescaling the lane's accumulators where
// a segment starts (see seg_start): three or five products per 16 dims
// instead of six, and no split of the record's values.
template <bool MS, int QB, int FL = EMS_LANES, bool PK = false, bool TR = false>
__global__ __launch_bounds__(256, (MS || TR) ? 3 : 4) void estimate_kernel(
    const float* __restrict__ Qp, int nq, int dk, const float* __restrict__ qn2,
    const SegEntry* __restrict__ segs, int n_kept, const uint8_t* __restrict__ codes,
    int64_t code_bytes, const float* __restrict__ factors, int64_t n, int prefix,
    const float* __restrict__ lbq, const float* __restrict__ qsum, const float* __restrict__ tau,
    uint8_t* __restrict__ stage, float* __restrict__ out, const u32x4* __restrict__ Qs, int qg) {
    __shared__ __attribute__((aligned(16))) float lds[EST_LDS_FLOATS];
    __shared__ uint64_t spread[256];      // bit i of the index -> bit 8 i
    // multi-stage: open-pair counts of alternate bound checks, list fills
    __shared__ int ms_open[2], ms_fill[2];
    // query slice term tm of buffer b, query row q, dims d..d+7: 16 bytes at
    // bq(b, tm, q, d)
    auto bq = [&](int b, int tm, int q, int d) {
        return reinterpret_cast<u32x4*>(reinterpret_cast<__bf16*>(lds) +
                                        ((b * 3 + tm) * EQ + q) * EROW + d);
    };
    static_assert(!(TR && MS), "the multi-stage scan keeps records as the A operand");
    const int t = threadIdx.x;
    {
        uint64_t v = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) v |= uint64_t((t >> i) & 1) << (8 * i);
        spread[t] = v;                    // blockDim.x == 256
        if (t < 2) {
            ms_open[t] = 0;
            ms_fill[t] = 0;
        }
    }
    __syncthreads();
    const int wave = t >> 6, lane = t & 63, li = lane & 31, lh = lane >> 5;
    const int64_t r0 = int64_t(blockIdx.x) * ER;
    const int q0 = blockIdx.y * EQ;

    // unpacking: record ur of the tile, dims 16 uh .. 16 uh + 15 of a k-step;
    // records past n read record n - 1 and are never stored
    // lane li + 32 lh of wave w unpacks record 32 w + li, dims 16 lh .. 16 lh + 15:
    // exactly its own A operand of the 32 x 32 x 2 MFMAs (row li, k = 16 lh + j
    // at step j), so the record tile never passes through LDS
    const int ur = 32 * wave + li, uh = lh;
    const int64_t ri = min(r0 + ur, n - 1);
    const uint8_t* rec = codes + ri * code_bytes;
    const float* fr = factors + ri * (n_kept + 1);
    // query staging: query qq of the tile, dims qd .. qd + 7 of a k-step
    const int qq = t >> 2, qd = (t & 3) * 8;
    const bool qlive = q0 + qq < nq;
    const float* qrow = Qp + int64_t(qlive ? q0 + qq : 0) * dk;

    // the k-step's raw inputs: plane words, the staged query dims as three
    // bf16 terms, the segment factor
    struct Raw { uint32_t w[16]; u32x4 q[3]; float fs; };
    // this lane's record operand of the current k-step: f_s (c - h) of its
    // 16 dims as three exact bf16 terms, for each half (dims 16 lh + 8 m ..
    // + 7); the A operand, or with TR the B operand
    u32x4 Areg[3][2];
    // TR: the record's operand is c - h as terms 0 (and 1 above 8 bits);
    // its accumulators hold the inner products divided by gsc, the factor
    // of the last segment taken; `use` is false in a skipped segment, whose
    // operand is zero; fmx is the largest factor magnitude seen
    bool use = true;
    float gsc = 1.f, fmx = 0.f;
    // bits of a segment the scan reads: all of them, or the first `prefix`
    // (progressive approximation, Section 3.2)
    auto used_bits = [&](int B) { return (prefix > 0 && prefix < B) ? prefix : B; };
    // plane words of this lane's 16 dims d0 .. d0 + 15 of segment e (zero
    // past its width)
    auto fetch_planes = [&](Raw& g, const SegEntry& e, int B, int d0) {
        const int W = e.width, pb = (W + 7) >> 3;
        const bool any = d0 < W, two = d0 + 8 < W;
        const uint8_t* pl = rec + e.code_off + (d0 >> 3);
        // both bytes of a lane's 16 dims in one 16-bit load when they are
        // inside the plane and 2-byte aligned (even record, segment and
        // plane offsets); otherwise byte loads
        const bool half = two && ((code_bytes | int64_t(e.code_off) | int64_t(pb)) & 1) == 0;
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            uint32_t w = 0u;
            if (p < B && any) {
                if (half) {
                    w = *reinterpret_cast<const uint16_t*>(pl + int64_t(p) * pb);
                } else {
                    w = pl[int64_t(p) * pb];
                    if (two) w |= uint32_t(pl[int64_t(p) * pb + 1]) << 8;
                }
            }
            g.w[p] = w;
        }
    };
    // the scan's pre-split query of kept dims kq + qd .. kq + qd + 7 (kq a
    // multiple of 8; dims past a segment meet zero codes, groups past D_kept
    // are zero)
    auto fetch_query = [&](Raw& g, int kq) {
        const u32x4* src = Qs + (int64_t(qlive ? q0 + qq : 0) * qg + ((kq + qd) >> 3)) * 3;
#pragma unroll
        for (int tm = 0; tm < 3; ++tm) g.q[tm] = qlive ? src[tm] : u32x4{0u, 0u, 0u, 0u};
    };
    auto fetch = [&](Raw& g, int si, int j0) {
        const SegEntry e = segs[si];
        const int W = e.width, B = used_bits(e.bits);
        fetch_planes(g, e, B, j0 + 16 * uh);
        if ((e.col & 7) == 0) {
            fetch_query(g, e.col + j0);
        } else {
            float qv[8];
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                const int j = j0 + qd + d;
                qv[d] = (qlive && j < W) ? qrow[e.col + j] : 0.f;
            }
            uint32_t t0[4], t1[4], t2[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) split3(qv[2 * k], qv[2 * k + 1], t0[k], t1[k], t2[k]);
            g.q[0] = u32x4{t0[0], t0[1], t0[2], t0[3]};
            g.q[1] = u32x4{t1[0], t1[1], t1[2], t1[3]};
            g.q[2] = u32x4{t2[0], t2[1], t2[2], t2[3]};
        }
        // the b-bit prefix estimates with the stored factor times 2^(B - b);
        // the factor changes only where a segment starts
        if (j0 == 0) g.fs = ldexpf(fr[si], e.bits - B);
    };
    // this lane's operand from its 16 dims d0 .. d0 + 15 of a segment of
    // width W read at B bits (zero past W), and the staged query slice
    auto put_core = [&](const Raw& g, int W, int B, int d0, int buf) {
        uint32_t c[16];
        // loops fully unrolled with a uniform predicate per plane, so g stays
        // in registers (a loop exit would index it dynamically)
        if (B <= 8) {
            // codes as the bytes of two words: each plane byte is spread to
            // one bit per byte by the table and shifted in (a code below
            // 2^8 never carries into the next byte)
            uint64_t lo = 0, hi = 0;
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                if (p < B) {
                    lo = (lo << 1) | spread[g.w[p] & 0xffu];
                    hi = (hi << 1) | spread[(g.w[p] >> 8) & 0xffu];
                }
            }
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                c[d] = uint32_t(lo >> (8 * d)) & 0xffu;
                c[8 + d] = uint32_t(hi >> (8 * d)) & 0xffu;
            }
        } else {
#pragma unroll
            for (int d = 0; d < 16; ++d) c[d] = 0u;
#pragma unroll
            for (int p = 0; p < 16; ++p) {
                if (p < B) {
#pragma unroll
                    for (int d = 0; d < 16; ++d) c[d] = (c[d] << 1) | ((g.w[p] >> d) & 1u);
                }
            }
        }
        // f_s (c - h) with h = (2^B - 1)/2; c - h is exact in FP32
        const float h = 0.5f * float((1 << B) - 1);
        float a[16];
        if constexpr (TR) {
            // c - h alone: 2c - (2^B - 1) is an odd integer below 2^B, so
            // c - h has at most B significant bits, exact as one bf16 term
            // for B <= 8 and as two (the rest below half an ulp of the
            // first) for B <= 16
#pragma unroll
            for (int d = 0; d < 16; ++d) a[d] = (use && d0 + d < W) ? float(c[d]) - h : 0.f;
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                uint32_t t0[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) t0[k] = pack_bf16x2(a[8 * m + 2 * k], a[8 * m + 2 * k + 1]);
                Areg[0][m] = u32x4{t0[0], t0[1], t0[2], t0[3]};
                uint32_t t1[4] = {0u, 0u, 0u, 0u};
                if (B > 8) {
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        t1[k] = pack_bf16x2(a[8 * m + 2 * k] - __uint_as_float(t0[k] << 16),
                                            a[8 * m + 2 * k + 1] - __uint_as_float(t0[k] & 0xffff0000u));
                }
                Areg[1][m] = u32x4{t1[0], t1[1], t1[2], t1[3]};
            }
        } else {
#pragma unroll
            for (int d = 0; d < 16; ++d) a[d] = (d0 + d < W) ? g.fs * (float(c[d]) - h) : 0.f;
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                uint32_t t0[4], t1[4], t2[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) split3(a[8 * m + 2 * k], a[8 * m + 2 * k + 1], t0[k], t1[k], t2[k]);
                Areg[0][m] = u32x4{t0[0], t0[1], t0[2], t0[3]};
                Areg[1][m] = u32x4{t1[0], t1[1], t1[2], t1[3]};
                Areg[2][m] = u32x4{t2[0], t2[1], t2[2], t2[3]};
            }
        }
#pragma unroll
        for (int tm = 0; tm < 3; ++tm) *bq(buf, tm, qq, qd) = g.q[tm];
    };
    auto put = [&](const Raw& g, int si, int j0, int buf) {
        const SegEntry e = segs[si];
        put_core(g, e.width, used_bits(e.bits), j0 + 16 * uh, buf);
    };
    // Packed k-steps (PK, plain scans of plans whose kept widths are all
    // multiples of 16): step kk covers kept dims EK kk .. EK kk + EK - 1
    // whichever segments hold them, so a 16-dim segment no longer pads a
    // step to 32.  The segment factor is part of each lane's operand, so the
    // two halves of a step may belong to different segments; each lane
    // follows its half with a cursor over the segments.
    int seg_l = 0;
    auto lane_seg = [&](int kk) -> int {   // -1 past D_kept
        const int kd = EK * kk + 16 * uh;
        if (kd >= dk) return -1;
        while (kd >= segs[seg_l].col + segs[seg_l].width) ++seg_l;
        return seg_l;
    };
    auto fetch_packed = [&](Raw& g, int kk) {
        const int sl = lane_seg(kk);
        if (sl >= 0) {
            const SegEntry e = segs[sl];
            const int B = used_bits(e.bits);
            fetch_planes(g, e, B, EK * kk + 16 * uh - e.col);
            g.fs = ldexpf(fr[sl], e.bits - B);
        } else {
#pragma unroll
            for (int p = 0; p < 16; ++p) g.w[p] = 0u;
            g.fs = 0.f;
        }
        fetch_query(g, EK * kk);
    };
    auto put_packed = [&](const Raw& g, int kk, int buf) {
        const int kd = EK * kk + 16 * uh;
        int W = 0, B = 1, d0 = 0;
        if (kd < dk) {
            const SegEntry e = segs[seg_l];
            W = e.width;
            B = used_bits(e.bits);
            d0 = kd - e.col;
        }
        put_core(g, W, B, d0, buf);
    };

    floatx16 acc[2];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[b][r] = 0.f;

    // lane's pairs: query q0 + 32 bj + li, for register r the record
    // r0 + 32 wave + 8 (r/4) + 4 lh + r%4; bit 16 bj + r of `open` is set
    // while that pair is live and not pruned (multi-stage mode only)
    auto rec_of = [&](int r) { return r0 + 32 * wave + 8 * (r >> 2) + 4 * lh + (r & 3); };
    uint32_t open = 0;
    float on2v[16];
    if constexpr (MS) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t i = rec_of(r);
            on2v[r] = i < n ? factors[i * (n_kept + 1) + n_kept] : 0.f;
#pragma unroll
            for (int bj = 0; bj < QB; ++bj)
                if (i < n && q0 + 32 * bj + li < nq) open |= 1u << (16 * bj + r);
        }
    }
    auto on2 = [&](int r) { return on2v[r]; };
    // the lane's records are rbase + roff(r)
    const int64_t rbase = r0 + 32 * wave + 4 * lh;
    auto roff = [](int r) { return 8 * (r >> 2) + (r & 3); };
    // rows of out (and stage) start 16-byte (4-byte) aligned
    const bool vec_ms = (n & 3) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0 &&
                        (reinterpret_cast<uintptr_t>(stage) & 3) == 0;
    // close the pairs whose bound before segment si exceeds their threshold;
    // returns the number of pairs of the workgroup still open
    int par = 0;
    auto prune = [&](int si) -> int {
#pragma unroll
        for (int bj = 0; bj < QB; ++bj) {
            const int q = q0 + 32 * bj + li;
            if (q >= nq) continue;
            const float lb = lbq[int64_t(q) * n_kept + si], th = tau[q];
            float* orow = out + int64_t(q) * n + rbase;
            uint8_t* srow = stage ? stage + int64_t(q) * n + rbase : nullptr;
            // records 4g .. 4g + 3 are consecutive: when all four close
            // here, one 16-byte value store and one 4-byte stage store
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const uint32_t gbits = 0xfu << (16 * bj + 4 * g);
                if ((open & gbits) == 0u) continue;
                float v[4];
                uint32_t close = 0u;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = 4 * g + e;
                    v[e] = (on2(r) - 2.f * acc[bj][r]) + lb;
                    if ((open & (1u << (16 * bj + r))) && v[e] > th) close |= 1u << (16 * bj + r);
                }
                if (close == 0u) continue;
                open &= ~close;
                const int o = roff(4 * g);
                if (close == gbits && vec_ms) {
                    *reinterpret_cast<float4*>(orow + o) = make_float4(v[0], v[1], v[2], v[3]);
                    if (srow) *reinterpret_cast<uint32_t*>(srow + o) = uint32_t(si) * 0x01010101u;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (close & (1u << (16 * bj + 4 * g + e))) {
                            orow[o + e] = v[e];
                            if (srow) srow[o + e] = uint8_t(si);
                        }
                }
            }
        }
        if (open != 0u) atomicAdd(&ms_open[par], __popc(open));
        __syncthreads();
        const int c = ms_open[par];
        // the other counter was last read before an earlier barrier, and
        // is next added to after a later one
        if (t == 0) ms_open[par ^ 1] = 0;
        par ^= 1;
        return c;
    };
    // the open pairs go to list 0 with their partial sums (key: query of the
    // tile << 8 | record of the tile); call after a bound check, when no
    // thread reads the query slices any more
    uint32_t* keys = reinterpret_cast<uint32_t*>(lds);   // [2][EMS_CAP]
    float* part = lds + 2 * EMS_CAP;                     // [2][EMS_CAP]
    auto to_list = [&]() {
        const int k = __popc(open);
        if (k > 0) {
            int slot = atomicAdd(&ms_fill[0], k);
#pragma unroll
            for (int bj = 0; bj < QB; ++bj)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    if (open & (1u << (16 * bj + r))) {
                        keys[slot] = uint32_t((32 * bj + li) << 8) |
                                     uint32_t(32 * wave + 8 * (r >> 2) + 4 * lh + (r & 3));
                        part[slot] = acc[bj][r];
                        ++slot;
                    }
        }
        open = 0u;
        __syncthreads();
    };

    // the k-steps in order: (segment s, first dim j0)
    int s = 0, j0 = 0;
    while (s < n_kept && segs[s].width <= 0) ++s;
    bool go = s < n_kept;
    int listed = 0;          // open pairs handed to the sparse finish
    if constexpr (MS) {
        if (go) {
            const int c = prune(s);
            go = c > 0;
            if (go && c <= EMS_CAP) {
                to_list();
                listed = c;
                go = false;
            }
        }
    }
    // one k-step's products: per half m the six products of the split
    // terms, smallest first (the projection's scheme), against queries li
    // and 32 + li
    auto mfma_step = [&](int buf) {
        constexpr int TA[6] = {2, 1, 0, 1, 0, 0};
        constexpr int TB[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            u32x4 B0[3], B1[3];
#pragma unroll
            for (int tm = 0; tm < 3; ++tm) {
                B0[tm] = *bq(buf, tm, li, 16 * lh + 8 * m);
                if (QB == 2) B1[tm] = *bq(buf, tm, 32 + li, 16 * lh + 8 * m);
            }
#pragma unroll
            for (int u = 0; u < 6; ++u) {
                acc[0] = mfma_bf16(Areg[TA[u]][m], B0[TB[u]], acc[0]);
                if (QB == 2) acc[1] = mfma_bf16(Areg[TA[u]][m], B1[TB[u]], acc[1]);
            }
        }
    };
    // TR, where segment s starts (its factor f: the lane's record's, times
    // 2^(B - b) for a prefix): the accumulators, done with the segments
    // before, are rescaled from gsc to f, so the products that follow need
    // no factor.  A zero factor, or one below 2^-60 of the largest seen,
    // skips the segment (zero operand, no rescale): its part of the inner
    // product is then below 2^-30 of ||o|| ||q - c|| (the code's norm is at
    // most 2^20 times another segment's, their cosines at least 2^-5), and
    // every accumulator holds its products times at most 2^60.  A NaN
    // factor propagates.
    auto seg_start = [&](float f) {
        const float af = fabsf(f);
        fmx = fmaxf(fmx, af);
        use = f != 0.f && !(af < 0x1p-60f * fmx);
        // no branch around the accumulators: a skipped segment scales by 1
        const float ratio = use ? gsc / f : 1.f;
        gsc = use ? f : gsc;
#pragma unroll
        for (int b = 0; b < QB; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[b][r] *= ratio;
    };
    // TR: one k-step's products, the query slices (queries li and 32 + li
    // of the tile) as the A operand and the lane's record as the B operand,
    // smallest first; `two`: the segment's codes take two terms
    auto mfma_step_tr = [&](int buf, bool two) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            // query term tm (2, 1, 0: smallest first) times the record's
            // terms; q2 c1, below 2^-24 of the product, is dropped
#pragma unroll
            for (int tm = 2; tm >= 0; --tm) {
                const u32x4 a0 = *bq(buf, tm, li, 16 * lh + 8 * m);
                u32x4 a1;
                if (QB == 2) a1 = *bq(buf, tm, 32 + li, 16 * lh + 8 * m);
                if (two && tm < 2) {
                    acc[0] = mfma_bf16(a0, Areg[1][m], acc[0]);
                    if (QB == 2) acc[1] = mfma_bf16(a1, Areg[1][m], acc[1]);
                }
                acc[0] = mfma_bf16(a0, Areg[0][m], acc[0]);
                if (QB == 2) acc[1] = mfma_bf16(a1, Areg[0][m], acc[1]);
            }
        }
    };
    if constexpr (PK) {
        static_assert(!MS, "packed k-steps are for the plain scan");
        static_assert(!TR, "packed k-steps take the six-product operand");
        const int nk = (dk + EK - 1) / EK;
        if (go && nk > 0) {
            Raw g;
            fetch_packed(g, 0);
            put_packed(g, 0, 0);
            __syncthreads();
            for (int kt = 0;; ++kt) {
                const int buf = kt & 1;
                const bool more = kt + 1 < nk;
                if (more) fetch_packed(g, kt + 1);
                mfma_step(buf);
                if (!more) break;
                put_packed(g, kt + 1, buf ^ 1);
                __syncthreads();
            }
        }
    } else if (go) {
        Raw g;
        fetch(g, s, j0);
        if constexpr (TR) seg_start(g.fs);
        put(g, s, j0, 0);
        __syncthreads();
        for (int kt = 0;; ++kt) {
            const int buf = kt & 1;
            if constexpr (MS) {
                if (kt > 0 && j0 == 0) {
                    const int c = prune(s);
                    if (c == 0) break;
                    if (c <= EMS_CAP) {
                        to_list();
                        listed = c;
                        break;
                    }
                }
            }
            // the next k-step
            int s1 = s, j1 = j0 + EK;
            if (j1 >= segs[s1].width) { ++s1; j1 = 0; }
            const bool more = s1 < n_kept;
            if (more) fetch(g, s1, j1);
            if constexpr (TR)
                mfma_step_tr(buf, used_bits(segs[s].bits) > 8);
            else
                mfma_step(buf);
            if (!more) break;
            if constexpr (TR) {
                if (j1 == 0) seg_start(g.fs);
            }
            put(g, s1, j1, buf ^ 1);
            __syncthreads();
            s = s1;
            j0 = j1;
        }
    }

    if constexpr (TR) {
        // lane: record r0 + 32 wave + li; for register r of block bj the
        // query q0 + 32 bj + 8 (r/4) + 4 lh + r%4, so each store writes 32
        // consecutive records per half-wave
        const int64_t i = r0 + 32 * wave + li;
        if (i < n) {
            const float o2 = factors[i * (n_kept + 1) + n_kept];
#pragma unroll
            for (int bj = 0; bj < QB; ++bj)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int q = q0 + 32 * bj + 8 * (r >> 2) + 4 * lh + (r & 3);
                    if (q < nq) out[int64_t(q) * n + i] = o2 + qn2[q] - 2.f * (gsc * acc[bj][r]);
                }
        }
    }
    // lane: query q0 + 32 bj + li; for register r the record
    // r0 + 32 wave + 8 (r/4) + 4 lh + r%4
    const bool vec_out = (n & 3) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0;
#pragma unroll
    for (int bj = 0; bj < (TR ? 0 : QB); ++bj) {
        const int q = q0 + 32 * bj + li;
        if (q >= nq) continue;
        const float qn = qn2[q];
        float* orow = out + int64_t(q) * n;
        if constexpr (MS) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t i = rec_of(r);
                if (open & (1u << (16 * bj + r))) {
                    orow[i] = on2(r) + qn - 2.f * acc[bj][r];
                    if (stage) stage[int64_t(q) * n + i] = uint8_t(n_kept);
                }
            }
        } else {
            // records 4g .. 4g + 3 of the lane are consecutive: one 16-byte
            // store when all four exist and the row is 16-byte aligned (one
            // store instruction then writes 32 B runs of 32 rows, not 4 B)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int64_t i0 = rec_of(4 * g);
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    v[e] = i0 + e < n ? factors[(i0 + e) * (n_kept + 1) + n_kept] + qn -
                                            2.f * acc[bj][4 * g + e]
                                      : 0.f;
                if (i0 + 3 < n && vec_out) {
                    *reinterpret_cast<float4*>(orow + i0) = make_float4(v[0], v[1], v[2], v[3]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (i0 + e < n) orow[i0 + e] = v[e];
                }
            }
        }
    }

    if constexpr (MS) {
        // sparse finish from segment s: list `cur` holds the pairs open at
        // its start (workgroup-uniform count `listed`)
        // a pair's chunks of 32 dims are shared by FL consecutive lanes
        const int sub = t & (FL - 1), grp = t / FL;
        int cur = 0;
        for (int si = s; listed > 0 && si < n_kept; ++si) {
            const SegEntry e = segs[si];
            const bool qvec = ((dk | e.col) & 3) == 0 && (reinterpret_cast<uintptr_t>(Qp) & 15) == 0;
            const bool last = si + 1 == n_kept;
            const float h = 0.5f * float((1 << e.bits) - 1);
            // a pair with partial sum acc after segment si: the full estimate
            // after the last segment, else closed by the bound before si + 1
            // or appended to the next list
            auto ms_close = [&](float o2, float acc, int q, int64_t oi, uint32_t key) {
                if (last) {
                    out[oi] = o2 + qn2[q] - 2.f * acc;
                    if (stage) stage[oi] = uint8_t(n_kept);
                    return;
                }
                const float v = (o2 - 2.f * acc) + lbq[int64_t(q) * n_kept + si + 1];
                if (v > tau[q]) {
                    out[oi] = v;
                    if (stage) stage[oi] = uint8_t(si + 1);
                } else {
                    const int slot = atomicAdd(&ms_fill[cur ^ 1], 1);
                    keys[(cur ^ 1) * EMS_CAP + slot] = key;
                    part[(cur ^ 1) * EMS_CAP + slot] = acc;
                }
            };
            constexpr int G = 256 / FL;            // lane groups
            for (int k = grp; k < listed; k += G) {
                const uint32_t key = keys[cur * EMS_CAP + k];
                const int q = q0 + int(key >> 8);
                const int64_t i = r0 + int(key & 255u);
                float S = pair_segment_any(e.bits, codes + i * code_bytes + e.code_off, e.width,
                                           Qp + int64_t(q) * dk + e.col, qvec, spread, sub, FL);
                // the group's lanes are consecutive: a butterfly leaves the
                // pair's sum in all of them
#pragma unroll
                for (int o = 1; o < FL; o <<= 1) S += __shfl_xor(S, o);
                if (sub != 0) continue;
                const float* fi = factors + i * (n_kept + 1);
                const float acc = part[cur * EMS_CAP + k] +
                                  fi[si] * (S - h * qsum[int64_t(q) * n_kept + si]);
                ms_close(fi[n_kept], acc, q, int64_t(q) * n + i, key);
            }
            __syncthreads();
            listed = ms_fill[cur ^ 1];
            // list `cur` is spent: its fill is cleared before anyone appends
            // to it again, two segments on
            if (t == 0) ms_fill[cur] = 0;
            __syncthreads();
            cur ^= 1;
        }
    }
}

// The scan's queries as exact three-term bf16 splits, once per scan rather
// than once per record tile: query q, kept dims 8 g .. 8 g + 7 at
// Qs[(q qg + g) 3 + term] (16 bytes per term); dims past D_kept are zero.
__global__ __launch_bounds__(256) void split_query_kernel(const float* __restrict__ Qp, int nq,
                                                          int dk, int qg, u32x4* __restrict__ Qs) {
    const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= int64_t(nq) * qg) return;
    const int64_t q = idx / qg;
    const int g = int(idx - q * qg);
    float v[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const int j = 8 * g + d;
        v[d] = j < dk ? Qp[q * dk + j] : 0.f;
    }
    uint32_t t0[4], t1[4], t2[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) split3(v[2 * k], v[2 * k + 1], t0[k], t1[k], t2[k]);
    Qs[idx * 3 + 0] = u32x4{t0[0], t0[1], t0[2], t0[3]};
    Qs[idx * 3 + 1] = u32x4{t1[0], t1[1], t1[2], t1[3]};
    Qs[idx * 3 + 2] = u32x4{t2[0], t2[1], t2[2], t2[3]};
}

// 8-dim query groups the split covers: the kept dims and the 32 more a
// segment's last k-step can read past D_kept
inline int query_groups(int dk) { return (dk + 7) / 8 + 4; }

// sigma_s of Section 4.3 for query blockIdx.y and kept segment blockIdx.x:
// ||S_s q'_s||, the standard deviation over the data of <o_s, q_s>.  The
// segment's rows are split into SIG_RB contiguous blocks (blockIdx.z), so a
// single query still fills the chip; each workgroup writes the sum of
// squares of its rows, and stage_bound_kernel adds the blocks in a fixed
// order.  A wave takes rows of the block (coalesced along the row), the
// query slice sits in LDS.  Block 0 also writes qsum: the plain sum of the
// slice, which turns the multi-stage sparse finish's sum of c_j q'_j into
// the segment's term.
constexpr int SIG_MAXW = 4096;
constexpr int SIG_RB = 8;
__global__ __launch_bounds__(256) void sigma_kernel(const float* __restrict__ Qp, int dk,
                                                    const SegEntry* __restrict__ segs, int n_kept,
                                                    const float* __restrict__ S,
                                                    float* __restrict__ sig_part,
                                                    float* __restrict__ qsum) {
    __shared__ float qs[SIG_MAXW];
    __shared__ float part[4], psum[4];
    const int si = blockIdx.x, q = blockIdx.y, rb = blockIdx.z;
    int64_t off = 0;
    for (int t = 0; t < si; ++t) off += int64_t(segs[t].width) * segs[t].width;
    const SegEntry e = segs[si];
    const int W = e.width;
    const float* qrow = Qp + int64_t(q) * dk + e.col;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float qt = 0.f;
    for (int j = threadIdx.x; j < W; j += 256) {
        qs[j] = qrow[j];
        qt += qrow[j];
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) qt += __shfl_xor(qt, d);
    if (lane == 0) psum[wave] = qt;
    __syncthreads();
    float v = 0.f;
    const int i0 = int(int64_t(W) * rb / SIG_RB), i1 = int(int64_t(W) * (rb + 1) / SIG_RB);
    for (int i = i0 + wave; i < i1; i += 4) {
        const float* row = S + off + int64_t(i) * W;
        float y = 0.f;
        for (int j = lane; j < W; j += 64) y = fmaf(row[j], qs[j], y);
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) y += __shfl_xor(y, d);
        v = fmaf(y, y, v);
    }
    if (lane == 0) part[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        sig_part[(int64_t(q) * n_kept + si) * SIG_RB + rb] = (part[0] + part[1]) + (part[2] + part[3]);
        if (rb == 0) qsum[int64_t(q) * n_kept + si] = (psum[0] + psum[1]) + (psum[2] + psum[3]);
    }
}

// lbq[q][s] = ||q - c||^2 - 2 m sum_{t >= s} sigma_t, one thread per query;
// sigma_t from sigma_kernel's row-block sums of squares, added in a fixed order
__global__ __launch_bounds__(256) void stage_bound_kernel(const float* __restrict__ sig_part,
                                                          const float* __restrict__ qn2, int nq,
                                                          int n_kept, float m,
                                                          float* __restrict__ lbq) {
    static_assert(SIG_RB == 8, "the fixed summation order below");
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    float t = 0.f;
    for (int si = n_kept - 1; si >= 0; --si) {
        const float* p = sig_part + (int64_t(q) * n_kept + si) * SIG_RB;
        t += sqrtf(((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7])));
        lbq[int64_t(q) * n_kept + si] = qn2[q] - 2.f * m * t;
    }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
saq_status hip_fail(hipError_t e, const char* what) {
    return saq::fail(SAQ_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// The plan must be uploaded, and to the current device: its buffer is read
// by the kernels launched there.
saq_status check_plan(const saq_plan* p, const char* what = "plan") {
    if (!p || p->dev == nullptr) return saq::fail(SAQ_EINVAL, std::string(what) + " not uploaded");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    if (dev != p->dev_id)
        return saq::fail(SAQ_EINVAL, std::string(what) + " uploaded on device " +
                                         std::to_string(p->dev_id) + ", current device " +
                                         std::to_string(dev));
    return SAQ_OK;
}

const u32x4* dev_Ms(const saq_plan* p) {
    return reinterpret_cast<const u32x4*>(static_cast<const char*>(p->dev) + p->layout.off_Ms);
}
const float* dev_c(const saq_plan* p) {
    return reinterpret_cast<const float*>(static_cast<const char*>(p->dev) + p->layout.off_c);
}
const SegEntry* dev_seg(const saq_plan* p) {
    return reinterpret_cast<const SegEntry*>(static_cast<const char*>(p->dev) + p->layout.off_seg);
}
const float* dev_S(const saq_plan* p) {
    return reinterpret_cast<const float*>(static_cast<const char*>(p->dev) + p->layout.off_S);
}

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

saq_status launch_project(const saq_plan* p, const float* X, int64_t n, float* O, int64_t ld,
                          int layout, float* norm2, hipStream_t st,
                          RefRows R = RefRows{nullptr, nullptr, 0}) {
    const int rows = p->acc64 ? gemm_rows<gemm_bi<true>()>() : gemm_rows<gemm_bi<false>()>();
    const int tiles_m = int((n + rows - 1) / rows);
    const int tiles_n = p->layout.n_pad / TN;
    // two halves of the XCDs when the pre-split M is larger than one L2 (4 MB)
    // and half of it fits
    const int64_t ms_bytes = int64_t(tiles_n) * (p->layout.k_pad / SK) * SCB * 16;
    const int halves = (tiles_n >= 2 && ms_bytes > (int64_t(4) << 20) && ms_bytes <= (int64_t(7) << 20)) ? 1 : 0;
    int64_t slots;
    if (!halves) {
        slots = int64_t((tiles_m + NXCD - 1) / NXCD) * tiles_n;
    } else {
        const int cm = tiles_n / 2, odd = tiles_n & 1;
        const int64_t rows = (tiles_m + NXCD / 2 - 1) / (NXCD / 2);
        const int64_t rows_mid = ((tiles_m + 1) / 2 + NXCD / 2 - 1) / (NXCD / 2);
        slots = rows * std::max(cm, tiles_n - cm - odd) + (odd ? rows_mid : 0);
    }
    const dim3 grid(unsigned(NXCD * slots));
    const bool vec = (p->D % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0) &&
                     ((reinterpret_cast<uintptr_t>(R.refs) & 15) == 0);
    if (layout == LAYOUT_DIMS && ((reinterpret_cast<uintptr_t>(O) & 15) != 0 || (ld % 4) != 0))
        return saq::fail(SAQ_EINVAL, "dims-major output needs a 16-byte aligned buffer and ld % 4 == 0");
    if (layout == LAYOUT_TILES && (reinterpret_cast<uintptr_t>(O) & 15) != 0)
        return saq::fail(SAQ_EINVAL, "tiled output needs a 16-byte aligned buffer");
#define SAQ_LAUNCH_PROJ(V, L, A, F)                                                               \
    hipLaunchKernelGGL((project_kernel<V, L, A, F>), grid, dim3(256), 0, st, X, n, p->D, dev_Ms(p),\
                       p->layout.k_pad, dev_c(p), p->D_kept, O, ld, norm2, tiles_m, tiles_n, R,  \
                       halves)
#define SAQ_LAUNCH_PROJ2(V, L, F) \
    do { if (p->acc64) SAQ_LAUNCH_PROJ(V, L, true, F); else SAQ_LAUNCH_PROJ(V, L, false, F); } while (0)
    // references per row exist for the tiled (encode) and row (query) layouts
    const bool ref = R.refs != nullptr;
    if (ref && layout == LAYOUT_DIMS)
        return saq::fail(SAQ_EUNSUPPORTED, "per-row references with the dims-major layout");
    if (layout == LAYOUT_TILES) {
        if (ref) {
            if (vec) SAQ_LAUNCH_PROJ2(true, LAYOUT_TILES, true); else SAQ_LAUNCH_PROJ2(false, LAYOUT_TILES, true);
        } else {
            if (vec) SAQ_LAUNCH_PROJ2(true, LAYOUT_TILES, false); else SAQ_LAUNCH_PROJ2(false, LAYOUT_TILES, false);
        }
    } else if (layout == LAYOUT_DIMS) {
        if (vec) SAQ_LAUNCH_PROJ2(true, LAYOUT_DIMS, false); else SAQ_LAUNCH_PROJ2(false, LAYOUT_DIMS, false);
    } else {
        if (ref) {
            if (vec) SAQ_LAUNCH_PROJ2(true, LAYOUT_ROWS, true); else SAQ_LAUNCH_PROJ2(false, LAYOUT_ROWS, true);
        } else {
            if (vec) SAQ_LAUNCH_PROJ2(true, LAYOUT_ROWS, false); else SAQ_LAUNCH_PROJ2(false, LAYOUT_ROWS, false);
        }
    }
#undef SAQ_LAUNCH_PROJ2
#undef SAQ_LAUNCH_PROJ
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SAQ_OK : hip_fail(e, "project_kernel launch");
}

constexpr size_t kMaxDynLds = 65536;

saq_status launch_quantize(const saq_plan* p, const float* O, int64_t ld, int layout, int64_t n,
                           const float* norm2, int rounds, uint8_t* codes, float* factors,
                           hipStream_t st) {
    const bool small = p->max_kept_b <= 8;
    // whole 32-dim blocks: a ragged last block's packed words may run past W
    const size_t lds = size_t(round_up(std::max(p->max_kept_w, 1), 32)) * 64 * (small ? 1 : 2);
    if (lds > kMaxDynLds)
        return saq::fail(SAQ_EUNSUPPORTED, "a kept segment is wider than the quantize kernel's "
                                           "LDS code buffer (1024 dims at <= 8 bits, 512 above)");
    const dim3 grid(unsigned((n + 63) / 64));
    // 4 when the codes base is 4-byte aligned, 2 when 2-byte aligned, else 1
    const uintptr_t cb = reinterpret_cast<uintptr_t>(codes);
    const int codes_align = (cb & 3) == 0 ? 4 : (cb & 1) == 0 ? 2 : 1;
#define SAQ_LAUNCH_Q(CT, L)                                                                       \
    hipLaunchKernelGGL((quantize_kernel<CT, L>), grid, dim3(64), lds, st, O, ld, n, dev_seg(p),   \
                       p->n_kept, norm2, rounds, codes, p->code_bytes, codes_align, factors)
    if (layout == LAYOUT_TILES) {
        if (small) SAQ_LAUNCH_Q(uint8_t, LAYOUT_TILES); else SAQ_LAUNCH_Q(uint16_t, LAYOUT_TILES);
    } else if (layout == LAYOUT_DIMS) {
        if (small) SAQ_LAUNCH_Q(uint8_t, LAYOUT_DIMS); else SAQ_LAUNCH_Q(uint16_t, LAYOUT_DIMS);
    } else {
        if (small) SAQ_LAUNCH_Q(uint8_t, LAYOUT_ROWS); else SAQ_LAUNCH_Q(uint16_t, LAYOUT_ROWS);
    }
#undef SAQ_LAUNCH_Q
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SAQ_OK : hip_fail(e, "quantize_kernel launch");
}

// workspace of saq_encode: O in the tiled layout ([ceil(n/64)][ld][64] with
// ld = D_kept) then norm2 [n]
int64_t enc_o_bytes(const saq_plan* p, int64_t n) {
    return round_up(std::max<int64_t>(n, 1), 64) * std::max(p->D_kept, 1) * 4;
}


struct BatchPlan {
    GemmArgs g{};
    QuantArgs q{};
    FusedArgs f{};
    int64_t gemm_blocks = 0, quant_blocks = 0, ws_need = 0;
    int waves = 1;
    int bi = 2;               // projection tile rows / 64
    bool fused = true;
    bool wide = false;
    bool any64 = false;       // some dataset takes FP64 k-tile totals
    size_t lds = 0;           // grouped: quantize LDS; fused: the kernel's dynamic LDS
};

// Lays out the workspace (per dataset: projected rows in the tiled layout
// and ||x - c||^2; then the fused launch's ticket) and fills the launch
// arguments of the chosen mode.  With ws == nullptr only the size is
// meaningful.
saq_status plan_batch(const saq_batch_item* items, int32_t count, int32_t rounds,
                      const saq_batch_tuning* tuning, void* ws, BatchPlan& B,
                      bool check_buffers = true) {
    if (!items || count <= 0 || count > BATCH_MAX)
        return saq::fail(SAQ_EINVAL, "batch must hold 1..16 datasets");
    if (rounds < 0) return saq::fail(SAQ_EINVAL, "rounds < 0");
    int wmax = 1;
    B.any64 = false;
    for (int i = 0; i < count; ++i) {
        const saq_batch_item& it = items[i];
        if (saq_status st = check_plan(it.plan, "batch plan"); st != SAQ_OK) return st;
        if (it.n < 0) return saq::fail(SAQ_EINVAL, "negative n");
        if (check_buffers && it.n > 0 && (!it.X_dev || !it.codes_dev || !it.factors_dev))
            return saq::fail(SAQ_EINVAL, "null buffer");
        if (it.n > 0) {
            // whole 32-dim blocks: a ragged last block's packed words may run past W
            wmax = std::max(wmax, int(round_up(it.plan->max_kept_w, 32)));
            B.wide |= it.plan->max_kept_b > 8;
            B.any64 |= it.plan->acc64;
        }
    }
    const size_t cs = B.wide ? 2 : 1;
    if (tuning && tuning->reserved != 0) return saq::fail(SAQ_EINVAL, "saq_batch_tuning.reserved must be 0");
    const int mode = tuning ? tuning->mode : SAQ_BATCH_FUSED;
    if (mode != SAQ_BATCH_FUSED && mode != SAQ_BATCH_GROUPED)
        return saq::fail(SAQ_EINVAL, "saq_batch_tuning.mode must be SAQ_BATCH_FUSED or SAQ_BATCH_GROUPED");
    B.fused = mode == SAQ_BATCH_FUSED;
    const int rows_req = tuning ? tuning->tile_rows : 0;
    if (rows_req != 0 && rows_req != 64 && rows_req != 128)
        return saq::fail(SAQ_EINVAL, "tile_rows must be 0, 64 or 128");
    if (rows_req == 128 && B.any64)
        return saq::fail(SAQ_EINVAL, "tile_rows 128 with a dataset that takes FP64 k-tile totals");
    B.bi = (B.any64 || rows_req == 64) ? 1 : 2;
    const int want = tuning && tuning->quant_waves > 0 ? tuning->quant_waves : 1;
    if (want != 1 && want != 2 && want != 4) return saq::fail(SAQ_EINVAL, "quant_waves must be 1, 2 or 4");
    if (size_t(wmax) * 64 * cs > kMaxDynLds)
        return saq::fail(SAQ_EUNSUPPORTED, "a kept segment is wider than the quantize kernel's "
                                           "LDS code buffer (1024 dims at <= 8 bits, 512 above)");
    if (B.fused) {
        // the item's quantize waves (4, 2 or the tile's BI) share the
        // workgroup's LDS with the projection tile
        int qw = 4;
        while (qw > B.bi && size_t(qw) * wmax * 64 * cs > kMaxDynLds) qw >>= 1;
        const size_t q = size_t(qw) * wmax * 64 * cs;
        const size_t g = size_t(B.bi == 1 ? split_lds_floats<1>() : split_lds_floats<2>()) * 4;
        if (q > kMaxDynLds)
            return saq::fail(SAQ_EUNSUPPORTED, "the fused launch's quantize waves need more than "
                                               "64 KiB of LDS at this tile shape (use tile_rows 64 "
                                               "or the grouped mode)");
        B.f.qwaves = qw;
        B.lds = std::max(q, g);
    } else {
        B.waves = want;
        while (B.waves > 1 && size_t(B.waves) * wmax * 64 * cs > kMaxDynLds) B.waves >>= 1;
        B.lds = size_t(B.waves) * wmax * 64 * cs;
    }
    const int xcd = !tuning || tuning->gemm_xcd_order != 0;

    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
    int64_t off = 0;
    auto take = [&](int64_t bytes) { const int64_t o = off; off += (bytes + 255) & ~int64_t(255); return o; };
    B.g.count = B.q.count = B.f.count = 0;
    B.g.xcd_order = xcd;
    B.q.rounds = B.f.rounds = rounds;
    B.q.wmax = B.f.wmax = wmax;
    B.f.items = 0;
    const int rows = 64 * B.bi;
    for (int i = 0; i < count; ++i) {
        const saq_batch_item& it = items[i];
        if (it.n == 0) continue;
        const saq_plan* p = it.plan;
        const int64_t ld = std::max(p->D_kept, 1);
        float* O = reinterpret_cast<float*>(base + take(enc_o_bytes(p, it.n)));
        float* nrm = reinterpret_cast<float*>(base + take(it.n * 4));
        const int vec = (p->D % 4 == 0) && ((reinterpret_cast<uintptr_t>(it.X_dev) & 15) == 0);
        const uintptr_t cb = reinterpret_cast<uintptr_t>(it.codes_dev);
        const int codes_align = (cb & 3) == 0 ? 4 : (cb & 1) == 0 ? 2 : 1;
        const int tiles_m = int((it.n + rows - 1) / rows), tiles_n = p->layout.n_pad / TN;
        GemmSet& G = B.g.set[B.g.count++];
        G.X = it.X_dev; G.n = it.n; G.D = p->D; G.acc64 = p->acc64 ? 1 : 0; G.vec = vec;
        G.Ms = dev_Ms(p); G.k_pad = p->layout.k_pad; G.cp = dev_c(p); G.dk = p->D_kept;
        G.tiles_m = tiles_m; G.tiles_n = tiles_n;
        G.O = O; G.ld = ld; G.norm2 = nrm;
        G.first_block = B.gemm_blocks;
        B.gemm_blocks += xcd ? int64_t(NXCD) * ((G.tiles_m + NXCD - 1) / NXCD) * G.tiles_n
                             : int64_t(G.tiles_m) * G.tiles_n;
        QuantSet& Q = B.q.set[B.q.count++];
        Q.O = O; Q.ld = ld; Q.n = it.n; Q.segs = dev_seg(p); Q.n_kept = p->n_kept; Q.norm2 = nrm;
        Q.codes = it.codes_dev; Q.code_bytes = p->code_bytes; Q.codes_align = codes_align;
        Q.factors = it.factors_dev;
        Q.first_block = B.quant_blocks;
        B.quant_blocks += (it.n + 64 * B.waves - 1) / (64 * B.waves);
        FusedSet& F = B.f.set[B.f.count++];
        F.X = it.X_dev; F.Ms = G.Ms; F.cp = G.cp; F.O = O; F.norm2 = nrm; F.segs = Q.segs;
        F.codes = it.codes_dev; F.factors = it.factors_dev;
        F.n = it.n; F.ld = ld; F.code_bytes = p->code_bytes; F.first_item = B.f.items;
        F.D = p->D; F.vec = vec; F.acc64 = G.acc64; F.k_pad = G.k_pad; F.dk = G.dk;
        F.tiles_m = tiles_m; F.tiles_n = tiles_n; F.n_kept = p->n_kept; F.codes_align = codes_align;
        if (B.fused) B.f.items += (it.n + 64 * B.f.qwaves - 1) / (64 * B.f.qwaves);
    }
    B.f.ticket = reinterpret_cast<unsigned long long*>(base + take(8));
    B.f.count = B.g.count;
    B.ws_need = off + 256;
    return SAQ_OK;
}

// Resident workgroups of a fused-launch instantiation on this device
template <class K>
saq_status fused_grid(K kernel, size_t lds, int64_t items, unsigned& grid) {
    int dev = 0, cus = 0, occ = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, 256, lds);
    if (e != hipSuccess) return hip_fail(e, "fused launch occupancy");
    const int64_t cap = int64_t(std::max(cus, 1)) * std::max(occ, 1);
    grid = unsigned(std::max<int64_t>(1, std::min(items, cap)));
    return SAQ_OK;
}
}  // namespace

extern "C" {

int64_t saq_plan_device_bytes(const saq_plan* p) { return p ? p->layout.bytes : -1; }

saq_status saq_plan_upload(saq_plan* p, void* dev_buf, void* stream) {
    if (!p || !dev_buf) return saq::fail(SAQ_EINVAL, "bad arguments");
    if ((reinterpret_cast<uintptr_t>(dev_buf) & 255) != 0)
        return saq::fail(SAQ_EINVAL, "plan buffer must be 256-byte aligned");
    const hipError_t e = hipMemcpyAsync(dev_buf, p->staging.data(), size_t(p->layout.bytes),
                                        hipMemcpyHostToDevice, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "plan upload");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    p->dev = dev_buf;
    p->dev_id = dev;
    return SAQ_OK;
}

int64_t saq_encode_workspace_bytes(const saq_plan* p, int64_t n) {
    if (!p || n < 0) return -1;
    return round_up(enc_o_bytes(p, n), 256) + round_up(std::max<int64_t>(n, 1), 64) * 4 + 256;
}

static saq_status check_layout(const saq_plan* p, int64_t n, int64_t ld, int32_t layout) {
    if (layout == LAYOUT_ROWS) {
        if (ld < p->D_kept) return saq::fail(SAQ_EINVAL, "ld < D_kept for the row layout");
    } else if (layout == LAYOUT_DIMS) {
        if (ld < n || (ld % 4) != 0) return saq::fail(SAQ_EINVAL, "dims layout needs ld >= n and ld % 4 == 0");
    } else if (layout == LAYOUT_TILES) {
        if (ld < p->D_kept) return saq::fail(SAQ_EINVAL, "ld < D_kept for the tiled layout");
    } else {
        return saq::fail(SAQ_EINVAL, "unknown layout");
    }
    return SAQ_OK;
}

saq_status saq_project(const saq_plan* p, const float* X, int64_t n, float* O, int64_t ld,
                       int32_t layout, float* norm2, void* stream) {
    if (saq_status st = check_plan(p); st != SAQ_OK) return st;
    if (n < 0) return saq::fail(SAQ_EINVAL, "bad sizes");
    if (n == 0) return SAQ_OK;
    if (saq_status s = check_layout(p, n, ld, layout); s != SAQ_OK) return s;
    if (!X || (!O && p->D_kept > 0)) return saq::fail(SAQ_EINVAL, "null buffer");
    return launch_project(p, X, n, O, ld, layout, norm2, static_cast<hipStream_t>(stream));
}

saq_status saq_quantize(const saq_plan* p, const float* O, int64_t ld, int32_t layout, int64_t n,
                        const float* norm2, int32_t rounds, uint8_t* codes, float* factors,
                        void* stream) {
    if (saq_status st = check_plan(p); st != SAQ_OK) return st;
    if (n < 0 || rounds < 0) return saq::fail(SAQ_EINVAL, "bad sizes");
    if (n == 0) return SAQ_OK;
    if (saq_status s = check_layout(p, n, ld, layout); s != SAQ_OK) return s;
    if ((!O && p->D_kept > 0) || !codes || !factors) return saq::fail(SAQ_EINVAL, "null buffer");
    return launch_quantize(p, O, ld, layout, n, norm2, rounds, codes, factors,
                           static_cast<hipStream_t>(stream));
}

}  // extern "C"

static saq_status encode_impl(const saq_plan* p, const float* X, int64_t n, int32_t rounds,
                              uint8_t* codes, float* factors, void* ws, int64_t ws_bytes,
                              void* stream, RefRows R) {
    if (saq_status st = check_plan(p); st != SAQ_OK) return st;
    if (n < 0 || rounds < 0) return saq::fail(SAQ_EINVAL, "bad sizes");
    if (n == 0) return SAQ_OK;
    if (!X || !codes || !factors || !ws) return saq::fail(SAQ_EINVAL, "null buffer");
    if (ws_bytes < saq_encode_workspace_bytes(p, n)) return saq::fail(SAQ_EINVAL, "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t ld = std::max(p->D_kept, 1);
    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
    float* O = reinterpret_cast<float*>(base);
    float* nrm = reinterpret_cast<float*>(base + round_up(enc_o_bytes(p, n), 256));
    // with nothing kept the projection kernel still runs its first column
    // tile (all padding) to produce ||x - c||^2
    saq_status s = launch_project(p, X, n, O, ld, LAYOUT_TILES, nrm, st, R);
    if (s != SAQ_OK) return s;
    return launch_quantize(p, O, ld, LAYOUT_TILES, n, nrm, rounds, codes, factors, st);
}

extern "C" {

saq_status saq_encode(const saq_plan* p, const float* X, int64_t n, int32_t rounds,
                      uint8_t* codes, float* factors, void* ws, int64_t ws_bytes, void* stream) {
    return encode_impl(p, X, n, rounds, codes, factors, ws, ws_bytes, stream,
                       RefRows{nullptr, nullptr, 0});
}

saq_status saq_encode_ref(const saq_plan* p, const float* X, int64_t n, const float* refs,
                          int32_t K, const int32_t* ref_ids, int32_t rounds, uint8_t* codes,
                          float* factors, void* ws, int64_t ws_bytes, void* stream) {
    if (K <= 0) return saq::fail(SAQ_EINVAL, "K must be positive");
    if (n > 0 && (!refs || !ref_ids)) return saq::fail(SAQ_EINVAL, "null reference buffer");
    return encode_impl(p, X, n, rounds, codes, factors, ws, ws_bytes, stream,
                       RefRows{refs, ref_ids, K});
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Encode without allocation: the workspace of saq_encode (the tiled
// projection and the norms) is a file-scope device array instead of a
// caller buffer.  Each GPU holds its own copy from the library's load until
// the process ends; its device address is looked up once per device and
// kept, and only that address is handed to kernels (the array's name is a
// host-side stand-in in host code).  Nothing in it must start at zero.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[SAQ_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device
saq_status scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return saq::fail(SAQ_EUNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (ptr == nullptr || (reinterpret_cast<uintptr_t>(ptr) & 255) != 0)
            return saq::fail(SAQ_EDEVICE, "scratch array has no aligned device address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SAQ_OK;
}
}  // namespace

extern "C" {

saq_status saq_encode_noalloc(const saq_plan* p, const float* X, int64_t n, int32_t rounds,
                              uint8_t* codes, float* factors, void* stream) {
    if (saq_status st = check_plan(p); st != SAQ_OK) return st;
    if (n < 0 || rounds < 0) return saq::fail(SAQ_EINVAL, "bad sizes");
    if (n == 0) return SAQ_OK;
    const int64_t need = saq_encode_workspace_bytes(p, n);
    if (need > SAQ_NOALLOC_SCRATCH_BYTES) {
        int64_t lo = 0, hi = n;      // the largest accepted n for this plan
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (saq_encode_workspace_bytes(p, mid) <= SAQ_NOALLOC_SCRATCH_BYTES) lo = mid; else hi = mid - 1;
        }
        return saq::fail(SAQ_EINVAL, "n = " + std::to_string(n) + " exceeds the no-allocation "
                         "scratch (" + std::to_string(SAQ_NOALLOC_SCRATCH_BYTES >> 20) +
                         " MiB holds at most " + std::to_string(lo) + " rows for this plan); "
                         "split the batch or use saq_encode with a workspace");
    }
    void* ws = nullptr;
    if (saq_status st = scratch_address(&ws); st != SAQ_OK) return st;
    return encode_impl(p, X, n, rounds, codes, factors, ws, SAQ_NOALLOC_SCRATCH_BYTES, stream,
                       RefRows{nullptr, nullptr, 0});
}

int64_t saq_encode_batched_workspace_bytes(const saq_batch_item* items, int32_t count,
                                           const saq_batch_tuning* tuning) {
    BatchPlan B;
    if (plan_batch(items, count, 0, tuning, nullptr, B, false) != SAQ_OK) return -1;
    return B.ws_need;
}

saq_status saq_encode_batched(const saq_batch_item* items, int32_t count, int32_t rounds,
                              const saq_batch_tuning* tuning, void* ws, int64_t ws_bytes,
                              void* stream) {
    if (!ws) return saq::fail(SAQ_EINVAL, "null workspace");
    BatchPlan B;
    if (saq_status s = plan_batch(items, count, rounds, tuning, ws, B); s != SAQ_OK) return s;
    if (ws_bytes < B.ws_need) return saq::fail(SAQ_EINVAL, "workspace too small");
    if (B.g.count == 0) return SAQ_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (B.fused) {
        hipLaunchKernelGGL(clear_ticket_kernel, dim3(1), dim3(64), 0, st, B.f.ticket);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "clear_ticket_kernel launch");
        unsigned grid = 1;
#define SAQ_LAUNCH_FUSED(BI, A64, CT)                                                              \
    do {                                                                                           \
        if (saq_status s2 = fused_grid(fused_encode_kernel<BI, A64, CT>, B.lds, B.f.items, grid);  \
            s2 != SAQ_OK)                                                                          \
            return s2;                                                                             \
        hipLaunchKernelGGL((fused_encode_kernel<BI, A64, CT>), dim3(grid), dim3(256), B.lds, st,   \
                           B.f);                                                                   \
    } while (0)
        if (B.any64) {
            if (B.wide) SAQ_LAUNCH_FUSED(1, true, uint16_t); else SAQ_LAUNCH_FUSED(1, true, uint8_t);
        } else if (B.bi == 1) {
            if (B.wide) SAQ_LAUNCH_FUSED(1, false, uint16_t); else SAQ_LAUNCH_FUSED(1, false, uint8_t);
        } else {
            if (B.wide) SAQ_LAUNCH_FUSED(2, false, uint16_t); else SAQ_LAUNCH_FUSED(2, false, uint8_t);
        }
#undef SAQ_LAUNCH_FUSED
        e = hipGetLastError();
        return e == hipSuccess ? SAQ_OK : hip_fail(e, "fused_encode_kernel launch");
    }
    // one instantiation per tile shape: the 64-row one also carries datasets
    // with FP64 k-tile totals, the 128-row one keeps three workgroups per CU
    if (B.bi == 1)
        hipLaunchKernelGGL(grouped_gemm_kernel<true>, dim3(unsigned(B.gemm_blocks)), dim3(256), 0, st, B.g);
    else
        hipLaunchKernelGGL(grouped_gemm_kernel<false>, dim3(unsigned(B.gemm_blocks)), dim3(256), 0, st, B.g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "grouped_gemm_kernel launch");
    const dim3 qb(unsigned(64 * B.waves));
    if (B.wide)
        hipLaunchKernelGGL(grouped_quantize_kernel<uint16_t>, dim3(unsigned(B.quant_blocks)), qb, B.lds, st, B.q);
    else
        hipLaunchKernelGGL(grouped_quantize_kernel<uint8_t>, dim3(unsigned(B.quant_blocks)), qb, B.lds, st, B.q);
    e = hipGetLastError();
    return e == hipSuccess ? SAQ_OK : hip_fail(e, "grouped_quantize_kernel launch");
}

int64_t saq_estimate_workspace_bytes(const saq_plan* p, int32_t nq) {
    if (!p || nq < 0) return -1;
    const int64_t q = std::max(nq, 1);
    // Qp [nq x D_kept], ||q - c||^2 [nq], the row-block sums of squares
    // behind sigma [nq x n_kept x 8], stage bounds and segment sums of q'
    // [nq x n_kept] each, then (16-byte aligned) the three-term bf16 split of
    // the queries [nq x query_groups x 3 x 16 bytes]
    const int64_t dk = std::max(p->D_kept, 1);
    return q * dk * 4 + q * 4 + (8 + 2) * q * std::max(p->n_kept, 1) * 4 + 16 +
           q * query_groups(int(dk)) * 48 + 512;
}

}  // extern "C"

static saq_status scan_impl(const saq_plan* p, const float* Q, int32_t nq, const float* ref,
                            const uint8_t* codes, const float* factors, int64_t n,
                            int32_t prefix_bits, float* out, void* ws, int64_t ws_bytes,
                            void* stream) {
    if (saq_status st = check_plan(p); st != SAQ_OK) return st;
    if (nq < 0 || n < 0) return saq::fail(SAQ_EINVAL, "bad sizes");
    if (prefix_bits < 0) return saq::fail(SAQ_EINVAL, "prefix_bits < 0");
    if (nq == 0 || n == 0) return SAQ_OK;
    if (!Q || !codes || !factors || !out || !ws) return saq::fail(SAQ_EINVAL, "null buffer");
    if (ws_bytes < saq_estimate_workspace_bytes(p, nq)) return saq::fail(SAQ_EINVAL, "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
    float* Qp = reinterpret_cast<float*>(base);
    const int dk = std::max(p->D_kept, 1), qg = query_groups(dk);
    float* qn2 = Qp + int64_t(nq) * dk;
    u32x4* Qs = reinterpret_cast<u32x4*>((reinterpret_cast<uintptr_t>(qn2 + nq) + 15) & ~uintptr_t(15));
    saq_status s = launch_project(p, Q, nq, Qp, dk, LAYOUT_ROWS, qn2, st, RefRows{ref, nullptr, 1});
    if (s != SAQ_OK) return s;
    hipLaunchKernelGGL(split_query_kernel, dim3(unsigned((int64_t(nq) * qg + 255) / 256)), dim3(256), 0,
                       st, Qp, nq, dk, qg, Qs);
    const dim3 grid(unsigned((n + ER - 1) / ER), unsigned((nq + EQ - 1) / EQ));
    // packed k-steps when every kept segment is a whole number of 16-dim
    // halves (each lane half then lies inside one segment) and packing saves
    // at least a quarter of the steps: a lane's segment then varies across
    // the wave, so its plane count and factor come from per-lane rather than
    // uniform loads, which only pays where many steps were half padding
    // (16-dim segments)
    bool packed = !p->kept.empty();
    int64_t seg_steps = 0;
    for (const SegEntry& e : p->kept) {
        packed = packed && (e.width % 16) == 0;
        seg_steps += (e.width + EK - 1) / EK;
    }
    packed = packed && 4 * ((int64_t(dk) + EK - 1) / EK) <= 3 * seg_steps;
    // otherwise segment by segment with the records as the B operand (TR)
#define SAQ_LAUNCH_SCAN(QB, PK, TR)                                                                 \
    hipLaunchKernelGGL((estimate_kernel<false, QB, EMS_LANES, PK, TR>), grid, dim3(256), 0, st, Qp, \
                       nq, dk, qn2, dev_seg(p), p->n_kept, codes, p->code_bytes, factors, n,       \
                       int(prefix_bits), nullptr, nullptr, nullptr, nullptr, out, Qs, qg)
    if (nq <= 32) {
        if (packed) SAQ_LAUNCH_SCAN(1, true, false); else SAQ_LAUNCH_SCAN(1, false, true);
    } else {
        if (packed) SAQ_LAUNCH_SCAN(2, true, false); else SAQ_LAUNCH_SCAN(2, false, true);
    }
#undef SAQ_LAUNCH_SCAN
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SAQ_OK : hip_fail(e, "estimate_kernel launch");
}


static saq_status multistage_impl(const saq_plan* p, const float* Q, int32_t nq, const float* ref,
                                  const uint8_t* codes, const float* factors, int64_t n,
                                  const float* tau, float m, float* out, uint8_t* stage, void* ws,
                                  int64_t ws_bytes, void* stream) {
    if (saq_status st = check_plan(p); st != SAQ_OK) return st;
    if (nq < 0 || n < 0) return saq::fail(SAQ_EINVAL, "bad sizes");
    if (!(m >= 0.f) || !std::isfinite(m)) return saq::fail(SAQ_EINVAL, "m must be finite and >= 0");
    if (p->S.empty())
        return saq::fail(SAQ_EINVAL, "plan has no variances: the multi-stage bound needs them");
    if (p->n_kept > 255) return saq::fail(SAQ_EUNSUPPORTED, "multi-stage scan: more than 255 kept segments");
    if (p->max_kept_w > SIG_MAXW)
        return saq::fail(SAQ_EUNSUPPORTED, "multi-stage scan: a kept segment wider than 4096 dims");
    if (nq == 0 || n == 0 || p->n_kept == 0) {
        if (nq > 0 && n > 0 && p->n_kept == 0)
            return saq::fail(SAQ_EUNSUPPORTED, "multi-stage scan: the plan keeps no segment");
        return SAQ_OK;
    }
    if (!Q || !codes || !factors || !tau || !out || !ws) return saq::fail(SAQ_EINVAL, "null buffer");
    if (ws_bytes < saq_estimate_workspace_bytes(p, nq)) return saq::fail(SAQ_EINVAL, "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
    const int dk = std::max(p->D_kept, 1);
    float* Qp = reinterpret_cast<float*>(base);
    float* qn2 = Qp + int64_t(nq) * dk;
    float* sig = qn2 + nq;                                 // [nq][n_kept][SIG_RB]
    float* lbq = sig + int64_t(nq) * p->n_kept * SIG_RB;
    float* qsum = lbq + int64_t(nq) * p->n_kept;
    const int qg = query_groups(dk);
    u32x4* Qs = reinterpret_cast<u32x4*>((reinterpret_cast<uintptr_t>(qsum + int64_t(nq) * p->n_kept) + 15) &
                                         ~uintptr_t(15));
    saq_status s = launch_project(p, Q, nq, Qp, dk, LAYOUT_ROWS, qn2, st, RefRows{ref, nullptr, 1});
    if (s != SAQ_OK) return s;
    hipLaunchKernelGGL(split_query_kernel, dim3(unsigned((int64_t(nq) * qg + 255) / 256)), dim3(256), 0,
                       st, Qp, nq, dk, qg, Qs);
    hipLaunchKernelGGL(sigma_kernel, dim3(unsigned(p->n_kept), unsigned(nq), SIG_RB), dim3(256), 0, st, Qp, dk,
                       dev_seg(p), p->n_kept, dev_S(p), sig, qsum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "sigma_kernel launch");
    hipLaunchKernelGGL(stage_bound_kernel, dim3(unsigned((nq + 255) / 256)), dim3(256), 0, st, sig, qn2,
                       nq, p->n_kept, m, lbq);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "stage_bound_kernel launch");
    const dim3 grid(unsigned((n + ER - 1) / ER), unsigned((nq + EQ - 1) / EQ));
    // one lane per open pair in the sparse finish when every kept segment is
    // a single 32-dim chunk
    const bool narrow = p->max_kept_w <= 32;
#define SAQ_LAUNCH_MS(QB, FL)                                                                     \
    hipLaunchKernelGGL((estimate_kernel<true, QB, FL>), grid, dim3(256), 0, st, Qp, nq, dk, qn2,  \
                       dev_seg(p), p->n_kept, codes, p->code_bytes, factors, n, 0, lbq, qsum, tau, \
                       stage, out, Qs, qg)
    if (nq <= 32) {
        if (narrow) SAQ_LAUNCH_MS(1, 1); else SAQ_LAUNCH_MS(1, EMS_LANES);
    } else {
        if (narrow) SAQ_LAUNCH_MS(2, 1); else SAQ_LAUNCH_MS(2, EMS_LANES);
    }
#undef SAQ_LAUNCH_MS
    e = hipGetLastError();
    return e == hipSuccess ? SAQ_OK : hip_fail(e, "estimate_kernel launch");
}

extern "C" {

saq_status saq_estimate_multistage(const saq_plan* p, const float* Q, int32_t nq,
                                   const uint8_t* codes, const float* factors, int64_t n,
                                   const float* tau, float m, float* out, uint8_t* stage, void* ws,
                                   int64_t ws_bytes, void* stream) {
    return multistage_impl(p, Q, nq, nullptr, codes, factors, n, tau, m, out, stage, ws, ws_bytes,
                           stream);
}

saq_status saq_estimate_multistage_ref(const saq_plan* p, const float* Q, int32_t nq,
                                       const float* ref, const uint8_t* codes,
                                       const float* factors, int64_t n, const float* tau, float m,
                                       float* out, uint8_t* stage, void* ws, int64_t ws_bytes,
                                       void* stream) {
    if (!ref && nq > 0 && n > 0) return saq::fail(SAQ_EINVAL, "null reference");
    return multistage_impl(p, Q, nq, ref, codes, factors, n, tau, m, out, stage, ws, ws_bytes,
                           stream);
}

saq_status saq_estimate_dist_prefix(const saq_plan* p, const float* Q, int32_t nq,
                                    const uint8_t* codes, const float* factors, int64_t n,
                                    int32_t prefix_bits, float* out, void* ws, int64_t ws_bytes,
                                    void* stream) {
    return scan_impl(p, Q, nq, nullptr, codes, factors, n, prefix_bits, out, ws, ws_bytes, stream);
}

saq_status saq_estimate_dist(const saq_plan* p, const float* Q, int32_t nq, const uint8_t* codes,
                             const float* factors, int64_t n, float* out, void* ws,
                             int64_t ws_bytes, void* stream) {
    return scan_impl(p, Q, nq, nullptr, codes, factors, n, 0, out, ws, ws_bytes, stream);
}

saq_status saq_estimate_dist_ref(const saq_plan* p, const float* Q, int32_t nq, const float* ref,
                                 const uint8_t* codes, const float* factors, int64_t n, float* out,
                                 void* ws, int64_t ws_bytes, void* stream) {
    if (!ref && nq > 0 && n > 0) return saq::fail(SAQ_EINVAL, "null reference");
    return scan_impl(p, Q, nq, ref, codes, factors, n, 0, out, ws, ws_bytes, stream);
}

}  // extern "C"
