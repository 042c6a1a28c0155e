// libsaq device fit: mean and covariance of the fit sample on the GPU
// (Section 4.1), for saq_covariance and saq_fit_plan_device.
//
//   mean_part_kernel / mean_reduce_kernel
//       FP64 column sums over fixed blocks of 4,096 sample rows, added in
//       block order: the same order as the host fit, so the mean is the
//       host fit's bit for bit.
//   cov_kernel
//       (1/m) sum_r (x_r - c)(x_r - c)^T as an FP64 matrix-core contraction
//       (v_mfma_f64_16x16x4_f64): one 64 x 64 output tile of the upper
//       triangle per workgroup, over one slice of the sample rows; rows are
//       staged in LDS as FP64 x - c, 32 rows per step, the next step's raw
//       FP32 values loaded during the current step's MFMAs.
//   cov_reduce_kernel
//       adds the row slices of each element in slice order, divides by m and
//       writes both triangles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "plan.hpp"

typedef double doublex4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int MEAN_ROWS = 4096;   // rows per partial mean (the host fit's block)
constexpr int CT = 64;            // covariance output tile
constexpr int CK = 32;            // sample rows per k-step
constexpr int CSTR = CT + 2;      // doubles per LDS row

__device__ __forceinline__ int64_t sample_row(int64_t i, int64_t n, int64_t m) {
    return m == n ? i : (i * n) / m;
}

__global__ __launch_bounds__(256) void mean_part_kernel(const float* __restrict__ X, int64_t n, int D,
                                                        int64_t m, double* __restrict__ part) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    const int64_t b = blockIdx.y;
    if (k >= D) return;
    double s = 0.0;
    const int64_t i1 = std::min<int64_t>(m, (b + 1) * MEAN_ROWS);
    for (int64_t i = b * MEAN_ROWS; i < i1; ++i) s += double(X[sample_row(i, n, m) * D + k]);
    part[b * D + k] = s;
}

__global__ __launch_bounds__(256) void mean_reduce_kernel(const double* __restrict__ part, int64_t nb,
                                                          int D, int64_t m, double* __restrict__ mu) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= D) return;
    double s = 0.0;
    for (int64_t b = 0; b < nb; ++b) s += part[b * D + k];
    mu[k] = s / double(m);
}

// Upper-triangle tile t (row block I <= column block J) of an nt x nt grid.
__device__ __forceinline__ void tile_of(int t, int nt, int& I, int& J) {
    I = 0;
    while (t >= nt - I) { t -= nt - I; ++I; }
    J = I + t;
}

// grid: (upper tiles, row slices).  part: [slices][D][D], only the upper
// tiles' elements written.  Wave w computes rows 32 (w/2) .. +31 and columns
// 32 (w%2) .. +31 of the tile as 2 x 2 blocks of 16 x 16.
__global__ __launch_bounds__(256) void cov_kernel(const float* __restrict__ X, int64_t n, int D,
                                                  int64_t m, const double* __restrict__ mu,
                                                  int64_t slice_rows, int vec,
                                                  double* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) double Ya[2][CK * CSTR];
    __shared__ __attribute__((aligned(16))) double Yb[2][CK * CSTR];
    const int nt = (D + CT - 1) / CT;
    int I, J;
    tile_of(blockIdx.x, nt, I, J);
    const int i0 = I * CT, j0 = J * CT;
    const int64_t r_begin = int64_t(blockIdx.y) * slice_rows;
    const int64_t r_end = std::min<int64_t>(m, r_begin + slice_rows);
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int wi = wave >> 1, wj = wave & 1;
    const int li = lane & 15, lk = lane >> 4;

    // staging: thread t loads row t/8 of the step, columns 8 (t%8) .. +7 of
    // both column blocks
    const int sr = t >> 3, sc = (t & 7) * 8;
    double ma[8], mb[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        ma[e] = (i0 + sc + e < D) ? mu[i0 + sc + e] : 0.0;
        mb[e] = (j0 + sc + e < D) ? mu[j0 + sc + e] : 0.0;
    }
    float ra[8], rb[8];
    // 8 consecutive floats of one row per column block: two 16-byte loads
    // when rows are 16-byte aligned and the 8 columns are inside D
    auto load8 = [&](const float* x, int c0, bool live, float (&r)[8]) {
        if (vec && live && c0 + 8 <= D) {
            const float4 u = *reinterpret_cast<const float4*>(x + c0);
            const float4 v = *reinterpret_cast<const float4*>(x + c0 + 4);
            r[0] = u.x; r[1] = u.y; r[2] = u.z; r[3] = u.w;
            r[4] = v.x; r[5] = v.y; r[6] = v.z; r[7] = v.w;
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) r[e] = (live && c0 + e < D) ? x[c0 + e] : 0.f;
        }
    };
    auto load = [&](int64_t r0) {
        const int64_t r = r0 + sr;
        const bool live = r < r_end;
        const float* x = X + (live ? sample_row(r, n, m) : 0) * int64_t(D);
        load8(x, i0 + sc, live, ra);
        load8(x, j0 + sc, live, rb);
    };
    auto store = [&](int64_t r0, int buf) {
        const bool live = r0 + sr < r_end;
        // x - c in FP64 (exact for FP32 x); rows past the slice and columns
        // past D are 0 and add nothing.  Stored as pairs (16-byte LDS writes).
        double2* ya = reinterpret_cast<double2*>(&Ya[buf][sr * CSTR + sc]);
        double2* yb = reinterpret_cast<double2*>(&Yb[buf][sr * CSTR + sc]);
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
            double2 va, vb;
            va.x = (live && i0 + sc + e < D) ? double(ra[e]) - ma[e] : 0.0;
            va.y = (live && i0 + sc + e + 1 < D) ? double(ra[e + 1]) - ma[e + 1] : 0.0;
            vb.x = (live && j0 + sc + e < D) ? double(rb[e]) - mb[e] : 0.0;
            vb.y = (live && j0 + sc + e + 1 < D) ? double(rb[e + 1]) - mb[e + 1] : 0.0;
            ya[e / 2] = va;
            yb[e / 2] = vb;
        }
    };

    doublex4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = doublex4{0.0, 0.0, 0.0, 0.0};

    if (r_begin < r_end) {
        load(r_begin);
        store(r_begin, 0);
        __syncthreads();
        for (int64_t r0 = r_begin, step = 0; r0 < r_end; r0 += CK, ++step) {
            const int buf = int(step & 1);
            const bool more = r0 + CK < r_end;
            if (more) load(r0 + CK);
            const double* A = Ya[buf];
            const double* B = Yb[buf];
#pragma unroll
            for (int k = 0; k < CK; k += 4) {
                // A[i][kk] = y_{r0+k+kk}[i0 + i], B[kk][j] = y_{r0+k+kk}[j0 + j]
                const double a0 = A[(k + lk) * CSTR + wi * 32 + li];
                const double a1 = A[(k + lk) * CSTR + wi * 32 + 16 + li];
                const double b0 = B[(k + lk) * CSTR + wj * 32 + li];
                const double b1 = B[(k + lk) * CSTR + wj * 32 + 16 + li];
                acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
            }
            if (more) store(r0 + CK, buf ^ 1);
            __syncthreads();
        }
    }
    // the FP64 16 x 16 result is row-interleaved: lane holds, for register
    // q, row 4 q + lane/16 and column lane%16 of each block
    double* P = part + int64_t(blockIdx.y) * D * D;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int col = j0 + wj * 32 + b * 16 + li;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = i0 + wi * 32 + a * 16 + 4 * q + lk;
                if (row < D && col < D) P[int64_t(row) * D + col] = acc[a][b][q];
            }
        }
}

// cov[i][j] = cov[j][i] = (sum over slices, in order) / m for i <= j
__global__ __launch_bounds__(256) void cov_reduce_kernel(const double* __restrict__ part, int slices,
                                                         int D, int64_t m, double* __restrict__ cov) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= int64_t(D) * D) return;
    const int i = int(e / D), j = int(e % D);
    if (i > j) return;
    double s = 0.0;
    for (int sl = 0; sl < slices; ++sl) s += part[int64_t(sl) * D * D + e];
    const double v = s / double(m);
    cov[int64_t(i) * D + j] = v;
    cov[int64_t(j) * D + i] = v;
}

struct CovShape {
    int64_t m = 0, nb = 0, slice_rows = 0;
    int nt = 0, tiles = 0, slices = 0;
    int64_t off_mpart = 0, off_part = 0, bytes = 0;
};

int64_t align256(int64_t v) { return (v + 255) & ~int64_t(255); }

CovShape cov_shape(int64_t n, int32_t D, int64_t fit_sample) {
    CovShape S;
    S.m = (fit_sample > 0 && fit_sample < n) ? fit_sample : n;
    S.nb = (S.m + MEAN_ROWS - 1) / MEAN_ROWS;
    S.nt = (D + CT - 1) / CT;
    S.tiles = S.nt * (S.nt + 1) / 2;
    // enough row slices to give the chip about 2,048 workgroups, each slice
    // at least 1,024 rows
    const int64_t want = std::max<int64_t>(1, (2048 + S.tiles - 1) / S.tiles);
    const int64_t most = std::max<int64_t>(1, S.m / 1024);
    S.slices = int(std::min<int64_t>(std::min<int64_t>(want, most), 64));
    S.slice_rows = ((S.m + S.slices - 1) / S.slices + CK - 1) / CK * CK;
    S.slices = int((S.m + S.slice_rows - 1) / S.slice_rows);
    S.off_mpart = 0;
    S.off_part = align256(S.nb * D * 8);
    S.bytes = S.off_part + int64_t(S.slices) * D * D * 8 + 256;
    return S;
}

saq_status hip_err(hipError_t e, const char* what) {
    return saq::fail(SAQ_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

saq_status run_covariance(const float* X, int64_t n, int32_t D, int64_t fit_sample, double* mu,
                          double* cov, void* ws, int64_t ws_bytes, hipStream_t st) {
    const CovShape S = cov_shape(n, D, fit_sample);
    if (ws_bytes < S.bytes) return saq::fail(SAQ_EINVAL, "workspace too small");
    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
    double* mpart = reinterpret_cast<double*>(base + S.off_mpart);
    double* part = reinterpret_cast<double*>(base + S.off_part);
    const unsigned cb = unsigned((D + 255) / 256);
    hipLaunchKernelGGL(mean_part_kernel, dim3(cb, unsigned(S.nb)), dim3(256), 0, st, X, n, D, S.m, mpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_err(e, "mean_part_kernel launch");
    hipLaunchKernelGGL(mean_reduce_kernel, dim3(cb), dim3(256), 0, st, mpart, S.nb, D, S.m, mu);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_err(e, "mean_reduce_kernel launch");
    const int vec = (D % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
    hipLaunchKernelGGL(cov_kernel, dim3(unsigned(S.tiles), unsigned(S.slices)), dim3(256), 0, st, X, n, D,
                       S.m, mu, S.slice_rows, vec, part);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_err(e, "cov_kernel launch");
    const int64_t el = int64_t(D) * D;
    hipLaunchKernelGGL(cov_reduce_kernel, dim3(unsigned((el + 255) / 256)), dim3(256), 0, st, part,
                       S.slices, D, S.m, cov);
    e = hipGetLastError();
    return e == hipSuccess ? SAQ_OK : hip_err(e, "cov_reduce_kernel launch");
}

// the fit's own buffers ahead of the covariance workspace: mean, covariance
int64_t fit_extra(int32_t D) { return align256(int64_t(D) * 8) + align256(int64_t(D) * D * 8); }

}  // namespace

extern "C" {

int64_t saq_covariance_workspace_bytes(int64_t n, int32_t D, int64_t fit_sample) {
    if (n <= 0 || D <= 0 || fit_sample < 0) return -1;
    return cov_shape(n, D, fit_sample).bytes;
}

saq_status saq_covariance(const float* X_dev, int64_t n, int32_t D, int64_t fit_sample,
                          double* mean_dev, double* cov_dev, void* ws_dev, int64_t ws_bytes,
                          void* stream) {
    if (n <= 0 || D <= 0 || fit_sample < 0) return saq::fail(SAQ_EINVAL, "bad sizes");
    if (!X_dev || !mean_dev || !cov_dev || !ws_dev) return saq::fail(SAQ_EINVAL, "null buffer");
    return run_covariance(X_dev, n, D, fit_sample, mean_dev, cov_dev, ws_dev, ws_bytes,
                          static_cast<hipStream_t>(stream));
}

int64_t saq_fit_workspace_bytes(int64_t n, int32_t D, const saq_plan_params* p) {
    if (!p || n <= 0 || D <= 0 || p->fit_sample < 0) return -1;
    return fit_extra(D) + cov_shape(n, D, p->fit_sample).bytes + 256;
}

saq_status saq_fit_plan_device(const float* X_dev, int64_t n, int32_t D, const saq_plan_params* p,
                               void* ws_dev, int64_t ws_bytes, void* stream, saq_plan** out) {
    if (!X_dev || !p || !out || !ws_dev || n <= 0 || D <= 0 || p->fit_sample < 0)
        return saq::fail(SAQ_EINVAL, "bad arguments");
    if (ws_bytes < saq_fit_workspace_bytes(n, D, p)) return saq::fail(SAQ_EINVAL, "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws_dev) + 255) & ~uintptr_t(255));
    double* mu = reinterpret_cast<double*>(base);
    double* cov = reinterpret_cast<double*>(base + align256(int64_t(D) * 8));
    char* rest = base + fit_extra(D);
    const int64_t rest_bytes = ws_bytes - (rest - static_cast<char*>(ws_dev));
    saq_status s = run_covariance(X_dev, n, D, p->fit_sample, mu, cov, rest, rest_bytes, st);
    if (s != SAQ_OK) return s;
    try {
        std::vector<double> hm(static_cast<size_t>(D)), hc(static_cast<size_t>(D) * D);
        hipError_t e = hipMemcpyAsync(hm.data(), mu, size_t(D) * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hc.data(), cov, size_t(D) * D * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_err(e, "copying the moments to the host");
        return saq::plan_from_moments(D, hm, hc, *p, out);
    } catch (const std::bad_alloc&) {
        return saq::fail(SAQ_ENOMEM, "out of host memory");
    }
}

}  // extern "C"
