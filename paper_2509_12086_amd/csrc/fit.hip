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
//   jacobi_*_kernel
//       the covariance's eigen-decomposition (the PCA basis of Section 4.1)
//       by the cyclic Jacobi method with a parallel ordering: in each round
//       the indices form n/2 disjoint pairs (the round-robin tournament
//       schedule), one plane rotation per pair zeroes that pair's
//       off-diagonal entry, and the rotations of a round commute, so
//       A <- J^T A J and V <- V J are applied at once: each thread takes one
//       2 x 2 block (pair P rows, pair Q columns) of A, B' = R_P^T B R_Q,
//       from one buffer into the other, and the 2 x 2 block of V in place.
//       n - 1 rounds make a sweep; sweeps repeat until the off-diagonal
//       mass is below FP64 rounding of the diagonal (Jacobi 1846; the
//       parallel ordering of Brent and Luk 1985; the rotation formulas of
//       Rutishauser, Numer. Math. 9, 1966).
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

// ---------------------------------------------------------------------------
// Cyclic Jacobi on the device.  N is n rounded up to even; a padded index
// has a zero row and column, so its rotations are the identity and its
// column of V stays a unit vector outside the first n rows and columns.
// ---------------------------------------------------------------------------
// the pair k (k < N/2) of round r of the round-robin schedule on N players:
// player N - 1 stays, the others rotate
__device__ __forceinline__ void jacobi_pair(int N, int r, int k, int& a, int& b) {
    if (k == 0) {
        a = r;
        b = N - 1;
    } else {
        const int m = N - 1;
        a = (r + k) % m;
        b = (r - k + m) % m;
    }
    if (a > b) {
        const int t = a;
        a = b;
        b = t;
    }
}

// (c, s) of R = [[c, s], [-s, c]] with (R^T [[app, apq], [apq, aqq]] R)[0][1] = 0,
// the smaller of the two angles
__device__ __forceinline__ void jacobi_rotation(double app, double aqq, double apq, double& c,
                                                double& s) {
    if (apq == 0.0) {
        c = 1.0;
        s = 0.0;
        return;
    }
    const double th = (aqq - app) / (2.0 * apq);
    double t;
    if (fabs(th) > 1e150) {
        t = 0.5 / th;
    } else {
        t = 1.0 / (fabs(th) + sqrt(th * th + 1.0));
        if (th < 0.0) t = -t;
    }
    c = 1.0 / sqrt(t * t + 1.0);
    s = t * c;
}

__global__ __launch_bounds__(256) void jacobi_init_kernel(const double* __restrict__ C, int n, int N,
                                                          double* __restrict__ A,
                                                          double* __restrict__ V) {
    const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= int64_t(N) * N) return;
    const int i = int(idx / N), j = int(idx % N);
    A[idx] = (i < n && j < n) ? C[int64_t(i) * n + j] : 0.0;
    V[idx] = i == j ? 1.0 : 0.0;
}

// one round: thread (kp, kq) maps block (pair kp rows, pair kq columns) of
// Ain into Aout, and rotates columns of pair kq in rows of pair kp of V
__global__ __launch_bounds__(256) void jacobi_round_kernel(const double* __restrict__ Ain,
                                                           double* __restrict__ Aout,
                                                           double* __restrict__ V, int N, int r) {
    const int h = N / 2;
    const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= int64_t(h) * h) return;
    const int kp = int(idx / h), kq = int(idx % h);
    int p0, p1, q0, q1;
    jacobi_pair(N, r, kp, p0, p1);
    jacobi_pair(N, r, kq, q0, q1);
    auto at = [&](int i, int j) { return Ain[int64_t(i) * N + j]; };
    double cp, sp, cq, sq;
    jacobi_rotation(at(p0, p0), at(p1, p1), at(p0, p1), cp, sp);
    jacobi_rotation(at(q0, q0), at(q1, q1), at(q0, q1), cq, sq);
    const double b00 = at(p0, q0), b01 = at(p0, q1), b10 = at(p1, q0), b11 = at(p1, q1);
    // rows: R_P^T B
    const double r00 = cp * b00 - sp * b10, r01 = cp * b01 - sp * b11;
    const double r10 = sp * b00 + cp * b10, r11 = sp * b01 + cp * b11;
    // columns: (R_P^T B) R_Q
    double n00 = r00 * cq - r01 * sq, n01 = r00 * sq + r01 * cq;
    double n10 = r10 * cq - r11 * sq, n11 = r10 * sq + r11 * cq;
    if (kp == kq) n01 = n10 = 0.0;   // the pair's own entry, zero by construction
    Aout[int64_t(p0) * N + q0] = n00;
    Aout[int64_t(p0) * N + q1] = n01;
    Aout[int64_t(p1) * N + q0] = n10;
    Aout[int64_t(p1) * N + q1] = n11;
    // V <- V R_Q on rows p0, p1 (every row belongs to exactly one pair)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int64_t row = int64_t(e ? p1 : p0) * N;
        const double v0 = V[row + q0], v1 = V[row + q1];
        V[row + q0] = v0 * cq - v1 * sq;
        V[row + q1] = v0 * sq + v1 * cq;
    }
}

// per-block sums of squares: off-diagonal entries, diagonal entries
__global__ __launch_bounds__(256) void jacobi_off_kernel(const double* __restrict__ A, int N,
                                                         double* __restrict__ part) {
    __shared__ double so[256], sd[256];
    double off = 0.0, dg = 0.0;
    for (int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x; idx < int64_t(N) * N;
         idx += int64_t(gridDim.x) * 256) {
        const double a = A[idx];
        if (idx / N == idx % N) dg += a * a;
        else off += a * a;
    }
    so[threadIdx.x] = off;
    sd[threadIdx.x] = dg;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) {
            so[threadIdx.x] += so[threadIdx.x + w];
            sd[threadIdx.x] += sd[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = so[0];
        part[2 * blockIdx.x + 1] = sd[0];
    }
}

// w[j] = A[j][j], Vout = the first n rows and columns of V
__global__ __launch_bounds__(256) void jacobi_finish_kernel(const double* __restrict__ A,
                                                            const double* __restrict__ V, int n,
                                                            int N, double* __restrict__ w,
                                                            double* __restrict__ Vout) {
    const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= int64_t(n) * n) return;
    const int i = int(idx / n), j = int(idx % n);
    Vout[idx] = V[int64_t(i) * N + j];
    if (i == j) w[i] = A[int64_t(i) * N + i];
}

constexpr int JACOBI_OFF_BLOCKS = 256;
constexpr int JACOBI_MAX_SWEEPS = 40;

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

int64_t jacobi_bytes(int32_t n) {
    const int64_t N = n + (n & 1);
    return 3 * align256(N * N * 8) + align256(int64_t(JACOBI_OFF_BLOCKS) * 2 * 8) + 256;
}

// eigen-decomposition of the symmetric C [n x n] (device): w [n] in the
// Jacobi order, V [n x n] row-major with eigenvector j in column j; waits
// for `st` once per sweep (the convergence test)
saq_status run_jacobi(const double* C, int32_t n, double* w, double* V, void* ws, int64_t ws_bytes,
                      hipStream_t st) {
    if (ws_bytes < jacobi_bytes(n)) return saq::fail(SAQ_EINVAL, "workspace too small");
    const int N = n + (n & 1);
    const int64_t el = int64_t(N) * N;
    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
    double* A[2] = {reinterpret_cast<double*>(base), reinterpret_cast<double*>(base + align256(el * 8))};
    double* Vw = reinterpret_cast<double*>(base + 2 * align256(el * 8));
    double* part = reinterpret_cast<double*>(base + 3 * align256(el * 8));
    const unsigned gel = unsigned((el + 255) / 256);
    const unsigned gpair = unsigned((int64_t(N / 2) * (N / 2) + 255) / 256);
    hipLaunchKernelGGL(jacobi_init_kernel, dim3(gel), dim3(256), 0, st, C, n, N, A[0], Vw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_err(e, "jacobi_init_kernel launch");
    std::vector<double> hp(size_t(JACOBI_OFF_BLOCKS) * 2);
    int cur = 0;
    bool converged = false;
    for (int sweep = 0; sweep < JACOBI_MAX_SWEEPS && !converged; ++sweep) {
        for (int r = 0; r + 1 < N; ++r) {
            hipLaunchKernelGGL(jacobi_round_kernel, dim3(gpair), dim3(256), 0, st, A[cur], A[cur ^ 1],
                               Vw, N, r);
            cur ^= 1;
        }
        e = hipGetLastError();
        if (e != hipSuccess) return hip_err(e, "jacobi_round_kernel launch");
        hipLaunchKernelGGL(jacobi_off_kernel, dim3(JACOBI_OFF_BLOCKS), dim3(256), 0, st, A[cur], N, part);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), part, hp.size() * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_err(e, "jacobi convergence test");
        double off = 0.0, dg = 0.0;
        for (int b = 0; b < JACOBI_OFF_BLOCKS; ++b) {
            off += hp[2 * b];
            dg += hp[2 * b + 1];
        }
        // below FP64 rounding of the diagonal: further rotations change
        // nothing in the eigenvalues' leading 15 digits
        converged = off <= 1e-30 * dg;
    }
    if (!converged) return saq::fail(SAQ_EINVAL, "Jacobi eigen-decomposition did not converge");
    hipLaunchKernelGGL(jacobi_finish_kernel, dim3(unsigned((int64_t(n) * n + 255) / 256)), dim3(256), 0,
                       st, A[cur], Vw, n, N, w, V);
    e = hipGetLastError();
    return e == hipSuccess ? SAQ_OK : hip_err(e, "jacobi_finish_kernel launch");
}

// the fit's own buffers ahead of the covariance workspace: mean,
// covariance, eigenvalues, eigenvectors, then the Jacobi workspace
int64_t fit_extra(int32_t D) {
    return align256(int64_t(D) * 8) + align256(int64_t(D) * D * 8) + align256(int64_t(D) * 8) +
           align256(int64_t(D) * D * 8) + jacobi_bytes(D);
}

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

int64_t saq_sym_eigen_workspace_bytes(int32_t n) {
    if (n <= 0) return -1;
    return jacobi_bytes(n);
}

saq_status saq_sym_eigen_device(const double* A_dev, int32_t n, double* w_dev, double* V_dev,
                                void* ws_dev, int64_t ws_bytes, void* stream) {
    if (n <= 0) return saq::fail(SAQ_EINVAL, "bad size");
    if (!A_dev || !w_dev || !V_dev || !ws_dev) return saq::fail(SAQ_EINVAL, "null buffer");
    return run_jacobi(A_dev, n, w_dev, V_dev, ws_dev, ws_bytes, static_cast<hipStream_t>(stream));
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
    const int64_t dv = align256(int64_t(D) * 8), dm = align256(int64_t(D) * D * 8);
    double* mu = reinterpret_cast<double*>(base);
    double* cov = reinterpret_cast<double*>(base + dv);
    double* w = reinterpret_cast<double*>(base + dv + dm);
    double* V = reinterpret_cast<double*>(base + 2 * dv + dm);
    char* jws = base + 2 * dv + 2 * dm;
    char* rest = base + fit_extra(D);
    const int64_t rest_bytes = ws_bytes - (rest - static_cast<char*>(ws_dev));
    saq_status s = run_covariance(X_dev, n, D, p->fit_sample, mu, cov, rest, rest_bytes, st);
    if (s != SAQ_OK) return s;
    s = run_jacobi(cov, D, w, V, jws, jacobi_bytes(D), st);
    if (s != SAQ_OK) return s;
    try {
        std::vector<double> hm(static_cast<size_t>(D)), hw(static_cast<size_t>(D)),
            hv(static_cast<size_t>(D) * D);
        hipError_t e = hipMemcpyAsync(hm.data(), mu, size_t(D) * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(hw.data(), w, size_t(D) * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hv.data(), V, size_t(D) * D * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_err(e, "copying the basis to the host");
        // the plan search on the host, from the device's basis (sorted there)
        return saq_plan_from_basis(hm.data(), hv.data(), hw.data(), D, p, out);
    } catch (const std::bad_alloc&) {
        return saq::fail(SAQ_ENOMEM, "out of host memory");
    }
}

}  // extern "C"
