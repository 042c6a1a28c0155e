// Host half of libsaq.so: the plan fit (Sections 4.1-4.2), plan objects and
// their serialisation.  Everything here runs once per dataset and budget, in
// FP64; the device path reads the result as data.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <numeric>
#include <string>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "plan.hpp"

namespace saq {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

saq_status fail(saq_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

static int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

DeviceLayout device_layout(const saq_plan& p) {
    DeviceLayout L;
    L.n_pad = std::max(kGemmTileN, (p.D_kept + kGemmTileN - 1) / kGemmTileN * kGemmTileN);
    L.k_pad = (p.D + kGemmTileK - 1) / kGemmTileK * kGemmTileK;
    L.off_Ms = 0;
    const int64_t split_chunks = int64_t(L.n_pad / kGemmTileN) * (L.k_pad / kSplitK) * kSplitChunks;
    L.off_c = align256(L.off_Ms + split_chunks * 16);
    L.off_seg = align256(L.off_c + int64_t(L.k_pad) * 4);
    L.off_S = align256(L.off_seg + int64_t(std::max(p.n_kept, 1)) * int64_t(sizeof(SegEntry)));
    L.bytes = align256(L.off_S + int64_t(std::max<size_t>(p.S.size(), 1)) * 4);
    return L;
}

// bf16 with round-to-nearest-even of a finite FP32 value (its upper 16 bits
// after rounding), and the FP32 value of a bf16
static uint16_t bf16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
static float bf16_value(uint16_t h) {
    const uint32_t u = uint32_t(h) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

void build_staging(saq_plan& p) {
    p.layout = device_layout(p);
    const DeviceLayout& L = p.layout;
    p.staging.assign(size_t(L.bytes), 0);
    // M_split: each entry of M, zero padded to [n_pad x k_pad], as three bf16
    // terms, in the GEMM's chunk order
    uint16_t* Ms = reinterpret_cast<uint16_t*>(p.staging.data() + L.off_Ms);
    const int ksteps = L.k_pad / kSplitK;
    for (int tile = 0; tile < L.n_pad / kGemmTileN; ++tile)
        for (int ks = 0; ks < ksteps; ++ks)
            for (int half = 0; half < 2; ++half)
                for (int row = 0; row < kGemmTileN; ++row)
                    for (int e = 0; e < 8; ++e) {
                        const int r = tile * kGemmTileN + row, k = ks * kSplitK + 8 * half + e;
                        float v = (r < p.D_kept && k < p.D) ? p.M[int64_t(r) * p.D + k] : 0.0f;
                        for (int term = 0; term < 3; ++term) {
                            const uint16_t h = bf16_rne(v);
                            const int64_t chunk = (int64_t(tile) * ksteps + ks) * kSplitChunks +
                                                  term * 2 * kGemmTileN + half * kGemmTileN + row;
                            Ms[chunk * 8 + e] = h;
                            v -= bf16_value(h);          // exact: the remainder fits in FP32
                        }
                    }
    float* c = reinterpret_cast<float*>(p.staging.data() + L.off_c);
    std::memcpy(c, p.c.data(), size_t(p.D) * 4);
    std::memcpy(p.staging.data() + L.off_seg, p.kept.data(), p.kept.size() * sizeof(SegEntry));
    if (!p.S.empty()) std::memcpy(p.staging.data() + L.off_S, p.S.data(), p.S.size() * 4);
}

// The blocks S_s for kept segments without a rotation: diag(sqrt(var)) of
// the dims' own variances (empty if every variance is 0, i.e. unknown).
static std::vector<float> diagonal_spread(const std::vector<int32_t>& widths,
                                          const std::vector<int32_t>& bits,
                                          const std::vector<double>& var) {
    bool any = false;
    for (double v : var) any = any || v != 0.0;
    std::vector<float> S;
    if (!any) return S;
    int col = 0;
    for (size_t s = 0; s < widths.size(); ++s) {
        const int W = widths[s];
        if (bits[s] > 0) {
            const size_t base = S.size();
            S.resize(base + size_t(W) * W, 0.0f);
            for (int i = 0; i < W; ++i)
                S[base + size_t(i) * W + i] = float(std::sqrt(std::max(var[size_t(col + i)], 0.0)));
        }
        col += W;
    }
    return S;
}

// ---------------------------------------------------------------------------
// Symmetric eigen-decomposition in FP64: Householder reduction to tridiagonal
// form followed by QL iterations with implicit Wilkinson shifts (the classic
// textbook pair).  The Givens rotations of the QL phase are recorded and
// applied to the accumulated basis in parallel over row blocks.
// ---------------------------------------------------------------------------

struct Rot { int32_t i; double c, s; };

// Apply recorded Givens rotations (in order) to the rows i, i+1 of Zt (the
// transposed basis, n x n row-major), in parallel over column blocks so that
// each rotation is a contiguous two-row update.
static void apply_rotations(std::vector<double>& Zt, int n, const std::vector<Rot>& rots) {
    if (rots.empty()) return;
    const int64_t nrot = int64_t(rots.size());
    const int CB = 128;
#pragma omp parallel for schedule(dynamic, 1)
    for (int k0 = 0; k0 < n; k0 += CB) {
        const int k1 = std::min(n, k0 + CB);
        for (int64_t t = 0; t < nrot; ++t) {
            const Rot& R = rots[size_t(t)];
            double* zi = &Zt[size_t(R.i) * n];
            double* zj = zi + n;
            for (int k = k0; k < k1; ++k) {
                const double f = zj[k];
                zj[k] = R.s * zi[k] + R.c * f;
                zi[k] = R.c * zi[k] - R.s * f;
            }
        }
    }
}

// A: n x n symmetric row-major (destroyed).  On return w holds the
// eigenvalues in descending order and V (n x n row-major) the matching
// eigenvectors in its columns.
static bool sym_eigen(std::vector<double>& A, int n, std::vector<double>& w, std::vector<double>& V) {
    std::vector<double> d(n), e(n, 0.0);
    std::vector<std::vector<double>> hv(size_t(std::max(n, 1)));   // Householder vectors
    std::vector<double> hs(size_t(std::max(n, 1)), 0.0);            // 2 / |v|^2 (0 = identity)
    std::vector<double> p(n), q(n);
    // reduce row k (k = n-1 .. 2): zero a[k][0..k-2] with a reflector on 0..k-1
    for (int k = n - 1; k >= 2; --k) {
        double* row = &A[size_t(k) * n];
        double nrm = 0.0;
        for (int j = 0; j < k; ++j) nrm += row[j] * row[j];
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) { e[k] = 0.0; continue; }
        const double alpha = row[k - 1] > 0 ? -nrm : nrm;
        std::vector<double>& v = hv[size_t(k)];
        v.assign(row, row + k);
        v[k - 1] -= alpha;
        double vv = 0.0;
        for (int j = 0; j < k; ++j) vv += v[j] * v[j];
        if (vv == 0.0) { e[k] = row[k - 1]; continue; }
        const double beta = 2.0 / vv;
        hs[size_t(k)] = beta;
        // p = beta * A v over the leading k x k block
#pragma omp parallel for schedule(static)
        for (int i = 0; i < k; ++i) {
            const double* ai = &A[size_t(i) * n];
            double s = 0.0;
            for (int j = 0; j < k; ++j) s += ai[j] * v[j];
            p[i] = beta * s;
        }
        double vp = 0.0;
        for (int i = 0; i < k; ++i) vp += v[i] * p[i];
        const double K = 0.5 * beta * vp;
        for (int i = 0; i < k; ++i) q[i] = p[i] - K * v[i];
#pragma omp parallel for schedule(static)
        for (int i = 0; i < k; ++i) {
            double* ai = &A[size_t(i) * n];
            for (int j = 0; j < k; ++j) ai[j] -= v[i] * q[j] + q[i] * v[j];
        }
        e[k] = alpha;
    }
    if (n >= 2) e[1] = A[size_t(1) * n + 0];
    for (int i = 0; i < n; ++i) d[i] = A[size_t(i) * n + i];
    // basis Z = H_{n-1} ... H_2 applied to I (H_k acts on rows 0..k-1 from
    // the left).  Applied in ascending k, the rows 0..k-1 are still zero
    // outside columns 0..k-1, so each step updates a k x k block; it is done
    // as row-contiguous sweeps in parallel over column blocks.
    V.assign(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) V[size_t(i) * n + i] = 1.0;
    for (int k = 2; k < n; ++k) {
        if (hs[size_t(k)] == 0.0) continue;
        const std::vector<double>& v = hv[size_t(k)];
        const double beta = hs[size_t(k)];
        const int JB = 64;
#pragma omp parallel for schedule(static)
        for (int j0 = 0; j0 < k; j0 += JB) {
            const int j1 = std::min(k, j0 + JB);
            double w[64];
            for (int j = j0; j < j1; ++j) w[j - j0] = 0.0;
            for (int i = 0; i < k; ++i) {
                const double vi = v[i];
                const double* row = &V[size_t(i) * n];
                for (int j = j0; j < j1; ++j) w[j - j0] += vi * row[j];
            }
            for (int j = j0; j < j1; ++j) w[j - j0] *= beta;
            for (int i = 0; i < k; ++i) {
                const double vi = v[i];
                double* row = &V[size_t(i) * n];
                for (int j = j0; j < j1; ++j) row[j] -= vi * w[j - j0];
            }
        }
    }
    hv.clear();
    // the QL rotations act on columns of V: work on its transpose
    {
        std::vector<double> T(size_t(n) * n);
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) T[size_t(j) * n + i] = V[size_t(i) * n + j];
        V.swap(T);
    }
    // QL with implicit shifts on (d, e); e[i] couples i and i+1 after the shift.
    // This is the published implicit-shift QL iteration for symmetric
    // tridiagonal matrices (Bowdler, Martin, Reinsch and Wilkinson, "The QR
    // and QL algorithms for symmetric matrices", Numer. Math. 11, 1968; the
    // EISPACK routine tql2), with its usual variable names: a Wilkinson-type
    // shift from the leading 2 x 2 block, then a chase of plane rotations
    // (c, s) from the bottom of the unreduced block up; the rotations are
    // recorded and applied to the basis in batches.
    for (int i = 1; i < n; ++i) e[i - 1] = e[i];
    if (n > 0) e[n - 1] = 0.0;
    std::vector<Rot> rots;
    rots.reserve(1 << 20);
    const double eps = std::numeric_limits<double>::epsilon();
    for (int l = 0; l < n; ++l) {
        int iter = 0, m;
        do {
            for (m = l; m < n - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= eps * dd) break;
            }
            if (m != l) {
                if (++iter > 60) return false;
                double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                double r = std::hypot(g, 1.0);
                g = d[m] - d[l] + e[l] / (g + (g >= 0 ? std::fabs(r) : -std::fabs(r)));
                double s = 1.0, c = 1.0, pp = 0.0;
                int i;
                bool early = false;
                for (i = m - 1; i >= l; --i) {
                    double f = s * e[i], b = c * e[i];
                    r = std::hypot(f, g);
                    e[i + 1] = r;
                    if (r == 0.0) { d[i + 1] -= pp; e[m] = 0.0; early = true; break; }
                    s = f / r;
                    c = g / r;
                    g = d[i + 1] - pp;
                    r = (d[i] - g) * s + 2.0 * c * b;
                    pp = s * r;
                    d[i + 1] = g + pp;
                    g = c * r - b;
                    rots.push_back(Rot{i, c, s});
                }
                if (early) continue;
                d[l] -= pp;
                e[l] = g;
                e[m] = 0.0;
            }
            if (rots.size() >= (size_t(1) << 20)) { apply_rotations(V, n, rots); rots.clear(); }
        } while (m != l);
    }
    apply_rotations(V, n, rots);
    // sort descending; V now holds eigenvector j in its row j
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return d[a] > d[b]; });
    w.resize(n);
    std::vector<double> V2(size_t(n) * n);
    for (int j = 0; j < n; ++j) w[j] = d[ord[j]];
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V2[size_t(i) * n + j] = V[size_t(ord[j]) * n + i];
    V.swap(V2);
    return true;
}

// ---------------------------------------------------------------------------
// Plan search (Section 4.2).  ERROR(Seg, B) = 2^-B * sum_{i in Seg} sigma_i^2
// (Eq. seg-err without the constant 1/pi).  Algorithm 2 gives the minimum over
// plans within the quota; a second pass adds the segment count to the state
// and keeps the fewest segments whose error is within (1 + eps) of it.
// Dimensions are handled in units of g (the last unit may be shorter), costs
// in units of the gcd of the unit widths.
// ---------------------------------------------------------------------------

struct DPResult { std::vector<int32_t> widths, bits; double err, min_err; int64_t quota, used; };

static saq_status plan_search(const std::vector<double>& sig2, const saq_plan_params& P, DPResult& out) {
    const int D = int(sig2.size());
    const int g = P.granularity;
    if (g <= 0) return fail(SAQ_EINVAL, "granularity must be positive");
    if (P.max_bits < 0 || P.max_bits > 16) return fail(SAQ_EINVAL, "max_bits must be in 0..16");
    if (P.max_width < 0 || (P.max_width % g) != 0)
        return fail(SAQ_EINVAL, "max_width must be a non-negative multiple of granularity");
    if (!(P.bits_per_dim >= 0.0) || P.bits_per_dim > 16.0) return fail(SAQ_EINVAL, "bits_per_dim out of range");
    std::vector<int> uw;
    for (int a = 0; a < D; a += g) uw.push_back(std::min(g, D - a));
    const int nu = int(uw.size());
    int qg = 0;
    for (int w : uw) qg = std::gcd(qg, w);
    const int64_t quota = int64_t(std::floor(P.bits_per_dim * D + 1e-9));
    const int nq = int(quota / qg) + 1;
    std::vector<int> pos(nu + 1, 0);
    for (int j = 0; j < nu; ++j) pos[j + 1] = pos[j] + uw[j];
    std::vector<double> pre(D + 1, 0.0);
    for (int i = 0; i < D; ++i) pre[i + 1] = pre[i] + std::max(sig2[i], 0.0);
    std::vector<double> S(nu + 1);
    for (int j = 0; j <= nu; ++j) S[j] = pre[pos[j]];
    const int mwu = P.max_width ? P.max_width / g : nu;
    const double inf = std::numeric_limits<double>::infinity();
    std::vector<double> pw(P.max_bits + 1);
    for (int b = 0; b <= P.max_bits; ++b) pw[b] = std::ldexp(1.0, -b);

    auto relax = [&](const std::vector<double>& src, std::vector<double>& dst,
                     std::vector<int32_t>* back, int d, int d2) {
        const int width = pos[d2] - pos[d];
        const double ssum = S[d2] - S[d];
        const double* sp = &src[size_t(d) * nq];
        double* dp = &dst[size_t(d2) * nq];
        for (int b = 0; b <= P.max_bits; ++b) {
            if (b > 0 && d2 - d > mwu) continue;
            const int cq = b * width / qg;
            if (cq >= nq) continue;
            const double add = ssum * pw[b];
            for (int q = 0; q + cq < nq; ++q) {
                const double cand = sp[q] + add;
                if (cand < dp[q + cq]) {
                    dp[q + cq] = cand;
                    if (back) (*back)[size_t(d2) * nq + q + cq] = (d << 8) | b;
                }
            }
        }
    };

    // Algorithm 2: E[d][Q] best error over the first d units with exactly Q
    // cost units; every reachable E[d] is extended by one segment.
    std::vector<double> E(size_t(nu + 1) * nq, inf);
    E[0] = 0.0;
    for (int d = 0; d < nu; ++d) {
        bool any = false;
        for (int q = 0; q < nq; ++q) any |= std::isfinite(E[size_t(d) * nq + q]);
        if (!any) continue;
        for (int d2 = d + 1; d2 <= nu; ++d2) relax(E, E, nullptr, d, d2);
    }
    double min_err = inf;
    for (int q = 0; q < nq; ++q) min_err = std::min(min_err, E[size_t(nu) * nq + q]);
    if (!std::isfinite(min_err)) return fail(SAQ_EINVAL, "no plan fits the bit quota");

    // segment-count layers: layer k = plans with exactly k+1 segments
    std::vector<double> prev(size_t(nu + 1) * nq, inf), cur;
    prev[0] = 0.0;
    std::vector<std::vector<int32_t>> backs;
    int kstar = -1, qstar = -1;
    for (int k = 0; k < nu; ++k) {
        cur.assign(size_t(nu + 1) * nq, inf);
        backs.emplace_back(size_t(nu + 1) * nq, -1);
        std::vector<int32_t>& bk = backs.back();
#pragma omp parallel for schedule(dynamic, 1)
        for (int d2 = 1; d2 <= nu; ++d2)
            for (int d = 0; d < d2; ++d) relax(prev, cur, &bk, d, d2);
        double best = inf;
        int bq = -1;
        for (int q = 0; q < nq; ++q)
            if (cur[size_t(nu) * nq + q] < best) { best = cur[size_t(nu) * nq + q]; bq = q; }
        if (best <= (1.0 + P.seg_eps) * min_err) { kstar = k; qstar = bq; break; }
        prev.swap(cur);
    }
    if (kstar < 0) return fail(SAQ_EINVAL, "plan search did not converge");
    out.widths.clear(); out.bits.clear();
    int d2 = nu, q = qstar;
    for (int k = kstar; k >= 0; --k) {
        const int32_t bd = backs[size_t(k)][size_t(d2) * nq + q];
        const int d = bd >> 8, b = bd & 255;
        out.widths.push_back(pos[d2] - pos[d]);
        out.bits.push_back(b);
        q -= b * (pos[d2] - pos[d]) / qg;
        d2 = d;
    }
    std::reverse(out.widths.begin(), out.widths.end());
    std::reverse(out.bits.begin(), out.bits.end());
    out.err = 0.0;
    out.used = 0;
    int a = 0;
    for (size_t s = 0; s < out.widths.size(); ++s) {
        out.err += (pre[a + out.widths[s]] - pre[a]) * std::ldexp(1.0, -out.bits[s]);
        out.used += int64_t(out.widths[s]) * out.bits[s];
        a += out.widths[s];
    }
    out.min_err = min_err;
    out.quota = quota;
    return SAQ_OK;
}

// ---------------------------------------------------------------------------
// Random orthonormal matrices for the per-segment rotation (Section 4.1).
// Gaussian entries from SplitMix64 used as a counter-based generator
// (Steele, Lea & Flood, OOPSLA 2014: output i = mix(seed + (i+1) * gamma)),
// Box-Muller, then Gram-Schmidt orthonormalisation (QR with a positive
// diagonal in R, which makes Q Haar distributed; Mezzadri 2007).
// ---------------------------------------------------------------------------

static uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double gauss_at(uint64_t seed, uint64_t i) {
    const uint64_t a = splitmix64_at(seed, 2 * i), b = splitmix64_at(seed, 2 * i + 1);
    const double u1 = (double((a >> 11) + 1)) * 0x1.0p-53;   // (0, 1]
    const double u2 = double(b >> 11) * 0x1.0p-53;           // [0, 1)
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586476925 * u2);
}

// W x W orthonormal matrix, row-major
static std::vector<double> haar(int W, uint64_t seed) {
    std::vector<double> G(size_t(W) * W);
    for (int64_t i = 0; i < int64_t(W) * W; ++i) G[size_t(i)] = gauss_at(seed, uint64_t(i));
    // Gram-Schmidt on the columns of G, twice for orthogonality in FP64
    std::vector<double> Q(size_t(W) * W, 0.0);
    std::vector<double> col(W);
    for (int j = 0; j < W; ++j) {
        for (int i = 0; i < W; ++i) col[i] = G[size_t(i) * W + j];
        for (int pass = 0; pass < 2; ++pass)
            for (int k = 0; k < j; ++k) {
                double dot = 0.0;
                for (int i = 0; i < W; ++i) dot += Q[size_t(i) * W + k] * col[i];
                for (int i = 0; i < W; ++i) col[i] -= dot * Q[size_t(i) * W + k];
            }
        double nn = 0.0;
        for (int i = 0; i < W; ++i) nn += col[i] * col[i];
        nn = std::sqrt(nn);
        for (int i = 0; i < W; ++i) Q[size_t(i) * W + j] = col[i] / nn;
    }
    return Q;
}

static saq_status validate_segments(int32_t D, const std::vector<int32_t>& w, const std::vector<int32_t>& b) {
    int64_t s = 0;
    for (size_t i = 0; i < w.size(); ++i) {
        if (w[i] <= 0) return fail(SAQ_EINVAL, "segment width must be positive");
        if (b[i] < 0 || b[i] > 16) return fail(SAQ_EINVAL, "segment bits must be in 0..16");
        s += w[i];
    }
    if (s != D) return fail(SAQ_EINVAL, "segment widths must sum to D");
    return SAQ_OK;
}

static saq_status make_plan(int32_t D, const std::vector<double>& mean, const std::vector<double>& V,
                            const std::vector<double>& lam, const saq_plan_params& P, saq_plan** out) {
    DPResult r;
    saq_status st = plan_search(lam, P, r);
    if (st != SAQ_OK) return st;
    std::unique_ptr<saq_plan> p(new saq_plan());
    p->D = D;
    p->widths = r.widths;
    p->bits = r.bits;
    p->params = P;
    p->model_error = r.err;
    p->min_error = r.min_err;
    p->quota = r.quota;
    p->used = r.used;
    p->var = lam;
    p->c.resize(D);
    for (int i = 0; i < D; ++i) p->c[i] = float(mean[i]);
    int dk = 0;
    for (size_t s = 0; s < r.widths.size(); ++s) if (r.bits[s] > 0) dk += r.widths[s];
    p->M.assign(size_t(dk) * D, 0.0f);
    int col = 0, row = 0;
    for (size_t s = 0; s < r.widths.size(); ++s) {
        const int W = r.widths[s];
        if (r.bits[s] > 0) {
            std::vector<double> R;
            if (P.rotate_segments) R = haar(W, P.seed * 0x100000001B3ull + uint64_t(s) + 1);
            // spread block: S_s[i][j] = sqrt(lambda_{col+i}) R_s[j][i]
            const size_t sb = p->S.size();
            p->S.resize(sb + size_t(W) * W, 0.0f);
            for (int i = 0; i < W; ++i) {
                const double sl = std::sqrt(std::max(lam[size_t(col + i)], 0.0));
                for (int j = 0; j < W; ++j)
                    p->S[sb + size_t(i) * W + j] =
                        float(sl * (P.rotate_segments ? R[size_t(j) * W + i] : (i == j ? 1.0 : 0.0)));
            }
            // rows of M: R_s * V[:, col .. col+W)^T
#pragma omp parallel for schedule(static)
            for (int j = 0; j < W; ++j) {
                for (int k = 0; k < D; ++k) {
                    double acc;
                    if (P.rotate_segments) {
                        acc = 0.0;
                        for (int t = 0; t < W; ++t) acc += R[size_t(j) * W + t] * V[size_t(k) * D + col + t];
                    } else {
                        acc = V[size_t(k) * D + col + j];
                    }
                    p->M[size_t(row + j) * D + k] = float(acc);
                }
            }
            row += W;
        }
        col += W;
    }
    p->derive();
    *out = p.release();
    return SAQ_OK;
}

saq_status plan_from_moments(int32_t D, const std::vector<double>& mean, std::vector<double> C,
                             const saq_plan_params& P, saq_plan** out) {
    try {
        std::vector<double> lam, V;
        if (!sym_eigen(C, D, lam, V)) return fail(SAQ_EINVAL, "eigen-decomposition did not converge");
        return make_plan(D, mean, V, lam, P, out);
    } catch (const std::bad_alloc&) {
        return fail(SAQ_ENOMEM, "out of host memory");
    }
}

}  // namespace saq

using namespace saq;

void saq_plan::derive() {
    D_kept = 0; n_kept = 0; max_kept_w = 0; max_kept_b = 0; code_bytes = 0;
    kept.clear();
    for (size_t s = 0; s < widths.size(); ++s) {
        if (bits[s] > 0) {
            kept.push_back(SegEntry{D_kept, widths[s], bits[s], int32_t(code_bytes)});
            D_kept += widths[s];
            code_bytes += int64_t(bits[s]) * ((widths[s] + 7) / 8);
            max_kept_w = std::max(max_kept_w, widths[s]);
            max_kept_b = std::max(max_kept_b, bits[s]);
            ++n_kept;
        }
    }
    if (var.empty()) var.assign(size_t(D), 0.0);
    // FP32 accumulation over the whole input dimension measurably breaks
    // code parity for long inputs and fine grids (D = 3072 with 9-bit
    // segments: 3e-4 of codes differ, against 4e-5 with FP64 k-tile totals);
    // auto mode takes the FP64 totals there
    const int mode = params.projection_accumulation;
    acc64 = mode == 2 || (mode == 0 && (D > 1024 || max_kept_b >= 8));
    build_staging(*this);
}

extern "C" {

void saq_default_params(saq_plan_params* p) {
    if (!p) return;
    p->bits_per_dim = 4.0;
    p->granularity = 16;
    p->max_bits = 9;
    p->max_width = 512;
    p->seg_eps = 1e-3;
    p->rotate_segments = 1;
    p->fit_sample = 65536;
    p->seed = 1;
    p->projection_accumulation = 0;
}

const char* saq_last_error(void) { return g_last_error.c_str(); }

saq_status saq_plan_from_basis(const double* mean, const double* eigvecs, const double* eigvals,
                               int32_t D, const saq_plan_params* p, saq_plan** out) {
    if (!mean || !eigvecs || !eigvals || !p || !out || D <= 0) return fail(SAQ_EINVAL, "bad arguments");
    try {
        std::vector<int> ord(D);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return eigvals[a] > eigvals[b]; });
        std::vector<double> V(size_t(D) * D), lam(D), mu(mean, mean + D);
        for (int j = 0; j < D; ++j) {
            lam[j] = eigvals[ord[j]];
            for (int i = 0; i < D; ++i) V[size_t(i) * D + j] = eigvecs[size_t(i) * D + ord[j]];
        }
        return make_plan(D, mu, V, lam, *p, out);
    } catch (const std::bad_alloc&) {
        return fail(SAQ_ENOMEM, "out of host memory");
    }
}

saq_status saq_fit_plan(const float* X, int64_t n, int32_t D, const saq_plan_params* p, saq_plan** out) {
    if (!X || !p || !out || n <= 0 || D <= 0) return fail(SAQ_EINVAL, "bad arguments");
    try {
        const int64_t m = (p->fit_sample > 0 && p->fit_sample < n) ? p->fit_sample : n;
        std::vector<int64_t> rows(static_cast<size_t>(m));
        for (int64_t i = 0; i < m; ++i) rows[size_t(i)] = (m == n) ? i : (i * n) / m;
        // mean: partial sums over fixed blocks of rows, added in block order,
        // so the result does not depend on the thread count or schedule
        std::vector<double> mu(D, 0.0);
        {
            const int64_t MB = 4096;
            const int64_t nb = (m + MB - 1) / MB;
            std::vector<double> part(size_t(nb) * D, 0.0);
#pragma omp parallel for schedule(static)
            for (int64_t b = 0; b < nb; ++b) {
                double* pb = &part[size_t(b) * D];
                for (int64_t i = b * MB; i < std::min(m, (b + 1) * MB); ++i) {
                    const float* x = X + rows[size_t(i)] * D;
                    for (int k = 0; k < D; ++k) pb[k] += double(x[k]);
                }
            }
            for (int64_t b = 0; b < nb; ++b)
                for (int k = 0; k < D; ++k) mu[k] += part[size_t(b) * D + k];
        }
        for (int k = 0; k < D; ++k) mu[k] /= double(m);
        // covariance (1/m) sum (x - c)(x - c)^T, blocked over rows; each block
        // is transposed so the inner products run over contiguous memory
        std::vector<double> C(size_t(D) * D, 0.0);
        const int RB = 256;
        std::vector<double> Yt(size_t(D) * RB);
        for (int64_t r0 = 0; r0 < m; r0 += RB) {
            const int rb = int(std::min<int64_t>(RB, m - r0));
#pragma omp parallel for schedule(static)
            for (int t = 0; t < rb; ++t) {
                const float* x = X + rows[size_t(r0 + t)] * D;
                for (int k = 0; k < D; ++k) Yt[size_t(k) * RB + t] = double(x[k]) - mu[k];
            }
#pragma omp parallel for schedule(dynamic, 4)
            for (int i = 0; i < D; ++i) {
                const double* yi = &Yt[size_t(i) * RB];
                for (int j = 0; j <= i; ++j) {
                    const double* yj = &Yt[size_t(j) * RB];
                    double s = 0.0;
                    for (int t = 0; t < rb; ++t) s += yi[t] * yj[t];
                    C[size_t(i) * D + j] += s;
                }
            }
        }
        for (int i = 0; i < D; ++i)
            for (int j = 0; j <= i; ++j) {
                const double v = C[size_t(i) * D + j] / double(m);
                C[size_t(i) * D + j] = v;
                C[size_t(j) * D + i] = v;
            }
        return plan_from_moments(D, mu, C, *p, out);
    } catch (const std::bad_alloc&) {
        return fail(SAQ_ENOMEM, "out of host memory");
    }
}

saq_status saq_plan_from_parts(int32_t D, int32_t n_seg, const int32_t* widths, const int32_t* bits,
                               const float* M, const float* c, const double* variances, saq_plan** out) {
    if (D <= 0 || n_seg <= 0 || !widths || !bits || !c || !out) return fail(SAQ_EINVAL, "bad arguments");
    std::vector<int32_t> w(widths, widths + n_seg), b(bits, bits + n_seg);
    saq_status st = validate_segments(D, w, b);
    if (st != SAQ_OK) return st;
    int64_t dk = 0;
    for (int s = 0; s < n_seg; ++s) if (b[s] > 0) dk += w[s];
    if (dk > 0 && !M) return fail(SAQ_EINVAL, "M is required when a segment has bits > 0");
    try {
        std::unique_ptr<saq_plan> p(new saq_plan());
        p->D = D;
        p->widths = w;
        p->bits = b;
        p->M.assign(M, M + dk * D);
        p->c.assign(c, c + D);
        if (variances) {
            p->var.assign(variances, variances + D);
            p->S = diagonal_spread(w, b, p->var);
        }
        saq_default_params(&p->params);
        p->params.granularity = 1;
        p->params.max_width = 0;
        for (int s = 0; s < n_seg; ++s) p->used += int64_t(w[s]) * b[s];
        p->quota = p->used;
        double e = 0.0;
        int a = 0;
        for (int s = 0; s < n_seg; ++s) {
            double ss = 0.0;
            if (variances) for (int i = a; i < a + w[s]; ++i) ss += variances[i];
            e += ss * std::ldexp(1.0, -b[s]);
            a += w[s];
        }
        p->model_error = p->min_error = e;
        p->derive();
        *out = p.release();
        return SAQ_OK;
    } catch (const std::bad_alloc&) {
        return fail(SAQ_ENOMEM, "out of host memory");
    }
}

saq_status saq_plan_info_get(const saq_plan* p, saq_plan_info* o) {
    if (!p || !o) return fail(SAQ_EINVAL, "bad arguments");
    o->D = p->D;
    o->D_kept = p->D_kept;
    o->n_seg = int32_t(p->widths.size());
    o->n_kept = p->n_kept;
    o->code_bytes = p->code_bytes;
    o->n_factors = p->n_kept + 1;
    o->max_kept_width = p->max_kept_w;
    o->max_kept_bits = p->max_kept_b;
    o->model_error = p->model_error;
    o->min_error = p->min_error;
    o->quota_bits = p->quota;
    o->used_bits = p->used;
    o->projection_fp64_totals = p->acc64 ? 1 : 0;
    return SAQ_OK;
}

saq_status saq_plan_segments(const saq_plan* p, int32_t* widths, int32_t* bits) {
    if (!p) return fail(SAQ_EINVAL, "bad arguments");
    if (widths) std::copy(p->widths.begin(), p->widths.end(), widths);
    if (bits) std::copy(p->bits.begin(), p->bits.end(), bits);
    return SAQ_OK;
}

saq_status saq_plan_arrays(const saq_plan* p, float* M, float* c, double* var) {
    if (!p) return fail(SAQ_EINVAL, "bad arguments");
    if (M) std::copy(p->M.begin(), p->M.end(), M);
    if (c) std::copy(p->c.begin(), p->c.end(), c);
    if (var) std::copy(p->var.begin(), p->var.end(), var);
    return SAQ_OK;
}

void saq_plan_free(saq_plan* p) { delete p; }

}  // extern "C"

// ---- serialisation --------------------------------------------------------
// "SAQPLAN1" | u32 version | i32 D | i32 n_seg | params | f64 model_error |
// f64 min_error | i64 quota | i64 used | i32 widths[n_seg] | i32 bits[n_seg] |
// f32 c[D] | f64 var[D] | f32 M[D_kept x D] | i64 n_S | f32 S[n_S] |
// u64 FNV-1a of all previous bytes.  Version 1 files end after M (no S).

namespace {
struct Writer {
    std::vector<unsigned char> buf;
    template <class T> void put(const T& v) {
        const unsigned char* b = reinterpret_cast<const unsigned char*>(&v);
        buf.insert(buf.end(), b, b + sizeof(T));
    }
    template <class T> void arr(const T* v, size_t n) {
        const unsigned char* b = reinterpret_cast<const unsigned char*>(v);
        buf.insert(buf.end(), b, b + n * sizeof(T));
    }
};
struct Reader {
    const unsigned char* p; size_t n, i = 0;
    template <class T> bool get(T& v) {
        if (i + sizeof(T) > n) return false;
        std::memcpy(&v, p + i, sizeof(T)); i += sizeof(T); return true;
    }
    template <class T> bool arr(T* v, size_t k) {
        if (k > (n - i) / sizeof(T)) return false;
        std::memcpy(v, p + i, k * sizeof(T)); i += k * sizeof(T); return true;
    }
};
uint64_t fnv1a(const unsigned char* p, size_t n) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < n; ++i) { h ^= p[i]; h *= 0x100000001b3ull; }
    return h;
}
const char kMagic[8] = {'S', 'A', 'Q', 'P', 'L', 'A', 'N', '1'};
}  // namespace

extern "C" {

saq_status saq_plan_save(const saq_plan* p, const char* path) {
    if (!p || !path) return fail(SAQ_EINVAL, "bad arguments");
    Writer w;
    w.arr(kMagic, 8);
    w.put(uint32_t(2));
    w.put(p->D);
    w.put(int32_t(p->widths.size()));
    w.put(p->params);
    w.put(p->model_error);
    w.put(p->min_error);
    w.put(p->quota);
    w.put(p->used);
    w.arr(p->widths.data(), p->widths.size());
    w.arr(p->bits.data(), p->bits.size());
    w.arr(p->c.data(), p->c.size());
    w.arr(p->var.data(), p->var.size());
    w.arr(p->M.data(), p->M.size());
    w.put(int64_t(p->S.size()));
    w.arr(p->S.data(), p->S.size());
    w.put(fnv1a(w.buf.data(), w.buf.size()));
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(SAQ_EIO, std::string("cannot open ") + path);
    const size_t k = std::fwrite(w.buf.data(), 1, w.buf.size(), f);
    const int rc = std::fclose(f);
    if (k != w.buf.size() || rc != 0) return fail(SAQ_EIO, "short write");
    return SAQ_OK;
}

saq_status saq_plan_load(const char* path, saq_plan** out) {
    if (!path || !out) return fail(SAQ_EINVAL, "bad arguments");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(SAQ_EIO, std::string("cannot open ") + path);
    std::vector<unsigned char> buf;
    unsigned char tmp[1 << 16];
    size_t k;
    while ((k = std::fread(tmp, 1, sizeof tmp, f)) > 0) buf.insert(buf.end(), tmp, tmp + k);
    std::fclose(f);
    if (buf.size() < 8 + 8 || std::memcmp(buf.data(), kMagic, 8) != 0) return fail(SAQ_EIO, "not a plan file");
    uint64_t want;
    std::memcpy(&want, buf.data() + buf.size() - 8, 8);
    if (fnv1a(buf.data(), buf.size() - 8) != want) return fail(SAQ_EIO, "plan file checksum mismatch");
    Reader r{buf.data() + 8, buf.size() - 16};
    uint32_t ver; int32_t D, ns;
    std::unique_ptr<saq_plan> p(new saq_plan());
    if (!r.get(ver) || (ver != 1 && ver != 2) || !r.get(D) || !r.get(ns) || D <= 0 || ns <= 0 ||
        ns > D)
        return fail(SAQ_EIO, "bad plan header");
    p->D = D;
    if (!r.get(p->params) || !r.get(p->model_error) || !r.get(p->min_error) || !r.get(p->quota) ||
        !r.get(p->used))
        return fail(SAQ_EIO, "truncated plan file");
    p->widths.resize(ns); p->bits.resize(ns);
    if (!r.arr(p->widths.data(), ns) || !r.arr(p->bits.data(), ns)) return fail(SAQ_EIO, "truncated plan file");
    if (validate_segments(D, p->widths, p->bits) != SAQ_OK) return fail(SAQ_EIO, "bad segments in plan file");
    int64_t dk = 0;
    for (int s = 0; s < ns; ++s) if (p->bits[s] > 0) dk += p->widths[s];
    p->c.resize(D); p->var.resize(D); p->M.resize(size_t(dk * D));
    if (!r.arr(p->c.data(), D) || !r.arr(p->var.data(), D) || !r.arr(p->M.data(), size_t(dk * D)))
        return fail(SAQ_EIO, "truncated plan file");
    if (ver >= 2) {
        int64_t ns2 = 0, want_s = 0;
        for (int s = 0; s < ns; ++s) if (p->bits[s] > 0) want_s += int64_t(p->widths[s]) * p->widths[s];
        if (!r.get(ns2) || (ns2 != 0 && ns2 != want_s)) return fail(SAQ_EIO, "bad spread blocks in plan file");
        p->S.resize(size_t(ns2));
        if (!r.arr(p->S.data(), size_t(ns2))) return fail(SAQ_EIO, "truncated plan file");
    }
    if (r.i != r.n) return fail(SAQ_EIO, "trailing bytes in plan file");
    p->derive();
    *out = p.release();
    return SAQ_OK;
}

const char* saq_version(void) { return "saq-mi355x 0.1 (gfx950)"; }

}  // extern "C"
