/*
 * SAQ oracle: a plain, slow, FP64 CPU implementation of the SAQ encode path
 * and its distance estimator.  TEST INFRASTRUCTURE ONLY: it exists to check
 * the device path and is never called by the product library.  It shares no
 * code, header or table with the device path; the quantization plan
 * (segments, bits, projection matrix M, reference vector c) is read as data.
 *
 * Paper: "SAQ: Pushing the Limits of Vector Quantization through Code
 * Adjustment and Dimension Segmentation" (SIGMOD'26, arXiv 2509.12086).
 *
 *   projection          Section 3.1, Eq. (rotate):  o = P (o_r - c)
 *   initial code        Section 3.1, Eq. (find_nearest_code) and the
 *                       midpoint grid on [-v_max, v_max] with 2^B cells
 *   code adjustment     Algorithm 1 (Adjustment of the LVQ quantized vector),
 *                       objective Eq. (adj-obj), O(1) incremental update
 *   stored factors      end of Section 3.1 (norm and <o_a, o>)
 *   segments            Section 4.1-4.2: each segment of the plan is
 *                       quantized on its own "just as a normal vector"
 *   estimator           Section 3.2, Eq. (estimator_inner_product), and its
 *                       progressive approximation from b-bit code prefixes
 *   multi-stage         Section 4.3: segments read in plan order, the unread
 *                       ones bounded by m sigma_Seg (Chebyshev)
 *
 * Readings where the paper is silent (the same list is kept in the design
 * notes of the repository):
 *   - o_i = +v_max gives floor(2^B) = 2^B, one past the last cell; the code
 *     is clamped to 2^B - 1 (the nearest midpoint, and the only value allowed
 *     by the range test of Algorithm 1).
 *   - v_max = 0 (all-zero segment): every code is 2^(B-1), no adjustment,
 *     and the rescale factor is 0.
 *   - Within a round, dimensions are visited in ascending order and +Delta is
 *     tried before -Delta, as Algorithm 1 lists them.  A move is accepted only
 *     on a strict increase of the cosine.
 *   - rounds < 0 means "repeat until a round accepts nothing".
 *   - The stored per-segment factor is f_s = ||o_s||^2 / <u_s, o_s> with
 *     u = code - (2^B - 1)/2, which equals ||o_s||^2 * Delta / <o_a, o_s>;
 *     the estimator then reads <o_s, q_s> ~= f_s * <u_s, q_s>.
 *
 * Everything is double precision.  OpenMP parallelism is over vectors only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SAQO_MAX_ROUNDS 64

/* One segment of one projected vector: Section 3.1 + Algorithm 1. */
static void caq_segment(const double *o, int W, int B, int rounds,
                        int32_t *code,          /* out: W codes            */
                        double *aux4,           /* out: v, Delta, <x,o>, ||o||^2 */
                        double *init_margin,    /* out or NULL: W          */
                        double *dec_margin,     /* out or NULL: W          */
                        int32_t *round_stats)   /* out or NULL: MAX_ROUNDS+1 */
{
    const double cells = ldexp(1.0, B);          /* 2^B */
    const int cmax = (int)cells - 1;
    double v = 0.0, oo = 0.0;
    for (int i = 0; i < W; ++i) {
        double a = fabs(o[i]);
        if (a > v) v = a;
        oo += o[i] * o[i];
    }
    if (round_stats)
        memset(round_stats, 0, sizeof(int32_t) * (SAQO_MAX_ROUNDS + 1));
    if (v == 0.0) {                 /* all-zero segment */
        for (int i = 0; i < W; ++i) {
            code[i] = (int32_t)(cmax + 1) / 2;
            if (init_margin) init_margin[i] = 0.5;
            if (dec_margin) dec_margin[i] = INFINITY;
        }
        aux4[0] = 0.0; aux4[1] = 0.0; aux4[2] = 0.0; aux4[3] = oo;
        return;
    }
    const double delta = 2.0 * v / cells;       /* Delta = 2 v_max / 2^B */

    /* initial code: c_i = floor((o_i + v_max) / Delta), clamped */
    double *x = (double *)malloc(sizeof(double) * (size_t)W);
    for (int i = 0; i < W; ++i) {
        double q = (o[i] + v) / delta;
        double f = floor(q);
        if (init_margin) {
            double fr = q - f;
            init_margin[i] = fr < 1.0 - fr ? fr : 1.0 - fr;
        }
        if (f > (double)cmax) f = (double)cmax;
        if (f < 0.0) f = 0.0;
        code[i] = (int32_t)f;
        /* quantized value: o_bar_i = Delta (c_i + 0.5) - v_max */
        x[i] = delta * ((double)code[i] + 0.5) - v;
        if (dec_margin) dec_margin[i] = INFINITY;
    }

    /* cosine objective L(x, o) = <x,o> / (||x|| ||o||), kept through the
       running sums <x,o> and ||x||^2 (one coordinate changes per move) */
    double xo = 0.0, xx = 0.0;
    for (int i = 0; i < W; ++i) { xo += x[i] * o[i]; xx += x[i] * x[i]; }
    const double onorm = sqrt(oo);
    double L = xo / (sqrt(xx) * onorm);

    int r_run = 0;
    for (int round = 0; rounds < 0 || round < rounds; ++round) {
        int accepted = 0;
        for (int i = 0; i < W; ++i) {
            for (int k = 0; k < 2; ++k) {
                const double d = k == 0 ? delta : -delta;
                const double xn = x[i] + d;
                if (!(xn >= -v && xn <= v)) continue;       /* range test */
                const double xo2 = xo + d * o[i];
                const double xx2 = xx - x[i] * x[i] + xn * xn;
                const double L2 = xo2 / (sqrt(xx2) * onorm);
                if (dec_margin) {
                    double m = fabs(L2 - L) / fabs(L);
                    if (m < dec_margin[i]) dec_margin[i] = m;
                }
                if (L2 > L) {
                    x[i] = xn; xo = xo2; xx = xx2; L = L2;
                    code[i] += k == 0 ? 1 : -1;
                    ++accepted;
                }
            }
        }
        if (round_stats && round < SAQO_MAX_ROUNDS) round_stats[round] = accepted;
        ++r_run;
        if (accepted == 0) break;       /* no later round can change anything */
        if (rounds < 0 && r_run >= 1000000) break;
    }
    if (round_stats) round_stats[SAQO_MAX_ROUNDS] = r_run;

    /* final code from the adjusted vector with Eq. (find_nearest_code) */
    double xo_f = 0.0;
    for (int i = 0; i < W; ++i) {
        double c2 = floor((x[i] + v) / delta);
        if (c2 > (double)cmax) c2 = (double)cmax;
        code[i] = (int32_t)c2;
        xo_f += x[i] * o[i];
    }
    aux4[0] = v; aux4[1] = delta; aux4[2] = xo_f; aux4[3] = oo;
    free(x);
}

/* Sets the OpenMP thread count for the caller's next parallel regions and
   returns the previous one, which restore_threads() puts back: a call with
   a thread count must not change it for other code in the process (the
   OpenMP runtime is shared with every other library loaded there). */
static int set_threads(int nthreads)
{
#ifdef _OPENMP
    const int prev = omp_get_max_threads();
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return prev;
#else
    (void)nthreads;
    return 1;
#endif
}

static void restore_threads(int prev)
{
#ifdef _OPENMP
    omp_set_num_threads(prev);
#else
    (void)prev;
#endif
}

/*
 * Quantize already-projected vectors O [n x Dk] (FP64, row-major) with the
 * kept segments (widths seg_w, bits seg_b > 0, in plan order, sum = Dk).
 * Outputs:
 *   codes   [n x Dk]  int32 final codes
 *   factors [n x nseg] f_s = ||o_s||^2 / <u_s, o_s>   (0 for v_max = 0)
 *   seg_aux [n x nseg x 4] (v_max, Delta, <o_a,o_s>, ||o_s||^2)   or NULL
 *   code_aux[n x Dk x 2]  (init margin, decision margin)         or NULL
 *   round_stats [n x nseg x (MAX_ROUNDS+1)]                      or NULL
 */
int saqo_quantize(const double *O, int64_t n, int32_t Dk,
                  int32_t nseg, const int32_t *seg_w, const int32_t *seg_b,
                  int32_t rounds, int32_t *codes, double *factors,
                  double *seg_aux, double *code_aux, int32_t *round_stats,
                  int nthreads)
{
    int sum = 0;
    for (int s = 0; s < nseg; ++s) {
        if (seg_w[s] <= 0 || seg_b[s] <= 0 || seg_b[s] > 24) return 1;
        sum += seg_w[s];
    }
    if (sum != Dk || n < 0) return 1;
    const int prev_threads = set_threads(nthreads);
#pragma omp parallel
    {
        double *im = (double *)malloc(sizeof(double) * (size_t)(Dk > 0 ? Dk : 1));
        double *dm = (double *)malloc(sizeof(double) * (size_t)(Dk > 0 ? Dk : 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < n; ++r) {
            int off = 0;
            for (int s = 0; s < nseg; ++s) {
                double aux[4];
                caq_segment(O + r * Dk + off, seg_w[s], seg_b[s], rounds,
                            codes + r * Dk + off, aux,
                            code_aux ? im : NULL, code_aux ? dm : NULL,
                            round_stats ? round_stats + (r * nseg + s) * (SAQO_MAX_ROUNDS + 1) : NULL);
                /* <u,o> = <o_a,o>/Delta ; f = ||o_s||^2 / <u,o> */
                factors[r * nseg + s] = aux[2] != 0.0 ? aux[3] * aux[1] / aux[2] : 0.0;
                if (seg_aux) memcpy(seg_aux + (r * nseg + s) * 4, aux, sizeof aux);
                if (code_aux)
                    for (int i = 0; i < seg_w[s]; ++i) {
                        code_aux[(r * Dk + off + i) * 2 + 0] = im[i];
                        code_aux[(r * Dk + off + i) * 2 + 1] = dm[i];
                    }
                off += seg_w[s];
            }
        }
        free(im); free(dm);
    }
    restore_threads(prev_threads);
    return 0;
}

/* o = M (x - c) in FP64 for n rows; also ||x - c||^2.  Eq. (rotate). */
int saqo_project(const float *X, int64_t n, int32_t D, const float *M, int32_t Dk,
                 const float *c, double *O, double *norm2, int nthreads)
{
    if (n < 0 || D <= 0 || Dk < 0) return 1;
    const int prev_threads = set_threads(nthreads);
#pragma omp parallel
    {
        double *xc = (double *)malloc(sizeof(double) * (size_t)D);
#pragma omp for schedule(static)
        for (int64_t r = 0; r < n; ++r) {
            double nn = 0.0;
            for (int k = 0; k < D; ++k) {
                xc[k] = (double)X[r * D + k] - (double)c[k];
                nn += xc[k] * xc[k];
            }
            norm2[r] = nn;
            for (int j = 0; j < Dk; ++j) {
                double acc = 0.0;
                const float *mj = M + (int64_t)j * D;
                for (int k = 0; k < D; ++k) acc += (double)mj[k] * xc[k];
                O[r * Dk + j] = acc;
            }
        }
        free(xc);
    }
    restore_threads(prev_threads);
    return 0;
}

/* Full encode: projection then quantization (see the two functions above). */
int saqo_encode(const float *X, int64_t n, int32_t D, const float *M, int32_t Dk,
                const float *c, int32_t nseg, const int32_t *seg_w, const int32_t *seg_b,
                int32_t rounds, int32_t *codes, double *factors, double *norm2,
                double *O_out, double *seg_aux, double *code_aux, int32_t *round_stats,
                int nthreads)
{
    double *O = O_out ? O_out : (double *)malloc(sizeof(double) * (size_t)(n * Dk > 0 ? n * Dk : 1));
    int rc = saqo_project(X, n, D, M, Dk, c, O, norm2, nthreads);
    if (rc == 0)
        rc = saqo_quantize(O, n, Dk, nseg, seg_w, seg_b, rounds, codes, factors,
                           seg_aux, code_aux, round_stats, nthreads);
    if (!O_out) free(O);
    return rc;
}

/*
 * Pack codes into the code string: per kept segment, B bit-planes, most
 * significant plane first; each plane holds bit (plane) of the W codes of the
 * segment, dimension i at byte i/8, bit i%8 of the plane; a plane occupies
 * ceil(W/8) bytes.  code_bytes is the record size (sum of B*ceil(W/8)).
 */
int saqo_pack(const int32_t *codes, int64_t n, int32_t Dk, int32_t nseg,
              const int32_t *seg_w, const int32_t *seg_b, uint8_t *out,
              int64_t code_bytes)
{
    int64_t need = 0;
    for (int s = 0; s < nseg; ++s) need += (int64_t)seg_b[s] * ((seg_w[s] + 7) / 8);
    if (need != code_bytes) return 1;
    memset(out, 0, (size_t)(n * code_bytes));
    for (int64_t r = 0; r < n; ++r) {
        uint8_t *rec = out + r * code_bytes;
        int64_t pos = 0;
        int off = 0;
        for (int s = 0; s < nseg; ++s) {
            const int W = seg_w[s], B = seg_b[s], pb = (W + 7) / 8;
            for (int p = B - 1; p >= 0; --p) {
                for (int i = 0; i < W; ++i)
                    if ((codes[r * Dk + off + i] >> p) & 1)
                        rec[pos + i / 8] |= (uint8_t)(1u << (i % 8));
                pos += pb;
            }
            off += W;
        }
    }
    return 0;
}

/*
 * Estimated squared distances d2[qi * n + r] between query rows Q and the
 * encoded data rows, Section 3.2:
 *   q' = M (q - c),  <o_s, q_s> ~= f_s <u_s, q'_s>,  u = code - (2^B - 1)/2,
 *   d2 = ||o||^2 + ||q - c||^2 - 2 sum_s f_s <u_s, q'_s>
 * (dimensions of dropped segments contribute nothing to the inner product;
 * ||o||^2 = ||x - c||^2 is the stored full norm).
 */
/* Estimator of Section 3.2, Eq. (estimator_inner_product), per segment:
 * <o_s, q_s> ~= <o_a, q_s> / <o_a, o_s> * ||o_s||^2 with o_a = Delta u, i.e.
 * f_s <u_s, q_s>.  prefix > 0 takes the progressive approximation of
 * Section 3.2 with b = min(prefix, B) bits per dimension: the prefix code
 * c_s = floor(c / 2^(B-b)) replaces c and Delta' = Delta 2^(B-b) replaces
 * Delta in o_a, so o_a becomes Delta' u' with u' = c_s - (2^b - 1)/2 while
 * the stored <o_a, o_s> is kept: the term is f_s 2^(B-b) <u'_s, q_s>. */
int saqo_estimate(const float *Q, int32_t nq, int32_t D, const float *M, int32_t Dk,
                  const float *c, int32_t nseg, const int32_t *seg_w, const int32_t *seg_b,
                  const int32_t *codes, const double *factors, const double *norm2,
                  int64_t n, int32_t prefix, double *d2, int nthreads)
{
    double *qp = (double *)malloc(sizeof(double) * (size_t)(nq * Dk > 0 ? nq * Dk : 1));
    double *qn = (double *)malloc(sizeof(double) * (size_t)(nq > 0 ? nq : 1));
    int rc = saqo_project(Q, nq, D, M, Dk, c, qp, qn, nthreads);
    if (rc) { free(qp); free(qn); return rc; }
#pragma omp parallel for schedule(static) collapse(2)
    for (int qi = 0; qi < nq; ++qi)
        for (int64_t r = 0; r < n; ++r) {
            double ip = 0.0;
            int off = 0;
            for (int s = 0; s < nseg; ++s) {
                const int B = seg_b[s];
                const int b = (prefix > 0 && prefix < B) ? prefix : B;
                const int shift = B - b;
                const double h = (ldexp(1.0, b) - 1.0) / 2.0;
                double uq = 0.0;
                for (int i = 0; i < seg_w[s]; ++i) {
                    const int cs = (int)floor((double)codes[r * Dk + off + i] / ldexp(1.0, shift));
                    uq += ((double)cs - h) * qp[(int64_t)qi * Dk + off + i];
                }
                ip += factors[r * nseg + s] * ldexp(1.0, shift) * uq;
                off += seg_w[s];
            }
            d2[(int64_t)qi * n + r] = norm2[r] + qn[qi] - 2.0 * ip;
        }
    free(qp); free(qn);
    return 0;
}

/*
 * Multi-stage estimator of Section 4.3.
 *
 * The kept segments are read in plan order, which is decreasing variance.
 * Before segment t is read, the segments already read give their Section 3.2
 * terms est_s = f_s <u_s, q'_s>.  The unread ones are bounded through
 * Chebyshev's inequality: |<o_s, q_s>| < m sigma_s with probability at least
 * 1 - 1/m^2, where
 *   sigma_s^2 = sum_{i in s} q[i]^2 sigma_i^2
 * is the variance over the data of the segment's inner product.  That sum
 * needs uncorrelated dimensions, so q[i] is the query's coordinate on PCA
 * axis i, P_i (q - c), and sigma_i^2 = lambda_i is that axis's variance.  The
 * inner product does not change under the per-segment rotation, so sigma_s
 * bounds the rotated segment as well.  The lower bound on the estimated
 * squared distance at stage t is
 *   LB_t = ||o||^2 + ||q - c||^2 - 2 (sum_{s<t} est_s + m sum_{s>=t} sigma_s).
 * A pair (query, record) is pruned at the first t < k with LB_t > tau[q]; it
 * then gets d2 = LB_t and stage = t (segments 0..t-1 were read).  A pair that
 * is never pruned gets the full estimate and stage = k.
 *
 * P [Dk x D] holds the PCA axes of the kept dimensions in plan order (rows,
 * unrotated) and lam [Dk] their variances.  sigma [nq x k] (optional) gets
 * sigma_s per query.
 */
int saqo_estimate_multistage(const float *Q, int32_t nq, int32_t D, const float *M, int32_t Dk,
                             const float *c, int32_t nseg, const int32_t *seg_w,
                             const int32_t *seg_b, const int32_t *codes, const double *factors,
                             const double *norm2, int64_t n, const double *P, const double *lam,
                             double m, const double *tau, double *d2, int32_t *stage,
                             double *sigma, int nthreads)
{
    if (nq < 0 || n < 0 || nseg < 0 || Dk < 0 || D <= 0 || !(m >= 0.0)) return 1;
    const size_t nqs = (size_t)(nq > 0 ? nq : 1);
    double *qp = (double *)malloc(sizeof(double) * nqs * (size_t)(Dk > 0 ? Dk : 1));
    double *qn = (double *)malloc(sizeof(double) * nqs);
    double *sg = (double *)malloc(sizeof(double) * nqs * (size_t)(nseg > 0 ? nseg : 1));
    int rc = saqo_project(Q, nq, D, M, Dk, c, qp, qn, nthreads);
    if (rc) { free(qp); free(qn); free(sg); return rc; }
    /* sigma_s from the query's PCA coordinates */
    for (int qi = 0; qi < nq; ++qi) {
        int off = 0;
        for (int s = 0; s < nseg; ++s) {
            double v = 0.0;
            for (int i = 0; i < seg_w[s]; ++i) {
                double y = 0.0;
                for (int k = 0; k < D; ++k)
                    y += P[(int64_t)(off + i) * D + k] * ((double)Q[(int64_t)qi * D + k] - (double)c[k]);
                v += lam[off + i] * y * y;
            }
            sg[(int64_t)qi * nseg + s] = sqrt(v);
            if (sigma) sigma[(int64_t)qi * nseg + s] = sqrt(v);
            off += seg_w[s];
        }
    }
#pragma omp parallel for schedule(static) collapse(2)
    for (int qi = 0; qi < nq; ++qi)
        for (int64_t r = 0; r < n; ++r) {
            const double *sq = sg + (int64_t)qi * nseg;
            double ip = 0.0;
            int t = 0, off = 0;
            double out = 0.0;
            for (; t < nseg; ++t) {
                double rest = 0.0;                  /* sum of sigma_s over s >= t */
                for (int s = t; s < nseg; ++s) rest += sq[s];
                const double lb = norm2[r] + qn[qi] - 2.0 * (ip + m * rest);
                if (lb > tau[qi]) { out = lb; break; }
                const double h = (ldexp(1.0, seg_b[t]) - 1.0) / 2.0;
                double uq = 0.0;
                for (int i = 0; i < seg_w[t]; ++i)
                    uq += ((double)codes[r * Dk + off + i] - h) * qp[(int64_t)qi * Dk + off + i];
                ip += factors[r * nseg + t] * uq;
                off += seg_w[t];
            }
            if (t == nseg) out = norm2[r] + qn[qi] - 2.0 * ip;
            d2[(int64_t)qi * n + r] = out;
            stage[(int64_t)qi * n + r] = t;
        }
    free(qp); free(qn); free(sg);
    return 0;
}

int saqo_max_rounds(void) { return SAQO_MAX_ROUNDS; }
