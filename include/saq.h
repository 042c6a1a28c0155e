/*
 * saq.h -- C ABI of the MI355X SAQ encoder (libsaq.so).
 *
 * SAQ: "Pushing the Limits of Vector Quantization through Code Adjustment and
 * Dimension Segmentation" (SIGMOD'26, arXiv 2509.12086).
 *
 * Conventions shared by every entry point
 *   - Status codes: every call returns saq_status; on failure
 *     saq_last_error() (thread-local) holds a message.  Nothing throws.
 *   - Device buffers (inputs, codes, factors, workspaces, the uploaded plan)
 *     are caller-owned device memory on the current HIP device.  The library
 *     allocates no device memory.  Plan handles are library-owned host
 *     objects, freed with saq_plan_free.
 *   - Asynchrony: device calls enqueue work on `stream` (a hipStream_t passed
 *     as void*, NULL = the default stream) and return; results are valid
 *     after the stream is synchronised, and inputs must stay alive until then.
 *   - n == 0 is a no-op.  Negative sizes, NULL required pointers, a workspace
 *     smaller than the matching *_workspace_bytes() or a plan that was not
 *     uploaded give SAQ_EINVAL; a failed launch gives SAQ_EDEVICE.
 *   - Inputs must be finite.  Non-finite inputs give unspecified codes but
 *     never an out-of-bounds access.
 *
 * Record layout (per encoded vector)
 *   codes   : code_bytes bytes.  For each kept segment (bits B > 0) in plan
 *             order, B bit-planes, most significant first; plane p holds bit
 *             p of the segment's W codes, dimension i at byte i/8, bit i%8;
 *             a plane takes ceil(W/8) bytes.  (The paper stores a B*D-bit
 *             string, end of Section 3.1; the plane order keeps every b-bit
 *             prefix a valid b-bit code, Section 3.2.)
 *   factors : n_kept + 1 floats: f_s = ||o_s||^2 / <u_s, o_s> for each kept
 *             segment (u = code - (2^B - 1)/2), then ||o||^2 = ||x - c||^2.
 *             The paper stores the norm and <o_a, o> (end of Section 3.1);
 *             f_s carries the same information for the estimator of
 *             Section 3.2: <o_s, q_s> ~= f_s <u_s, q_s>.
 */
#ifndef SAQ_H
#define SAQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SAQ_OK = 0,
    SAQ_EINVAL = 1,        /* bad argument */
    SAQ_ENOMEM = 2,        /* host allocation failed */
    SAQ_EDEVICE = 3,       /* HIP error (launch, copy) */
    SAQ_EUNSUPPORTED = 4,  /* valid but not supported by this library */
    SAQ_EIO = 5            /* plan file missing, truncated or corrupt */
} saq_status;

typedef struct saq_plan saq_plan;   /* opaque, library-owned */

/* Plan-search parameters (Sections 4.1-4.2). */
typedef struct {
    double   bits_per_dim;    /* average budget B; Q_quota = floor(B * D) bits */
    int32_t  granularity;     /* segment widths are multiples of g dims (paper: 64) */
    int32_t  max_bits;        /* allowed bits per dim: 0..max_bits (<= 16) */
    int32_t  max_width;       /* cap on the width of a segment with bits > 0, multiple of g (0 = none) */
    double   seg_eps;         /* fewest segments whose modelled error is <= (1 + seg_eps) * minimum (paper: 0.1 %) */
    int32_t  rotate_segments; /* 1: random orthonormal rotation inside each kept segment (Section 4.1) */
    int64_t  fit_sample;      /* rows used for mean/covariance (0 = all); an evenly spaced subset */
    uint64_t seed;            /* seeds the per-segment rotations */
    int32_t  projection_accumulation; /* 0 auto: FP64 k-tile totals when D > 1024 or a kept
                                         segment has >= 8 bits, else FP32; 1: FP32 throughout;
                                         2: FP32 per 32-wide k-tile, FP64 across tiles.  Every
                                         FP32 product is formed as six bf16 matrix-core
                                         products of operands split exactly into three bf16
                                         terms (each product within about two FP32
                                         unit roundoffs, 2^-23 relative). */
} saq_plan_params;

typedef struct {
    int32_t D;            /* input dimension */
    int32_t D_kept;       /* dims in segments with bits > 0 (rows of M) */
    int32_t n_seg;        /* all segments, including 0-bit ones */
    int32_t n_kept;       /* segments with bits > 0 */
    int64_t code_bytes;   /* bytes of one code record */
    int32_t n_factors;    /* floats of one factor record = n_kept + 1 */
    int32_t max_kept_width;
    int32_t max_kept_bits;
    double  model_error;  /* sum over segments of 2^-B * sum sigma_i^2 (Eq. seg-err without 1/pi) */
    double  min_error;    /* minimum of the model over all plans within the quota */
    int64_t quota_bits;   /* Q_quota */
    int64_t used_bits;    /* sum B * |Seg| */
    int32_t projection_fp64_totals; /* 1 when the projection adds its k-tiles in FP64 */
} saq_plan_info;

/* Defaults: B=4, g=16, max_bits=9, max_width=512, seg_eps=1e-3, rotation on,
   fit_sample=65536, seed=1, projection_accumulation=0 (auto). */
void saq_default_params(saq_plan_params* p);

/* Fit a plan on host rows X [n x D] (row-major FP32): mean c, covariance and
   its FP64 eigen-decomposition (Section 4.1, variances sorted descending),
   the plan search of Algorithm 2 with the fewest-segments rule (Section 4.2),
   per-segment random rotations, and M = blockdiag(R_s) P_kept rounded to FP32
   (Eq. rotate; PCA and rotation folded into one matrix as Section 5.2 notes).
   *out receives a new handle. */
saq_status saq_fit_plan(const float* X, int64_t n, int32_t D,
                        const saq_plan_params* p, saq_plan** out);

/* Mean and covariance of the fit sample on the device (Section 4.1): the
   same evenly spaced sample as saq_fit_plan (row i*n/m of X_dev for
   i < m = fit_sample, or every row when fit_sample is 0 or >= n), X_dev
   [n x D] FP32 row-major on the device.  mean_dev [D] FP64 is the host fit's
   mean bit for bit (fixed 4,096-row blocks added in block order); cov_dev
   [D x D] FP64 row-major = (1/m) sum (x - c)(x - c)^T, summed on the FP64
   matrix cores in a fixed order (run to run identical, equal to the host's
   covariance up to FP64 rounding).  ws_dev: saq_covariance_workspace_bytes
   bytes.  Asynchronous on `stream`. */
int64_t    saq_covariance_workspace_bytes(int64_t n, int32_t D, int64_t fit_sample);
saq_status saq_covariance(const float* X_dev, int64_t n, int32_t D, int64_t fit_sample,
                          double* mean_dev, double* cov_dev, void* ws_dev, int64_t ws_bytes,
                          void* stream);

/* Eigen-decomposition of a symmetric matrix on the device (the PCA basis
   of Section 4.1 from a covariance): A_dev [n x n] FP64 row-major (read
   only; the upper and lower triangles must agree), w_dev [n] the
   eigenvalues in no particular order, V_dev [n x n] FP64 row-major with the
   unit eigenvector of w_dev[j] in column j.  Cyclic Jacobi with a parallel
   (round-robin) ordering, in FP64, run until the off-diagonal mass is below
   1e-15 of the diagonal's; SAQ_EINVAL if that takes more than 40 sweeps.
   The call waits for `stream` once per sweep.  ws_dev:
   saq_sym_eigen_workspace_bytes(n) bytes (three n x n FP64 buffers). */
int64_t    saq_sym_eigen_workspace_bytes(int32_t n);
saq_status saq_sym_eigen_device(const double* A_dev, int32_t n, double* w_dev, double* V_dev,
                                void* ws_dev, int64_t ws_bytes, void* stream);

/* saq_fit_plan with the rows on the device: the mean and covariance from
   saq_covariance, their eigen-decomposition from saq_sym_eigen_device, then
   the basis (D + D x D values) is copied back (the call waits for `stream`)
   and the plan search runs on the host, as saq_plan_from_basis.
   ws_dev: saq_fit_workspace_bytes bytes. */
int64_t    saq_fit_workspace_bytes(int64_t n, int32_t D, const saq_plan_params* p);
saq_status saq_fit_plan_device(const float* X_dev, int64_t n, int32_t D,
                               const saq_plan_params* p, void* ws_dev, int64_t ws_bytes,
                               void* stream, saq_plan** out);

/* Same as saq_fit_plan from a given basis: mean [D], eigenvectors [D x D]
   row-major with eigenvector j in column j, eigenvalues [D] (any order; they
   are sorted descending together with their vectors). */
saq_status saq_plan_from_basis(const double* mean, const double* eigvecs,
                               const double* eigvals, int32_t D,
                               const saq_plan_params* p, saq_plan** out);

/* A plan given explicitly: n_seg segments (widths summing to D, bits in
   0..16), M [D_kept x D] FP32 row-major whose rows follow the kept segments
   in order, c [D] FP32, and optional per-dim variances [D] (may be NULL).
   The variances are taken as those of M's rows, which are assumed
   uncorrelated (the multi-stage bound of saq_estimate_multistage uses them;
   without them it returns SAQ_EINVAL). */
saq_status saq_plan_from_parts(int32_t D, int32_t n_seg, const int32_t* widths,
                               const int32_t* bits, const float* M, const float* c,
                               const double* variances, saq_plan** out);

saq_status saq_plan_info_get(const saq_plan* plan, saq_plan_info* out);
/* widths/bits: arrays of n_seg entries (all segments, plan order). */
saq_status saq_plan_segments(const saq_plan* plan, int32_t* widths, int32_t* bits);
/* M [D_kept x D], c [D], variances [D]; any output may be NULL. */
saq_status saq_plan_arrays(const saq_plan* plan, float* M, float* c, double* variances);
/* Versioned binary file with a checksum; load gives SAQ_EIO on a bad file. */
saq_status saq_plan_save(const saq_plan* plan, const char* path);
saq_status saq_plan_load(const char* path, saq_plan** out);
void saq_plan_free(saq_plan* plan);

/* Device-resident copy of the plan: saq_plan_device_bytes() bytes of
   caller-owned device memory, filled by saq_plan_upload (enqueued on stream;
   the host staging copy is kept by the plan until it is freed).  A plan can
   be uploaded again to another buffer; the last upload is the one used.
   Calls that use the plan must run with the upload's device current (the
   kernels read the buffer there); otherwise they return SAQ_EINVAL. */
int64_t    saq_plan_device_bytes(const saq_plan* plan);
saq_status saq_plan_upload(saq_plan* plan, void* dev_buf, void* stream);

/* Encode n rows X_dev [n x D] (row-major FP32, device): o = M (x - c) with a
   matrix-core GEMM at FP32 accuracy (Eq. rotate; the plan's
   projection_accumulation picks FP32 or FP64-total accumulation), then for
   every kept segment the grid quantization of Eq. (find_nearest_code) and
   `rounds` rounds of the code adjustment of Algorithm 1 (stopping early once
   a round changes nothing, which cannot alter the result), then the stored
   factors and the bit-plane record.  codes_dev [n x code_bytes], factors_dev [n x n_factors].
   ws_dev: saq_encode_workspace_bytes(plan, n) bytes of device scratch.
   A kept segment wider than the quantize kernel's LDS code buffer (1024 dims
   at <= 8 bits, 512 dims above) gives SAQ_EUNSUPPORTED. */
int64_t    saq_encode_workspace_bytes(const saq_plan* plan, int64_t n);
saq_status saq_encode(const saq_plan* plan, const float* X_dev, int64_t n, int32_t rounds,
                      uint8_t* codes_dev, float* factors_dev, void* ws_dev, int64_t ws_bytes,
                      void* stream);

/* saq_encode with a reference vector per record instead of the plan's c
   (Section 3.1's reference vector; the paper's experiments use the IVF
   centroid of each vector's list): record i encodes
     o_i = M (x_i - refs[ref_ids[i]]),  ||x_i - refs[ref_ids[i]]||^2
   with everything else as saq_encode.  refs_dev [K x D] FP32 row-major,
   ref_ids_dev [n] int32 on the device.  A record whose id is outside [0, K)
   is centered on row 0 and gets a NaN norm (its last factor), so it cannot
   pass unnoticed; nothing is read out of bounds.  The plan's M and segments
   should come from a fit on the residuals x - refs[id].  Same workspace as
   saq_encode.  SAQ_EINVAL for K <= 0 or null refs/ids with n > 0. */
saq_status saq_encode_ref(const saq_plan* plan, const float* X_dev, int64_t n,
                          const float* refs_dev, int32_t K, const int32_t* ref_ids_dev,
                          int32_t rounds, uint8_t* codes_dev, float* factors_dev, void* ws_dev,
                          int64_t ws_bytes, void* stream);

/* saq_encode for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
   the same kernels and records as saq_encode, with the workspace taken from
   a fixed device array of SAQ_NOALLOC_SCRATCH_BYTES that the library holds
   on each GPU it runs on until the process ends.  The call allocates and
   frees nothing.  n is accepted when saq_encode_workspace_bytes(plan, n) <=
   SAQ_NOALLOC_SCRATCH_BYTES (at D_kept = 864 about 19,000 rows); a larger n
   gives SAQ_EINVAL with the limit in saq_last_error(), and the caller splits
   the batch.  Inputs and outputs are as in saq_encode (caller-owned device
   buffers, asynchronous on `stream`).  Every call on one GPU uses the same
   array: calls that overlap on one GPU (other streams, other threads,
   another replay of a captured graph) race and must be ordered by the
   caller. */
#define SAQ_NOALLOC_SCRATCH_BYTES (64LL << 20)
saq_status saq_encode_noalloc(const saq_plan* plan, const float* X_dev, int64_t n,
                              int32_t rounds, uint8_t* codes_dev, float* factors_dev,
                              void* stream);

/* Layouts of a projected-row buffer O with leading dimension ld:
   SAQ_LAYOUT_ROWS:  element (vector i, kept dim j) at O[i * ld + j], ld >= D_kept
   SAQ_LAYOUT_DIMS:  element (vector i, kept dim j) at O[j * ld + i], ld >= n,
                     ld % 4 == 0 and O 16-byte aligned
   SAQ_LAYOUT_TILES: element (vector i, kept dim j) at
                     O[((i / 64) * ld + j) * 64 + i % 64], ld >= D_kept, O
                     16-byte aligned and holding ceil(n / 64) whole tiles of
                     ld x 64 floats (what saq_encode uses internally: the 64
                     vectors one wave quantizes are one tile, each kept dim 64
                     contiguous floats).  saq_project also fills the slots of
                     the last tile past n (with copies of row n - 1);
                     saq_quantize reads them and never uses their values. */
#define SAQ_LAYOUT_ROWS  0
#define SAQ_LAYOUT_DIMS  1
#define SAQ_LAYOUT_TILES 2

/* The projection step alone (the GEMM saq_encode runs):
   O = M (x_i - c) for the D_kept kept dims in the given layout, and
   norm2_dev[i] = ||x_i - c||^2 (may be NULL). */
saq_status saq_project(const saq_plan* plan, const float* X_dev, int64_t n,
                       float* O_dev, int64_t ld, int32_t layout, float* norm2_dev,
                       void* stream);

/* Everything after the projection (the second kernel saq_encode runs), on
   given projected rows O_dev in the given layout: quantization, adjustment,
   factors and packing exactly as in saq_encode.  norm2_dev gives the last
   factor (||x - c||^2); when NULL the squared norm of the kept dims is used. */
saq_status saq_quantize(const saq_plan* plan, const float* O_dev, int64_t ld, int32_t layout,
                        int64_t n, const float* norm2_dev, int32_t rounds, uint8_t* codes_dev,
                        float* factors_dev, void* stream);

/* Estimated squared distances (Section 3.2, Eq. estimator_inner_product)
   between nq query rows Q_dev [nq x D] and n encoded records:
     dist2_dev[q * n + i] = ||o_i||^2 + ||q - c||^2 - 2 sum_s f_s <u_s, q'_s>,
   q' = M (q - c).  ws_dev: saq_estimate_workspace_bytes(plan, nq) bytes. */
int64_t    saq_estimate_workspace_bytes(const saq_plan* plan, int32_t nq);
saq_status saq_estimate_dist(const saq_plan* plan, const float* Q_dev, int32_t nq,
                             const uint8_t* codes_dev, const float* factors_dev, int64_t n,
                             float* dist2_dev, void* ws_dev, int64_t ws_bytes, void* stream);

/* The same estimate from code prefixes (progressive approximation, Section
   3.2): every kept segment with B bits reads only its first
   b = min(prefix_bits, B) bit planes, i.e. the prefix codes
   c_s = floor(c / 2^(B-b)), which stand for the B-bit grid with
   Delta' = Delta 2^(B-b):
     dist2_dev[q * n + i] = ||o_i||^2 + ||q - c||^2
                            - 2 sum_s f_s 2^(B-b) <c_s - (2^b - 1)/2, q'_s>.
   prefix_bits = 0 (or >= every B) is saq_estimate_dist; < 0 gives
   SAQ_EINVAL.  Same workspace as saq_estimate_dist. */
saq_status saq_estimate_dist_prefix(const saq_plan* plan, const float* Q_dev, int32_t nq,
                                    const uint8_t* codes_dev, const float* factors_dev,
                                    int64_t n, int32_t prefix_bits, float* dist2_dev,
                                    void* ws_dev, int64_t ws_bytes, void* stream);

/* saq_estimate_dist over records encoded against one reference vector ref_dev
   [D] FP32 (one list of saq_encode_ref records, all with the same id): the
   queries are projected as q' = M (q - ref) and ||q - ref||^2 replaces
   ||q - c||^2.  Same workspace as saq_estimate_dist. */
saq_status saq_estimate_dist_ref(const saq_plan* plan, const float* Q_dev, int32_t nq,
                                 const float* ref_dev, const uint8_t* codes_dev,
                                 const float* factors_dev, int64_t n, float* dist2_dev,
                                 void* ws_dev, int64_t ws_bytes, void* stream);

/* Multi-stage estimate with Chebyshev pruning (Section 4.3).  The kept
   segments are read in plan order (decreasing variance).  Before segment t,
   the distance of a pair (query q, record i) is bounded from below by
     LB_t = ||o_i||^2 + ||q - c||^2 - 2 (sum_{s<t} f_s <u_s, q'_s> + m sum_{s>=t} sigma_s),
   with sigma_s^2 = sum_{j in s} lambda_j (P_j (q - c))^2 the variance over the
   data of the segment's inner product (P_j the PCA axis behind kept dim j,
   lambda_j its variance; the plan's per-segment rotation does not change
   it), so each unread segment exceeds m sigma_s with probability at most
   1/m^2.  The first t < k with LB_t > tau_dev[q] closes the pair:
     dist2_dev[q * n + i] = LB_t,        stage_dev[q * n + i] = t;
   a pair never closed gets the full Section 3.2 estimate and stage k (the
   number of kept segments), so the bits read for it are
   sum_{s < stage} B_s W_s.  tau_dev [nq] FP32 thresholds (e.g. the current
   k-th best distance; +inf closes nothing and gives saq_estimate_dist's
   values), m >= 0 (the paper's default is 4), stage_dev [nq x n] uint8 or
   NULL.  A workgroup stops reading codes once every pair it holds is
   closed.  Same workspace as saq_estimate_dist.
   Errors: SAQ_EINVAL for a plan without variances (saq_plan_from_parts
   without them), m < 0 or not finite; SAQ_EUNSUPPORTED for plans with more
   than 255 kept segments, a kept segment wider than 4096 dims, or none. */
saq_status saq_estimate_multistage(const saq_plan* plan, const float* Q_dev, int32_t nq,
                                   const uint8_t* codes_dev, const float* factors_dev,
                                   int64_t n, const float* tau_dev, float m, float* dist2_dev,
                                   uint8_t* stage_dev, void* ws_dev, int64_t ws_bytes,
                                   void* stream);

/* saq_estimate_multistage over one list of saq_encode_ref records with
   reference ref_dev [D] (as saq_estimate_dist_ref). */
saq_status saq_estimate_multistage_ref(const saq_plan* plan, const float* Q_dev, int32_t nq,
                                       const float* ref_dev, const uint8_t* codes_dev,
                                       const float* factors_dev, int64_t n, const float* tau_dev,
                                       float m, float* dist2_dev, uint8_t* stage_dev,
                                       void* ws_dev, int64_t ws_bytes, void* stream);

/* Batched encode: many datasets, each with its own uploaded plan (uneven
   segment widths and bits; the batching pattern stated for the method's
   encode path), in one launch for the whole batch however many datasets
   there are.  In the default mode a persistent grid (as many workgroups as
   stay resident) takes row blocks of every dataset from one atomic ticket;
   a workgroup projects its row block against all of the dataset's kept dims
   and then quantizes, adjusts and packs those rows itself, so no workgroup
   ever waits for another (a tiny kernel clears the ticket first).  The
   other mode runs two grouped launches: every dataset's projection tiles,
   then every dataset's quantize/adjust/pack blocks.  Every dataset gets
   exactly the records saq_encode would give it, in either mode and with any
   launch shape.  ws_dev: saq_encode_batched_workspace_bytes() bytes (the
   projected rows of all datasets and the ticket). */
#define SAQ_BATCH_MAX 16
typedef struct {
    const saq_plan* plan;      /* uploaded plan of this dataset */
    const float* X_dev;        /* [n x D] FP32 rows */
    int64_t n;                 /* rows (0 = nothing to do for this entry) */
    uint8_t* codes_dev;        /* [n x code_bytes] */
    float* factors_dev;        /* [n x n_factors] */
} saq_batch_item;

/* Launch shape (picked by the autotuner; zero fields take defaults). */
#define SAQ_BATCH_FUSED   0    /* one persistent fused launch (default) */
#define SAQ_BATCH_GROUPED 1    /* two grouped launches */
typedef struct {
    int32_t quant_waves;     /* grouped mode: waves (of 64 vectors) per quantize workgroup: 1, 2
                                or 4 (0: 1); halved while their LDS code buffers exceed 64 KiB */
    int32_t gemm_xcd_order;  /* grouped mode: 1 XCD-aware projection tile order (default),
                                0 row-major */
    int32_t mode;            /* SAQ_BATCH_FUSED or SAQ_BATCH_GROUPED */
    int32_t tile_rows;       /* projection tile rows: 0 auto, 64, or 128 (128 only when no
                                dataset accumulates its projection in FP64 k-tile totals) */
    int32_t reserved;        /* must be 0 */
} saq_batch_tuning;

int64_t    saq_encode_batched_workspace_bytes(const saq_batch_item* items, int32_t count,
                                              const saq_batch_tuning* tuning);
saq_status saq_encode_batched(const saq_batch_item* items, int32_t count, int32_t rounds,
                              const saq_batch_tuning* tuning, void* ws_dev, int64_t ws_bytes,
                              void* stream);

const char* saq_last_error(void);
const char* saq_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SAQ_H */
