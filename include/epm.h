/*
 * epm.h -- exact epipolar-guided matching on AMD Instinct MI355X (gfx950).
 *
 * Implements the data-parallel hot path of Nasypanyi & Rameau,
 * "Pixel-Accurate Epipolar Guided Matching":
 *
 *   1. epm_build_intervals   every image-2 keypoint's tolerance circle becomes
 *                            the angular interval between its two tangents
 *                            seen from the epipole (Sec. 4.1-4.2, Eq. 5-6,
 *                            Algorithm 1 preprocessing, Sec. 4.4 special
 *                            cases), laid out on the device sorted by angle;
 *   2. epm_query_candidates  every image-1 keypoint's epipolar line
 *                            l = F (x, y, 1)^T (Eq. 2) stabs those intervals
 *                            with its angle (Eq. 7, mod pi); each retrieved
 *                            candidate is confirmed by the FP64 point-line
 *                            test of Eq. 3, so the output is exactly the set
 *                            of Eq. 4, as CSR;
 *   3. epm_match             nearest-neighbour descriptor selection over each
 *                            candidate set, with an optional Lowe ratio test
 *                            (Sec. 4.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array argument is a DEVICE pointer owned by the caller (for
 *    instance the data_ptr() of a torch tensor).  The library never
 *    allocates device memory: all of its scratch lives in the caller's
 *    workspace (see epm_workspace_bytes), except for
 *    epm_query_match_noalloc, whose scratch is a fixed array of the library.
 *    Host-side bookkeeping lives in the opaque epm_index, released with
 *    epm_index_destroy.
 *  - `pairs` is a HOST array.  A batch of image pairs is concatenated along
 *    the keypoint axis: pair p owns image-1 rows [q_begin, q_begin + m) of
 *    kp1/desc1 and image-2 rows [k_begin, k_begin + n) of kp2/eps2/desc2.
 *    Slices must be in increasing order, contiguous and non-overlapping,
 *    starting at 0 (q_begin[0] = k_begin[0] = 0).
 *  - Keypoints are FP32 pixel coordinates (x, y), row-major [N][2], used as
 *    given (no half-pixel shift); keypoints outside the image are legal.
 *  - Work is enqueued on `stream` (0 = the null stream) and runs
 *    asynchronously, except where a call documents a host synchronisation.
 *  - Every call returns an epm_status and never throws.  Arguments are
 *    validated on the host before anything is launched; a failed validation
 *    launches nothing.
 *  - Column indices in the CSR are local to their pair (0 <= j < n_p).
 *  - Limits: num_pairs <= 65535; every m, n < 2^31; the batch totals of m and
 *    of n are each < 2^32.
 */
#ifndef EPM_H
#define EPM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EPM_OK = 0,
  EPM_ERR_ARG = 1,            /* null pointer, bad size or layout, bad option     */
  EPM_ERR_DEGENERATE_F = 2,   /* F non-finite, zero, or of rank <= 1: no epipole  */
  EPM_ERR_CAPACITY = 3,       /* col_indices too small; *nnz_host = required size */
  EPM_ERR_WORKSPACE = 4,      /* workspace too small or misaligned                */
  EPM_ERR_HIP = 5,            /* a HIP runtime call or kernel launch failed       */
  EPM_ERR_UNSUPPORTED = 6     /* valid request this build does not implement      */
} epm_status;

typedef enum {
  EPM_F32 = 0,       /* 128 x float32 per descriptor                              */
  EPM_BF16 = 1,      /* 128 x bfloat16 (uint16 bit patterns)                      */
  EPM_FP8_E4M3 = 2,  /* 128 x OCP float8 e4m3fn codes + one float32 scale per row */
  EPM_BIN256 = 3     /* 256-bit binary descriptor, 8 x uint32 per row             */
} epm_dtype;

/* Matching algorithm, passed in epm_match_opts.algo. */
typedef enum {
  EPM_ALGO_AUTO = 0,   /* tiled path for float types, gather path for binary       */
  EPM_ALGO_PLAIN = 1,  /* one wavefront per query, per-candidate descriptor gathers */
  EPM_ALGO_TILED = 2   /* angle-sorted query tiles against LDS-staged windows      */
} epm_algo;

/* One image pair, in host memory; an array of these is a batch. */
typedef struct {
  double F[9];        /* row-major F12: l2 = F (x1, y1, 1)^T, x2^T F x1 = 0 (Eq. 1-2) */
  int32_t w2, h2;     /* image-2 size in pixels: used for numerical normalisation only */
  int64_t q_begin, m; /* this pair's slice of the image-1 arrays                       */
  int64_t k_begin, n; /* this pair's slice of the image-2 arrays                       */
} epm_pair;

typedef struct epm_index epm_index;

/*
 * Device workspace needed to build an index over `pairs` and to run
 * epm_query_candidates / epm_match on it (bytes; the base must be 256-byte
 * aligned).  Returns 0 if `pairs` is invalid.
 */
size_t epm_workspace_bytes(const epm_pair* pairs, int32_t num_pairs);

/*
 * Preprocessing of Algorithm 1 (Sec. 4.2, Eq. 5-6; Sec. 4.4).
 *
 * kp2_xy    [N2][2] float32, N2 = sum of n over the batch.
 * eps2      [N2] float32 tolerance in pixels per image-2 keypoint, or NULL to
 *           use eps_scalar for every keypoint.  A tolerance that is not a
 *           positive finite number is accepted and handled exactly like the
 *           definition (such keypoints are simply always tested).
 * workspace device buffer of at least epm_workspace_bytes(pairs, num_pairs)
 *           bytes; it must stay alive and untouched while the index is used.
 * out       receives a new index (host object); release with
 *           epm_index_destroy.  On error *out is left NULL.
 *
 * Errors: EPM_ERR_ARG (null pointers, bad slices, eps_scalar not positive
 * finite when eps2 is NULL), EPM_ERR_DEGENERATE_F (pair without a finite or
 * infinite epipole: F non-finite, zero, or rank <= 1), EPM_ERR_WORKSPACE,
 * EPM_ERR_HIP.  The caller's kp2/eps2 buffers are only read while the work
 * enqueued here runs.
 */
epm_status epm_build_intervals(const epm_pair* pairs, int32_t num_pairs, const float* kp2_xy,
                               const float* eps2, float eps_scalar, void* workspace,
                               size_t workspace_bytes, epm_index** out, hipStream_t stream);

/*
 * Matching loop of Algorithm 1, candidate half (Sec. 4.2, Eq. 2-4, 7).
 *
 * kp1_xy       [N1][2] float32, N1 = sum of m over the batch.
 * row_offsets  [N1 + 1] int64 output: query i's candidates are
 *              col_indices[row_offsets[i] .. row_offsets[i+1]), ascending j.
 * col_indices  [capacity] int32 output, image-2 index local to the pair.
 * nnz_host     host pointer receiving the total number of candidates.
 *
 * The result is exactly { j : |a x_j + b y_j + c| <= eps_j sqrt(a^2 + b^2) }
 * evaluated in FP64 with a = (F0 x + F1 y) + F2, b, c alike (no FMA
 * contraction) -- Eq. 3-4 multiplied through by the positive denominator,
 * closed boundary.  A query whose line has a = b = 0 gets an empty row.
 *
 * Synchronises the host with `stream` once (to read nnz) when nnz_host is
 * not NULL.  If the total exceeds `capacity`, returns EPM_ERR_CAPACITY with
 * *nnz_host set to the required size and writes nothing at or beyond
 * col_indices[capacity]; row_offsets is complete, and a retry with a larger
 * buffer is valid.  With nnz_host == NULL nothing synchronises: the rows are
 * written up to `capacity` and row_offsets[N1] tells the caller whether the
 * buffer was large enough.
 */
epm_status epm_query_candidates(epm_index* idx, const float* kp1_xy, int64_t* row_offsets,
                                int32_t* col_indices, int64_t capacity, int64_t* nnz_host,
                                hipStream_t stream);

typedef struct {
  epm_algo algo;            /* EPM_ALGO_AUTO by default                           */
  int32_t check_capacity;   /* 1: col_capacity is the length of col_indices, and
                               the launch writes no output when row_offsets[N1]
                               exceeds it (an incomplete CSR, see
                               epm_query_candidates with nnz_host == NULL)      */
  int64_t col_capacity;
  int32_t reserved[4];      /* zero                                               */
  const float* qerr1;       /* BF16 / FP8: [N1] / [N2] per-row bounds on the norm of */
  const float* qerr2;       /* x - dequant(x^) (epm_rounding_error), both or neither;
                               tighter than the format's worst case, so fewer
                               candidates need exact distances.  NULL: the
                               format's bound (valid when the codes are rounded
                               to nearest from the masters).                     */
} epm_match_opts;

/*
 * Descriptor half of the matching loop (Sec. 4.3): for each query the
 * nearest candidate and the second-nearest distance.
 *
 * row_offsets/col_indices  the CSR written by epm_query_candidates for idx.
 * dtype, dim   EPM_F32/EPM_BF16/EPM_FP8_E4M3 with dim = 128, or EPM_BIN256
 *              with dim = 256 (bits).
 * desc1, desc2 [N1][..] / [N2][..] rows in the stored format.
 * scale1/2     FP8 per-row float32 scales (dequantised value = code * scale);
 *              NULL for other types.
 * desc1_f32/desc2_f32  float32 masters [N1][128] / [N2][128]; required for
 *              BF16/FP8 (final ranking is done on them), ignored otherwise.
 * ratio        0 = off; else Lowe's tau: accept iff best < (tau*tau) * second
 *              (float, FP32 arithmetic) or best < tau * second (binary).
 * best_idx     [N1] int32: local image-2 index, or -1 (empty row / rejected).
 * best_dist, second_dist  [N1] float32: squared L2 (canonical FP32 order:
 *              t = a_k - b_k, acc = fmaf(t, t, acc), k ascending) for float
 *              types, Hamming count for binary; +inf where absent.
 *              Ties are broken by the lower image-2 index.
 * opts         may be NULL (defaults).
 *
 * On angle tiles (EPM_ALGO_AUTO / TILED after a query on idx), FP32 and BF16
 * rows of the tiles whose last query had rows of more than 128 candidates
 * are ranked on MFMA against BF16 rows with a certified FP32 re-rank; a row
 * of the given CSR that differs from the tile's candidate set is evaluated
 * exactly.  Results are the same either way.
 *
 * Errors: EPM_ERR_ARG, EPM_ERR_HIP.  Asynchronous.
 */
epm_status epm_match(const epm_index* idx, const int64_t* row_offsets,
                     const int32_t* col_indices, epm_dtype dtype, int32_t dim,
                     const void* desc1, const void* desc2, const float* scale1,
                     const float* scale2, const float* desc1_f32, const float* desc2_f32,
                     float ratio, int32_t* best_idx, float* best_dist, float* second_dist,
                     const epm_match_opts* opts, hipStream_t stream);

/*
 * Storage formats of the reduced-precision path (a helper for callers that
 * hold FP32 descriptors): src [rows][dim] float32 ->
 *   EPM_BF16:     dst [rows][dim] uint16 bfloat16 bit patterns, round to
 *                 nearest even (scale unused, may be NULL);
 *   EPM_FP8_E4M3: dst [rows][dim] uint8 OCP E4M3FN codes and scale [rows]
 *                 float32 with scale = amax / 448 (1 for an all-zero row) and
 *                 code = round-to-nearest-even(x / scale), saturated at 448.
 * 1 <= dim <= 4096.  Errors: EPM_ERR_ARG (other dtypes, bad sizes, NULL).
 * Asynchronous.
 */
epm_status epm_quantize(const float* src, int64_t rows, int32_t dim, epm_dtype dtype, void* dst,
                        float* scale, hipStream_t stream);

/*
 * Per-row rounding error of reduced-precision descriptors against their FP32
 * masters: err[r] >= |src_r - dequant(codes_r)| (computed in FP64, inflated
 * by 1e-6), for the bound of the certified re-rank (epm_match_opts.qerr1/2).
 * src [rows][dim] float32; codes as epm_quantize writes them (EPM_BF16:
 * uint16 [rows][dim]; EPM_FP8_E4M3: uint8 [rows][dim] with scale [rows]).
 * Errors: EPM_ERR_ARG.  Asynchronous.
 */
epm_status epm_rounding_error(const float* src, int64_t rows, int32_t dim, epm_dtype dtype,
                              const void* codes, const float* scale, float* err,
                              hipStream_t stream);

/*
 * The two sides of the point-line test of Eq. 3 (multiplied through by the
 * denominator) for listed (query, keypoint) pairs, exactly as the candidate
 * search evaluates them on the device:
 *   num[t] = |a x_j + b y_j + c|,  rhs[t] = eps_j * sqrt(a*a + b*b),
 * with (a, b, c) = F (x_i, y_i, 1)^T as in epm_query_candidates.
 * F is a host array [9]; kp1/kp2/eps2/qi/kj/num/rhs are device arrays
 * (qi, kj index kp1 and kp2 directly); eps2 may be NULL (eps_scalar used).
 * A diagnostic for checking the FP64 arithmetic of the device against a
 * reference; it is not needed by the matching path.  Asynchronous.
 */
epm_status epm_point_line_terms(const double* F, const float* kp1_xy, const float* kp2_xy,
                                const float* eps2, float eps_scalar, const int64_t* qi,
                                const int64_t* kj, int64_t count, double* num, double* rhs,
                                hipStream_t stream);

/*
 * Descriptor distances of listed pairs exactly as the matching kernels
 * compute them (Sec. 4.3 selection; a diagnostic for stating the error of the
 * reduced-precision paths against a reference):
 *   EPM_F32:       out[t] = the canonical FP32 squared distance (t_k = a_k - b_k,
 *                  acc = fmaf(t_k, t_k, acc), k ascending) of rows qi[t] of
 *                  desc1 and kj[t] of desc2 ([N][128] float32);
 *   EPM_BF16 / EPM_FP8_E4M3: the MFMA approximation |q^|^2 + |w^|^2 - 2 s1 s2 q^.w^
 *                  of the codes (FP8 with per-row scales scale1/scale2; the
 *                  dot product on MFMA with FP32 accumulation), rounded to float.
 * dim must be 128.  Device arrays; asynchronous.  Errors: EPM_ERR_ARG.
 */
epm_status epm_descriptor_distances(epm_dtype dtype, int32_t dim, const void* desc1,
                                    const void* desc2, const float* scale1, const float* scale2,
                                    const int64_t* qi, const int64_t* kj, int64_t count,
                                    float* out, hipStream_t stream);

/*
 * epm_query_candidates followed by epm_match with FP32 descriptors (EPM_F32,
 * dim 128, tiled path), in one pass over the candidates (Algorithm 1 matching
 * loop with the selection of Sec. 4.3): every query's hits are ranked while
 * they are still on chip, so the CSR is not read back for them.  Outputs are
 * identical to the two calls: the CSR (with the same capacity and nnz_host
 * contract as epm_query_candidates) and best_idx / best_dist / second_dist
 * (as epm_match, ratio 0 = off).  When nnz_host is NULL and the candidates
 * exceed `capacity`, the match outputs are incomplete (row_offsets[N1] tells);
 * with nnz_host, EPM_ERR_CAPACITY is returned as in epm_query_candidates.
 */
epm_status epm_query_match(epm_index* idx, const float* kp1_xy, int64_t* row_offsets,
                           int32_t* col_indices, int64_t capacity, int64_t* nnz_host,
                           const float* desc1, const float* desc2, float ratio,
                           int32_t* best_idx, float* best_dist, float* second_dist,
                           hipStream_t stream);

/*
 * epm_query_match with BF16 descriptors (Algorithm 1 matching loop, selection
 * of Sec. 4.3): desc1/desc2 are BF16 codes [N][128] (uint16 bit patterns) that
 * must be the round-to-nearest-even values of the FP32 masters
 * desc1_f32/desc2_f32 [N][128] (as epm_quantize writes them).  Every query's
 * hits are scored on MFMA against the BF16 rows of its tile's window while
 * they are still on chip; each score gives certified lower and upper bounds
 * on the exact canonical FP32 distance of the masters (the format's rounding
 * bound for the image-2 rows, the measured rounding error of the query row,
 * the FP32 accumulation bound), and only the candidates whose lower bound is
 * not above the row's second-smallest upper bound are evaluated exactly on
 * the masters.  Outputs -- the CSR with the capacity and nnz_host contract of
 * epm_query_candidates, best_idx / best_dist / second_dist -- are identical
 * to epm_query_candidates + epm_match(EPM_F32) on the masters; rows whose
 * bounds cannot be certified are matched exactly (counted by
 * epm_get_match_stats).  Errors: EPM_ERR_ARG, EPM_ERR_CAPACITY, EPM_ERR_HIP.
 */
epm_status epm_query_match_bf16(epm_index* idx, const float* kp1_xy, int64_t* row_offsets,
                                int32_t* col_indices, int64_t capacity, int64_t* nnz_host,
                                const uint16_t* desc1, const uint16_t* desc2,
                                const float* desc1_f32, const float* desc2_f32, float ratio,
                                int32_t* best_idx, float* best_dist, float* second_dist,
                                hipStream_t stream);

/*
 * epm_query_match with the image-2 descriptors stored as FP8 (Algorithm 1
 * matching loop, selection of Sec. 4.3): desc2 holds OCP E4M3FN codes
 * [N2][128] with one float32 scale per row in scale2 [N2] (dequantised value
 * = code * scale, as epm_quantize writes them), err2 [N2] a bound on the
 * norm of each row's rounding error |x - code * scale| (as epm_rounding_error
 * writes it from the masters), and desc1_f32 / desc2_f32 [N][128] the FP32
 * masters.  The queries are rounded to BF16 on chip from their masters.
 * Every query's hits are scored on MFMA against the FP8 rows of its tile's
 * window (decoded exactly to BF16) while they are on chip; each score gives
 * certified lower and upper bounds on the exact canonical FP32 distance of
 * the masters (err2 for the image-2 row, the measured rounding error of the
 * query row, the FP32 accumulation bound), and only the candidates whose
 * lower bound is not above the row's second-smallest upper bound are
 * evaluated exactly on the masters.  Outputs -- the CSR with the capacity and
 * nnz_host contract of epm_query_candidates, best_idx / best_dist /
 * second_dist -- are identical to epm_query_candidates + epm_match(EPM_F32)
 * on the masters whenever err2 bounds the rounding errors; rows whose bounds
 * cannot be certified are matched exactly (counted by epm_get_match_stats).
 * desc2, scale2, err2 and desc2_f32 may be NULL only when N2 = 0.
 * Errors: EPM_ERR_ARG, EPM_ERR_CAPACITY, EPM_ERR_HIP.
 */
epm_status epm_query_match_fp8(epm_index* idx, const float* kp1_xy, int64_t* row_offsets,
                               int32_t* col_indices, int64_t capacity, int64_t* nnz_host,
                               const uint8_t* desc2, const float* scale2, const float* err2,
                               const float* desc1_f32, const float* desc2_f32, float ratio,
                               int32_t* best_idx, float* best_dist, float* second_dist,
                               hipStream_t stream);

/*
 * Allocation-free form of epm_build_intervals followed by epm_query_match,
 * for callers that cannot allocate device memory or hand over a workspace
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Inputs and outputs are those of the two calls (pairs in host
 * memory; kp1, kp2, eps2, FP32 descriptors, CSR and match outputs in device
 * memory, owned by the caller) and the results are identical to theirs.
 *
 * Instead of a workspace the index lives in the library's own device array
 * of EPM_NOALLOC_SCRATCH_BYTES bytes, one per GPU, which exists from the
 * time the library's code is loaded on that GPU until the process ends.  A
 * batch whose index needs more (epm_workspace_bytes(pairs, num_pairs) >
 * EPM_NOALLOC_SCRATCH_BYTES) is refused with EPM_ERR_WORKSPACE before
 * anything is enqueued.  No call allocates device memory: the first call on
 * a device (with that device current) looks up the array's address and
 * creates two events, later calls reuse them.
 *
 * Every call on one GPU uses that GPU's one array, which keeps whatever the
 * last call left in it; each call rebuilds everything it reads.  Calls in
 * sequence on one stream are safe; calls that overlap on one GPU (on
 * different streams, or from threads racing each other) race and give
 * undefined results.  Host synchronisation: as epm_query_match with
 * nnz_host; besides, a call waits for the table upload of the call two
 * before it when the host runs that far ahead of the stream.
 * Errors: as epm_build_intervals and epm_query_match; EPM_ERR_UNSUPPORTED on
 * a device ordinal >= 64.
 */
#define EPM_NOALLOC_SCRATCH_BYTES (64u << 20)
epm_status epm_query_match_noalloc(const epm_pair* pairs, int32_t num_pairs, const float* kp1_xy,
                                   const float* kp2_xy, const float* eps2, float eps_scalar,
                                   int64_t* row_offsets, int32_t* col_indices, int64_t capacity,
                                   int64_t* nnz_host, const float* desc1, const float* desc2,
                                   float ratio, int32_t* best_idx, float* best_dist,
                                   float* second_dist, hipStream_t stream);

/*
 * Work distribution of the angle-tile kernels (the stabbing pass of
 * epm_query_candidates and the tiled paths of epm_match).  All zero (the
 * default of a new index) launches one workgroup per tile of 64 angle-sorted
 * queries.  A persistent launch starts `*_workgroups` workgroups that take
 * tiles from a device queue until it is empty; with lpt = 1 the queue holds
 * the tiles longest first (cost = queries x angle-window records of the
 * tile, bucketed by powers of two), which keeps batches of very uneven pairs
 * from ending on one long tile.  Results never depend on these settings.
 */
typedef struct {
  int32_t stab_workgroups;   /* 0: one per tile; > 0: persistent launch        */
  int32_t match_workgroups;  /* 0: one per tile; > 0: persistent launch        */
  int32_t lpt;               /* persistent launches: 1 = longest tiles first   */
  int32_t stab_chunk;        /* tile shape of the stabbing pass: window records
                                staged in LDS per round, 256, 512 or 1024
                                (0: 256 for the fused BF16 pass, 512 for the
                                others); larger rounds need fewer barriers,
                                smaller ones less LDS                          */
  int32_t reserved[4];       /* zero                                           */
} epm_sched;

/* Profiling aid: with start and stop not NULL, later epm_query_candidates /
 * epm_query_match calls on idx record `start` right before the stabbing-tile
 * kernel and `stop` right after it, and epm_match calls record them around
 * its matching kernel, on the call's stream, so a caller can time that kernel
 * alone with hipEventElapsedTime.  NULL, NULL turns it off.  Errors:
 * EPM_ERR_ARG (idx NULL, or only one event given). */
epm_status epm_index_set_timing_events(epm_index* idx, hipEvent_t start, hipEvent_t stop);

/* Which kernel of epm_query_candidates / epm_query_match the timing events
 * bracket: the stabbing-tile kernel (the default) or the wide-row kernel
 * that writes (and, in epm_query_match, matches) the rows with more than 128
 * candidates -- the dominant kernel at tolerances of tens of pixels.
 * Host only.  Errors: EPM_ERR_ARG (idx NULL, unknown kernel). */
typedef enum { EPM_TIMED_STAB = 0, EPM_TIMED_WIDE = 1 } epm_timed_kernel;
epm_status epm_index_set_timing_kernel(epm_index* idx, epm_timed_kernel kernel);

/* Sets the work distribution used by later calls on idx (host only).
 * Errors: EPM_ERR_ARG (NULL, negative counts, lpt not 0/1, stab_chunk not
 * 0/256/512/1024, reserved != 0). */
epm_status epm_index_set_sched(epm_index* idx, const epm_sched* sched);

/*
 * Batched execution under a HIP graph (many image pairs per launch).
 *
 * epm_batch_create builds an index over `pairs` (as epm_build_intervals), then
 * records the whole per-batch pipeline -- interval build, query sort,
 * stabbing with the FP64 test, CSR compaction and descriptor matching
 * (Algorithm 1, preprocessing and matching loop) -- for the buffers named in
 * `desc` into one HIP graph: kernels only, no host synchronisation, no
 * memset or memcpy nodes.  The interval build and the query keys with their
 * sort are two branches of the graph (they read disjoint inputs and write
 * disjoint buffers) that join before the first kernel reading the records.
 * FP32 and BF16 descriptors on the tiled path use the fused passes of
 * epm_query_match and epm_query_match_bf16.
 * epm_batch_launch replays it on a stream; every
 * replay recomputes every output from the current contents of the input
 * buffers, so new keypoints and descriptors of the same sizes can be written
 * between replays.  The slices are fixed at creation; F is too unless
 * desc->F_dev is given, in which case the graph's first node recomputes the
 * pair setup of Algorithm 1 (e2 = null(F^T), the pencil basis) on the device
 * from F_dev on every replay.  A replayed F that is non-finite, zero or of
 * rank <= 1 gets no pencil: its pair's queries are then tested against every
 * keypoint of the pair (scanned_queries counts them), so the CSR still is
 * exactly the set of Eq. 4.
 *
 * The CSR capacity cannot be checked on the host inside a graph: rows are
 * written up to `capacity` and nothing is read past it; when the total
 * exceeds it, the match outputs of that replay are incomplete and
 * epm_batch_nnz reports EPM_ERR_CAPACITY.  The buffers in `desc` and the
 * workspace must stay alive, and must not be used by other work, while the
 * batch exists.  Replays of one batch on different streams race.
 */
typedef struct {
  const float* kp1_xy;       /* [N1][2]                                              */
  const float* kp2_xy;       /* [N2][2]                                              */
  const float* eps2;         /* [N2] or NULL                                         */
  float eps_scalar;          /* used when eps2 == NULL                               */
  int64_t* row_offsets;      /* [N1 + 1] output                                      */
  int32_t* col_indices;      /* [capacity] output                                    */
  int64_t capacity;
  epm_dtype dtype;           /* matching, as in epm_match                            */
  int32_t dim;
  const void* desc1;
  const void* desc2;
  const float* scale1;
  const float* scale2;
  const float* desc1_f32;
  const float* desc2_f32;
  float ratio;
  int32_t* best_idx;         /* [N1] outputs                                         */
  float* best_dist;
  float* second_dist;
  epm_algo algo;             /* matching algorithm                                   */
  epm_sched sched;           /* work distribution of the tile kernels                */
  const double* F_dev;       /* [num_pairs][9] row-major F in device memory, or NULL:
                                when set, every replay first redoes the pair setup
                                (epipole, pencil basis) on the device from it, so new
                                F of the same pairs may be written between replays */
  const float* err2;         /* EPM_FP8_E4M3 with a tiled algorithm: [N2] bounds on the
                                image-2 rows' rounding errors, as for
                                epm_query_match_fp8; when set the graph runs that
                                fused pass (desc2 / scale2 the FP8 rows, desc1_f32 /
                                desc2_f32 the masters; desc1 and scale1 unused).
                                NULL: the separate FP8 match with the format's bound */
} epm_batch_desc;

typedef struct epm_batch epm_batch;

/* Creates the batch (host setup and one upload of its tables on `stream`;
 * the graph itself is recorded on a private stream and launches nothing).
 * workspace: at least epm_workspace_bytes(pairs, num_pairs), 256-byte
 * aligned.  Errors: as epm_build_intervals and epm_match, EPM_ERR_HIP when
 * the graph cannot be recorded.  On error *out is NULL. */
epm_status epm_batch_create(const epm_pair* pairs, int32_t num_pairs, const epm_batch_desc* desc,
                            void* workspace, size_t workspace_bytes, epm_batch** out,
                            hipStream_t stream);

/* Replays the recorded pipeline on `stream` (asynchronous). */
epm_status epm_batch_launch(epm_batch* batch, hipStream_t stream);

/* Waits for `stream` and reads the total number of candidates of the last
 * replay into *nnz; returns EPM_ERR_CAPACITY when it exceeded the capacity
 * (the match outputs of that replay are then not valid). */
epm_status epm_batch_nnz(epm_batch* batch, int64_t* nnz, hipStream_t stream);

/* The batch's index, for epm_get_query_stats / epm_get_match_stats after a
 * replay (they then read the counters of the last replay). */
const epm_index* epm_batch_index(const epm_batch* batch);

/* Releases the graph and the host objects (not the caller's buffers). */
void epm_batch_destroy(epm_batch* batch);

/*
 * Learned per-keypoint tolerance.  The candidate test (Eq. 3-4) takes one
 * tolerance per image-2 keypoint; Sec. 6 leaves predicting it from keypoint
 * attributes as future work.  These calls implement that predictor: a
 * 6 -> 64 -> 64 -> 1 ReLU network
 *     eps_j = clamp(softplus(z_j), 0.5, 8) px
 * over the features
 *     f_j = (scale, response, orientation, (x - W/2)/(W/2), (y - H/2)/(W/2),
 *            log1p(min(|p_j - e2| / diag, 1000)))
 * (W, H, diag: image-2 size and diagonal; e2: image-2 epipole, at infinity
 * giving the clipped value), trained on the device with a pinball (quantile)
 * loss of the unclamped softplus(z) against point-line residuals of matches
 * the method accepted, and Adam.  The output feeds eps2 of
 * epm_build_intervals; a fixed scalar tolerance remains the fallback.
 *
 * Parameters: EPM_EPS_NPARAM float32 values, W1 [64][6], b1 [64], W2 [64][64],
 * b2 [64], w3 [64], b3 (row-major, one row per output unit).
 */
#define EPM_EPS_NPARAM 4673

/* Workspace of epm_eps_features (num_pairs > 0) and epm_eps_grad: bytes,
 * 256-byte aligned base. */
size_t epm_eps_workspace_bytes(int32_t num_pairs);

/* features [N2][6] float32 for the image-2 keypoints of `pairs` (slices as in
 * epm_build_intervals).  attrs [N2][3] float32: scale (px), detector
 * response, orientation (rad).  Does not wait for `stream`: the per-pair
 * epipole table goes up from a library-held host image (a call waits only
 * when eight uploads of the device are still pending).  Errors: EPM_ERR_ARG,
 * EPM_ERR_DEGENERATE_F, EPM_ERR_WORKSPACE, EPM_ERR_HIP. */
epm_status epm_eps_features(const epm_pair* pairs, int32_t num_pairs, const float* kp2_xy,
                            const float* attrs, float* features, void* workspace,
                            size_t workspace_bytes, hipStream_t stream);

/* eps2[j] for n feature rows: BF16 weights (round to nearest even from
 * `params`), FP32 activations and accumulation.  Asynchronous. */
epm_status epm_eps_infer(const float* features, int64_t n, const float* params, float* eps2,
                         hipStream_t stream);

/* Gradient of the mean pinball loss (level q in (0, 1)) of softplus(z) over a
 * minibatch: sample t uses slot s = sample_idx[t], target[s] and feature row
 * feat_index[s] (or s when feat_index is NULL).  features [num_rows][6];
 * target and feat_index [num_slots].  A sample whose slot or row lies
 * outside those arrays contributes nothing (the mean still divides by
 * batch).  grad [EPM_EPS_NPARAM] and loss [1] are device outputs.  FP32,
 * deterministic: the same inputs give the same bits.  batch >= 1.
 * Asynchronous. */
epm_status epm_eps_grad(const float* features, int64_t num_rows, const int64_t* feat_index,
                        const float* target, int64_t num_slots, const int32_t* sample_idx,
                        int32_t batch, float q, const float* params, float* grad, float* loss,
                        void* workspace, size_t workspace_bytes, hipStream_t stream);

/* One Adam step (step number >= 1) on params with moments m, v (device,
 * EPM_EPS_NPARAM each; start from zeros).  Asynchronous. */
epm_status epm_eps_adam(float* params, float* m, float* v, const float* grad, int32_t step,
                        float lr, float beta1, float beta2, float eps, hipStream_t stream);

/* Residual targets: for each query with best_idx[i] in [0, n) of its pair
 * (a match of the last epm_match on idx), the point-line distance of Eq. 3 in
 * FP64 (the same evaluation as the candidate test), rounded to float32, and
 * the global image-2 row of the match in feat_index[i] (may be NULL); -1 in
 * both for other queries.  Asynchronous. */
epm_status epm_match_residuals(const epm_index* idx, const float* kp1_xy, const float* kp2_xy,
                               const int32_t* best_idx, float* residual, int64_t* feat_index,
                               hipStream_t stream);

/*
 * Per-keypoint tolerance from the uncertainty of the relative pose (the
 * noise-sensitivity setting of the paper's experiments, Sec. 5; per-keypoint
 * tolerances are its Sec. 6 future work).  For each pair the caller gives the
 * estimated pose and the covariance of theta = (w, tau) around it, with
 * R(theta) = Exp([w]x) R and t(theta) = t + tau (w in radians).  The signed
 * distance of Eq. 3, d = x2^T F(theta) x1 / |(F(theta) x1)_12| with
 * F(theta) = K2^-T [t(theta)]x R(theta) K1^-1 (Eq. 1), spreads to first order
 * by s^2 = g^T Sigma g, g = grad_theta d at the estimate.  An image-2
 * keypoint's partner lies on its reverse epipolar line F^T x2 inside image 1
 * ([0, w1] x [0, h1]).  With a scene depth range (0 < zmin < zmax, zmax may
 * be +inf; camera-2 depths) the partners considered are the image-1
 * projections K1 R^T (K2^-1 x2 - rho t) at 16 inverse depths rho evenly spaced
 * over [1/zmax, 1/zmin], those in front of camera 1 and inside image 1;
 * without one (zmin = 0), or when none of those is inside image 1, 16 evenly
 * spaced points of the segment (the line's point nearest the image centre
 * when it misses the image).  Points where (F x1)_12 vanishes are skipped.
 * The largest s over the points gives
 *     eps2[j] = min(eps0 + k_sigma * max s, eps_max)   (pixels, FP64, rounded).
 * The result feeds eps2 of epm_build_intervals, where every candidate is
 * still decided by the exact test of Eq. 3 at that tolerance.
 *
 * pairs: slices as in epm_build_intervals (F itself is taken from the
 * priors); priors: [num_pairs]; kp2_xy [N2][2]; eps2 [N2] output.  Requires
 * eps0 >= 0, k_sigma >= 0, eps_max >= eps0 finite, zmin = 0 or finite with
 * zmax > zmin.  workspace: at least
 * epm_pose_eps_workspace_bytes(num_pairs), 256-byte aligned.  Does not
 * wait for `stream` (the per-pair table goes up as in epm_eps_features).
 * Errors:
 * EPM_ERR_ARG, EPM_ERR_DEGENERATE_F (singular intrinsics, non-finite pose or
 * covariance, F = 0), EPM_ERR_WORKSPACE, EPM_ERR_HIP.
 */
typedef struct {
  double K1[9], K2[9];  /* intrinsics of the two cameras, row-major         */
  double R[9];          /* estimated relative rotation, X2 = R X1 + t (Eq. 1) */
  double t[3];          /* estimated translation                           */
  double cov[36];       /* 6 x 6 covariance of (w, tau), row-major          */
  int32_t w1, h1;       /* image-1 size                                     */
  double zmin, zmax;    /* scene depth range in camera 2 (m); zmin = 0: none */
} epm_pose_prior;

size_t epm_pose_eps_workspace_bytes(int32_t num_pairs);
epm_status epm_pose_eps(const epm_pair* pairs, const epm_pose_prior* priors, int32_t num_pairs,
                        const float* kp2_xy, float eps0, float k_sigma, float eps_max,
                        float* eps2, void* workspace, size_t workspace_bytes,
                        hipStream_t stream);

/* Counters of the last epm_query_candidates call on an index. */
typedef struct {
  int64_t queries;          /* image-1 queries                                       */
  int64_t empty_queries;    /* zero lines (a = b = 0): empty rows                     */
  int64_t scanned_queries;  /* lines missing the epipole by more than the intervals
                               absorb: tested against every keypoint of their pair   */
  int64_t records_scanned;  /* (query, record) pairs tested: the records of the angle
                               window that can meet the key span of the query's
                               group of 16 angle-sorted queries                     */
  int64_t angle_hits;       /* of those, inside the record's angular interval        */
  int64_t candidates;       /* confirmed by the FP64 test (= nnz)                     */
} epm_query_stats;

/*
 * Reads the counters of the last epm_query_candidates on idx (waits for the
 * stream that call used).  angle_hits >= candidates always holds; the ratio
 * is the selectivity of the angular filter.
 */
epm_status epm_get_query_stats(const epm_index* idx, epm_query_stats* out);

/* Counters of the last reduced-precision (BF16 / FP8) epm_match on an index. */
typedef struct {
  int64_t queries;        /* image-1 queries                                         */
  int64_t reranked_rows;  /* rows ranked on MFMA bounds with a few candidates re-ranked */
  int64_t fallback_rows;  /* of those, not certified: every candidate evaluated exactly */
  int64_t long_rows;      /* rows beyond a tile's 8192-entry list: evaluated exactly  */
  int64_t exact_distances; /* epm_query_match_bf16 / _fp8: exact FP32 distances of the re-rank */
} epm_match_stats;

/*
 * Reads the counters of the last BF16/FP8 (or FP32 on angle tiles) epm_match
 * on idx, or of the rows with more than 128 candidates of the last
 * epm_query_match on idx (ranked on MFMA with BF16 copies of the FP32 rows;
 * long_rows is then 0), and waits for the stream that call used.  fallback_rows / reranked_rows is the rate at which
 * the four re-ranked candidates could not be certified to contain the exact
 * best and second; those rows are then evaluated exactly, so results never
 * depend on it.
 */
epm_status epm_get_match_stats(const epm_index* idx, epm_match_stats* out);

/*
 * Mutual guided matching (Sec. 4.3 with the classical cross-check): the
 * caller matches image 1 against image 2 on idx (F, pairs as built) and
 * image 2 against image 1 on a second index built with the transposed
 * matrices and the roles of the images swapped (image-1 sizes, m and n
 * exchanged).  This keeps a match only when it is mutual:
 *   mutual[i] = best12[i]  if best21[k_begin + best12[i]] == i - q_begin
 *               -1         otherwise (no match, rejected, or not mutual)
 * best12 [N1] and mutual [N1] are indexed like the queries of idx; best21
 * [N2] by the global image-2 row, holding image-1 indices local to the pair
 * (as epm_match writes them on the reversed index).  Device pointers, no
 * host synchronisation.  Errors: EPM_ERR_ARG, EPM_ERR_HIP.
 */
epm_status epm_mutual_check(const epm_index* idx, const int32_t* best12, const int32_t* best21,
                            int32_t* mutual, hipStream_t stream);

/*
 * GMS validation of the matches of idx (grid-based motion statistics, the
 * filter the paper's experiments apply with the threshold set to 6; Sec. 4.3
 * cites the method).  Single-grid form: both images are cut into grid x grid
 * cells (cell of a point: floor(x grid / W), clamped); every image-1 cell's
 * motion is the image-2 cell receiving most of its matches (ties to the
 * lowest row-major index); the cell passes when the matches from its 3 x 3
 * neighbourhood to the neighbourhood of its motion (same offsets) number S
 * with S^2 * cells > alpha^2 * total, total the matches of the neighbourhood
 * cells and cells their count (cells outside a grid are left out).  A match
 * is kept when it follows its cell's motion and the cell passes.
 *
 * size1       host [P][2] int32: image-1 width and height of every pair
 *             (image-2 sizes are those given to epm_build_intervals).
 * grid        1 .. 32 (20 in GMS); alpha > 0 (6 in the paper).
 * kp1_xy, kp2_xy  the keypoints of the batch, as for the query and the index.
 * best_idx    [N1] matches (local image-2 index or -1), e.g. from epm_match.
 * out_idx     [N1] the kept matches, -1 elsewhere (may not alias best_idx).
 * workspace   caller-owned device memory of epm_gms_workspace_bytes(idx,
 *             grid) bytes, 256-byte aligned.
 * No host synchronisation (the pair table goes up as in epm_eps_features).
 * Errors: EPM_ERR_ARG, EPM_ERR_WORKSPACE, EPM_ERR_HIP.
 */
size_t epm_gms_workspace_bytes(const epm_index* idx, int32_t grid);
epm_status epm_gms(const epm_index* idx, const int32_t* size1, int32_t grid, float alpha,
                   const float* kp1_xy, const float* kp2_xy, const int32_t* best_idx,
                   int32_t* out_idx, void* workspace, size_t workspace_bytes,
                   hipStream_t stream);

/* Releases the host object; the device workspace stays owned by the caller. */
void epm_index_destroy(epm_index* idx);

/* Static, never NULL. */
const char* epm_status_string(epm_status s);

/* Library version string, static. */
const char* epm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EPM_H */
