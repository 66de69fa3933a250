/*
 * CPU oracle for exact epipolar-guided matching -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is a plain, slow, obviously correct restatement of what the
 * matching path computes.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code, header or
 * constant with the GPU library.
 *
 * Built with -O2 -ffp-contract=off: every floating-point operation below is
 * one IEEE-754 correctly rounded operation, evaluated left to right exactly
 * as written.
 *
 * Paper: Nasypanyi & Rameau, "Pixel-Accurate Epipolar Guided Matching".
 *   - Section 3, Eq. 2: epipolar line l_i = F p~_i.
 *   - Section 3, Eq. 3: point-line distance |a x + b y + c| / sqrt(a^2+b^2).
 *   - Section 3, Eq. 4: candidate set = { j : dist(l_i, p_j) <= eps }.
 *   - Section 4.3: descriptor comparison restricted to the candidate set,
 *     nearest neighbour, optional Lowe ratio test.
 *
 * Readings where the paper is silent (each one is listed with its reason in
 * the design notes of the repository):
 *   - eps belongs to the image-2 keypoint (per-keypoint tolerance, Sec. 4.2
 *     and Sec. 6); a scalar eps means all eps_j are equal.
 *   - The boundary is closed (Eq. 3 uses <=).  The comparison is Eq. 3
 *     multiplied through by the positive denominator:
 *         |a x_j + b y_j + c| <= eps_j * sqrt(a*a + b*b)
 *     with a = (F0*x + F1*y) + F2 etc., FP64, no contraction, IEEE sqrt.
 *   - A query whose line has a = b = 0 (the query sits on the image-1
 *     epipole, or the line is the line at infinity) has no well-defined
 *     distance: its candidate set is empty and it is flagged degenerate.
 *   - Float descriptors: squared L2 in a canonical FP32 order,
 *         t_k = a_k - b_k;  acc = fmaf(t_k, t_k, acc), k = 0..D-1, acc0 = +0.
 *   - Binary descriptors: Hamming distance = sum of popcount(a_w ^ b_w).
 *   - Selection: candidates ordered by (distance, j); best is the first,
 *     second the next.  Empty row: best = -1, both distances +inf.
 *     Singleton row: second = +inf.
 *   - Ratio test with tau > 0 (float): accept iff best < (tau*tau) * second,
 *     all in FP32; (binary): accept iff (float)best < tau * (float)second.
 *     A rejection sets best_idx = -1 and keeps both distances.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------ */
/* A minimal parallel-for over [0, count): contiguous chunks per thread. */

typedef void (*range_fn)(void* ctx, int64_t begin, int64_t end);

typedef struct {
    range_fn fn;
    void* ctx;
    int64_t begin, end;
} chunk_t;

static void* run_chunk(void* p) {
    chunk_t* c = (chunk_t*)p;
    c->fn(c->ctx, c->begin, c->end);
    return NULL;
}

int oracle_default_threads(void) {
    long n = sysconf(_SC_NPROCESSORS_ONLN);
    return n > 0 ? (int)n : 1;
}

static void parallel_for(int64_t count, int nthreads, range_fn fn, void* ctx) {
    if (nthreads <= 0) nthreads = oracle_default_threads();
    if (nthreads > 256) nthreads = 256;
    if (count < (int64_t)nthreads * 4 || nthreads == 1) {
        fn(ctx, 0, count);
        return;
    }
    pthread_t th[256];
    chunk_t ch[256];
    int64_t step = (count + nthreads - 1) / nthreads;
    int used = 0;
    for (int t = 0; t < nthreads; ++t) {
        int64_t b = (int64_t)t * step, e = b + step;
        if (b >= count) break;
        if (e > count) e = count;
        ch[t].fn = fn;
        ch[t].ctx = ctx;
        ch[t].begin = b;
        ch[t].end = e;
        pthread_create(&th[t], NULL, run_chunk, &ch[t]);
        ++used;
    }
    for (int t = 0; t < used; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------ */
/* Eq. 2: l = F (x, y, 1)^T, each component evaluated left to right.    */

static void epipolar_line(const double F[9], double x, double y, double* a, double* b,
                          double* c) {
    *a = F[0] * x + F[1] * y + F[2];
    *b = F[3] * x + F[4] * y + F[5];
    *c = F[6] * x + F[7] * y + F[8];
}

/* Eq. 3-4, multiplied through by sqrt(a^2 + b^2) > 0; closed boundary. */
static int is_candidate(double a, double b, double c, double x, double y, double eps) {
    double num = fabs(a * x + b * y + c);
    double rhs = eps * sqrt(a * a + b * b);
    return num <= rhs;
}

typedef struct {
    const double* F;
    const float* kp1;
    const float* kp2;
    int64_t n;
    const float* eps2;
    float eps_scalar;
    int64_t* counts;       /* pass 1 */
    const int64_t* offs;   /* pass 2 */
    int32_t* cols;         /* pass 2 */
    uint8_t* degenerate;
} cand_ctx;

static double eps_of(const cand_ctx* c, int64_t j) {
    return (double)(c->eps2 ? c->eps2[j] : c->eps_scalar);
}

static void cand_count(void* p, int64_t i0, int64_t i1) {
    cand_ctx* c = (cand_ctx*)p;
    for (int64_t i = i0; i < i1; ++i) {
        double a, b, cc;
        epipolar_line(c->F, (double)c->kp1[2 * i], (double)c->kp1[2 * i + 1], &a, &b, &cc);
        int64_t k = 0;
        int degen = (a == 0.0 && b == 0.0);
        if (!degen) {
            for (int64_t j = 0; j < c->n; ++j)
                k += is_candidate(a, b, cc, (double)c->kp2[2 * j], (double)c->kp2[2 * j + 1],
                                  eps_of(c, j));
        }
        c->counts[i] = k;
        if (c->degenerate) c->degenerate[i] = (uint8_t)degen;
    }
}

static void cand_fill(void* p, int64_t i0, int64_t i1) {
    cand_ctx* c = (cand_ctx*)p;
    for (int64_t i = i0; i < i1; ++i) {
        double a, b, cc;
        epipolar_line(c->F, (double)c->kp1[2 * i], (double)c->kp1[2 * i + 1], &a, &b, &cc);
        if (a == 0.0 && b == 0.0) continue;
        int64_t o = c->offs[i];
        for (int64_t j = 0; j < c->n; ++j)
            if (is_candidate(a, b, cc, (double)c->kp2[2 * j], (double)c->kp2[2 * j + 1],
                             eps_of(c, j)))
                c->cols[o++] = (int32_t)j;
    }
}

/*
 * Brute-force candidate sets (Eq. 4) for one image pair as CSR, rows in
 * ascending j.  If the total exceeds `capacity`, nothing is written to
 * col_indices, *nnz receives the required size and 1 is returned.
 */
int oracle_candidates(const double F[9], const float* kp1, int64_t m, const float* kp2,
                      int64_t n, const float* eps2, float eps_scalar, int64_t* row_offsets,
                      int32_t* col_indices, int64_t capacity, int64_t* nnz,
                      uint8_t* degenerate, int nthreads) {
    int64_t* counts = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    cand_ctx c = {F, kp1, kp2, n, eps2, eps_scalar, counts, NULL, NULL, degenerate};
    parallel_for(m, nthreads, cand_count, &c);
    row_offsets[0] = 0;
    for (int64_t i = 0; i < m; ++i) row_offsets[i + 1] = row_offsets[i] + counts[i];
    free(counts);
    *nnz = row_offsets[m];
    if (*nnz > capacity) return 1;
    c.offs = row_offsets;
    c.cols = col_indices;
    parallel_for(m, nthreads, cand_fill, &c);
    return 0;
}

/* Eq. 3 distances for listed (i, j) pairs, FP64 (for boundary-band reports). */
void oracle_point_line_dist(const double F[9], const float* kp1, const float* kp2,
                            const int64_t* qi, const int64_t* kj, int64_t count, double* out) {
    for (int64_t t = 0; t < count; ++t) {
        double a, b, c;
        int64_t i = qi[t], j = kj[t];
        epipolar_line(F, (double)kp1[2 * i], (double)kp1[2 * i + 1], &a, &b, &c);
        double num = fabs(a * (double)kp2[2 * j] + b * (double)kp2[2 * j + 1] + c);
        out[t] = num / sqrt(a * a + b * b);
    }
}

/* Both sides of the Eq. 3 comparison for listed (i, j) pairs. */
void oracle_candidate_terms(const double F[9], const float* kp1, const float* kp2,
                            const float* eps2, float eps_scalar, const int64_t* qi,
                            const int64_t* kj, int64_t count, double* num, double* rhs) {
    for (int64_t t = 0; t < count; ++t) {
        double a, b, c;
        int64_t i = qi[t], j = kj[t];
        double eps = (double)(eps2 ? eps2[j] : eps_scalar);
        epipolar_line(F, (double)kp1[2 * i], (double)kp1[2 * i + 1], &a, &b, &c);
        num[t] = fabs(a * (double)kp2[2 * j] + b * (double)kp2[2 * j + 1] + c);
        rhs[t] = eps * sqrt(a * a + b * b);
    }
}

/* ------------------------------------------------------------------ */
/* Descriptor distances.                                               */

float oracle_desc_dist_f32(const float* a, const float* b, int dim) {
    float acc = 0.0f;
    for (int k = 0; k < dim; ++k) {
        float t = a[k] - b[k];
        acc = fmaf(t, t, acc);
    }
    return acc;
}

double oracle_desc_dist_f64(const float* a, const float* b, int dim) {
    double acc = 0.0;
    for (int k = 0; k < dim; ++k) {
        double t = (double)a[k] - (double)b[k];
        acc += t * t;
    }
    return acc;
}

static uint32_t popcount32(uint32_t v) {
    uint32_t c = 0;
    while (v) {
        c += v & 1u;
        v >>= 1;
    }
    return c;
}

uint32_t oracle_hamming(const uint32_t* a, const uint32_t* b, int words) {
    uint32_t h = 0;
    for (int w = 0; w < words; ++w) h += popcount32(a[w] ^ b[w]);
    return h;
}

typedef struct {
    float d;
    int32_t j;
} cand_t;

static int cmp_cand(const void* x, const void* y) {
    const cand_t* p = (const cand_t*)x;
    const cand_t* q = (const cand_t*)y;
    if (p->d < q->d) return -1;
    if (p->d > q->d) return 1;
    return (p->j > q->j) - (p->j < q->j);
}

typedef struct {
    int binary;
    const void* d1;
    const void* d2;
    int dim; /* floats, or u32 words */
    const int64_t* offs;
    const int32_t* cols;
    const int64_t* col_base; /* optional per-row offset added to col (batched pairs) */
    const int64_t* row_base1; /* optional: desc1 row of query i (default i) */
    float ratio;
    int32_t* best_idx;
    float* best_d;
    float* second_d;
} match_ctx;

static void match_rows(void* p, int64_t i0, int64_t i1) {
    match_ctx* c = (match_ctx*)p;
    cand_t* buf = NULL;
    int64_t cap = 0;
    for (int64_t i = i0; i < i1; ++i) {
        int64_t b = c->offs[i], e = c->offs[i + 1], k = e - b;
        if (k > cap) {
            cap = k;
            buf = (cand_t*)realloc(buf, sizeof(cand_t) * (size_t)cap);
        }
        int64_t qi = c->row_base1 ? c->row_base1[i] : i;
        int64_t base = c->col_base ? c->col_base[i] : 0;
        for (int64_t t = 0; t < k; ++t) {
            int64_t j = base + c->cols[b + t];
            float d;
            if (c->binary) {
                const uint32_t* A = (const uint32_t*)c->d1 + qi * c->dim;
                const uint32_t* B = (const uint32_t*)c->d2 + j * c->dim;
                d = (float)oracle_hamming(A, B, c->dim);
            } else {
                const float* A = (const float*)c->d1 + qi * c->dim;
                const float* B = (const float*)c->d2 + j * c->dim;
                d = oracle_desc_dist_f32(A, B, c->dim);
            }
            buf[t].d = d;
            buf[t].j = c->cols[b + t];
        }
        qsort(buf, (size_t)k, sizeof(cand_t), cmp_cand);
        int32_t bi = k > 0 ? buf[0].j : -1;
        float bd = k > 0 ? buf[0].d : INFINITY;
        float sd = k > 1 ? buf[1].d : INFINITY;
        if (c->ratio > 0.0f && bi >= 0) {
            int accept;
            if (c->binary) {
                accept = bd < c->ratio * sd;
            } else {
                float thr = c->ratio * c->ratio;
                accept = bd < thr * sd;
            }
            if (!accept) bi = -1;
        }
        c->best_idx[i] = bi;
        c->best_d[i] = bd;
        c->second_d[i] = sd;
    }
    free(buf);
}

/*
 * Nearest neighbour over each candidate row (Section 4.3).  Float rows use
 * the canonical FP32 squared distance; binary rows (binary != 0) the Hamming
 * distance over `dim` u32 words.  col_base/row_base1 may be NULL.
 */
void oracle_match(int binary, const void* desc1, const void* desc2, int dim,
                  const int64_t* row_offsets, const int32_t* col_indices,
                  const int64_t* col_base, const int64_t* row_base1, int64_t m, float ratio,
                  int32_t* best_idx, float* best_d, float* second_d, int nthreads) {
    match_ctx c = {binary, desc1, desc2, dim, row_offsets, col_indices, col_base, row_base1,
                   ratio, best_idx, best_d, second_d};
    parallel_for(m, nthreads, match_rows, &c);
}

/* FP64 squared distances for listed (i, j) pairs, for error reports. */
void oracle_desc_dist_f64_pairs(const float* desc1, const float* desc2, int dim,
                                const int64_t* qi, const int64_t* kj, int64_t count,
                                double* out) {
    for (int64_t t = 0; t < count; ++t)
        out[t] = oracle_desc_dist_f64(desc1 + qi[t] * dim, desc2 + kj[t] * dim, dim);
}
