/*
 * FP64 CPU oracle for CSR sparse x dense matrix multiplication.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this file; only the tests, the package smoke check and the CPU
 * baseline leg of the benchmark use it. It shares no code with the GPU
 * library and includes none of its headers.
 *
 * Everything here is the plain definition written out, slow and obviously
 * correct:
 *   - the product C = A*B with A m-by-k in CSR (row offsets, column
 *     indices, values) and B k-by-n dense row-major (paper, Sec. 1 and the
 *     input/output statement of Algorithm 1);
 *   - the elementwise normaliser N = |A|*|B| used to judge rounding error;
 *   - the two gradients of L = <dC, A*B>: dB = A^T dC and
 *     dvals[p] = <dC[row(p),:], B[col(p),:]>;
 *   - the CSR of A^T by a stable counting sort;
 *   - the merge-path coordinates of Sec. 4 (2-D search on the diagonals of
 *     the merge of row offsets with nonzero indices), both by a sequential
 *     walk of the merge and by binary search;
 *   - the nonzero split of Sec. 4 (equal nonzeros per piece, start row by
 *     a 1-D binary search on the row offsets);
 *   - the paper's mean-row-length heuristic of Sec. 5.4.
 *
 * Inputs arrive in their storage type (fp64, fp32, bf16 or fp16 bit
 * patterns) and are widened exactly to double. Sums run in CSR order in
 * double; no blocking or reordering.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_F64 = 0, OR_F32 = 1, OR_BF16 = 2, OR_F16 = 3 };

/* bf16 is the upper half of an IEEE binary32 pattern. */
static double or_bf16_to_double(uint16_t h) {
    uint32_t bits = ((uint32_t)h) << 16;
    float f;
    memcpy(&f, &bits, sizeof f);
    return (double)f;
}

/* IEEE 754 binary16: 1 sign bit, 5 exponent bits (bias 15), 10 fraction
 * bits; exponent 0 encodes zero/subnormals, 31 encodes inf/nan. */
static double or_f16_to_double(uint16_t h) {
    int sign = (h >> 15) & 1;
    int e = (h >> 10) & 0x1f;
    int f = h & 0x3ff;
    double v;
    if (e == 0)
        v = ldexp((double)f, -24);
    else if (e == 31)
        v = f ? NAN : INFINITY;
    else
        v = ldexp((double)(1024 + f), e - 25);
    return sign ? -v : v;
}

static double or_load(const void* base, int64_t idx, int dt) {
    switch (dt) {
    case OR_F64: return ((const double*)base)[idx];
    case OR_F32: return (double)((const float*)base)[idx];
    case OR_BF16: return or_bf16_to_double(((const uint16_t*)base)[idx]);
    case OR_F16: return or_f16_to_double(((const uint16_t*)base)[idx]);
    default: return NAN;
    }
}

double oracle_decode(const void* base, int64_t idx, int dt) { return or_load(base, idx, dt); }

static void or_set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* One output row: C[i,c] = sum_{p in row i} vals[p] * B[colind[p], c], with
 * the sum taken in CSR order. If absval, sums |vals[p]| * |B[..]| instead. */
static void or_row(int64_t i, int64_t n, const int32_t* rowptr, const int32_t* colind,
                   const void* vals, int vdt, const void* B, int bdt, int64_t ldb,
                   double* out, int absval) {
    for (int64_t c = 0; c < n; ++c) out[c] = 0.0;
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        double a = or_load(vals, p, vdt);
        int64_t r = colind[p];
        if (absval) a = fabs(a);
        for (int64_t c = 0; c < n; ++c) {
            double b = or_load(B, r * ldb + c, bdt);
            if (absval) b = fabs(b);
            out[c] += a * b;
        }
    }
}

/* C (m-by-n, row stride ldc, doubles) = A * B. Rows are independent, so the
 * result does not depend on nthreads. Returns 0, or -1 on bad arguments. */
int oracle_spmm(int64_t m, int64_t k, int64_t n, const int32_t* rowptr, const int32_t* colind,
                const void* vals, int vdt, const void* B, int bdt, int64_t ldb, double* C,
                int64_t ldc, int absval, int nthreads) {
    (void)k;
    if (m < 0 || n < 0 || ldb < n || ldc < n) return -1;
    or_set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < m; ++i)
        or_row(i, n, rowptr, colind, vals, vdt, B, bdt, ldb, C + i * ldc, absval);
    return 0;
}

/* The same product restricted to a list of rows: out[t, :] = (A*B)[rows[t], :]. */
int oracle_spmm_rows(int64_t n, const int32_t* rowptr, const int32_t* colind, const void* vals,
                     int vdt, const void* B, int bdt, int64_t ldb, const int64_t* rows,
                     int64_t nrows, double* out, int absval, int nthreads) {
    if (n < 0 || ldb < n) return -1;
    or_set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nrows; ++t)
        or_row(rows[t], n, rowptr, colind, vals, vdt, B, bdt, ldb, out + t * n, absval);
    return 0;
}

/* Product over a semiring (Sec. 1: SpMM as an instance of the GraphBLAS
 * matrix product on a semiring): C[i,c] = (+)_{p in row i} vals[p] (x)
 * B[colind[p], c], with (+, x, identity) one of
 *   0: (+, *, 0)          the ordinary product
 *   1: (min, +, +inf)     shortest-path relaxation
 *   2: (max, +, -inf)
 *   3: (max, *, -inf)
 * Rows without entries give the identity. */
int oracle_spmm_semiring(int64_t m, int64_t n, const int32_t* rowptr, const int32_t* colind,
                         const void* vals, int vdt, const void* B, int bdt, int64_t ldb,
                         double* C, int64_t ldc, int semiring) {
    if (m < 0 || n < 0 || ldb < n || ldc < n || semiring < 0 || semiring > 3) return -1;
    const double ident = semiring == 0 ? 0.0 : semiring == 1 ? INFINITY : -INFINITY;
    for (int64_t i = 0; i < m; ++i) {
        double* out = C + i * ldc;
        for (int64_t c = 0; c < n; ++c) out[c] = ident;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            double a = or_load(vals, p, vdt);
            int64_t r = colind[p];
            for (int64_t c = 0; c < n; ++c) {
                double b = or_load(B, r * ldb + c, bdt);
                switch (semiring) {
                case 0: out[c] += a * b; break;
                case 1: out[c] = fmin(out[c], a + b); break;
                case 2: out[c] = fmax(out[c], a + b); break;
                default: out[c] = fmax(out[c], a * b); break;
                }
            }
        }
    }
    return 0;
}

/* dB (k-by-n, doubles, row stride n) = A^T * dC, accumulated by scattering
 * each row of A in CSR order: dB[colind[p], :] += vals[p] * dC[i, :]. */
int oracle_spmm_t(int64_t m, int64_t k, int64_t n, const int32_t* rowptr, const int32_t* colind,
                  const void* vals, int vdt, const void* dC, int cdt, int64_t ldc, double* dB,
                  int absval) {
    if (m < 0 || k < 0 || n < 0 || ldc < n) return -1;
    for (int64_t t = 0; t < k * n; ++t) dB[t] = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            double a = or_load(vals, p, vdt);
            if (absval) a = fabs(a);
            double* dst = dB + (int64_t)colind[p] * n;
            for (int64_t c = 0; c < n; ++c) {
                double g = or_load(dC, i * ldc + c, cdt);
                if (absval) g = fabs(g);
                dst[c] += a * g;
            }
        }
    }
    return 0;
}

/* dvals[p] = sum_c dC[row(p), c] * B[colind[p], c]: the gradient of
 * <dC, A*B> with respect to the stored values of A (sampled dense-dense
 * product on A's pattern). */
int oracle_sddmm(int64_t m, int64_t n, const int32_t* rowptr, const int32_t* colind,
                 const void* dC, int cdt, int64_t ldc, const void* B, int bdt, int64_t ldb,
                 double* dvals, int absval, int nthreads) {
    if (m < 0 || n < 0 || ldc < n || ldb < n) return -1;
    or_set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int64_t r = colind[p];
            double s = 0.0;
            for (int64_t c = 0; c < n; ++c) {
                double g = or_load(dC, i * ldc + c, cdt);
                double b = or_load(B, r * ldb + c, bdt);
                if (absval) { g = fabs(g); b = fabs(b); }
                s += g * b;
            }
            dvals[p] = s;
        }
    }
    return 0;
}

/* CSR of A^T by a stable counting sort over column indices. Row j of A^T
 * lists the rows i of A with a nonzero in column j, in increasing i (CSR
 * order of A), and perm[q] is the position in A's arrays of A^T's q-th
 * nonzero, so that AT_vals[q] = vals[perm[q]]. */
int oracle_transpose(int64_t m, int64_t k, const int32_t* rowptr, const int32_t* colind,
                     int32_t* at_rowptr, int32_t* at_colind, int32_t* perm) {
    if (m < 0 || k < 0) return -1;
    int64_t nnz = rowptr[m];
    int64_t* cursor = (int64_t*)calloc((size_t)k + 1, sizeof(int64_t));
    if (!cursor) return -2;
    for (int64_t p = 0; p < nnz; ++p) {
        int64_t c = colind[p];
        if (c < 0 || c >= k) { free(cursor); return -1; }
        cursor[c + 1]++;
    }
    for (int64_t c = 0; c < k; ++c) cursor[c + 1] += cursor[c];
    for (int64_t c = 0; c <= k; ++c) at_rowptr[c] = (int32_t)cursor[c];
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int64_t q = cursor[colind[p]]++;
            at_colind[q] = (int32_t)i;
            perm[q] = (int32_t)p;
        }
    }
    free(cursor);
    return 0;
}

/* ---- merge-path coordinates (Sec. 4, merge path of Merrill and Garland) ----
 *
 * The two sorted lists being merged are the row ends a[i] = rowptr[i+1]
 * (i < m) and the nonzero indices b[j] = j (j < nnz). At merge state (i, j)
 * the next item is the end of row i when i < m and (j == nnz or a[i] <= j),
 * otherwise nonzero j, which belongs to row i. Ties therefore go to the row
 * end, which lets empty rows finish before any nonzero of a later row. The
 * coordinate of diagonal d is the state reached after d items.
 */

/* Every coordinate of the merge, by walking it one item at a time:
 * coords[2d] = i, coords[2d+1] = j for d = 0 .. m + nnz. */
int oracle_merge_walk(int64_t m, const int32_t* rowptr, int32_t* coords) {
    if (m < 0) return -1;
    int64_t nnz = rowptr[m];
    int64_t i = 0, j = 0;
    for (int64_t d = 0; d <= m + nnz; ++d) {
        coords[2 * d] = (int32_t)i;
        coords[2 * d + 1] = (int32_t)j;
        if (d == m + nnz) break;
        if (i < m && (j == nnz || rowptr[i + 1] <= j))
            ++i;
        else
            ++j;
    }
    return 0;
}

/* The coordinate of one diagonal by binary search: i is the number of row
 * ends among the first d merged items. Row end x precedes exactly
 * min(a[x], nnz) = a[x] nonzeros, so it is among the first d items iff
 * x + a[x] < d; that predicate is monotone in x, and i counts the x for
 * which it holds within the feasible range [max(0, d - nnz), min(d, m)]. */
int oracle_merge_search(int64_t m, const int32_t* rowptr, int64_t d, int64_t* i_out,
                        int64_t* j_out) {
    int64_t nnz = rowptr[m];
    if (d < 0 || d > m + nnz) return -1;
    int64_t lo = d - nnz > 0 ? d - nnz : 0;
    int64_t hi = d < m ? d : m;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if ((int64_t)rowptr[mid + 1] + mid < d)
            lo = mid + 1;
        else
            hi = mid;
    }
    *i_out = lo;
    *j_out = d - lo;
    return 0;
}

/* Partition of the merge into pieces of W items: diagonals
 * d_p = min(p * W, m + nnz) for p = 0 .. P, P = ceil((m + nnz) / W)
 * (P = 0 when m + nnz = 0, leaving the single coordinate (0, 0)). */
int64_t oracle_merge_num_parts(int64_t m, int64_t nnz, int64_t W) {
    if (W <= 0) return -1;
    return (m + nnz + W - 1) / W;
}

int oracle_merge_partition(int64_t m, const int32_t* rowptr, int64_t W, int32_t* coords) {
    if (m < 0 || W <= 0) return -1;
    int64_t nnz = rowptr[m];
    int64_t P = oracle_merge_num_parts(m, nnz, W);
    for (int64_t p = 0; p <= P; ++p) {
        int64_t d = p * W < m + nnz ? p * W : m + nnz;
        int64_t i, j;
        oracle_merge_search(m, rowptr, d, &i, &j);
        coords[2 * p] = (int32_t)i;
        coords[2 * p + 1] = (int32_t)j;
    }
    return 0;
}

/* ---- nonzero split (Sec. 4, item (a) of the load-balancing schemes) ----
 *
 * Every piece gets the same number W of nonzeros: piece p starts at
 * nonzero j_p = min(p * W, nnz), and a 1-D binary search on the row offsets
 * finds the row it starts in, i.e. the row holding nonzero j_p. Expressed as
 * a state of the merge above, piece p starts at (i_p, j_p) with i_p the
 * number of rows whose end rowptr[i+1] is <= j_p (those rows, empty ones
 * included, are finished before nonzero j_p is taken). The first piece
 * starts at (0, 0) so that it also finishes the leading empty rows, and the
 * last piece ends at (m, nnz). P = ceil(nnz / W), at least 1 when m > 0
 * (a matrix without nonzeros is one piece of empty rows); P = 0 when m = 0.
 */
int64_t oracle_nz_num_parts(int64_t m, int64_t nnz, int64_t W) {
    if (W <= 0) return -1;
    if (m == 0) return 0;
    int64_t P = (nnz + W - 1) / W;
    return P > 0 ? P : 1;
}

/* Number of rows whose end is <= j: the 1-D binary search on row offsets. */
static int64_t or_rows_ended_by(int64_t m, const int32_t* rowptr, int64_t j) {
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if ((int64_t)rowptr[mid + 1] <= j)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

int oracle_nz_partition(int64_t m, const int32_t* rowptr, int64_t W, int32_t* coords) {
    if (m < 0 || W <= 0) return -1;
    int64_t nnz = rowptr[m];
    int64_t P = oracle_nz_num_parts(m, nnz, W);
    coords[0] = 0;
    coords[1] = 0;
    for (int64_t p = 1; p <= P; ++p) {
        int64_t j = p * W < nnz ? p * W : nnz;
        coords[2 * p] = (int32_t)(p == P ? m : or_rows_ended_by(m, rowptr, j));
        coords[2 * p + 1] = (int32_t)j;
    }
    return 0;
}

/* Sec. 5.4: with d the mean row length nnz / m, use the merge-based kernel
 * when d < 9.35 and row splitting otherwise. Returns 1 for merge-based,
 * 0 for row split (also for m == 0, where there is nothing to do). */
int oracle_heuristic_merge(int64_t m, int64_t nnz) {
    if (m <= 0) return 0;
    double d = (double)nnz / (double)m;
    return d < 9.35 ? 1 : 0;
}
