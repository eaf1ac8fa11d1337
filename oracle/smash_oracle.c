/*
 * smash_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU reference for the sparse product
 * C = A * B on CSR operands.  It exists so that tests, the smoke check and the
 * benchmark's CPU-baseline leg can check and time the GPU library against an
 * independent implementation.  It shares no code, header, table or helper
 * with the GPU library and must never be linked into it.
 *
 * What it computes (Background chapter, eq. "inner_product"): every output
 * entry is c_ij = sum_k a_ik * b_kj.  It is evaluated in the row-wise
 * (Gustavson) order of eq. "row_wise", C[i,:] = sum_k A[i,k] * B[k,:]: for
 * each stored a_ik, in storage order, the whole row k of B is scaled and
 * merged into a dense accumulator indexed by column ("sparse accumulator",
 * Gustavson 1978).  That is the definition written out; nothing is blocked,
 * fused or reordered.
 *
 * Readings taken where the paper is silent:
 *   - the structure of C is the structural product {(i,j) : some k has a_ik
 *     and b_kj stored}; entries whose products cancel to 0.0 are kept;
 *   - output columns are ascending and unique within a row;
 *   - sums are accumulated in long double (x87 80-bit on x86-64), in
 *     ascending k then ascending j order, and rounded to double once, so the
 *     oracle's own rounding error is negligible next to FP32/FP64 tolerances;
 *   - for every entry the oracle also reports absmass = sum |a_ik * b_kj|
 *     and the term count m = #{k : a_ik and b_kj stored}; tolerances are
 *     stated relative to absmass.
 *
 * Inputs are int32 CSR with double values (FP32 inputs are widened exactly by
 * the caller; the product of two widened FP32 values is exact in double).
 * Preconditions checked by oracle_validate(): row_ptr[0] = 0, row_ptr
 * nondecreasing, 0 <= col < cols, columns strictly ascending in each row.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct {
    int64_t rows, cols;
    const int32_t *rp, *ci;
    const double *v;
} ocsr;

/* ------------------------------------------------------------ validation */

/* 0 = valid; 1 = row_ptr[0] != 0; 2 = row_ptr decreasing; 3 = column out of
 * range; 4 = columns not strictly ascending in a row; 5 = negative size. */
int oracle_validate(int64_t rows, int64_t cols, const int32_t *rp, const int32_t *ci)
{
    if (rows < 0 || cols < 0) return 5;
    if (rp[0] != 0) return 1;
    for (int64_t i = 0; i < rows; ++i) {
        if (rp[i + 1] < rp[i]) return 2;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] < 0 || ci[p] >= cols) return 3;
            if (p > rp[i] && ci[p] <= ci[p - 1]) return 4;
        }
    }
    return 0;
}

/* -------------------------------------------------- per-thread accumulator */

typedef struct {
    long double *sum;   /* running sum per column                         */
    double *absm;       /* running sum of |product| per column            */
    int64_t *terms;     /* number of products merged per column           */
    int64_t *stamp;     /* visit number of the last row that touched column */
    int64_t visit;      /* rows merged so far by this accumulator         */
    int32_t *touched;   /* columns touched by the current row             */
} spa;

static int spa_init(spa *s, int64_t n)
{
    size_t nn = (size_t)(n > 0 ? n : 1);
    s->sum = (long double *)malloc(nn * sizeof(long double));
    s->absm = (double *)malloc(nn * sizeof(double));
    s->terms = (int64_t *)malloc(nn * sizeof(int64_t));
    s->stamp = (int64_t *)calloc(nn, sizeof(int64_t));
    s->touched = (int32_t *)malloc(nn * sizeof(int32_t));
    s->visit = 0;
    return s->sum && s->absm && s->terms && s->stamp && s->touched;
}

static void spa_free(spa *s)
{
    free(s->sum); free(s->absm); free(s->terms); free(s->stamp); free(s->touched);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Merge row i of C = A*B into the accumulator; returns the number of
 * distinct columns and leaves them, ascending, in s->touched. */
static int64_t spa_row(spa *s, const ocsr *A, const ocsr *B, int64_t i, int with_values)
{
    int64_t cnt = 0;
    const int64_t mark = ++s->visit;   /* fresh for every row merged, even a repeated one */
    for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) {
        const int64_t k = A->ci[p];
        const double a = with_values ? A->v[p] : 0.0;
        for (int64_t q = B->rp[k]; q < B->rp[k + 1]; ++q) {
            const int32_t j = B->ci[q];
            if (s->stamp[j] != mark) {
                s->stamp[j] = mark;
                s->touched[cnt++] = j;
                s->sum[j] = 0.0L;
                s->absm[j] = 0.0;
                s->terms[j] = 0;
            }
            if (with_values) {
                const double prod = a * B->v[q];
                s->sum[j] += (long double)prod;
                s->absm[j] += fabs(prod);
            }
            s->terms[j] += 1;
        }
    }
    qsort(s->touched, (size_t)cnt, sizeof(int32_t), cmp_i32);
    return cnt;
}

/* ------------------------------------------------------------- threading */

typedef struct {
    const ocsr *A, *B;
    const int64_t *sel;       /* selected rows, or NULL for 0..nsel-1      */
    int64_t nsel;
    int64_t next;             /* shared dynamic row counter                */
    int mode;                 /* 0 = count, 1 = fill                       */
    int64_t *nnz_out;         /* mode 0: per selected row                  */
    const int64_t *off;       /* mode 1: output offset per selected row    */
    int32_t *col_out;
    double *val_out, *abs_out;
    int64_t *terms_out;
    int failed;
} job;

static void *worker(void *arg)
{
    job *J = (job *)arg;
    spa s;
    if (!spa_init(&s, J->B->cols)) {
        __atomic_store_n(&J->failed, 1, __ATOMIC_SEQ_CST);
        spa_free(&s);
        return NULL;
    }
    const int64_t block = 16;
    for (;;) {
        int64_t r0 = __atomic_fetch_add(&J->next, block, __ATOMIC_RELAXED);
        if (r0 >= J->nsel) break;
        int64_t r1 = r0 + block < J->nsel ? r0 + block : J->nsel;
        for (int64_t r = r0; r < r1; ++r) {
            int64_t i = J->sel ? J->sel[r] : r;
            int64_t cnt = spa_row(&s, J->A, J->B, i, J->mode == 1);
            if (J->mode == 0) {
                J->nnz_out[r] = cnt;
            } else {
                int64_t o = J->off[r];
                for (int64_t t = 0; t < cnt; ++t) {
                    int32_t j = s.touched[t];
                    J->col_out[o + t] = j;
                    J->val_out[o + t] = (double)s.sum[j];
                    if (J->abs_out) J->abs_out[o + t] = s.absm[j];
                    if (J->terms_out) J->terms_out[o + t] = s.terms[j];
                }
            }
        }
    }
    spa_free(&s);
    return NULL;
}

static int run_job(job *J, int threads)
{
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t tid[256];
    int started = 0;
    for (int t = 1; t < threads; ++t) {
        if (pthread_create(&tid[t], NULL, worker, J) != 0) break;
        ++started;
    }
    worker(J);
    for (int t = 1; t <= started; ++t) pthread_join(tid[t], NULL);
    return J->failed ? -1 : 0;
}

/* Number of distinct columns of each selected row of A*B.
 * sel == NULL selects rows 0..nsel-1.  Returns 0, or -1 on allocation failure. */
int oracle_row_nnz(int64_t a_rows, int64_t a_cols, const int32_t *a_rp, const int32_t *a_ci,
                   int64_t b_rows, int64_t b_cols, const int32_t *b_rp, const int32_t *b_ci,
                   const int64_t *sel, int64_t nsel, int64_t *nnz_out, int threads)
{
    ocsr A = {a_rows, a_cols, a_rp, a_ci, NULL};
    ocsr B = {b_rows, b_cols, b_rp, b_ci, NULL};
    job J;
    memset(&J, 0, sizeof J);
    J.A = &A; J.B = &B; J.sel = sel; J.nsel = nsel; J.mode = 0; J.nnz_out = nnz_out;
    return run_job(&J, threads);
}

/* Columns, values, absmass and term counts of each selected row of A*B.
 * Row r of the selection is written at [off[r], off[r] + nnz_r) of the
 * output arrays, which the caller sizes from oracle_row_nnz.  abs_out and
 * terms_out may be NULL.  Returns 0, or -1 on allocation failure. */
int oracle_fill(int64_t a_rows, int64_t a_cols, const int32_t *a_rp, const int32_t *a_ci, const double *a_v,
                int64_t b_rows, int64_t b_cols, const int32_t *b_rp, const int32_t *b_ci, const double *b_v,
                const int64_t *sel, int64_t nsel, const int64_t *off,
                int32_t *col_out, double *val_out, double *abs_out, int64_t *terms_out, int threads)
{
    ocsr A = {a_rows, a_cols, a_rp, a_ci, a_v};
    ocsr B = {b_rows, b_cols, b_rp, b_ci, b_v};
    job J;
    memset(&J, 0, sizeof J);
    J.A = &A; J.B = &B; J.sel = sel; J.nsel = nsel; J.mode = 1; J.off = off;
    J.col_out = col_out; J.val_out = val_out; J.abs_out = abs_out; J.terms_out = terms_out;
    return run_job(&J, threads);
}
