/* Threaded CSR sparse matrix-vector product y = A u in FP64 (OpenMP): the
 * matrix-based operator application the paper compares the matrix-free
 * evaluation against (Sec. 3.2), timed on the host's cores as the CPU
 * baseline.  TEST INFRASTRUCTURE ONLY, like the rest of oracle/: only the
 * tests and the CPU-baseline leg of the benchmark load it.
 *
 * y_i = sum over the stored entries (i, j) of row i, in storage order, of
 * a_ij u_j.  Rows are split into equal contiguous ranges, one per thread;
 * every row is summed by one thread in storage order, so the result does not
 * depend on the thread count.  The matrix and the vectors are copied into
 * buffers that each thread first touches for its own rows (the pages then
 * sit on the memory node of the thread that reads them).
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t n, nnz;
  int64_t* ptr;  /* [n + 1] */
  int32_t* col;  /* [nnz] */
  double* val;   /* [nnz] */
  double* u;     /* [n] */
  double* y;     /* [n] */
} spmv_t;

static void row_range(int64_t n, int t, int nt, int64_t* lo, int64_t* hi) {
  *lo = n * t / nt;
  *hi = n * (t + 1) / nt;
}

static void product(spmv_t* m) {
#pragma omp parallel
  {
    int64_t lo, hi;
    row_range(m->n, omp_get_thread_num(), omp_get_num_threads(), &lo, &hi);
    for (int64_t i = lo; i < hi; ++i) {
      double s = 0.0;
      for (int64_t k = m->ptr[i]; k < m->ptr[i + 1]; ++k) s += m->val[k] * m->u[m->col[k]];
      m->y[i] = s;
    }
  }
}

/* Square matrix of n rows in CSR form (host arrays, copied) and the input
 * vector u.  Returns NULL when a buffer cannot be allocated. */
void* spmv_create(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, const double* u) {
  spmv_t* m = (spmv_t*)calloc(1, sizeof(spmv_t));
  if (!m) return NULL;
  m->n = n;
  m->nnz = ptr[n];
  m->ptr = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
  m->col = (int32_t*)malloc((size_t)(m->nnz > 0 ? m->nnz : 1) * sizeof(int32_t));
  m->val = (double*)malloc((size_t)(m->nnz > 0 ? m->nnz : 1) * sizeof(double));
  m->u = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  m->y = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  if (!m->ptr || !m->col || !m->val || !m->u || !m->y) {
    free(m->ptr), free(m->col), free(m->val), free(m->u), free(m->y), free(m);
    return NULL;
  }
  m->ptr[n] = ptr[n];
#pragma omp parallel
  {
    int64_t lo, hi;
    row_range(n, omp_get_thread_num(), omp_get_num_threads(), &lo, &hi);
    for (int64_t i = lo; i < hi; ++i) {
      m->ptr[i] = ptr[i];
      m->u[i] = u[i];
      m->y[i] = 0.0;
    }
    if (hi > lo) {
      memcpy(m->col + ptr[lo], col + ptr[lo], (size_t)(ptr[hi] - ptr[lo]) * sizeof(int32_t));
      memcpy(m->val + ptr[lo], val + ptr[lo], (size_t)(ptr[hi] - ptr[lo]) * sizeof(double));
    }
  }
  return m;
}

void spmv_destroy(void* h) {
  spmv_t* m = (spmv_t*)h;
  if (!m) return;
  free(m->ptr), free(m->col), free(m->val), free(m->u), free(m->y), free(m);
}

/* One product; y_out (host [n]) receives A u. */
void spmv_apply(void* h, double* y_out) {
  spmv_t* m = (spmv_t*)h;
  product(m);
  memcpy(y_out, m->y, (size_t)m->n * sizeof(double));
}

/* `warmup` untimed products, then `runs` timed ones; seconds[k] is the wall
 * time of product k. */
void spmv_time(void* h, int warmup, int runs, double* seconds) {
  spmv_t* m = (spmv_t*)h;
  for (int k = 0; k < warmup; ++k) product(m);
  for (int k = 0; k < runs; ++k) {
    const double t0 = omp_get_wtime();
    product(m);
    seconds[k] = omp_get_wtime() - t0;
  }
}

/* Threads a parallel region uses (OMP_NUM_THREADS, else the cores available). */
int spmv_threads(void) { return omp_get_max_threads(); }
