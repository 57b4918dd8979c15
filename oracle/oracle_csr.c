/* Plain CSR sparse matrix-vector product of the oracle's assembled matrices,
 * threaded with OpenMP (static schedule over rows), for timing the oracle on
 * a host's cores.  TEST INFRASTRUCTURE ONLY: used by the CPU-baseline leg of
 * the benchmark; nothing in the product links it.
 *
 * y_i = sum_{j in row i} data_j x_{indices_j}, summed in the stored order of
 * the row (the order of a sequential CSR product). */
#include <stdint.h>
#include <omp.h>

void csr_spmv(int64_t n, const int64_t *indptr, const int32_t *indices, const double *data,
              const double *x, double *y, int threads)
{
#pragma omp parallel for schedule(static) num_threads(threads)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t q = indptr[i]; q < indptr[i + 1]; ++q) s += data[q] * x[indices[q]];
        y[i] = s;
    }
}

/* `warm` untimed products, then `reps` timed ones; times[r] = seconds of
 * product r (wall clock). */
void csr_spmv_bench(int64_t n, const int64_t *indptr, const int32_t *indices, const double *data,
                    const double *x, double *y, int threads, int warm, int reps, double *times)
{
    for (int r = 0; r < warm; ++r) csr_spmv(n, indptr, indices, data, x, y, threads);
    for (int r = 0; r < reps; ++r) {
        const double t0 = omp_get_wtime();
        csr_spmv(n, indptr, indices, data, x, y, threads);
        times[r] = omp_get_wtime() - t0;
    }
}

int csr_max_threads(void) { return omp_get_max_threads(); }
