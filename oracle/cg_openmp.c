/*
 * cg_openmp.c -- plain fp64 conjugate gradients (section 3's recurrences for x,
 * r, p, alpha and beta, no preconditioner) on every host core: the multi-core
 * CPU speed baseline timed beside the GPU solver.  Not part of the parity
 * oracle, which is single-threaded.
 *
 * TEST INFRASTRUCTURE ONLY: the benchmark's CPU-baseline leg and the test suite
 * load it; the product path never does.
 *
 * Row-parallel SpMV and vector updates (OpenMP, static schedule).  Every inner
 * product is first summed over fixed chunks of CHUNK consecutive rows, each in
 * ascending row order, and the chunk sums are then added in chunk order by one
 * thread, so the result does not depend on the number of threads.  The inner
 * products are fused with the loop that produces their operand (p.q with the
 * SpMV, r.r with the x and r updates).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>

#define CHUNK 8192

static double sum_chunks(const double *part, int64_t nc)
{
    double t = 0.0;
    for (int64_t c = 0; c < nc; ++c) t += part[c];
    return t;
}

/* x: initial guess in, solution out.  Stops when sqrt(r.r)/||b|| <= tol (the
 * recursive residual) or after maxit iterations.  Returns the threads used. */
int cgomp_solve(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, const double *b,
                double *x, double tol, int32_t maxit, int32_t *iters_out, double *relres_out)
{
    const int64_t nc = (n + CHUNK - 1) / CHUNK;
    size_t bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *r = malloc(bytes), *p = malloc(bytes), *q = malloc(bytes);
    double *part = malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
    int threads = 1;

#pragma omp parallel
    {
#pragma omp single
        threads = omp_get_num_threads();
    }

#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t e = (c + 1) * CHUNK < n ? (c + 1) * CHUNK : n;
        double s = 0.0;
        for (int64_t i = c * CHUNK; i < e; ++i) s += b[i] * b[i];
        part[c] = s;
    }
    const double bnorm = sqrt(sum_chunks(part, nc));

#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t e = (c + 1) * CHUNK < n ? (c + 1) * CHUNK : n;
        double s = 0.0;
        for (int64_t i = c * CHUNK; i < e; ++i) {
            double acc = 0.0;
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) acc += v[k] * x[ci[k]];
            r[i] = b[i] - acc;
            p[i] = r[i];
            s += r[i] * r[i];
        }
        part[c] = s;
    }
    double sigma = sum_chunks(part, nc);
    int32_t k = 0;
    while (k < maxit && sqrt(sigma) / bnorm > tol) {
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nc; ++c) {
            const int64_t e = (c + 1) * CHUNK < n ? (c + 1) * CHUNK : n;
            double s = 0.0;
            for (int64_t i = c * CHUNK; i < e; ++i) {
                double acc = 0.0;
                for (int64_t kk = rp[i]; kk < rp[i + 1]; ++kk) acc += v[kk] * p[ci[kk]];
                q[i] = acc;
                s += p[i] * acc;
            }
            part[c] = s;
        }
        const double alpha = sigma / sum_chunks(part, nc);
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nc; ++c) {
            const int64_t e = (c + 1) * CHUNK < n ? (c + 1) * CHUNK : n;
            double s = 0.0;
            for (int64_t i = c * CHUNK; i < e; ++i) {
                x[i] += alpha * p[i];
                r[i] -= alpha * q[i];
                s += r[i] * r[i];
            }
            part[c] = s;
        }
        const double sn = sum_chunks(part, nc);
        const double beta = sn / sigma;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        sigma = sn;
        k++;
    }
    *iters_out = k;
    *relres_out = sqrt(sigma) / bnorm;
    free(r); free(p); free(q); free(part);
    return threads;
}
