/*
 * Oracle helper (test infrastructure only; never linked into the product).
 *
 * Sequential FP64 evaluation of the p-stable hash of Section 4.1 (Eq. hash_fn):
 *     h(v) = floor((alpha . v + beta) / r)
 * with the dot product summed in FP64 in index order 0..D-1. Each product of
 * two fp32 values is exact in FP64, so this value does not depend on whether a
 * multiply-add is fused. Codes outside the int32 range saturate.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC orc_seq.c -o liborc_seq.so
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>

/* Threads of the OpenMP loops below (timing of the oracle at one thread and
 * at many). */
void orc_set_threads(int n)
{
    omp_set_num_threads(n > 0 ? n : 1);
}

void orc_codes(const float* V, int64_t n, int D, const float* A, const float* beta,
               int m, double w, int32_t* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        const float* v = V + r * (int64_t)D;
        for (int j = 0; j < m; ++j) {
            const float* a = A + (int64_t)j * D;
            double s = 0.0;
            for (int i = 0; i < D; ++i)
                s = s + (double)a[i] * (double)v[i];
            double t = (s + (double)beta[j]) / w;
            double f = floor(t);
            int32_t c;
            if (f >= 2147483647.0)
                c = INT32_MAX;
            else if (f <= -2147483648.0)
                c = INT32_MIN;
            else
                c = (int32_t)f;
            out[r * (int64_t)m + j] = c;
        }
    }
}

/* Sequential FP64 squared l2 distance of one query row q[D] to rows Y[n, D]:
 * d = sum_i (q_i - y_i)^2, each difference, square and sum rounded in FP64,
 * accumulated in index order. */
void orc_sqdist(const float* q, const float* Y, const int64_t* rows, int64_t n, int D,
                double* out)
{
    for (int64_t r = 0; r < n; ++r) {
        const float* y = Y + rows[r] * (int64_t)D;
        double s = 0.0;
        for (int i = 0; i < D; ++i) {
            double d = (double)q[i] - (double)y[i];
            double sq = d * d;
            s = s + sq;
        }
        out[r] = s;
    }
}
