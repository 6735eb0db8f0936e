/*
 * FP64 reference ("oracle") loops for the coverage-flow hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code with the HIP kernels.
 *
 * These are the O(N^2) sums of the method written out plainly in double
 * precision, one output point at a time, parallelised only across output
 * points (OpenMP).  No tiling, no fusion, no reordering of the sums beyond
 * "max first, then sum" for the log-sum-exp.  The iteration logic that calls
 * them lives in oracle/sinkhorn.py and oracle/svgd.py.
 *
 *   orc_lse      : for query i,  z_ij = h_j - |xq_i - xk_j|^2 / eps,
 *                  lse_i = log sum_j exp(z_ij)                      (Sec. II-B,
 *                  eq. 5: the dual (soft-min) update of entropic OT under the
 *                  squared-norm cost), optionally the soft-min-weighted mean
 *                  offset  bary_i = sum_j softmax_j(z_i.) (xk_j - xq_i).
 *   orc_svgd_phi : eq. 4 with the RBF kernel k(s,s') = exp(-|s-s'|^2 / h).
 *   orc_pair_count : number of pairs i<j with squared distance < thr and <= thr
 *                  (used to certify a pairwise-distance median).
 */
#include <math.h>
#include <stdint.h>

static double sqdist(int d, const double* a, const double* b) {
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = a[k] - b[k];
        s += t * t;
    }
    return s;
}

void orc_lse(int d, int64_t nq, const double* xq, int64_t nk, const double* xk,
             const double* h, double eps, double* lse, double* bary) {
#pragma omp parallel for schedule(static) if (nq * nk > 65536)
    for (int64_t i = 0; i < nq; ++i) {
        const double* xi = xq + i * d;
        /* pass 1: the largest exponent */
        double m = -INFINITY;
        for (int64_t j = 0; j < nk; ++j) {
            double z = h[j] - sqdist(d, xi, xk + j * d) / eps;
            if (z > m) m = z;
        }
        /* pass 2: shifted sum (and weighted offsets) */
        double s = 0.0;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < nk; ++j) {
            const double* xj = xk + j * d;
            double e = exp(h[j] - sqdist(d, xi, xj) / eps - m);
            s += e;
            if (bary)
                for (int k = 0; k < d; ++k) acc[k] += e * (xj[k] - xi[k]);
        }
        lse[i] = m + log(s);
        if (bary)
            for (int k = 0; k < d; ++k) bary[i * d + k] = acc[k] / s;
    }
}

void orc_svgd_phi(int d, int64_t n, const double* x, const double* score, double h, double* phi) {
#pragma omp parallel for schedule(static) if (n * n > 65536)
    for (int64_t i = 0; i < n; ++i) {
        const double* xi = x + i * d;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            const double* xj = x + j * d;
            double kij = exp(-sqdist(d, xi, xj) / h);
            for (int k = 0; k < d; ++k)
                acc[k] += kij * score[j * d + k] + kij * (2.0 / h) * (xi[k] - xj[k]);
        }
        for (int k = 0; k < d; ++k) phi[i * d + k] = acc[k] / (double)n;
    }
}

void orc_pair_count(int d, int64_t n, const double* x, double thr, int64_t* n_lt, int64_t* n_le) {
    int64_t lt = 0, le = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : lt, le)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            double s = sqdist(d, x + i * d, x + j * d);
            lt += s < thr;
            le += s <= thr;
        }
    *n_lt = lt;
    *n_le = le;
}
