/*
 * FP64 reference ("oracle") loops for the coverage-flow hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code with the HIP kernels.
 *
 * These are the O(N^2) sums of the method written out plainly in double
 * precision, one output point at a time, parallelised only across output
 * points (OpenMP), and the log-sum-exp's loop over keys also across vector lanes
 * (OpenMP simd).  No tiling, no fusion, no reordering of the sums beyond "max
 * first, then sum" for the log-sum-exp and the lanes' partial sums.  The iteration logic that calls
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
#include <stdlib.h>

/* glibc's vector exp (libmvec) for the simd loops of orc_lse; each lane is the
 * correctly rounded exp to within a few ulp. */
#pragma omp declare simd notinbranch
double exp(double);

static double sqdist(int d, const double* a, const double* b) {
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = a[k] - b[k];
        s += t * t;
    }
    return s;
}

/* One query row of orc_lse, for a fixed d (inlined with d = 2 or 3 so that the
 * loops over keys vectorise; the key coordinates come one array per axis).
 * Pass 1 takes the largest exponent, pass 2 the shifted sum (and the weighted
 * offsets).  The sums run over all keys; only the order in which the vector
 * lanes add their terms differs from a one-at-a-time loop. */
static inline __attribute__((always_inline)) void lse_row(
    int d, const double* xi, int64_t nk, const double* k0, const double* k1, const double* k2,
    const double* h, double eps, double* lse_i, double* bary_i) {
    double m = -INFINITY;
#pragma omp simd reduction(max : m)
    for (int64_t j = 0; j < nk; ++j) {
        double t0 = xi[0] - k0[j], t1 = xi[1] - k1[j];
        double c = t0 * t0 + t1 * t1;
        if (d == 3) {
            double t2 = xi[2] - k2[j];
            c += t2 * t2;
        }
        double z = h[j] - c / eps;
        m = z > m ? z : m;
    }
    double s = 0.0, a0 = 0.0, a1 = 0.0, a2 = 0.0;
    if (!bary_i) {
#pragma omp simd reduction(+ : s)
        for (int64_t j = 0; j < nk; ++j) {
            double t0 = xi[0] - k0[j], t1 = xi[1] - k1[j];
            double c = t0 * t0 + t1 * t1;
            if (d == 3) {
                double t2 = xi[2] - k2[j];
                c += t2 * t2;
            }
            s += exp(h[j] - c / eps - m);
        }
    } else {
#pragma omp simd reduction(+ : s, a0, a1, a2)
        for (int64_t j = 0; j < nk; ++j) {
            double t0 = xi[0] - k0[j], t1 = xi[1] - k1[j];
            double c = t0 * t0 + t1 * t1;
            double t2 = 0.0;
            if (d == 3) {
                t2 = xi[2] - k2[j];
                c += t2 * t2;
            }
            double e = exp(h[j] - c / eps - m);
            s += e;
            a0 -= e * t0;            /* e * (y_j - x_i) */
            a1 -= e * t1;
            if (d == 3) a2 -= e * t2;
        }
        bary_i[0] = a0 / s;
        bary_i[1] = a1 / s;
        if (d == 3) bary_i[2] = a2 / s;
    }
    *lse_i = m + log(s);
}

void orc_lse(int d, int64_t nq, const double* xq, int64_t nk, const double* xk,
             const double* h, double eps, double* lse, double* bary) {
    /* key coordinates, one array per axis */
    double* kc = (double*)malloc(sizeof(double) * (size_t)d * (size_t)nk);
    for (int k = 0; k < d; ++k)
        for (int64_t j = 0; j < nk; ++j) kc[k * nk + j] = xk[j * d + k];
    const double* k2 = d == 3 ? kc + 2 * nk : kc;
#pragma omp parallel for schedule(static) if (nq * nk > 65536)
    for (int64_t i = 0; i < nq; ++i) {
        if (d == 2)
            lse_row(2, xq + 2 * i, nk, kc, kc + nk, k2, h, eps, lse + i, bary ? bary + 2 * i : 0);
        else
            lse_row(3, xq + 3 * i, nk, kc, kc + nk, k2, h, eps, lse + i, bary ? bary + 3 * i : 0);
    }
    free(kc);
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
