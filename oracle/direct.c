/*
 * Direct summation of polyharmonic-spline kernel sums (oracle; TEST
 * INFRASTRUCTURE ONLY: called by the test-suite, the smoke check and the
 * benchmark's CPU baseline, never by the library).
 *
 * out[i] = sum_j c[j] * phi(|t_i - x_j|) for every target t_i, with the basis
 * of eq. phs_fun: phi(r) = r^k for odd k, r^k log r for even k, and phi(0) = 0
 * (a target that coincides with a node gets nothing from it).  This is the
 * kernel part of the interpolant of eq. phs_interp and, with t = x, a row of
 * the matvec M c.
 *
 * Plain FP64, no reassociation: r = sqrt(dx*dx + dy*dy) with each operation
 * rounded (built with -ffp-contract=off), r^k by repeated multiplication, and
 * each row summed in source order with Neumaier's compensated summation.  Rows
 * are independent and split over OpenMP threads.
 */
#include <math.h>
#include <stdint.h>

static double phi(int k, double r) {
  if (r == 0.0) return 0.0;
  double rk = 1.0;
  for (int e = 0; e < k; ++e) rk *= r;
  return (k % 2 == 1) ? rk : rk * log(r);
}

void oracle_direct_sums(int k, int64_t n, const double *xs, const double *c, int64_t m,
                        const double *ts, double *out) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < m; ++i) {
    const double tx = ts[2 * i], ty = ts[2 * i + 1];
    double s = 0.0, comp = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      const double dx = tx - xs[2 * j], dy = ty - xs[2 * j + 1];
      const double r = sqrt(dx * dx + dy * dy);
      const double term = c[j] * phi(k, r);
      const double t = s + term;
      if (fabs(s) >= fabs(term)) comp += (s - t) + term;
      else comp += (term - t) + s;
      s = t;
    }
    out[i] = s + comp;
  }
}

int oracle_direct_threads(void) {
  int t = 1;
#pragma omp parallel
  {
#pragma omp single
    {
#ifdef _OPENMP
      extern int omp_get_num_threads(void);
      t = omp_get_num_threads();
#endif
    }
  }
  return t;
}
