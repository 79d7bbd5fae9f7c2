/* The oracle's banded LU (oracle/band_lu.c) on small random systems, built
 * with gcc under AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers.py: factor, forward and transposed solves, residuals
 * checked against the dense matrix.  Prints "ok" or the failure. */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t oracle_band_lu(int64_t n, int64_t kl, int64_t ku, double complex* ab, int64_t ldab, int64_t* ipiv);
void oracle_band_solve(int64_t n, int64_t kl, int64_t ku, const double complex* ab, int64_t ldab,
                       const int64_t* ipiv, int trans, int64_t nrhs, double complex* b, int64_t ldb);

static double urand(unsigned* s) {
  *s = *s * 1664525u + 1013904223u;
  return (double)(*s >> 8) / 16777216.0 - 0.5;
}

int main(void) {
  const int64_t sizes[][3] = {{1, 0, 0}, {5, 1, 2}, {17, 3, 3}, {40, 7, 5}, {64, 8, 8}};
  unsigned seed = 12345u;
  for (int t = 0; t < 5; ++t) {
    const int64_t n = sizes[t][0], kl = sizes[t][1], ku = sizes[t][2];
    const int64_t ldab = 2 * kl + ku + 1, kv = kl + ku;
    double complex* A = calloc((size_t)(n * n), sizeof(double complex));
    double complex* ab = calloc((size_t)(n * ldab), sizeof(double complex));
    int64_t* ipiv = calloc((size_t)n, sizeof(int64_t));
    double complex* x = calloc((size_t)(2 * n), sizeof(double complex));
    for (int64_t c = 0; c < n; ++c)
      for (int64_t r = c - ku; r <= c + kl; ++r)
        if (r >= 0 && r < n) {
          const double complex v = urand(&seed) + I * urand(&seed) + (r == c ? 0.5 : 0.0);
          A[r * n + c] = v;
          ab[c * ldab + kv + r - c] = v;
        }
    if (oracle_band_lu(n, kl, ku, ab, ldab, ipiv) != 0) { printf("FAIL singular n=%ld\n", (long)n); return 1; }
    for (int trans = 0; trans < 2; ++trans) {
      for (int64_t i = 0; i < 2 * n; ++i) x[i] = (double)(i % 7) - 3.0 + I * (double)(i % 3);
      double complex* b = malloc((size_t)(2 * n) * sizeof(double complex));
      for (int64_t i = 0; i < 2 * n; ++i) b[i] = x[i];
      oracle_band_solve(n, kl, ku, ab, ldab, ipiv, trans, 2, x, n);
      for (int64_t k = 0; k < 2; ++k) {
        double rn = 0, bn = 0;
        for (int64_t r = 0; r < n; ++r) {
          double complex s = 0;
          for (int64_t c = 0; c < n; ++c) s += (trans ? A[c * n + r] : A[r * n + c]) * x[k * n + c];
          rn += cabs(s - b[k * n + r]) * cabs(s - b[k * n + r]);
          bn += cabs(b[k * n + r]) * cabs(b[k * n + r]);
        }
        if (!(sqrt(rn) <= 1e-10 * sqrt(bn) + 1e-300)) { printf("FAIL residual n=%ld trans=%d\n", (long)n, trans); return 1; }
      }
      free(b);
    }
    free(A); free(ab); free(ipiv); free(x);
  }
  printf("ok\n");
  return 0;
}
