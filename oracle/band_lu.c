/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.  Not part of the GPU product path.
 *
 * Plain complex128 banded LU factorisation with partial (row) pivoting and the
 * two triangular-solve sequences the paper writes down:
 *   forward  x   = U^-1 L^-1 b          (Eq. 5, applied with the row interchanges)
 *   adjoint  x   = (L^T)^-1 (U^T)^-1 g   (Eq. 6, the transposed factors, no refactor)
 * Section II of the paper states the method solves A E = b by LU with back
 * substitution and reuses the same factors, transposed, for A^T E_adj = g.
 *
 * Band storage (column major, leading dimension ldab = 2*kl + ku + 1):
 *   A(i, j) lives at ab[(kl + ku + i - j) + j * ldab]
 * for max(0, j - ku) <= i <= min(n - 1, j + kl).  The first kl rows of every
 * column are workspace for the fill that row interchanges create; the caller
 * zeroes them.  Unblocked, unthreaded, written for clarity, not speed.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>

typedef double complex zc;

static inline int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }
static inline int64_t imax(int64_t a, int64_t b) { return a > b ? a : b; }

#define AB(r, c) ab[(kv + (r) - (c)) + (c) * ldab]

/* Returns 0 on success, j+1 if column j has an exactly zero pivot. */
int64_t oracle_band_lu(int64_t n, int64_t kl, int64_t ku, zc *ab, int64_t ldab,
                       int64_t *ipiv)
{
    const int64_t kv = kl + ku; /* row of the diagonal inside a band column */
    int64_t ju = 0;             /* last column touched by interchanges so far */
    for (int64_t j = 0; j < n; ++j) {
        const int64_t km = imin(kl, n - 1 - j);
        /* pivot: largest modulus in column j on or below the diagonal */
        int64_t jp = 0;
        double amax = cabs(AB(j, j));
        for (int64_t i = 1; i <= km; ++i) {
            double a = cabs(AB(j + i, j));
            if (a > amax) { amax = a; jp = i; }
        }
        ipiv[j] = j + jp;
        if (amax == 0.0) return j + 1;
        ju = imax(ju, imin(j + ku + jp, n - 1));
        if (jp != 0) {
            for (int64_t c = j; c <= ju; ++c) {
                zc t = AB(j, c);
                AB(j, c) = AB(j + jp, c);
                AB(j + jp, c) = t;
            }
        }
        /* multipliers l_ij = a_ij / a_jj */
        const zc inv = 1.0 / AB(j, j);
        for (int64_t i = 1; i <= km; ++i) AB(j + i, j) *= inv;
        /* rank-1 update of the trailing block rows j+1..j+km, columns j+1..ju */
        for (int64_t c = j + 1; c <= ju; ++c) {
            const zc a = AB(j, c);
            if (a == 0.0) continue;
            zc *col = &AB(j, c);
            const zc *l = &AB(j, j);
            for (int64_t i = 1; i <= km; ++i) col[i] -= l[i] * a;
        }
    }
    return 0;
}

/*
 * Solve with the factors from oracle_band_lu, in place on b (n x nrhs, column
 * major, leading dimension ldb).  trans = 0 solves A x = b, trans = 1 solves
 * A^T x = b (plain transpose, no conjugation).
 */
void oracle_band_solve(int64_t n, int64_t kl, int64_t ku, const zc *ab,
                       int64_t ldab, const int64_t *ipiv, int trans,
                       int64_t nrhs, zc *b, int64_t ldb)
{
    const int64_t kv = kl + ku;
    for (int64_t r = 0; r < nrhs; ++r) {
        zc *x = b + r * ldb;
        if (!trans) {
            /* L^-1 with the interchanges in the order they were made */
            for (int64_t j = 0; j < n; ++j) {
                const int64_t km = imin(kl, n - 1 - j);
                const int64_t p = ipiv[j];
                if (p != j) { zc t = x[j]; x[j] = x[p]; x[p] = t; }
                const zc xj = x[j];
                for (int64_t i = 1; i <= km; ++i) x[j + i] -= AB(j + i, j) * xj;
            }
            /* U^-1: U has kl + ku superdiagonals after the interchanges */
            for (int64_t j = n - 1; j >= 0; --j) {
                x[j] /= AB(j, j);
                const zc xj = x[j];
                for (int64_t i = imax(0, j - kv); i < j; ++i) x[i] -= AB(i, j) * xj;
            }
        } else {
            /* (U^T)^-1: forward substitution with the rows of U */
            for (int64_t j = 0; j < n; ++j) {
                zc s = x[j];
                for (int64_t i = imax(0, j - kv); i < j; ++i) s -= AB(i, j) * x[i];
                x[j] = s / AB(j, j);
            }
            /* (L^T)^-1 with the interchanges undone in reverse order */
            for (int64_t j = n - 1; j >= 0; --j) {
                const int64_t km = imin(kl, n - 1 - j);
                zc s = x[j];
                for (int64_t i = 1; i <= km; ++i) s -= AB(j + i, j) * x[j + i];
                x[j] = s;
                const int64_t p = ipiv[j];
                if (p != j) { zc t = x[j]; x[j] = x[p]; x[p] = t; }
            }
        }
    }
}
