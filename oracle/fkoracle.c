/*
 * FP64 reference implementation of the FK-table convolution (test
 * infrastructure only).
 *
 * Plain loops over the definitions, in double precision, in a fixed order
 * per output element.  OpenMP splits the work over output elements only, so
 * every result is independent of the thread count.  Nothing here is shared
 * with the HIP library: this file includes no header of it and is built by
 * gcc on its own.
 *
 * Index names: datapoint i, flavours a, b, grid points alpha, beta,
 * replica r.  Eq. (1) of Section 3 writes the same sum with grid indices
 * (i, j) and flavour indices (alpha, beta).
 *
 * Layouts (row-major, replica fastest):
 *   DIS table      mask[F] (uint8), fk[N][nact][X]  active flavours ascending
 *   hadronic table mask[F][F],      fk[N][np][X][X] active (a,b) row-major
 *   PDF            pdf[F][X][R]
 *   observables    out[N][R]
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX3(a, b, c, B, C) (((size_t)(a) * (B) + (b)) * (C) + (c))

static int active_flavours(int F, const uint8_t *mask, int *flav) {
  int n = 0;
  for (int a = 0; a < F; ++a)
    if (mask[a]) flav[n++] = a;
  return n;
}

static int active_pairs(int F, const uint8_t *mask, int *pa, int *pb) {
  int n = 0;
  for (int a = 0; a < F; ++a)
    for (int b = 0; b < F; ++b)
      if (mask[a * F + b]) {
        pa[n] = a;
        pb[n] = b;
        ++n;
      }
  return n;
}

/*
 * DIS observable (Section 3; the linear, one-PDF case of the convolution
 * whose values Table 1 lists under "DIS"):
 *   T[i,r] = sum_{a active} sum_alpha FK[i,a,alpha] f[a,alpha,r]
 */
void oracle_dis(int N, int F, int X, const uint8_t *mask, const double *fk,
                int R, const double *pdf, double *out) {
  int flav[256];
  int nact = active_flavours(F, mask, flav);
#pragma omp parallel for schedule(static)
  for (long ir = 0; ir < (long)N * R; ++ir) {
    int i = (int)(ir / R), r = (int)(ir % R);
    double acc = 0.0;
    for (int c = 0; c < nact; ++c)
      for (int al = 0; al < X; ++al)
        acc += fk[IDX3(i, c, al, nact, X)] * pdf[IDX3(flav[c], al, r, X, R)];
    out[ir] = acc;
  }
}

/*
 * Hadronic observable, Eq. (1) of Section 3, written as a bilinear form
 * with a left and a right PDF (both equal to f in the paper):
 *   s[i,r] = sum_{(a,b) active} sum_{alpha,beta}
 *              FK[i,a,b,alpha,beta] fl[a,alpha,r] fr[b,beta,r]
 */
void oracle_had_bilinear(int N, int F, int X, const uint8_t *mask,
                         const double *fk, int R, const double *pdfl,
                         const double *pdfr, double *out) {
  int *pa = (int *)malloc(sizeof(int) * F * F);
  int *pb = (int *)malloc(sizeof(int) * F * F);
  int np = active_pairs(F, mask, pa, pb);
#pragma omp parallel for schedule(static)
  for (long ir = 0; ir < (long)N * R; ++ir) {
    int i = (int)(ir / R), r = (int)(ir % R);
    double acc = 0.0;
    for (int c = 0; c < np; ++c) {
      const double *blk = fk + ((size_t)i * np + c) * X * X;
      for (int al = 0; al < X; ++al) {
        double fa = pdfl[IDX3(pa[c], al, r, X, R)];
        for (int be = 0; be < X; ++be)
          acc += blk[(size_t)al * X + be] * fa * pdfr[IDX3(pb[c], be, r, X, R)];
      }
    }
    out[ir] = acc;
  }
  free(pa);
  free(pb);
}

void oracle_had(int N, int F, int X, const uint8_t *mask, const double *fk,
                int R, const double *pdf, double *out) {
  oracle_had_bilinear(N, F, X, mask, fk, R, pdf, pdf, out);
}

/*
 * Gradient of L = sum_{i,r} gbar[i,r] T[i,r] with respect to the PDF, the
 * quantity the custom operator of Section 3 returns beside the convolution
 * (Table 1, "Gradient" rows):
 *   g[a,alpha,r] = sum_i gbar[i,r] FK[i,a,alpha]          (a active)
 * Inactive flavours get 0.
 */
void oracle_dis_grad(int N, int F, int X, const uint8_t *mask,
                     const double *fk, int R, const double *gbar, double *g) {
  int flav[256];
  int nact = active_flavours(F, mask, flav);
  int cof[256];
  for (int a = 0; a < F; ++a) cof[a] = -1;
  for (int c = 0; c < nact; ++c) cof[flav[c]] = c;
#pragma omp parallel for schedule(static)
  for (long o = 0; o < (long)F * X * R; ++o) {
    int a = (int)(o / ((long)X * R));
    int al = (int)((o / R) % X);
    int r = (int)(o % R);
    double acc = 0.0;
    if (cof[a] >= 0)
      for (int i = 0; i < N; ++i)
        acc += gbar[(size_t)i * R + r] * fk[IDX3(i, cof[a], al, nact, X)];
    g[o] = acc;
  }
}

/*
 * Gradient of L = sum_{i,r} gbar[i,r] sigma[i,r] for the hadronic form:
 *   g[p,r] = sum_i gbar[i,r] ( sum_q FK[i,p,q] f[q,r] + sum_q FK[i,q,p] f[q,r] )
 * with p = (a,alpha), q = (b,beta); the first term differentiates the left
 * PDF factor of Eq. (1), the second the right one.  General (non-symmetric)
 * FK and masks are allowed.
 */
void oracle_had_grad(int N, int F, int X, const uint8_t *mask,
                     const double *fk, int R, const double *pdf,
                     const double *gbar, double *g) {
  int *pa = (int *)malloc(sizeof(int) * F * F);
  int *pb = (int *)malloc(sizeof(int) * F * F);
  int np = active_pairs(F, mask, pa, pb);
#pragma omp parallel for schedule(static)
  for (long o = 0; o < (long)F * X * R; ++o) {
    int a = (int)(o / ((long)X * R));
    int al = (int)((o / R) % X);
    int r = (int)(o % R);
    double acc = 0.0;
    for (int i = 0; i < N; ++i) {
      double gi = gbar[(size_t)i * R + r];
      double s = 0.0;
      for (int c = 0; c < np; ++c) {
        const double *blk = fk + ((size_t)i * np + c) * X * X;
        if (pa[c] == a) /* d/d f_left: row alpha of the block */
          for (int be = 0; be < X; ++be)
            s += blk[(size_t)al * X + be] * pdf[IDX3(pb[c], be, r, X, R)];
        if (pb[c] == a) /* d/d f_right: column alpha of the block */
          for (int ap = 0; ap < X; ++ap)
            s += blk[(size_t)ap * X + al] * pdf[IDX3(pa[c], ap, r, X, R)];
      }
      acc += gi * s;
    }
    g[o] = acc;
  }
  free(pa);
  free(pb);
}

/*
 * Cholesky factor of one SPD block, C = L L^T, L lower triangular
 * (Cholesky-Banachiewicz order: row by row, left to right).  Returns 0 on
 * success, -(row+1) when a pivot is not positive.  The strict upper
 * triangle of L is set to zero.
 */
int oracle_cholesky(int n, const double *C, double *L) {
  memset(L, 0, sizeof(double) * (size_t)n * n);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = C[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      if (i == j) {
        if (!(s > 0.0)) return -(i + 1);
        L[(size_t)i * n + i] = sqrt(s);
      } else {
        L[(size_t)i * n + j] = s / L[(size_t)j * n + j];
      }
    }
  }
  return 0;
}

/*
 * chi2 over block-diagonal covariance.  For every block with factor L and
 * every replica r:
 *   e = sigma - D,  y = L^{-1} e (forward substitution),  chi2_r += y.y,
 *   w = L^{-T} y (back substitution),  dchi2/dsigma = 2 w  (= 2 C^{-1} e).
 * Blocks are visited in order; ``Lpacked`` holds the n_k x n_k factors one
 * after the other.  ``dchi2`` may be NULL.
 */
void oracle_chi2(int nblocks, const int *block_n, const double *Lpacked,
                 int R, const double *sigma, const double *data,
                 double *chi2, double *dchi2) {
  for (int r = 0; r < R; ++r) chi2[r] = 0.0;
  size_t loff = 0, roff = 0;
  for (int k = 0; k < nblocks; ++k) {
    int n = block_n[k];
    const double *L = Lpacked + loff;
    double *part = (double *)calloc((size_t)R, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int r = 0; r < R; ++r) {
      double *y = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
      for (int i = 0; i < n; ++i) {
        double s = sigma[(roff + i) * (size_t)R + r] - data[roff + i];
        for (int j = 0; j < i; ++j) s -= L[(size_t)i * n + j] * y[j];
        y[i] = s / L[(size_t)i * n + i];
      }
      double c = 0.0;
      for (int i = 0; i < n; ++i) c += y[i] * y[i];
      part[r] = c;
      if (dchi2) {
        for (int i = n - 1; i >= 0; --i) {
          double s = y[i];
          for (int j = i + 1; j < n; ++j) s -= L[(size_t)j * n + i] * y[j];
          y[i] = s / L[(size_t)i * n + i];
        }
        for (int i = 0; i < n; ++i) dchi2[(roff + i) * (size_t)R + r] = 2.0 * y[i];
      }
      free(y);
    }
    for (int r = 0; r < R; ++r) chi2[r] += part[r];
    free(part);
    loff += (size_t)n * n;
    roff += (size_t)n;
  }
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads for the parallel loops that follow (timing only: every output is
   computed by one thread, so results do not depend on the count). */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}
