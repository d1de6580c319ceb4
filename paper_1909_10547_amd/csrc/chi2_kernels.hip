// FP64 chi2 over a block-diagonal experimental covariance on gfx950.
//
//   chi2_r = (sigma_r - D)^T C^{-1} (sigma_r - D),   C = blockdiag(C_b)
//
// Set-up (once per covariance): C_b = L_b L_b^T (right-looking Cholesky, one
// workgroup per block) and the triangular inverse M_b = L_b^{-1} (one wave
// per 64 columns).  Per call: y = M e (e = sigma - D, lower-triangular
// product), chi2_r = sum y^2, and the gradient 2 C^{-1} e = 2 M^T y
// (upper-triangular product).  Everything is binary64; partial sums are
// reduced in a fixed order.
#include "fk_internal.h"

namespace fk {

constexpr int kCT = 32;  // rows/columns per chi2 tile

__global__ void __launch_bounds__(256)
    chol_kernel(const int32_t *__restrict__ nb, const int64_t *__restrict__ off,
                double *__restrict__ A, int32_t *__restrict__ flag) {
  const int b = blockIdx.x;
  const int n = nb[b];
  double *a = A + off[b];
  __shared__ double piv;
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      double d = a[(size_t)j * n + j];
      if (!(d > 0.0)) {
        if (flag[b] == 0) flag[b] = j + 1;
        d = 1.0;
      }
      d = sqrt(d);
      a[(size_t)j * n + j] = d;
      piv = d;
    }
    __syncthreads();
    const double inv = 1.0 / piv;
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) a[(size_t)i * n + j] *= inv;
    __syncthreads();
    // trailing update of the lower triangle, rows/cols j+1..n-1
    const int m = n - j - 1;
    const long tri = (long)m * (m + 1) / 2;
    for (long idx = threadIdx.x; idx < tri; idx += blockDim.x) {
      int ii = (int)((sqrt(8.0 * (double)idx + 1.0) - 1.0) * 0.5);
      while ((long)ii * (ii + 1) / 2 > idx) --ii;
      while ((long)(ii + 1) * (ii + 2) / 2 <= idx) ++ii;
      const int kk = (int)(idx - (long)ii * (ii + 1) / 2);
      const int r = j + 1 + ii, c = j + 1 + kk;
      a[(size_t)r * n + c] -= a[(size_t)r * n + j] * a[(size_t)c * n + j];
    }
    __syncthreads();
  }
}

// Columns j of M = L^{-1}: M[j][j] = 1/L[j][j],
// M[i][j] = -(sum_{k=j}^{i-1} L[i][k] M[k][j]) / L[i][i] for i > j.
// M is zero-initialised, so the sum may start at the chunk's first column.
__global__ void __launch_bounds__(64)
    trtri_kernel(const int32_t *__restrict__ nb, const int64_t *__restrict__ off,
                 const double *__restrict__ L, double *__restrict__ M) {
  const int b = blockIdx.y;
  const int n = nb[b];
  const int j0 = blockIdx.x * 64;
  if (j0 >= n) return;
  const int j = j0 + threadIdx.x;
  const double *l = L + off[b];
  double *m = M + off[b];
  for (int i = j0; i < n; ++i) {
    double s = 0.0;
    const double *li = l + (size_t)i * n;
    for (int k = j0; k < i; ++k) s += li[k] * (j < n ? m[(size_t)k * n + j] : 0.0);
    if (j < n) {
      if (i == j)
        m[(size_t)i * n + j] = 1.0 / li[i];
      else if (i > j)
        m[(size_t)i * n + j] = -s / li[i];
    }
  }
}

// zero the strict upper triangle of L (the factorisation leaves C there)
__global__ void clear_upper_kernel(const int32_t *__restrict__ nb, const int64_t *__restrict__ off,
                                   double *__restrict__ A) {
  const int b = blockIdx.y;
  const int n = nb[b];
  double *a = A + off[b];
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < (long)n * n;
       idx += (long)gridDim.x * blockDim.x) {
    const int r = (int)(idx / n), c = (int)(idx % n);
    if (c > r) a[idx] = 0.0;
  }
}

// y = M e for one 32-row tile of a block and 32 columns; also the tile's
// column sums of y^2.
__global__ void __launch_bounds__(256)
    trmm_lower_kernel(const int32_t *__restrict__ rt_block, const int32_t *__restrict__ rt_row,
                      const int32_t *__restrict__ nb, const int64_t *__restrict__ off,
                      const int32_t *__restrict__ roff, const double *__restrict__ M,
                      const float *__restrict__ sigma, const double *__restrict__ data, int R,
                      int c0, int ncols, double *__restrict__ y, double *__restrict__ part) {
  __shared__ double sm[kCT][kCT + 1];
  __shared__ double se[kCT][kCT + 1];
  __shared__ double sq[8][kCT];
  const int rt = blockIdx.x;
  const int b = rt_block[rt], r0 = rt_row[rt];
  const int n = nb[b];
  const double *m = M + off[b];
  const int base = roff[b];
  const int tc = threadIdx.x & 31, tr = threadIdx.x >> 5;  // column, row group of 4
  const int col = blockIdx.y * kCT + tc;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int kend = min(n, r0 + kCT);
  for (int k0 = 0; k0 < kend; k0 += kCT) {
    for (int i = threadIdx.x; i < kCT * kCT; i += 256) {
      const int rr = i / kCT, cc = i % kCT;
      const int gr = r0 + rr, gk = k0 + cc;
      sm[rr][cc] = (gr < n && gk < n) ? m[(size_t)gr * n + gk] : 0.0;
      const int ek = k0 + rr, ec = blockIdx.y * kCT + cc;
      double e = 0.0;
      if (ek < n && ec < ncols)
        e = (double)sigma[(size_t)(base + ek) * R + c0 + ec] - data[base + ek];
      se[rr][cc] = e;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kCT; ++kk) {
      const double ev = se[kk][tc];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += sm[4 * tr + q][kk] * ev;
    }
    __syncthreads();
  }
  double ss = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int gr = r0 + 4 * tr + q;
    if (gr < n && col < ncols) {
      y[(size_t)(base + gr) * kRpMax + col] = acc[q];
      ss += acc[q] * acc[q];
    }
  }
  sq[tr][tc] = ss;
  __syncthreads();
  if (tr == 0) {
    double t = 0.0;
    for (int g = 0; g < 8; ++g) t += sq[g][tc];
    part[(size_t)rt * kRpMax + col] = t;
  }
}

__global__ void chi2_reduce_kernel(int nrt, const double *__restrict__ part, int c0, int ncols,
                                   double *__restrict__ chi2) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncols) return;
  double t = 0.0;
  for (int rt = 0; rt < nrt; ++rt) t += part[(size_t)rt * kRpMax + col];
  chi2[c0 + col] = t;
}

// w = M^T y for one 32-row tile (rows k of w) and 32 columns; writes 2w.
__global__ void __launch_bounds__(256)
    trmm_upper_kernel(const int32_t *__restrict__ rt_block, const int32_t *__restrict__ rt_row,
                      const int32_t *__restrict__ nb, const int64_t *__restrict__ off,
                      const int32_t *__restrict__ roff, const double *__restrict__ M,
                      const double *__restrict__ y, int R, int c0, int ncols,
                      float *__restrict__ dchi2) {
  __shared__ double sm[kCT][kCT + 1];  // sm[i][k] = M[i0+i][k0+k]
  __shared__ double sy[kCT][kCT + 1];
  const int rt = blockIdx.x;
  const int b = rt_block[rt], k0 = rt_row[rt];
  const int n = nb[b];
  const double *m = M + off[b];
  const int base = roff[b];
  const int tc = threadIdx.x & 31, tr = threadIdx.x >> 5;
  const int col = blockIdx.y * kCT + tc;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i0 = k0; i0 < n; i0 += kCT) {
    for (int i = threadIdx.x; i < kCT * kCT; i += 256) {
      const int rr = i / kCT, cc = i % kCT;
      const int gi = i0 + rr, gk = k0 + cc;
      sm[rr][cc] = (gi < n && gk < n) ? m[(size_t)gi * n + gk] : 0.0;
      const int yc = blockIdx.y * kCT + cc;
      sy[rr][cc] = (gi < n && yc < ncols) ? y[(size_t)(base + gi) * kRpMax + yc] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int ii = 0; ii < kCT; ++ii) {
      const double yv = sy[ii][tc];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += sm[ii][4 * tr + q] * yv;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int gk = k0 + 4 * tr + q;
    if (gk < n && col < ncols) dchi2[(size_t)(base + gk) * R + c0 + col] = (float)(2.0 * acc[q]);
  }
}

hipError_t launch_cholesky(int nblocks, const int32_t *d_n, const int64_t *d_off, double *d_a,
                           double *d_linv, int32_t *d_flag, int maxn, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(chol_kernel, dim3(nblocks), dim3(256), 0, s, d_n, d_off, d_a, d_flag);
  hipLaunchKernelGGL(clear_upper_kernel, dim3(64, nblocks), dim3(256), 0, s, d_n, d_off, d_a);
  hipLaunchKernelGGL(trtri_kernel, dim3((maxn + 63) / 64, nblocks), dim3(64), 0, s, d_n, d_off,
                     (const double *)d_a, d_linv);
  return hipGetLastError();
}

hipError_t launch_chi2(int nblocks, int nrt, const int32_t *d_rt_block, const int32_t *d_rt_row,
                       const int32_t *d_n, const int64_t *d_off, const int32_t *d_roff,
                       const double *d_linv, const float *sigma, const double *data, int R,
                       int c0, int ncols, double *d_y, double *d_part, double *chi2,
                       float *dchi2, hipStream_t s) {
  (void)nblocks;
  if (nrt <= 0) return hipSuccess;
  const dim3 grid(nrt, (ncols + kCT - 1) / kCT);
  hipLaunchKernelGGL(trmm_lower_kernel, grid, dim3(256), 0, s, d_rt_block, d_rt_row, d_n, d_off,
                     d_roff, d_linv, sigma, data, R, c0, ncols, d_y, d_part);
  hipLaunchKernelGGL(chi2_reduce_kernel, dim3((ncols + 127) / 128), dim3(128), 0, s, nrt, d_part,
                     c0, ncols, chi2);
  if (dchi2)
    hipLaunchKernelGGL(trmm_upper_kernel, grid, dim3(256), 0, s, d_rt_block, d_rt_row, d_n, d_off,
                       d_roff, d_linv, (const double *)d_y, R, c0, ncols, dchi2);
  return hipGetLastError();
}

}  // namespace fk
