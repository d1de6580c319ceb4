// FP64 chi2 over a block-diagonal experimental covariance on gfx950.
//
//   chi2_r = (sigma_r - D)^T C^{-1} (sigma_r - D),   C = blockdiag(C_b)
//
// Set-up (once per covariance): C_b = L_b L_b^T (right-looking Cholesky, one
// workgroup per block) and the triangular inverse M_b = L_b^{-1} (one wave
// per 64 columns).  Per call: y = M e (e = sigma - D, lower-triangular
// product), chi2_r = sum y^2, and the gradient 2 C^{-1} e = 2 M^T y
// (upper-triangular product).  Both products are split along k into
// entries of a few 32 x 32 tiles, so that every block's rows are worked on
// by many workgroups at once.  Everything is binary64; partial sums are
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

// chi2 of one replica column per workgroup: thread t adds the row tiles
// t, t + 256, ... in order, then a fixed-shape tree over the threads.
__global__ void __launch_bounds__(256)
    chi2_reduce_kernel(int nrt, const double *__restrict__ part, int c0, double *__restrict__ chi2) {
  __shared__ double sh[256];
  const int col = blockIdx.x;
  double t = 0.0;
  for (int rt = threadIdx.x; rt < nrt; rt += 256) t += part[(size_t)rt * kRpMax + col];
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) chi2[c0 + col] = sh[0];
}

// Split products.  A work entry {rt, t0, t1, slot} (slot = the entry's
// index in its list) asks for the partial product of row tile rt (32 rows
// of its block) over the k tiles [t0, t1):
//   lower: P = M[rows, k] e[k, cols]        (k tiles up to the diagonal)
//   upper: P = M[i, rows]^T y[i, cols]      (i tiles from the diagonal on)
// written to slot [32][kRpMax].  The entries of one row tile are added in
// list order by split_reduce_kernel, so the result is a fixed-order sum.
// A workgroup computes 32 rows x 32 columns on the FP64 matrix cores: wave
// (wr, wc) owns the 16 x 16 quarter (rows 16 wr.., columns 16 wc..) and
// steps through k four at a time with v_mfma_f64_16x16x4f64 (lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds rows
// l / 16 + 4 v, v = 0..3, of column l % 16 of the result: unlike the FP32
// form, whose rows are 4 (l / 16) + v).  The tiles of the next k step are
// read into registers while the current ones are multiplied.
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <bool UPPER>
__global__ void __launch_bounds__(256)
    trmm_split_kernel(const int4 *__restrict__ work, const int32_t *__restrict__ rt_block,
                      const int32_t *__restrict__ rt_row, const int32_t *__restrict__ nb,
                      const int64_t *__restrict__ off, const int32_t *__restrict__ roff,
                      const double *__restrict__ M, const float *__restrict__ sigma,
                      const double *__restrict__ data, const double *__restrict__ y, int R,
                      int c0, int ncols, double *__restrict__ spart) {
  __shared__ double sm[kCT][kCT + 1];  // lower: M[r0 + r][k0 + k]; upper: M[k0 + k][r0 + r]
  __shared__ double so[kCT][kCT + 1];  // operand [k][column]
  const int4 wk = work[blockIdx.x];
  const int rt = wk.x, t0 = wk.y, t1 = wk.z, slot = wk.w;
  const int b = rt_block[rt], r0 = rt_row[rt];
  const int n = nb[b];
  const double *m = M + off[b];
  const int base = roff[b];
  const int tc = threadIdx.x & 31, tr = threadIdx.x >> 5;
  // this thread's four elements of each 32 x 32 tile: (tr + 8 q, tc)
  double vm[4], vo[4];
  auto fetch = [&](int t) {
    const int k0 = t * kCT;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int rr = tr + 8 * q, cc = tc;
      // M tile: lower reads M[r0 + rr][k0 + cc]; upper reads M[k0 + rr][r0 + cc]
      const int gi = UPPER ? k0 + rr : r0 + rr, gk = UPPER ? r0 + cc : k0 + cc;
      vm[q] = (gi < n && gk < n) ? m[(size_t)gi * n + gk] : 0.0;
      // operand tile row k0 + rr, column blockIdx.y * 32 + cc
      const int ok = k0 + rr, oc = blockIdx.y * kCT + cc;
      double v = 0.0;
      if (ok < n && oc < ncols) {
        if (UPPER)
          v = y[(size_t)(base + ok) * kRpMax + oc];
        else
          v = (double)sigma[(size_t)(base + ok) * R + c0 + oc] - data[base + ok];
      }
      vo[q] = v;
    }
  };
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  fetch(t0);
  for (int t = t0; t < t1; ++t) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sm[tr + 8 * q][tc] = vm[q];
      so[tr + 8 * q][tc] = vo[q];
    }
    __syncthreads();
    if (t + 1 < t1) fetch(t + 1);
#pragma unroll
    for (int ks = 0; ks < kCT; ks += 4) {
      const int k = ks + lk, row = 16 * wr + li;
      const double a = UPPER ? sm[k][row] : sm[row][k];
      const double bv = so[k][16 * wc + li];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
    }
  }
  double *dst = spart + (size_t)slot * kCT * kRpMax + blockIdx.y * kCT + 16 * wc + li;
#pragma unroll
  for (int v = 0; v < 4; ++v) dst[(size_t)(16 * wr + lk + 4 * v) * kRpMax] = acc[v];
}

// Sum of the entries of each row tile in list order.  Lower: y and the
// tile's column sums of y^2; upper: 2 M^T y into the float gradient.
template <bool UPPER>
__global__ void __launch_bounds__(256)
    split_reduce_kernel(const int32_t *__restrict__ wptr,
                        const int32_t *__restrict__ rt_block, const int32_t *__restrict__ rt_row,
                        const int32_t *__restrict__ nb, const int32_t *__restrict__ roff,
                        const double *__restrict__ spart, int R, int c0, int ncols,
                        double *__restrict__ y, double *__restrict__ part,
                        float *__restrict__ dchi2) {
  __shared__ double sq[8][kCT];
  const int rt = blockIdx.x;
  const int b = rt_block[rt], r0 = rt_row[rt];
  const int n = nb[b];
  const int base = roff[b];
  const int tc = threadIdx.x & 31, tr = threadIdx.x >> 5;
  const int col = blockIdx.y * kCT + tc;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // an entry's slot is its index in the list
  for (int e = wptr[rt]; e < wptr[rt + 1]; ++e) {
    const double *src = spart + (size_t)e * kCT * kRpMax;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] += src[(size_t)(4 * tr + q) * kRpMax + col];
  }
  double ss = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int gr = r0 + 4 * tr + q;
    if (gr < n && col < ncols) {
      if (UPPER) {
        dchi2[(size_t)(base + gr) * R + c0 + col] = (float)(2.0 * acc[q]);
      } else {
        y[(size_t)(base + gr) * kRpMax + col] = acc[q];
        ss += acc[q] * acc[q];
      }
    }
  }
  if (UPPER) return;
  sq[tr][tc] = ss;
  __syncthreads();
  if (tr == 0) {
    double t = 0.0;
    for (int g = 0; g < 8; ++g) t += sq[g][tc];
    part[(size_t)rt * kRpMax + col] = t;
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

hipError_t launch_chi2(const Chi2Plan &P, const double *d_linv, const float *sigma,
                       const double *data, int R, int c0, int ncols, double *chi2, float *dchi2,
                       hipStream_t s) {
  if (P.nrt <= 0) return hipSuccess;
  const int nct = (ncols + kCT - 1) / kCT;
  hipLaunchKernelGGL(trmm_split_kernel<false>, dim3(P.nlw, nct), dim3(256), 0, s, P.d_lw,
                     P.d_rt_block, P.d_rt_row, P.d_n, P.d_off, P.d_roff, d_linv, sigma, data,
                     (const double *)nullptr, R, c0, ncols, P.d_spart);
  hipLaunchKernelGGL(split_reduce_kernel<false>, dim3(P.nrt, nct), dim3(256), 0, s, P.d_lptr,
                     P.d_rt_block, P.d_rt_row, P.d_n, P.d_roff,
                     (const double *)P.d_spart, R, c0, ncols, P.d_y, P.d_part, (float *)nullptr);
  hipLaunchKernelGGL(chi2_reduce_kernel, dim3(ncols), dim3(256), 0, s, P.nrt, P.d_part, c0, chi2);
  if (dchi2) {
    hipLaunchKernelGGL(trmm_split_kernel<true>, dim3(P.nuw, nct), dim3(256), 0, s, P.d_uw,
                       P.d_rt_block, P.d_rt_row, P.d_n, P.d_off, P.d_roff, d_linv,
                       (const float *)nullptr, (const double *)nullptr, (const double *)P.d_y, R,
                       c0, ncols, P.d_spart);
    hipLaunchKernelGGL(split_reduce_kernel<true>, dim3(P.nrt, nct), dim3(256), 0, s, P.d_uptr,
                       P.d_rt_block, P.d_rt_row, P.d_n, P.d_roff,
                       (const double *)P.d_spart, R, c0, ncols, (double *)nullptr,
                       (double *)nullptr, dchi2);
  }
  return hipGetLastError();
}

}  // namespace fk
