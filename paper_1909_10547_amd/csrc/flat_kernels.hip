// The flattened form of the hadronic convolution that Table 3 of the paper
// times: the PDF enters as a "luminosity" matrix L[K][R] with one row per
// (active flavour pair c = (a, b), x index alpha, x index beta), K = npairs
// * nx * nx (49 pairs on a 27-point grid give the table's K = 35721), and the
// observables are the plain product out[N][R] = FK[N][K] L[K][R].  This is
// the like-for-like counterpart of Table 3; the main path never forms L
// (it contracts S f on the matrix cores and dots with f in the epilogue).
//
// Kernels (FP32 in, FP32 accumulation, fixed summation order):
//  * lumi_kernel: L[(c, alpha, beta)][r] = f[a_c][alpha][r] f[b_c][beta][r].
//  * flat_stream_kernel: few rows or few columns (N <= 16 or R <= 16).  The
//    product is bound by streaming FK or L from HBM, so it runs on the
//    vector units: a block owns up to NB rows, CW columns and a chunk of
//    K; its 256 threads are CW columns x (256 / CW) k-lanes, each thread
//    accumulates the block's rows of its column over k = lane (mod lanes),
//    and the lanes are combined by a fixed tree in LDS.
//  * flat_mfma_kernel: N > 16 and R > 16, a dense product on the matrix
//    cores: 128 x 128 output tiles per workgroup (2 x 2 waves of 64 x 64),
//    stages of 32 k double-buffered through LDS, v_mfma_f32_16x16x4f32.
// Both write partial sums per K-chunk when K is split over workgroups;
// flat_reduce_kernel adds the chunks in order.
#include <algorithm>

#include "runtime.h"

namespace fk {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kFlatThreads = 256;

__global__ void __launch_bounds__(kFlatThreads)
    lumi_kernel(FlatPairs pairs, int nx, int R, const float *__restrict__ pdf,
                float *__restrict__ lum, int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * kFlatThreads + threadIdx.x;
  if (idx >= total) return;
  const int r = (int)(idx % R);
  const int64_t k = idx / R;
  const int xx = nx * nx;
  const int c = (int)(k / xx);
  const int rem = (int)(k - (int64_t)c * xx);
  const int al = rem / nx, be = rem - al * nx;
  const int a = pairs.ab[c] >> 6, b = pairs.ab[c] & 63;
  lum[idx] = pdf[((int64_t)a * nx + al) * R + r] * pdf[((int64_t)b * nx + be) * R + r];
}

// NB rows x (CW * VEC) columns x one K-chunk per block; thread (c, kl)
// owns columns VEC*c .. VEC*c+VEC-1 of the block (one 16-byte load of L when
// VEC = 4) and k = kl (mod KL); see the file comment.
template <int NB, int CW, int VEC>
__global__ void __launch_bounds__(kFlatThreads)
    flat_stream_kernel(const float *__restrict__ fk, const float *__restrict__ lum, int64_t N,
                       int64_t K, int64_t R, int64_t kchunk, float *__restrict__ part) {
  constexpr int KL = kFlatThreads / CW;
  __shared__ float red[kFlatThreads * NB * VEC];
  const int t = threadIdx.x, c = t % CW;
  // with CW = 64 the k-lane is the wave index: uniform, so the FK loads
  // are the same address for the whole wave
  const int kl = CW % 64 == 0 ? __builtin_amdgcn_readfirstlane(t / CW) : t / CW;
  const int64_t col = ((int64_t)blockIdx.x * CW + c) * VEC;
  const int64_t n0 = (int64_t)blockIdx.y * NB;
  const int nrows = (int)std::min<int64_t>(NB, N - n0);
  const int64_t k0 = (int64_t)blockIdx.z * kchunk;
  const int64_t k1 = std::min(K, k0 + kchunk);
  float acc[NB][VEC];
#pragma unroll
  for (int n = 0; n < NB; ++n)
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[n][v] = 0.f;
  const float *frow = fk + n0 * K;
  for (int64_t k = k0 + kl; k < k1; k += KL) {
    float l[VEC];
    if (VEC == 4) {
      // R % 4 == 0 for this form (the host checks), so col < R covers all four
      const float4 v4 = col < R ? *(const float4 *)(lum + k * R + col) : float4{0.f, 0.f, 0.f, 0.f};
      l[0] = v4.x;
      l[1 % VEC] = v4.y;
      l[2 % VEC] = v4.z;
      l[3 % VEC] = v4.w;
    } else {
      l[0] = col < R ? lum[k * R + col] : 0.f;
    }
#pragma unroll
    for (int n = 0; n < NB; ++n)
      if (n < nrows) {
        const float a = frow[n * K + k];
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[n][v] += a * l[v];
      }
  }
#pragma unroll
  for (int n = 0; n < NB; ++n)
#pragma unroll
    for (int v = 0; v < VEC; ++v) red[((kl * NB + n) * CW + c) * VEC + v] = acc[n][v];
  __syncthreads();
  // fixed tree over the k-lanes: lane j adds lane j + s
  for (int s = KL / 2; s > 0; s >>= 1) {
    if (kl < s) {
#pragma unroll
      for (int n = 0; n < NB; ++n)
#pragma unroll
        for (int v = 0; v < VEC; ++v)
          red[((kl * NB + n) * CW + c) * VEC + v] += red[(((kl + s) * NB + n) * CW + c) * VEC + v];
    }
    __syncthreads();
  }
  if (kl == 0) {
    float *dst = part + ((int64_t)blockIdx.z * N + n0) * R;
    for (int n = 0; n < nrows; ++n)
#pragma unroll
      for (int v = 0; v < VEC; ++v)
        if (col + v < R) dst[n * R + col + v] = red[(n * CW + c) * VEC + v];
  }
}

// 128 x 128 output tile per workgroup, K-chunk blockIdx.z; see the file
// comment.  Four waves in 2 x 2, each 64 x 64 = 4 x 4 tiles of
// v_mfma_f32_16x16x4f32.  K advances in stages of 32 through two LDS
// buffers: the global loads of stage s + 1 are in flight while stage s is
// multiplied, and one barrier per stage separates the two.  Inside a stage,
// k-step q of lane group g takes k = 16 (q / 4) + 4 g + q % 4 (any order
// that A and B share is the same sum), so a lane reads its A values of four
// k-steps as one 16-byte LDS read.  VB = 4 loads L in 16-byte vectors (R %
// 4 == 0 and a 16-byte aligned L), VB = 1 element by element.
constexpr int kMT = 128, kBK = 32, kApad = kBK + 4, kBpad = kMT + 4;

template <int VB>
__global__ void __launch_bounds__(kFlatThreads)
    flat_mfma_kernel(const float *__restrict__ fk, const float *__restrict__ lum, int64_t N,
                     int64_t K, int64_t R, int64_t kchunk, float *__restrict__ part) {
  __shared__ __attribute__((aligned(16))) float As[2][kMT][kApad];  // [row][k]
  __shared__ __attribute__((aligned(16))) float Bs[2][kBK][kBpad];  // [k][column]
  const int t = threadIdx.x, w = t >> 6, lane = t & 63, g = lane >> 4, l16 = lane & 15;
  const int64_t m0 = (int64_t)blockIdx.y * kMT, c0 = (int64_t)blockIdx.x * kMT;
  const int64_t ks = (int64_t)blockIdx.z * kchunk, ke = std::min(K, ks + kchunk);
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
  // A: thread t loads k = t % 32 of rows t / 32 + 8 p; B: k-row t / 32 + 8 p
  // (VB = 4: columns 4 (t % 32) .. + 3; VB = 1: columns t % 32 + 32 j)
  const int ak = t & 31, ar = t >> 5;
  constexpr int kBL = VB == 4 ? 4 : 16;
  float ra[16], rb[kBL * VB];
  auto load = [&](int64_t kk) {
    const int64_t gk = kk + ak;
#pragma unroll
    for (int p = 0; p < 16; ++p) {
      const int64_t gr = m0 + ar + 8 * p;
      ra[p] = gr < N && gk < ke ? fk[gr * K + gk] : 0.f;
    }
    if (VB == 4) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int64_t gk2 = kk + ar + 8 * p, gc = c0 + 4 * ak;
        const float4 v = gk2 < ke && gc < R ? *(const float4 *)(lum + gk2 * R + gc) : float4{0.f, 0.f, 0.f, 0.f};
        rb[4 * p] = v.x;
        rb[4 * p + 1] = v.y;
        rb[4 * p + 2] = v.z;
        rb[4 * p + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t gk2 = kk + ar + 8 * p, gc = c0 + ak + 32 * j;
          rb[4 * p + j] = gk2 < ke && gc < R ? lum[gk2 * R + gc] : 0.f;
        }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < 16; ++p) As[buf][ar + 8 * p][ak] = ra[p];
    if (VB == 4) {
#pragma unroll
      for (int p = 0; p < 4; ++p)
        *(f32x4 *)&Bs[buf][ar + 8 * p][4 * ak] = f32x4{rb[4 * p], rb[4 * p + 1], rb[4 * p + 2], rb[4 * p + 3]};
    } else {
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int j = 0; j < 4; ++j) Bs[buf][ar + 8 * p][ak + 32 * j] = rb[4 * p + j];
    }
  };
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int nst = (int)((ke - ks + kBK - 1) / kBK);
  load(ks);
  store(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    if (st + 1 < nst) load(ks + (int64_t)(st + 1) * kBK);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      f32x4 a[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = *(const f32x4 *)&As[buf][wm + 16 * i + l16][16 * h + 4 * g];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = Bs[buf][16 * h + 4 * g + q][wn + 16 * j + l16];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][q], b[j], acc[i][j], 0, 0, 0);
      }
    }
    if (st + 1 < nst) store(buf ^ 1);
    __syncthreads();
  }
  float *dst = part + (int64_t)blockIdx.z * N * R;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t row = m0 + wm + 16 * i + 4 * g + q, col = c0 + wn + 16 * j + l16;
        if (row < N && col < R) dst[row * R + col] = acc[i][j][q];
      }
}

// Sum of the K-chunks of every output, chunk after chunk.
__global__ void __launch_bounds__(kFlatThreads)
    flat_reduce_kernel(const float *__restrict__ part, int ks, int64_t nr, float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kFlatThreads + threadIdx.x;
  if (i >= nr) return;
  float s = 0.f;
  for (int z = 0; z < ks; ++z) s += part[(int64_t)z * nr + i];
  out[i] = s;
}

// The same for few outputs and many chunks: one wave per output, lane j
// sums chunks j, j + 64, ... in order, then a fixed tree over the lanes.
__global__ void __launch_bounds__(64)
    flat_reduce_wave_kernel(const float *__restrict__ part, int ks, int64_t nr, float *__restrict__ out) {
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x;
  float s = 0.f;
  for (int z = lane; z < ks; z += 64) s += part[(int64_t)z * nr + i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) out[i] = s;
}

}  // namespace

FlatPlan flat_plan(int64_t N, int64_t K, int64_t R, int ncu) {
  FlatPlan p;
  p.mfma = N > 16 && R > 16;
  int64_t tiles;
  int64_t min_chunk;
  if (p.mfma) {
    p.gx = (R + kMT - 1) / kMT;
    p.gy = (N + kMT - 1) / kMT;
    tiles = p.gx * p.gy;
    min_chunk = 4 * kBK;  // at least four stages per workgroup
  } else {
    p.nb = N <= 8 ? 8 : 16;
    p.cw = 1;
    while (p.cw < R && p.cw < 64) p.cw *= 2;
    // wide outputs: four columns per thread, one 16-byte load of L
    p.vec = (R >= 256 && R % 4 == 0) ? 4 : 1;
    p.gx = (R + p.cw * p.vec - 1) / (p.cw * p.vec);
    p.gy = (N + p.nb - 1) / p.nb;
    tiles = p.gx * p.gy;
    min_chunk = 16 * (kFlatThreads / p.cw);  // at least 16 k per thread
  }
  // split K until the grid has about 16 workgroups per compute unit (4 for
  // the matrix-core tiles, which hold 2 per unit at a time)
  const int64_t want = (p.mfma ? 4LL : 16LL) * ncu;
  int64_t ks = std::max<int64_t>(1, want / std::max<int64_t>(tiles, 1));
  ks = std::min<int64_t>(ks, std::max<int64_t>(1, (K + min_chunk - 1) / min_chunk));
  ks = std::min<int64_t>(ks, 65535);
  int64_t chunk = (K + ks - 1) / ks;
  const int64_t q = p.mfma ? kBK : 1;
  chunk = (chunk + q - 1) / q * q;
  p.kchunk = chunk;
  p.ks = (int)((K + chunk - 1) / chunk);
  p.work_bytes = p.ks > 1 ? (uint64_t)p.ks * N * R * sizeof(float) : 0;
  return p;
}

hipError_t launch_lumi(const FlatPairs &pairs, int nx, int R, const float *pdf, float *lum,
                       hipStream_t s) {
  const int64_t total = (int64_t)pairs.n * nx * nx * R;
  if (total <= 0) return hipSuccess;
  const int64_t blocks = (total + kFlatThreads - 1) / kFlatThreads;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lumi_kernel, dim3((unsigned)blocks), dim3(kFlatThreads), 0, s, pairs, nx, R,
                     pdf, lum, total);
  return hipGetLastError();
}

hipError_t launch_flat(const FlatPlan &p, int64_t N, int64_t K, int64_t R, const float *fk,
                       const float *lum, float *out, float *work, hipStream_t s) {
  float *part = p.ks > 1 ? work : out;
  const dim3 grid((unsigned)p.gx, (unsigned)p.gy, (unsigned)p.ks);
  if (p.mfma) {
    if (R % 4 == 0 && ((uintptr_t)lum & 15) == 0)
      hipLaunchKernelGGL(flat_mfma_kernel<4>, grid, dim3(kFlatThreads), 0, s, fk, lum, N, K, R,
                         p.kchunk, part);
    else
      hipLaunchKernelGGL(flat_mfma_kernel<1>, grid, dim3(kFlatThreads), 0, s, fk, lum, N, K, R,
                         p.kchunk, part);
  } else {
#define FK_FLAT(NB, CW)                                                                          \
  if (p.vec == 4)                                                                                  \
    hipLaunchKernelGGL((flat_stream_kernel<NB, CW, 4>), grid, dim3(kFlatThreads), 0, s, fk, lum, N, \
                       K, R, p.kchunk, part);                                                       \
  else                                                                                             \
    hipLaunchKernelGGL((flat_stream_kernel<NB, CW, 1>), grid, dim3(kFlatThreads), 0, s, fk, lum, N, \
                       K, R, p.kchunk, part)
#define FK_FLAT_CW(NB)                      \
  switch (p.cw) {                           \
    case 1: FK_FLAT(NB, 1); break;          \
    case 2: FK_FLAT(NB, 2); break;          \
    case 4: FK_FLAT(NB, 4); break;          \
    case 8: FK_FLAT(NB, 8); break;          \
    case 16: FK_FLAT(NB, 16); break;        \
    case 32: FK_FLAT(NB, 32); break;        \
    case 64: FK_FLAT(NB, 64); break;        \
    default: return hipErrorInvalidValue;   \
  }
    if (p.nb == 8) {
      FK_FLAT_CW(8);
    } else {
      FK_FLAT_CW(16);
    }
#undef FK_FLAT_CW
#undef FK_FLAT
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || p.ks == 1) return e;
  const int64_t nr = N * R;
  if (nr <= 16384 && p.ks >= 64)
    hipLaunchKernelGGL(flat_reduce_wave_kernel, dim3((unsigned)nr), dim3(64), 0, s, work, p.ks, nr, out);
  else
    hipLaunchKernelGGL(flat_reduce_kernel, dim3((unsigned)((nr + kFlatThreads - 1) / kFlatThreads)),
                       dim3(kFlatThreads), 0, s, work, p.ks, nr, out);
  return hipGetLastError();
}

}  // namespace fk
