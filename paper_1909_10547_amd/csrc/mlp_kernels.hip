// The PDF as the output of a neural network sampled on the x-grid, its
// gradient with respect to the network parameters, and the gradient-descent
// update: the steps either side of the convolution in a fit (Section 2: the
// fit trains a network parametrisation of the PDF by gradient descent;
// Section 3: the network generates the PDF on the grid that the FK tables
// are convolved with).  Every replica has its own network:
//
//   in(x)  = (x, ln x)
//   a1     = tanh(W1 in + b1)          [h1]
//   a2     = tanh(W2 a1 + b2)          [h2]
//   f_a(x) = x^alpha_a (1-x)^beta_a (W3 a2 + b3)_a
//
// Parameters of replica r at params[r][P] in the order W1 [h1][2], b1 [h1],
// W2 [h2][h1], b2 [h2], W3 [F][h2], b3 [F].  One workgroup per replica; the
// replica's parameters are staged in LDS.  Forward: thread alpha evaluates
// the network at x_alpha and writes f[a][alpha][r].  Backward: thread alpha
// runs the network and the reverse pass at x_alpha (the deltas of every
// layer into LDS), then thread p sums parameter p's gradient over alpha in
// order.  FP32 throughout.
#include <algorithm>

#include "runtime.h"

namespace fk {

namespace {

constexpr int kMlpThreads = 256;

struct MlpArgs {
  int F, X, h1, h2, P;
  const float *xin;  // [2][X]: x, ln x
  const float *pre;  // [F][X]: x^alpha (1-x)^beta
};

__device__ __forceinline__ void stage_params(float *sp, const float *params, int P, int r) {
  for (int p = threadIdx.x; p < P; p += kMlpThreads) sp[p] = params[(size_t)r * P + p];
}

// the two hidden layers at x index ``al`` into a1[h1], a2[h2]
__device__ __forceinline__ void hidden(const MlpArgs &A, const float *sp, int al, float *a1,
                                       float *a2) {
  const float *W1 = sp, *b1 = W1 + 2 * A.h1, *W2 = b1 + A.h1, *b2 = W2 + A.h2 * A.h1;
  const float x0 = A.xin[al], x1 = A.xin[A.X + al];
  for (int j = 0; j < A.h1; ++j) a1[j] = tanhf(W1[2 * j] * x0 + W1[2 * j + 1] * x1 + b1[j]);
  for (int k = 0; k < A.h2; ++k) {
    float z = b2[k];
    for (int j = 0; j < A.h1; ++j) z += W2[k * A.h1 + j] * a1[j];
    a2[k] = tanhf(z);
  }
}

__global__ void __launch_bounds__(kMlpThreads)
    mlp_forward_kernel(MlpArgs A, const float *__restrict__ params, int R, float *__restrict__ pdf) {
  extern __shared__ float sm[];
  const int r = blockIdx.x, al = threadIdx.x;
  float *sp = sm;
  stage_params(sp, params, A.P, r);
  __syncthreads();
  if (al >= A.X) return;
  float *a1 = sp + A.P + al * (A.h1 + A.h2), *a2 = a1 + A.h1;  // this thread's activations
  hidden(A, sp, al, a1, a2);
  const float *W3 = sp + 2 * A.h1 + A.h1 + A.h2 * A.h1 + A.h2, *b3 = W3 + A.F * A.h2;
  for (int a = 0; a < A.F; ++a) {
    float o = b3[a];
    for (int k = 0; k < A.h2; ++k) o += W3[a * A.h2 + k] * a2[k];
    pdf[((size_t)a * A.X + al) * R + r] = A.pre[a * A.X + al] * o;
  }
}

__global__ void __launch_bounds__(kMlpThreads)
    mlp_backward_kernel(MlpArgs A, const float *__restrict__ params, const float *__restrict__ gpdf,
                        int R, float *__restrict__ gparams) {
  extern __shared__ float sm[];
  const int r = blockIdx.x, t = threadIdx.x;
  const int h1 = A.h1, h2 = A.h2, F = A.F, X = A.X;
  float *sp = sm;
  float *a1 = sp + A.P;       // [X][h1]
  float *a2 = a1 + X * h1;    // [X][h2]
  float *d1 = a2 + X * h2;    // [X][h1]
  float *d2 = d1 + X * h1;    // [X][h2]
  float *dout = d2 + X * h2;  // [X][F]
  stage_params(sp, params, A.P, r);
  __syncthreads();
  const float *W1 = sp, *b1 = W1 + 2 * h1, *W2 = b1 + h1, *b2 = W2 + h2 * h1, *W3 = b2 + h2;
  (void)b1;
  (void)b2;
  if (t < X) {
    const int al = t;
    float *A1 = a1 + al * h1, *A2 = a2 + al * h2, *D1 = d1 + al * h1, *D2 = d2 + al * h2,
          *DO = dout + al * F;
    hidden(A, sp, al, A1, A2);
    for (int a = 0; a < F; ++a) DO[a] = gpdf[((size_t)a * X + al) * R + r] * A.pre[a * X + al];
    for (int k = 0; k < h2; ++k) {
      float s = 0.f;
      for (int a = 0; a < F; ++a) s += W3[a * h2 + k] * DO[a];
      D2[k] = s * (1.f - A2[k] * A2[k]);
    }
    for (int j = 0; j < h1; ++j) {
      float s = 0.f;
      for (int k = 0; k < h2; ++k) s += W2[k * h1 + j] * D2[k];
      D1[j] = s * (1.f - A1[j] * A1[j]);
    }
  }
  __syncthreads();
  // parameter p: its gradient summed over the grid points in order
  const int oW1 = 0, ob1 = 2 * h1, oW2 = ob1 + h1, ob2 = oW2 + h2 * h1, oW3 = ob2 + h2,
            ob3 = oW3 + F * h2;
  for (int p = t; p < A.P; p += kMlpThreads) {
    float g = 0.f;
    if (p < ob1) {
      const int j = (p - oW1) >> 1, i = (p - oW1) & 1;
      for (int al = 0; al < X; ++al) g += d1[al * h1 + j] * A.xin[i * X + al];
    } else if (p < oW2) {
      const int j = p - ob1;
      for (int al = 0; al < X; ++al) g += d1[al * h1 + j];
    } else if (p < ob2) {
      const int k = (p - oW2) / h1, j = (p - oW2) % h1;
      for (int al = 0; al < X; ++al) g += d2[al * h2 + k] * a1[al * h1 + j];
    } else if (p < oW3) {
      const int k = p - ob2;
      for (int al = 0; al < X; ++al) g += d2[al * h2 + k];
    } else if (p < ob3) {
      const int a = (p - oW3) / h2, k = (p - oW3) % h2;
      for (int al = 0; al < X; ++al) g += dout[al * F + a] * a2[al * h2 + k];
    } else {
      const int a = p - ob3;
      for (int al = 0; al < X; ++al) g += dout[al * F + a];
    }
    gparams[(size_t)r * A.P + p] = g;
  }
}

__global__ void __launch_bounds__(kMlpThreads)
    sgd_kernel(float *__restrict__ params, const float *__restrict__ grad, int64_t n, float lr) {
  const int64_t i = (int64_t)blockIdx.x * kMlpThreads + threadIdx.x;
  if (i < n) params[i] -= lr * grad[i];
}

}  // namespace

size_t mlp_lds_bytes(int F, int X, int h1, int h2, bool backward) {
  const size_t P = (size_t)mlp_nparams(F, h1, h2);
  if (backward) return (P + (size_t)X * (2 * h1 + 2 * h2 + F)) * sizeof(float);
  return (P + (size_t)X * (h1 + h2)) * sizeof(float);
}

int mlp_nparams(int F, int h1, int h2) { return 2 * h1 + h1 + h2 * h1 + h2 + F * h2 + F; }

hipError_t launch_mlp_forward(const MlpDev &m, const float *params, int R, float *pdf, hipStream_t s) {
  const MlpArgs A{m.F, m.X, m.h1, m.h2, mlp_nparams(m.F, m.h1, m.h2), m.d_xin, m.d_pre};
  const size_t lds = mlp_lds_bytes(m.F, m.X, m.h1, m.h2, false);
  hipError_t e = hipSuccess;
  if (lds > 65536)
    e = hipFuncSetAttribute((const void *)mlp_forward_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(R), dim3(kMlpThreads), lds, s, A, params, R, pdf);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const MlpDev &m, const float *params, const float *gpdf, int R,
                               float *gparams, hipStream_t s) {
  const MlpArgs A{m.F, m.X, m.h1, m.h2, mlp_nparams(m.F, m.h1, m.h2), m.d_xin, m.d_pre};
  const size_t lds = mlp_lds_bytes(m.F, m.X, m.h1, m.h2, true);
  hipError_t e = hipSuccess;
  if (lds > 65536)
    e = hipFuncSetAttribute((const void *)mlp_backward_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_backward_kernel, dim3(R), dim3(kMlpThreads), lds, s, A, params, gpdf, R, gparams);
  return hipGetLastError();
}

hipError_t launch_sgd(float *params, const float *grad, int64_t n, float lr, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sgd_kernel, dim3((unsigned)((n + kMlpThreads - 1) / kMlpThreads)), dim3(kMlpThreads),
                     0, s, params, grad, n, lr);
  return hipGetLastError();
}

}  // namespace fk
