// Learned pool screener kernels (float32): per-operator features, the
// 16 -> 128 -> 128 -> 1 ReLU MLP forward and backward passes, mean squared
// error and Adam.  Parameters are one flat vector:
//   W1[16][128] | b1[128] | W2[128][128] | b2[128] | W3[128] | b3[1]
// (row-major, input index first).  Each block handles 32 rows; the backward
// pass writes per-block partial gradients that a second kernel sums in block
// order, so results are deterministic.
#include "swcs_internal.h"

namespace swcs {

constexpr int kIn = kMlpIn, kH = kMlpHidden, kRows = kMlpRowsPerBlock;
constexpr int oW1 = 0, ob1 = oW1 + kIn * kH, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH,
              ob3 = oW3 + kH;

__global__ void __launch_bounds__(256)
k_features(const OpDesc* __restrict__ ops, long long K, const double* __restrict__ fock,
           const double* __restrict__ eri, int n, const double* __restrict__ occ,
           const float* __restrict__ prev_absg, const float* __restrict__ age,
           const float* __restrict__ count, float* __restrict__ feat) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const OpDesc op = ops[k];
  const int idx[4] = {op.P, op.Q, op.R, op.S};
  const double norm = occ[2 * n];
  float f[16];
  for (int t = 0; t < 16; ++t) f[t] = 0.0f;
  for (int t = 0; t < 4; ++t) {
    if (idx[t] >= 0) {
      const int p = idx[t] >> 1;
      f[t] = (float)fock[p * n + p];
      f[5 + t] = (float)(occ[idx[t]] / norm);
    }
  }
  if (op.R < 0) {
    f[4] = (float)fabs(fock[(op.P >> 1) * n + (op.Q >> 1)]);
    f[12] = 1.0f;
  } else {
    const int p = op.P >> 1, q = op.Q >> 1, r = op.R >> 1, s = op.S >> 1;
    f[4] = (float)fabs(eri[((size_t)(p * n + r) * n + q) * n + s]);
    if (((op.P ^ op.Q) & 1) == 0) f[13] = 1.0f; else f[14] = 1.0f;
  }
  const float g = prev_absg[k];
  f[9] = g;
  f[10] = log10f(g + 1e-16f);
  f[11] = age[k] / 10.0f;
  f[15] = count[k];
  float4* out = (float4*)(feat + 16 * k);
  out[0] = make_float4(f[0], f[1], f[2], f[3]);
  out[1] = make_float4(f[4], f[5], f[6], f[7]);
  out[2] = make_float4(f[8], f[9], f[10], f[11]);
  out[3] = make_float4(f[12], f[13], f[14], f[15]);
}

// Closed-shell Fock matrix f_pq = h_pq + sum_{j < n_occ} [2 (pq|jj) - (pj|jq)].
__global__ void k_fock(const double* __restrict__ h, const double* __restrict__ eri, int n,
                       int n_occ, double* __restrict__ fock) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  const int p = t / n, q = t % n;
  double v = h[t];
  for (int j = 0; j < n_occ; ++j)
    v += 2.0 * eri[((size_t)(p * n + q) * n + j) * n + j] - eri[((size_t)(p * n + j) * n + j) * n + q];
  fock[t] = v;
}

__global__ void __launch_bounds__(256)
k_mlp_forward(const float* __restrict__ W, const float* __restrict__ x, long long B,
              float* __restrict__ y, float* __restrict__ act) {
  __shared__ float sx[kRows][kIn];
  __shared__ float a1[kRows][kH + 1];
  __shared__ float a2[kRows][kH + 1];
  __shared__ float yp[kRows][8];
  const long long r0 = (long long)blockIdx.x * kRows;
  const int tid = threadIdx.x;
  for (int t = tid; t < kRows * kIn; t += 256) {
    const long long r = r0 + t / kIn;
    sx[t / kIn][t % kIn] = (r < B) ? x[r * kIn + t % kIn] : 0.0f;
  }
  __syncthreads();
  const int u = tid & (kH - 1);
  const int rb = tid >> 7;  // 0 or 1
  {
    float acc[kRows / 2];
    const float b = W[ob1 + u];
    for (int j = 0; j < kRows / 2; ++j) acc[j] = b;
    for (int i = 0; i < kIn; ++i) {
      const float w = W[oW1 + i * kH + u];
      for (int j = 0; j < kRows / 2; ++j) acc[j] += sx[rb + 2 * j][i] * w;
    }
    for (int j = 0; j < kRows / 2; ++j) a1[rb + 2 * j][u] = fmaxf(acc[j], 0.0f);
  }
  __syncthreads();
  {
    float acc[kRows / 2];
    const float b = W[ob2 + u];
    for (int j = 0; j < kRows / 2; ++j) acc[j] = b;
    for (int k = 0; k < kH; ++k) {
      const float w = W[oW2 + k * kH + u];
      for (int j = 0; j < kRows / 2; ++j) acc[j] += a1[rb + 2 * j][k] * w;
    }
    for (int j = 0; j < kRows / 2; ++j) a2[rb + 2 * j][u] = fmaxf(acc[j], 0.0f);
  }
  __syncthreads();
  {
    const int r = tid >> 3, c = tid & 7;
    float s = 0.0f;
    for (int k = c * 16; k < c * 16 + 16; ++k) s += a2[r][k] * W[oW3 + k];
    yp[r][c] = s;
  }
  __syncthreads();
  if (tid < kRows) {
    float s = W[ob3];
    for (int c = 0; c < 8; ++c) s += yp[tid][c];
    if (r0 + tid < B) y[r0 + tid] = s;
  }
  if (act) {
    for (int t = tid; t < kRows * kH; t += 256) {
      const int r = t / kH, k = t % kH;
      if (r0 + r < B) {
        act[(r0 + r) * (2 * kH) + k] = a1[r][k];
        act[(r0 + r) * (2 * kH) + kH + k] = a2[r][k];
      }
    }
  }
}

// Per-block partial gradient of sum_b dy_b y_b into partial[block][P].
__global__ void __launch_bounds__(256)
k_mlp_backward_partial(const float* __restrict__ W, const float* __restrict__ x,
                       const float* __restrict__ act, const float* __restrict__ dy, long long B,
                       float* __restrict__ partial) {
  __shared__ float sx[kRows][kIn];
  __shared__ float a1[kRows][kH + 1];
  __shared__ float dz2[kRows][kH + 1];
  __shared__ float dz1[kRows][kH + 1];
  __shared__ float sdy[kRows];
  const long long r0 = (long long)blockIdx.x * kRows;
  const int tid = threadIdx.x;
  float* out = partial + (size_t)blockIdx.x * kMlpParams;
  for (int t = tid; t < kRows * kIn; t += 256) {
    const long long r = r0 + t / kIn;
    sx[t / kIn][t % kIn] = (r < B) ? x[r * kIn + t % kIn] : 0.0f;
  }
  if (tid < kRows) sdy[tid] = (r0 + tid < B) ? dy[r0 + tid] : 0.0f;
  for (int t = tid; t < kRows * kH; t += 256) {
    const int r = t / kH, k = t % kH;
    const bool ok = r0 + r < B;
    a1[r][k] = ok ? act[(r0 + r) * (2 * kH) + k] : 0.0f;
    const float a2v = ok ? act[(r0 + r) * (2 * kH) + kH + k] : 0.0f;
    dz2[r][k] = a2v;  // stash a2 here for the W3 gradient
  }
  __syncthreads();
  // dW3, db3 and dz2 = dy * W3 * [a2 > 0]
  if (tid < kH) {
    float s = 0.0f;
    for (int r = 0; r < kRows; ++r) s += dz2[r][tid] * sdy[r];
    out[oW3 + tid] = s;
  }
  if (tid == kH) {
    float s = 0.0f;
    for (int r = 0; r < kRows; ++r) s += sdy[r];
    out[ob3] = s;
  }
  __syncthreads();
  for (int t = tid; t < kRows * kH; t += 256) {
    const int r = t / kH, k = t % kH;
    const float a2v = dz2[r][k];
    dz2[r][k] = (a2v > 0.0f) ? sdy[r] * W[oW3 + k] : 0.0f;
  }
  __syncthreads();
  // dW2[k][u] = sum_r a1[r][k] dz2[r][u], db2
  for (int t = tid; t < kH * kH; t += 256) {
    const int k = t / kH, u = t % kH;
    float s = 0.0f;
    for (int r = 0; r < kRows; ++r) s += a1[r][k] * dz2[r][u];
    out[oW2 + t] = s;
  }
  if (tid < kH) {
    float s = 0.0f;
    for (int r = 0; r < kRows; ++r) s += dz2[r][tid];
    out[ob2 + tid] = s;
  }
  // dz1[r][k] = (sum_u dz2[r][u] W2[k][u]) [a1 > 0]
  for (int t = tid; t < kRows * kH; t += 256) {
    const int r = t / kH, k = t % kH;
    float s = 0.0f;
    for (int u = 0; u < kH; ++u) s += dz2[r][u] * W[oW2 + k * kH + u];
    dz1[r][k] = (a1[r][k] > 0.0f) ? s : 0.0f;
  }
  __syncthreads();
  for (int t = tid; t < kIn * kH; t += 256) {
    const int i = t / kH, k = t % kH;
    float s = 0.0f;
    for (int r = 0; r < kRows; ++r) s += sx[r][i] * dz1[r][k];
    out[oW1 + t] = s;
  }
  if (tid < kH) {
    float s = 0.0f;
    for (int r = 0; r < kRows; ++r) s += dz1[r][tid];
    out[ob1 + tid] = s;
  }
}

__global__ void k_sum_partials_f32(const float* __restrict__ partial, long long rows, long long P,
                                   float* __restrict__ out) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float s = 0.0f;
  for (long long b = 0; b < rows; ++b) s += partial[b * P + p];
  out[p] = s;
}

__global__ void __launch_bounds__(256)
k_mse(const float* __restrict__ y, const float* __restrict__ t, long long B, float* __restrict__ dy,
      float* __restrict__ loss) {
  __shared__ float red[256];
  float s = 0.0f;
  const float inv = 1.0f / (float)B;
  for (long long i = threadIdx.x; i < B; i += 256) {
    const float r = y[i] - t[i];
    s += r * r;
    dy[i] = 2.0f * r * inv;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] * inv;
}

__global__ void k_adam(float* __restrict__ W, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, long long P, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  W[i] -= lr * mh / (sqrtf(vh) + eps);
}

hipError_t launch_fock(const double* h, const double* eri, int n, int n_occ, double* fock,
                       hipStream_t stream) {
  hipLaunchKernelGGL(k_fock, dim3((n * n + 255) / 256), dim3(256), 0, stream, h, eri, n, n_occ, fock);
  return hipGetLastError();
}

hipError_t launch_features(const OpDesc* ops, long long K, const double* fock, const double* eri,
                           int n, const double* occ, const float* prev_absg, const float* age,
                           const float* count, float* feat, hipStream_t stream) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, stream, ops, K,
                     fock, eri, n, occ, prev_absg, age, count, feat);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* W, const float* x, long long B, float* y, float* act,
                              hipStream_t stream) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((B + kRows - 1) / kRows)), dim3(256), 0, stream,
                     W, x, B, y, act);
  return hipGetLastError();
}

long long mlp_backward_partial_rows(long long B) { return (B + kRows - 1) / kRows; }

hipError_t launch_mlp_backward(const float* W, const float* x, const float* act, const float* dy,
                               long long B, float* dW, float* partial, long long partial_rows,
                               hipStream_t stream) {
  const long long blocks = mlp_backward_partial_rows(B);
  if (blocks > partial_rows) return hipErrorInvalidValue;
  if (B > 0)
    hipLaunchKernelGGL(k_mlp_backward_partial, dim3((unsigned)blocks), dim3(256), 0, stream, W, x,
                       act, dy, B, partial);
  hipLaunchKernelGGL(k_sum_partials_f32, dim3((unsigned)((kMlpParams + 255) / 256)), dim3(256), 0,
                     stream, partial, blocks, (long long)kMlpParams, dW);
  return hipGetLastError();
}

hipError_t launch_mse(const float* y, const float* t, long long B, float* dy, float* loss,
                      hipStream_t stream) {
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, stream, y, t, B, dy, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* W, float* m, float* v, const float* g, long long P, float lr,
                       float b1, float b2, float eps, int step, hipStream_t stream) {
  const float c1 = 1.0f - powf(b1, (float)step);
  const float c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, stream, W, m, v, g, P,
                     lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace swcs
