// Learned pool screener kernels (float32): per-operator features, the
// 16 -> 128 -> 128 -> 1 ReLU MLP forward and backward passes, mean squared
// error and Adam.  Parameters are one flat vector:
//   W1[16][128] | b1[128] | W2[128][128] | b2[128] | W3[128] | b3[1]
// (row-major, input index first).  The backward pass writes per-block
// partial gradients that a second kernel sums in block order, so results are
// deterministic.
#include "swcs_internal.h"

namespace swcs {

constexpr int kIn = kMlpIn, kH = kMlpHidden;
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

// The dense layers run on the FP32 matrix cores: one 16x16x4 step adds
// A (16x4) times B (4x16) to a 16x16 accumulator held as four floats per
// lane.  Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[4 (l / 16) + r][l % 16] in acc[r].
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline f32x4 mma4(float a, float b, f32x4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}

// LDS row strides (floats): 132 spreads the 16 rows a lane group reads in the
// "row = l % 16" pattern over distinct banks, 144 spreads the 4 rows of the
// "row = l / 16" pattern.
constexpr int kStrideRowLane = kH + 4;
constexpr int kStrideColLane = kH + 16;
constexpr int kFwdRows = 64;       // rows per block iteration, 16 per wavefront
constexpr int kBwdRows = 32;       // rows per block iteration of the backward pass
constexpr int kMlpMaxBlocks = 256;

// Forward pass: a1 = relu(x W1 + b1), a2 = relu(a1 W2 + b2), y = a2 W3 + b3;
// act (optional) receives [a1 | a2] per row for the backward pass.  Each
// wavefront computes 16 rows: 8 column tiles of 16, 4 k-steps for layer 1 and
// 32 for layer 2; the weights are staged in LDS once per block.
__global__ void __launch_bounds__(256)
k_mlp_forward(const float* __restrict__ W, const float* __restrict__ x, long long B,
              float* __restrict__ y, float* __restrict__ act) {
  __shared__ float w1s[kIn][kStrideColLane];
  __shared__ float w2s[kH][kStrideColLane];
  __shared__ float a1t[4][16][kStrideRowLane];
  __shared__ float b1s[kH], b2s[kH], w3s[kH];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  for (int t = tid; t < kIn * kH; t += 256) w1s[t / kH][t % kH] = W[oW1 + t];
  for (int t = tid; t < kH * kH; t += 256) w2s[t / kH][t % kH] = W[oW2 + t];
  if (tid < kH) {
    b1s[tid] = W[ob1 + tid];
    b2s[tid] = W[ob2 + tid];
    w3s[tid] = W[oW3 + tid];
  }
  const float b3 = W[ob3];
  __syncthreads();
  const long long groups = (B + kFwdRows - 1) / kFwdRows;
  for (long long g = blockIdx.x; g < groups; g += gridDim.x) {
    const long long r0 = g * kFwdRows + 16 * wave;
    {
      const long long ra = r0 + li;
      float xa[4];
      for (int s = 0; s < 4; ++s) xa[s] = (ra < B) ? x[ra * kIn + 4 * s + lk] : 0.0f;
      for (int t = 0; t < 8; ++t) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int s = 0; s < 4; ++s) acc = mma4(xa[s], w1s[4 * s + lk][16 * t + li], acc);
        for (int r = 0; r < 4; ++r)
          a1t[wave][4 * lk + r][16 * t + li] = fmaxf(acc[r] + b1s[16 * t + li], 0.0f);
      }
    }
    __syncthreads();
    f32x4 acc[8];
    for (int t = 0; t < 8; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int s = 0; s < kH / 4; ++s) {
      const float a = a1t[wave][li][4 * s + lk];
      for (int t = 0; t < 8; ++t) acc[t] = mma4(a, w2s[4 * s + lk][16 * t + li], acc[t]);
    }
    float ys[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int t = 0; t < 8; ++t) {
      const int col = 16 * t + li;
      for (int r = 0; r < 4; ++r) {
        const float a2 = fmaxf(acc[t][r] + b2s[col], 0.0f);
        acc[t][r] = a2;
        ys[r] += a2 * w3s[col];
      }
    }
    for (int r = 0; r < 4; ++r)
      for (int off = 1; off < 16; off <<= 1) ys[r] += __shfl_xor(ys[r], off);
    if (li == 0) {
      for (int r = 0; r < 4; ++r) {
        const long long row = r0 + 4 * lk + r;
        if (row < B) y[row] = ys[r] + b3;
      }
    }
    if (act) {
      for (int t = 0; t < 8; ++t) {
        for (int r = 0; r < 4; ++r) {
          const long long row = r0 + 4 * lk + r;
          if (row < B) {
            act[row * (2 * kH) + 16 * t + li] = a1t[wave][4 * lk + r][16 * t + li];
            act[row * (2 * kH) + kH + 16 * t + li] = acc[t][r];
          }
        }
      }
    }
    __syncthreads();
  }
}

// Per-block partial gradient of sum_b dy_b y_b into partial[block][P].  Per
// group of 32 rows:
//   dz2 = dy W3^T [a2 > 0]               (elementwise, thread per column)
//   dz1 = (dz2 W2^T) [a1 > 0]            (matrix cores, wavefront w: columns 32w..32w+31)
//   dW2 += a1^T dz2, dW1 += x^T dz1      (matrix cores, wavefront w: rows 32w.. of dW2,
//                                         columns 32w.. of dW1; accumulators in registers)
// plus the column sums for b1, b2, W3 and b3.  Fixed summation order.
__global__ void __launch_bounds__(256)
k_mlp_backward_partial(const float* __restrict__ W, const float* __restrict__ x,
                       const float* __restrict__ act, const float* __restrict__ dy, long long B,
                       float* __restrict__ partial) {
  __shared__ float w2s[kH][kStrideRowLane];
  __shared__ float a1s[kBwdRows][kStrideColLane];
  __shared__ float dz2s[kBwdRows][kStrideRowLane];
  __shared__ float dz1s[kBwdRows][kStrideColLane];
  __shared__ float xs[kBwdRows][kIn];
  __shared__ float dys[kBwdRows];
  __shared__ float red[3][2][kH];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  const int u = tid & (kH - 1), half = tid >> 7;
  for (int t = tid; t < kH * kH; t += 256) w2s[t / kH][t % kH] = W[oW2 + t];
  const float w3u = W[oW3 + u];
  f32x4 acc2[2][8], acc1[2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 8; ++j) acc2[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  acc1[0] = acc1[1] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  float gW3 = 0.0f, gb2 = 0.0f, gb1 = 0.0f, gb3 = 0.0f;
  const long long groups = (B + kBwdRows - 1) / kBwdRows;
  for (long long g = blockIdx.x; g < groups; g += gridDim.x) {
    const long long r0 = g * kBwdRows;
    __syncthreads();  // previous group consumed; w2s staged
    for (int t = tid; t < kBwdRows * kIn; t += 256) {
      const long long r = r0 + t / kIn;
      xs[t / kIn][t % kIn] = (r < B) ? x[r * kIn + t % kIn] : 0.0f;
    }
    if (tid < kBwdRows) dys[tid] = (r0 + tid < B) ? dy[r0 + tid] : 0.0f;
    for (int r = half; r < kBwdRows; r += 2) {
      const long long row = r0 + r;
      const bool ok = row < B;
      const float a1v = ok ? act[row * (2 * kH) + u] : 0.0f;
      const float a2v = ok ? act[row * (2 * kH) + kH + u] : 0.0f;
      const float d = ok ? dy[row] : 0.0f;
      const float z = (a2v > 0.0f) ? d * w3u : 0.0f;
      a1s[r][u] = a1v;
      dz2s[r][u] = z;
      gW3 += a2v * d;
      gb2 += z;
    }
    __syncthreads();
    if (tid == 0)
      for (int r = 0; r < kBwdRows; ++r) gb3 += dys[r];
    {
      f32x4 acc[2][2];
      for (int i = 0; i < 2; ++i) acc[i][0] = acc[i][1] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      for (int s = 0; s < kH / 4; ++s) {
        const float a0 = dz2s[li][4 * s + lk], a1 = dz2s[16 + li][4 * s + lk];
        for (int t = 0; t < 2; ++t) {
          const float b = w2s[32 * wave + 16 * t + li][4 * s + lk];
          acc[0][t] = mma4(a0, b, acc[0][t]);
          acc[1][t] = mma4(a1, b, acc[1][t]);
        }
      }
      for (int i = 0; i < 2; ++i)
        for (int t = 0; t < 2; ++t)
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * i + 4 * lk + r, col = 32 * wave + 16 * t + li;
            dz1s[row][col] = (a1s[row][col] > 0.0f) ? acc[i][t][r] : 0.0f;
          }
    }
    __syncthreads();
    for (int r = half; r < kBwdRows; r += 2) gb1 += dz1s[r][u];
    for (int s = 0; s < kBwdRows / 4; ++s) {
      const int rr = 4 * s + lk;
      const float a0 = a1s[rr][32 * wave + li], a1 = a1s[rr][32 * wave + 16 + li];
      for (int j = 0; j < 8; ++j) {
        const float b = dz2s[rr][16 * j + li];
        acc2[0][j] = mma4(a0, b, acc2[0][j]);
        acc2[1][j] = mma4(a1, b, acc2[1][j]);
      }
      const float ax = xs[rr][li];
      for (int t = 0; t < 2; ++t) acc1[t] = mma4(ax, dz1s[rr][32 * wave + 16 * t + li], acc1[t]);
    }
  }
  red[0][half][u] = gW3;
  red[1][half][u] = gb2;
  red[2][half][u] = gb1;
  __syncthreads();
  float* out = partial + (size_t)blockIdx.x * kMlpParams;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 8; ++j)
      for (int r = 0; r < 4; ++r)
        out[oW2 + (32 * wave + 16 * i + 4 * lk + r) * kH + 16 * j + li] = acc2[i][j][r];
  for (int t = 0; t < 2; ++t)
    for (int r = 0; r < 4; ++r) out[oW1 + (4 * lk + r) * kH + 32 * wave + 16 * t + li] = acc1[t][r];
  if (tid < kH) {
    out[oW3 + tid] = red[0][0][tid] + red[0][1][tid];
    out[ob2 + tid] = red[1][0][tid] + red[1][1][tid];
    out[ob1 + tid] = red[2][0][tid] + red[2][1][tid];
  }
  if (tid == 0) out[ob3] = gb3;
}

__global__ void k_sum_partials_f32(const float* __restrict__ partial, long long rows, long long P,
                                   float* __restrict__ out) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float s = 0.0f;
  for (long long b = 0; b < rows; ++b) s += partial[b * P + p];
  out[p] = s;
}

// Mean squared error and its gradient dy = 2 (y - t) / B: per-block partial
// sums of squares, then one block adds them in block order.
__global__ void __launch_bounds__(256)
k_mse_partial(const float* __restrict__ y, const float* __restrict__ t, long long B,
              float* __restrict__ dy, float* __restrict__ partial) {
  __shared__ float red[256];
  float s = 0.0f;
  const float inv = 1.0f / (float)B;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < B; i += (long long)gridDim.x * 256) {
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
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_mse_finish(const float* __restrict__ partial, int nblocks, long long B,
                             float* __restrict__ loss) {
  if (threadIdx.x != 0) return;
  float s = 0.0f;
  for (int b = 0; b < nblocks; ++b) s += partial[b];
  *loss = s / (float)B;
}

// Screener targets t = log10(|g| + 1e-12) (float64 arithmetic, float32 result).
// v[i] += sign * feat[i * 16 + col]: the screener's score and target offset
// by one feature column (log10 of the last exact |g|).
__global__ void k_add_feature(float* __restrict__ v, const float* __restrict__ feat, long long n, int col,
                              float sign, float scale) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = scale * v[i] + sign * feat[i * 16 + col];
}

__global__ void k_log_abs(const double* __restrict__ g, long long n, float* __restrict__ t) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] = (float)log10(fabs(g[i]) + 1e-12);
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
  const long long groups = (B + kFwdRows - 1) / kFwdRows;
  const unsigned grid = (unsigned)(groups < kMlpMaxBlocks ? groups : kMlpMaxBlocks);
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(256), 0, stream, W, x, B, y, act);
  return hipGetLastError();
}

long long mlp_backward_partial_rows(long long B) {
  const long long groups = (B + kBwdRows - 1) / kBwdRows;
  return groups < kMlpMaxBlocks ? groups : kMlpMaxBlocks;
}

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

int mse_partial_count(long long B) {
  const long long blocks = (B + 255) / 256;
  return (int)(blocks < kMlpMaxBlocks ? (blocks < 1 ? 1 : blocks) : kMlpMaxBlocks);
}

hipError_t launch_mse(const float* y, const float* t, long long B, float* dy, float* loss,
                      float* partial, hipStream_t stream) {
  const int nb = mse_partial_count(B);
  hipLaunchKernelGGL(k_mse_partial, dim3(nb), dim3(256), 0, stream, y, t, B, dy, partial);
  hipLaunchKernelGGL(k_mse_finish, dim3(1), dim3(64), 0, stream, partial, nb, B, loss);
  return hipGetLastError();
}

hipError_t launch_log_abs(const double* g, long long n, float* t, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_log_abs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, g, n, t);
  return hipGetLastError();
}

hipError_t launch_add_feature(float* v, const float* feat, long long n, int col, float sign, float scale,
                              hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_feature, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, v, feat, n, col,
                     sign, scale);
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
