// Learned off-line stage: a small 3D CNN from a cell's medium (8^3 voxels
// of log sigma, log rho) to the Cholesky factors of its deep S-fraction
// blocks, trained on the GPU by the kernels below (forward, backward, Adam)
// and evaluated with bfloat16 operands and float accumulation.
//
// Network: conv3d(2 -> C, 3^3, zero padding) + ReLU, 2^3 average pooling,
// dense(64 C -> H) + ReLU, dense(H -> P). Loss: mean squared error over the
// batch and the P normalised outputs. Parameters are one float vector
// [W1 (C,2,3,3,3), b1 (C), W2 (H, 64 C), b2 (H), W3 (P, H), b3 (P)], all
// row-major; inputs x are [n][channel][z][y][x].
//
// Every reduction (bias gradients, weight gradients of the convolution,
// the loss) is summed in a fixed order, so training is deterministic.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "sfrom.h"
#include "sfrom_internal.h"

namespace sfrom_impl {

namespace {

constexpr int VOX = 8, NVOX = 512, NPOOL = 64;

__device__ inline float round_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

// C[M x N] = op(A) op(B) (+ beta C), row-major; op(A) is M x K (A stored
// K x M when TA), op(B) is K x N (B stored N x K when TB). RND rounds both
// operands to bfloat16 (the products are then exact in float).
template <bool TA, bool TB, bool RND>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A, int lda,
                                              const float* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
                                              float beta) {
  __shared__ float As[16][68];
  __shared__ float Bs[16][68];
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  float acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.f;
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = threadIdx.x; e < 1024; e += 256) {
      // consecutive threads walk the contiguous dimension of each operand
      int kk, ii;
      if (TA) { kk = e >> 6; ii = e & 63; } else { ii = e >> 4; kk = e & 15; }
      const int gi = i0 + ii, gk = k0 + kk;
      float va = 0.f;
      if (gi < M && gk < K) va = TA ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk];
      As[kk][ii] = RND ? round_bf16(va) : va;
      int kb, jj;
      if (TB) { jj = e >> 4; kb = e & 15; } else { kb = e >> 6; jj = e & 63; }
      const int gj = j0 + jj, gkb = k0 + kb;
      float vb = 0.f;
      if (gj < N && gkb < K) vb = TB ? B[(int64_t)gj * ldb + gkb] : B[(int64_t)gkb * ldb + gj];
      Bs[kb][jj] = RND ? round_bf16(vb) : vb;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[kk][ty * 4 + r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx * 4 + c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = fmaf(a[r], b[c], acc[r][c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + ty * 4 + r;
    if (i >= M) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = j0 + tx * 4 + c;
      if (j >= N) continue;
      float* p = C + (int64_t)i * ldc + j;
      *p = (beta != 0.f) ? acc[r][c] + beta * (*p) : acc[r][c];
    }
  }
}

template <bool TA, bool TB, bool RND>
hipError_t gemm(int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C, int ldc, float beta,
                hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const dim3 grid((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL((k_gemm<TA, TB, RND>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, beta);
  return hipGetLastError();
}

// z1[n][co][v] = b1[co] + sum_ci sum_taps W1[co][ci][tap] x[n][ci][v + tap]
template <bool RND>
__global__ __launch_bounds__(256) void k_conv_fwd(const float* __restrict__ x, const float* __restrict__ W1,
                                                  const float* __restrict__ b1, float* __restrict__ z1, int n,
                                                  int C) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)n * C * NVOX) return;
  const int v = (int)(gid % NVOX);
  const int co = (int)((gid / NVOX) % C);
  const int64_t s = gid / ((int64_t)NVOX * C);
  const int z = v >> 6, y = (v >> 3) & 7, xx = v & 7;
  float acc = b1[co];
  for (int ci = 0; ci < 2; ++ci) {
    const float* xi = x + (s * 2 + ci) * NVOX;
    const float* w = W1 + (co * 2 + ci) * 27;
    for (int dz = 0; dz < 3; ++dz) {
      const int zz = z + dz - 1;
      if (zz < 0 || zz >= VOX) continue;
      for (int dy = 0; dy < 3; ++dy) {
        const int yy = y + dy - 1;
        if (yy < 0 || yy >= VOX) continue;
        for (int dx = 0; dx < 3; ++dx) {
          const int x3 = xx + dx - 1;
          if (x3 < 0 || x3 >= VOX) continue;
          float a = w[(dz * 3 + dy) * 3 + dx], b = xi[(zz * VOX + yy) * VOX + x3];
          if (RND) { a = round_bf16(a); b = round_bf16(b); }
          acc = fmaf(a, b, acc);
        }
      }
    }
  }
  z1[gid] = acc;
}

// p[n][c*64 + pv] = mean of relu(z1) over the 2^3 voxels of pooled cell pv
__global__ __launch_bounds__(256) void k_pool_fwd(const float* __restrict__ z1, float* __restrict__ p, int n, int C) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)n * C * NPOOL) return;
  const int pv = (int)(gid % NPOOL);
  const int64_t nc = gid / NPOOL;
  const int pz = pv >> 4, py = (pv >> 2) & 3, px = pv & 3;
  const float* zc = z1 + nc * NVOX;
  float s = 0.f;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int c = 0; c < 2; ++c) s += fmaxf(zc[((2 * pz + a) * VOX + 2 * py + b) * VOX + 2 * px + c], 0.f);
  p[gid] = 0.125f * s;
}

// z[i][j] += b[j]; h[i][j] = relu(z[i][j]) when h is given
__global__ __launch_bounds__(256) void k_bias_act(float* __restrict__ z, const float* __restrict__ b,
                                                  float* __restrict__ h, int rows, int cols) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)rows * cols) return;
  const float v = z[gid] + b[gid % cols];
  z[gid] = v;
  if (h) h[gid] = fmaxf(v, 0.f);
}

// dy = 2 (y - t) / (rows cols); per-block partial sums of (y - t)^2
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             float* __restrict__ dy, double* __restrict__ part, int64_t count) {
  __shared__ double sh[256];
  double acc = 0.0;
  const float scale = 2.f / (float)count;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) {
    const float r = y[i] - t[i];
    dy[i] = scale * r;
    acc += (double)r * r;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ part, int np, int64_t count,
                                                   float* __restrict__ loss) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(sh[0] / (double)count);
}

// out[j] = sum_i d[i][j] (column sums, rows summed in order)
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ d, float* __restrict__ out, int rows,
                                                int cols) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= cols) return;
  float s = 0.f;
  for (int i = 0; i < rows; ++i) s += d[(int64_t)i * cols + j];
  out[j] = s;
}

// d[i] *= (z[i] > 0)
__global__ __launch_bounds__(256) void k_relu_bwd(float* __restrict__ d, const float* __restrict__ z, int64_t count) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid < count && !(z[gid] > 0.f)) d[gid] = 0.f;
}

// dz1[n][c][v] = dp[n][c*64 + pool(v)] / 8 * (z1 > 0)
__global__ __launch_bounds__(256) void k_pool_bwd(const float* __restrict__ dp, const float* __restrict__ z1,
                                                  float* __restrict__ dz1, int n, int C) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)n * C * NVOX) return;
  const int v = (int)(gid % NVOX);
  const int64_t nc = gid / NVOX;
  const int z = v >> 6, y = (v >> 3) & 7, x = v & 7;
  const int pv = ((z >> 1) * 4 + (y >> 1)) * 4 + (x >> 1);
  dz1[gid] = (z1[gid] > 0.f) ? 0.125f * dp[nc * NPOOL + pv] : 0.f;
}

// gW1[co][ci][tap] = sum_{n,v} dz1[n][co][v] x[n][ci][v + tap]  (one block per
// weight; block C*54 + co computes gb1[co] = sum dz1[n][co][.])
__global__ __launch_bounds__(256) void k_conv_bwd(const float* __restrict__ dz1, const float* __restrict__ x,
                                                  float* __restrict__ gW1, float* __restrict__ gb1, int n, int C) {
  __shared__ double sh[256];
  const int wid = blockIdx.x;
  const bool bias = wid >= C * 54;
  int co, ci = 0, dz = 0, dy = 0, dx = 0;
  if (bias) {
    co = wid - C * 54;
  } else {
    co = wid / 54;
    const int r = wid % 54;
    ci = r / 27;
    dz = (r % 27) / 9; dy = (r % 9) / 3; dx = r % 3;
  }
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)n * NVOX; e += 256) {
    const int64_t s = e / NVOX;
    const int v = (int)(e % NVOX);
    const float g = dz1[(s * C + co) * NVOX + v];
    if (bias) { acc += g; continue; }
    const int z = (v >> 6) + dz - 1, y = ((v >> 3) & 7) + dy - 1, xx = (v & 7) + dx - 1;
    if (z < 0 || z >= VOX || y < 0 || y >= VOX || xx < 0 || xx >= VOX) continue;
    acc += (double)g * x[(s * 2 + ci) * NVOX + (z * VOX + y) * VOX + xx];
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (bias) gb1[co] = (float)sh[0];
    else gW1[wid] = (float)sh[0];
  }
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int64_t n, float lr, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
}

// out = y * sd + mu per output column
__global__ __launch_bounds__(256) void k_unscale(const float* __restrict__ y, const float* __restrict__ mu,
                                                 const float* __restrict__ sd, float* __restrict__ out, int rows,
                                                 int cols) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)rows * cols) return;
  const int j = (int)(gid % cols);
  out[gid] = y[gid] * sd[j] + mu[j];
}

__global__ __launch_bounds__(256) void k_fill(float* __restrict__ p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

inline dim3 grid1(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

}  // namespace sfrom_impl

using namespace sfrom_impl;

struct sfrom_surrogate {
  int device = -1;
  hipStream_t stream = nullptr;
  std::string err;
  int C = 0, H = 0, P = 0;
  int64_t n_params = 0, oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
  float *theta = nullptr, *grad = nullptr, *am = nullptr, *av = nullptr;
  float *mu = nullptr, *sd = nullptr;
  int64_t adam_t = 0;
  bool have_params = false, have_scale = false;
  int cap = 0;
  float *z1 = nullptr, *p = nullptr, *z2 = nullptr, *h2 = nullptr, *y = nullptr;
  float *dy = nullptr, *dh = nullptr, *dp = nullptr, *dz1 = nullptr, *loss = nullptr;
  double* part = nullptr;
};

namespace {

struct SFail {
  int code;
};

#define S_HIP(call)                                                                       \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      s->err = std::string("HIP error in " #call ": ") + hipGetErrorString(e_);          \
      throw SFail{SFROM_EDEVICE};                                                         \
    }                                                                                     \
  } while (0)
#define S_REQ(cond, code, msg) \
  do {                                 \
    if (!(cond)) {                     \
      s->err = (msg);                  \
      throw SFail{code};               \
    }                                  \
  } while (0)

template <typename T>
T* s_alloc(sfrom_surrogate* s, int64_t n) {
  void* p = nullptr;
  if (n <= 0) n = 1;
  const hipError_t e = hipMalloc(&p, (size_t)n * sizeof(T));
  if (e != hipSuccess) {
    s->err = "device allocation failed";
    throw SFail{SFROM_ENOMEM};
  }
  return static_cast<T*>(p);
}
template <typename T>
void s_free(T*& p) {
  if (p) hipFree(p);
  p = nullptr;
}

void free_scratch(sfrom_surrogate* s) {
  s_free(s->z1); s_free(s->p); s_free(s->z2); s_free(s->h2); s_free(s->y);
  s_free(s->dy); s_free(s->dh); s_free(s->dp); s_free(s->dz1); s_free(s->loss); s_free(s->part);
  s->cap = 0;
}

void ensure_cap(sfrom_surrogate* s, int n) {
  if (n <= s->cap) return;
  free_scratch(s);
  const int64_t C = s->C, H = s->H, P = s->P;
  s->z1 = s_alloc<float>(s, n * C * NVOX);
  s->dz1 = s_alloc<float>(s, n * C * NVOX);
  s->p = s_alloc<float>(s, n * C * NPOOL);
  s->dp = s_alloc<float>(s, n * C * NPOOL);
  s->z2 = s_alloc<float>(s, n * H);
  s->h2 = s_alloc<float>(s, n * H);
  s->dh = s_alloc<float>(s, n * H);
  s->y = s_alloc<float>(s, n * P);
  s->dy = s_alloc<float>(s, n * P);
  s->loss = s_alloc<float>(s, 1);
  s->part = s_alloc<double>(s, 1024);
  s->cap = n;
}

// y (n x P, normalised outputs) of the network for inputs x
void forward(sfrom_surrogate* s, const float* x, int n, bool bf16) {
  ensure_cap(s, n);
  const int C = s->C, H = s->H, P = s->P, C64 = C * NPOOL;
  const hipStream_t st = s->stream;
  const float* th = s->theta;
  if (bf16) hipLaunchKernelGGL(k_conv_fwd<true>, grid1((int64_t)n * C * NVOX), dim3(256), 0, st, x, th + s->oW1, th + s->ob1, s->z1, n, C);
  else hipLaunchKernelGGL(k_conv_fwd<false>, grid1((int64_t)n * C * NVOX), dim3(256), 0, st, x, th + s->oW1, th + s->ob1, s->z1, n, C);
  S_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_pool_fwd, grid1((int64_t)n * C64), dim3(256), 0, st, s->z1, s->p, n, C);
  S_HIP(hipGetLastError());
  if (bf16) S_HIP((gemm<false, true, true>(n, H, C64, s->p, C64, th + s->oW2, C64, s->z2, H, 0.f, st)));
  else S_HIP((gemm<false, true, false>(n, H, C64, s->p, C64, th + s->oW2, C64, s->z2, H, 0.f, st)));
  hipLaunchKernelGGL(k_bias_act, grid1((int64_t)n * H), dim3(256), 0, st, s->z2, th + s->ob2, s->h2, n, H);
  S_HIP(hipGetLastError());
  if (bf16) S_HIP((gemm<false, true, true>(n, P, H, s->h2, H, th + s->oW3, H, s->y, P, 0.f, st)));
  else S_HIP((gemm<false, true, false>(n, P, H, s->h2, H, th + s->oW3, H, s->y, P, 0.f, st)));
  hipLaunchKernelGGL(k_bias_act, grid1((int64_t)n * P), dim3(256), 0, st, s->y, th + s->ob3, (float*)nullptr, n, P);
  S_HIP(hipGetLastError());
}

// loss and gradient (into s->grad) for inputs x and normalised targets t
void loss_grad(sfrom_surrogate* s, const float* x, const float* t, int n) {
  forward(s, x, n, false);
  const int C = s->C, H = s->H, P = s->P, C64 = C * NPOOL;
  const hipStream_t st = s->stream;
  const float* th = s->theta;
  float* g = s->grad;
  const int64_t cnt = (int64_t)n * P;
  const int nb = (int)std::min<int64_t>(1024, (cnt + 255) / 256);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, st, s->y, t, s->dy, s->part, cnt);
  S_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, s->part, nb, cnt, s->loss);
  S_HIP(hipGetLastError());
  // dense 2
  S_HIP((gemm<true, false, false>(P, H, n, s->dy, P, s->h2, H, g + s->oW3, H, 0.f, st)));
  hipLaunchKernelGGL(k_colsum, grid1(P), dim3(256), 0, st, s->dy, g + s->ob3, n, P);
  S_HIP(hipGetLastError());
  S_HIP((gemm<false, false, false>(n, H, P, s->dy, P, th + s->oW3, H, s->dh, H, 0.f, st)));
  hipLaunchKernelGGL(k_relu_bwd, grid1((int64_t)n * H), dim3(256), 0, st, s->dh, s->z2, (int64_t)n * H);
  S_HIP(hipGetLastError());
  // dense 1
  S_HIP((gemm<true, false, false>(H, C64, n, s->dh, H, s->p, C64, g + s->oW2, C64, 0.f, st)));
  hipLaunchKernelGGL(k_colsum, grid1(H), dim3(256), 0, st, s->dh, g + s->ob2, n, H);
  S_HIP(hipGetLastError());
  S_HIP((gemm<false, false, false>(n, C64, H, s->dh, H, th + s->oW2, C64, s->dp, C64, 0.f, st)));
  // pooling, ReLU and convolution
  hipLaunchKernelGGL(k_pool_bwd, grid1((int64_t)n * C * NVOX), dim3(256), 0, st, s->dp, s->z1, s->dz1, n, C);
  S_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_conv_bwd, dim3(C * 54 + C), dim3(256), 0, st, s->dz1, x, g + s->oW1, g + s->ob1, n, C);
  S_HIP(hipGetLastError());
}

}  // namespace

namespace sfrom_impl {

int surrogate_outputs(const sfrom_surrogate* s) { return s->P; }

hipError_t surrogate_predict(sfrom_surrogate* s, const float* x, int n, float* out) {
  try {
    if (!s->have_params || !s->have_scale) return hipErrorInvalidValue;
    forward(s, x, n, true);
    hipLaunchKernelGGL(k_unscale, grid1((int64_t)n * s->P), dim3(256), 0, s->stream, s->y, s->mu, s->sd, out, n, s->P);
    return hipGetLastError();
  } catch (const SFail&) {
    return hipErrorUnknown;
  }
}

}  // namespace sfrom_impl

#define S_BEGIN(s)                     \
  if (!(s)) return SFROM_EINVAL;       \
  try {                                \
    (s)->err.clear();                  \
    if ((s)->device >= 0) hipSetDevice((s)->device);
#define S_END(s)                       \
  }                                    \
  catch (const SFail& f) {             \
    return f.code;                     \
  }                                    \
  catch (...) {                        \
    (s)->err = "unexpected error";     \
    return SFROM_EDEVICE;              \
  }                                    \
  return SFROM_OK;

extern "C" {

int sfrom_surrogate_create(sfrom_surrogate_t** out, int32_t device, void* hip_stream, int32_t conv_ch,
                           int32_t hidden, int32_t n_out) {
  if (!out) return SFROM_EINVAL;
  *out = nullptr;
  if (conv_ch <= 0 || hidden <= 0 || n_out <= 0 || device < 0) return SFROM_EINVAL;
  int nd = 0;
  if (hipGetDeviceCount(&nd) != hipSuccess || device >= nd) return SFROM_EDEVICE;
  auto* s = new sfrom_surrogate;
  s->device = device;
  s->stream = static_cast<hipStream_t>(hip_stream);
  s->C = conv_ch; s->H = hidden; s->P = n_out;
  const int64_t C = conv_ch, H = hidden, P = n_out;
  s->oW1 = 0;
  s->ob1 = s->oW1 + C * 54;
  s->oW2 = s->ob1 + C;
  s->ob2 = s->oW2 + H * C * NPOOL;
  s->oW3 = s->ob2 + H;
  s->ob3 = s->oW3 + P * H;
  s->n_params = s->ob3 + P;
  try {
    hipSetDevice(device);
    s->theta = s_alloc<float>(s, s->n_params);
    s->grad = s_alloc<float>(s, s->n_params);
    s->am = s_alloc<float>(s, s->n_params);
    s->av = s_alloc<float>(s, s->n_params);
    s->mu = s_alloc<float>(s, P);
    s->sd = s_alloc<float>(s, P);
  } catch (const SFail& f) {
    sfrom_surrogate_destroy(s);
    return f.code;
  }
  *out = s;
  return SFROM_OK;
}

void sfrom_surrogate_destroy(sfrom_surrogate_t* s) {
  if (!s) return;
  if (s->device >= 0) hipSetDevice(s->device);
  if (s->stream) hipStreamSynchronize(s->stream);
  else hipDeviceSynchronize();
  free_scratch(s);
  s_free(s->theta); s_free(s->grad); s_free(s->am); s_free(s->av); s_free(s->mu); s_free(s->sd);
  delete s;
}

const char* sfrom_surrogate_last_error(const sfrom_surrogate_t* s) { return s ? s->err.c_str() : "null handle"; }

int sfrom_surrogate_param_count(const sfrom_surrogate_t* s, int64_t* n) {
  if (!s || !n) return SFROM_EINVAL;
  *n = s->n_params;
  return SFROM_OK;
}

int sfrom_surrogate_set_params(sfrom_surrogate_t* s, const float* theta) {
  S_BEGIN(s)
  S_REQ(theta != nullptr, SFROM_EINVAL, "null parameters");
  for (int64_t i = 0; i < s->n_params; ++i) S_REQ(std::isfinite(theta[i]), SFROM_ENONFINITE, "non-finite parameter");
  S_HIP(hipMemcpyAsync(s->theta, theta, s->n_params * sizeof(float), hipMemcpyHostToDevice, s->stream));
  hipLaunchKernelGGL(k_fill, grid1(s->n_params), dim3(256), 0, s->stream, s->am, s->n_params, 0.f);
  hipLaunchKernelGGL(k_fill, grid1(s->n_params), dim3(256), 0, s->stream, s->av, s->n_params, 0.f);
  S_HIP(hipGetLastError());
  S_HIP(hipStreamSynchronize(s->stream));
  s->adam_t = 0;
  s->have_params = true;
  S_END(s)
}

int sfrom_surrogate_get_params(sfrom_surrogate_t* s, float* theta) {
  S_BEGIN(s)
  S_REQ(theta != nullptr && s->have_params, SFROM_ESTATE, "no parameters set");
  S_HIP(hipMemcpyAsync(theta, s->theta, s->n_params * sizeof(float), hipMemcpyDeviceToHost, s->stream));
  S_HIP(hipStreamSynchronize(s->stream));
  S_END(s)
}

int sfrom_surrogate_set_scale(sfrom_surrogate_t* s, const float* mu, const float* sd) {
  S_BEGIN(s)
  S_REQ(mu && sd, SFROM_EINVAL, "null scale");
  for (int j = 0; j < s->P; ++j) {
    S_REQ(std::isfinite(mu[j]) && std::isfinite(sd[j]), SFROM_ENONFINITE, "non-finite scale");
    S_REQ(sd[j] > 0.f, SFROM_EINVAL, "scale must be positive");
  }
  S_HIP(hipMemcpyAsync(s->mu, mu, s->P * sizeof(float), hipMemcpyHostToDevice, s->stream));
  S_HIP(hipMemcpyAsync(s->sd, sd, s->P * sizeof(float), hipMemcpyHostToDevice, s->stream));
  S_HIP(hipStreamSynchronize(s->stream));
  s->have_scale = true;
  S_END(s)
}

int sfrom_surrogate_gradients(sfrom_surrogate_t* s, const float* x, const float* t, int32_t n, float* loss,
                              float* grad) {
  S_BEGIN(s)
  S_REQ(x && t && n > 0, SFROM_EINVAL, "bad batch");
  S_REQ(s->have_params, SFROM_ESTATE, "no parameters set");
  loss_grad(s, x, t, n);
  if (loss) S_HIP(hipMemcpyAsync(loss, s->loss, sizeof(float), hipMemcpyDeviceToHost, s->stream));
  if (grad) S_HIP(hipMemcpyAsync(grad, s->grad, s->n_params * sizeof(float), hipMemcpyDeviceToHost, s->stream));
  S_HIP(hipStreamSynchronize(s->stream));
  S_END(s)
}

int sfrom_surrogate_train_step(sfrom_surrogate_t* s, const float* x, const float* t, int32_t n, float lr,
                               float* loss) {
  S_BEGIN(s)
  S_REQ(x && t && n > 0 && lr > 0.f, SFROM_EINVAL, "bad batch or learning rate");
  S_REQ(s->have_params, SFROM_ESTATE, "no parameters set");
  loss_grad(s, x, t, n);
  s->adam_t += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)s->adam_t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)s->adam_t)));
  hipLaunchKernelGGL(k_adam, grid1(s->n_params), dim3(256), 0, s->stream, s->theta, s->grad, s->am, s->av,
                     s->n_params, lr, c1, c2);
  S_HIP(hipGetLastError());
  if (loss) {
    S_HIP(hipMemcpyAsync(loss, s->loss, sizeof(float), hipMemcpyDeviceToHost, s->stream));
    S_HIP(hipStreamSynchronize(s->stream));
  }
  S_END(s)
}

int sfrom_surrogate_forward(sfrom_surrogate_t* s, const float* x, int32_t n, int32_t bf16, float* y) {
  S_BEGIN(s)
  S_REQ(x && y && n > 0, SFROM_EINVAL, "bad batch");
  S_REQ(s->have_params, SFROM_ESTATE, "no parameters set");
  forward(s, x, n, bf16 != 0);
  S_HIP(hipMemcpyAsync(y, s->y, (size_t)n * s->P * sizeof(float), hipMemcpyDeviceToDevice, s->stream));
  S_HIP(hipStreamSynchronize(s->stream));
  S_END(s)
}

}  // extern "C"
