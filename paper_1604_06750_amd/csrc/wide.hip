// Off-line band factorisation and shifted solves for cells with wide bands.
//
// The shifted solves with the cell matrix dominate the off-line cost and
// one Cholesky factorisation serves all of them (Sec. 4.2); for large cells
// (tens of thousands of nodes, half bandwidths of a thousand and more) the
// one-workgroup-per-cell kernels of offline.hip would leave most of the GPU
// idle and stream the band through one CU, so here the factorisation and
// the solves are blocked into panels of WB columns and spread over many
// workgroups per cell:
//
//   C = -(A_i + s B_i) = L L^T (band storage: column c holds L[c..c+w][c])
//   for each panel [j0, j0 + nb):
//     L11 = chol(C11)                               (k_wide_potrf)
//     L21 = C21 L11^{-T}                            (k_wide_trsm)
//     C22 -= L21 L21^T over the trailing band window  (k_wide_update, 64x64
//                                                      tiles of the window)
//   L L^T X = R (R = B q_j, n x b column-major):
//     forward, per panel:  Y1 = L11^{-1} R1; R2 -= L21 Y1
//     backward, per panel from the last: X1 = L11^{-T} (Y1 - L21^T X2)
//
// The result equals the unblocked band factorisation up to rounding order
// and uses the same storage, so every later kernel of the build is shared.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "sfrom_internal.h"

namespace sfrom_impl {

constexpr int WB = 64;      // panel width and tile edge
constexpr int WNT = 256;    // threads of the tiled kernels
constexpr int WST_NOTNSD = 1;   // status code of a non-positive pivot (as the other build kernels)

// Entry (r, c), c <= r <= c + w, of the band (zero outside the band or the
// matrix).
__device__ inline double band_at(const double* band, int ld, int w, int n, int64_t r, int64_t c) {
  return (r < n && c < n && r >= c && r - c <= w) ? band[c * ld + (r - c)] : 0.0;
}

// Band of C = -(A_i + s B_i), one workgroup per (cell, 256 columns): the
// workgroup zeroes its columns and fills them from the upper entries of the
// same CSR rows (C is symmetric), so no two workgroups write one column.
__global__ __launch_bounds__(WNT) void k_wide_assemble(BuildBatch bb) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  const int n = c.n, w = c.w, ld = w + 1;
  const int c0 = blockIdx.y * WNT;
  if (c0 >= n) return;
  const int c1 = min(n, c0 + WNT);
  double* band = bb.d_work + c.band_off;
  for (int64_t idx = threadIdx.x; idx < (int64_t)(c1 - c0) * ld; idx += WNT) band[(int64_t)c0 * ld + idx] = 0.0;
  __syncthreads();
  const int cc = c0 + threadIdx.x;
  if (cc < c1) {
    const int32_t* rp = bb.d_rowptr + c.rp_off;
    const int32_t* col = bb.d_col + c.csr_off;
    const double* a = bb.d_a + c.csr_off;
    const double* bd = bb.d_bdiag + c.b_off;
    for (int k = rp[cc]; k < rp[cc + 1]; ++k) {
      const int r = col[k];
      if (r >= cc && r - cc <= w) band[(int64_t)cc * ld + (r - cc)] = -(a[k] + (r == cc ? bb.shift * bd[cc] : 0.0));
    }
  }
}

// LDS copy of the nb x nb diagonal block of the panel at j0 (lower part,
// s[j][k] = C(j0 + j, j0 + k), identity beyond nb), stride WB + 1.
__device__ inline void load_diag(const double* band, int ld, int w, int n, int j0, int nb, double* s) {
  for (int idx = threadIdx.x; idx < WB * WB; idx += blockDim.x) {
    const int j = idx % WB, k = idx / WB;
    double v = 0.0;
    if (j < nb && k < nb) v = (j >= k) ? band_at(band, ld, w, n, j0 + j, j0 + k) : 0.0;
    else if (j == k) v = 1.0;
    s[j * (WB + 1) + k] = v;
  }
}

// In-place Cholesky of the LDS block (lower), column by column; a
// non-positive or non-finite pivot sets *bad and is replaced by 1.
__device__ inline void lds_potrf(double* s, int nb, int* bad) {
  for (int k = 0; k < nb; ++k) {
    if (threadIdx.x == 0) {
      const double d = s[k * (WB + 1) + k];
      if (!(d > 0.0) || !isfinite(d)) { *bad = 1; s[k * (WB + 1) + k] = 1.0; }
      else s[k * (WB + 1) + k] = sqrt(d);
    }
    __syncthreads();
    const double inv = 1.0 / s[k * (WB + 1) + k];
    for (int j = k + 1 + threadIdx.x; j < nb; j += blockDim.x) s[j * (WB + 1) + k] *= inv;
    __syncthreads();
    const int m = nb - k - 1;
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
      const int j = k + 1 + idx / m, i = k + 1 + idx % m;
      if (i <= j) s[j * (WB + 1) + i] -= s[j * (WB + 1) + k] * s[i * (WB + 1) + k];
    }
    __syncthreads();
  }
}

// Rows [r0, r0 + 64) of the panel's L21 (columns j0 .. j0 + nb - 1) into LDS
// as t[k][row] (zero outside the matrix or the band).
__device__ inline void load_l21(const double* band, int ld, int w, int n, int j0, int nb, int64_t r0, double* t) {
  for (int idx = threadIdx.x; idx < WB * WB; idx += blockDim.x) {
    const int rr = idx % WB, k = idx / WB;
    t[k * WB + rr] = (k < nb) ? band_at(band, ld, w, n, r0 + rr, j0 + k) : 0.0;
  }
}

typedef double doublex4 __attribute__((ext_vector_type(4)));
constexpr int TLD = WB + 1;   // stride of a staged 64 x 64 result tile (padded against bank conflicts)

// 64 x 64 product tile on the FP64 matrix instructions (four waves):
// acc[c] += sum_k a[k][row] b[k][col] over K (rounded up to 4; the LDS
// arrays a[64][64], b[64][64] hold zeros beyond K). Wave w owns rows
// 16 w .. 16 w + 15 and accumulator c columns 16 c .. 16 c + 15; the
// instruction takes A(i, k) from lane i + 16 k and B(k, j) from lane
// j + 16 k, and leaves C(g + 4 r, j) in register r of lane j + 16 g.
__device__ inline void tile_mfma(doublex4 (&acc)[4], const double* a, const double* b, int K) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, li = lane & 15;
  const int K4 = (K + 3) & ~3;
  for (int k0 = 0; k0 < K4; k0 += 4) {
    const double av = a[(k0 + g) * WB + 16 * w + li];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double bv = b[(k0 + g) * WB + 16 * c + li];
      acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[c], 0, 0, 0);
    }
  }
}

// The tile into LDS as t[col][row] (stride TLD), so that a coalesced pass
// over rows can apply it; the caller synchronises before reading t.
__device__ inline void tile_stage(const doublex4 (&acc)[4], double* t) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, li = lane & 15;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) t[(16 * c + li) * TLD + 16 * w + g + 4 * r] = acc[c][r];
}

// Panel j0, first launch: factor the diagonal block in LDS, store it, and
// store the inverse of the factor (64 x 64, identity beyond nb; M[i + 64 j]
// = L11^{-1}(i, j)): the panel's triangular solves become products with it
// (the block is a diagonal block of the Cholesky factor of a positive
// definite band matrix, so its inverse is as well conditioned as the block).
__global__ __launch_bounds__(WNT) void k_wide_potrf(BuildBatch bb, int j0) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  const int n = c.n, w = c.w, ld = w + 1;
  if (j0 >= n || c.status) return;
  const int nb = min(WB, n - j0);
  double* band = bb.d_work + c.band_off;
  __shared__ double s[WB * (WB + 1)];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  load_diag(band, ld, w, n, j0, nb, s);
  __syncthreads();
  lds_potrf(s, nb, &bad);
  for (int idx = threadIdx.x; idx < nb * nb; idx += WNT) {
    const int j = idx % nb, k = idx / nb;
    if (j >= k && j - k <= w) band[(int64_t)(j0 + k) * ld + (j - k)] = s[j * (WB + 1) + k];
  }
  if (threadIdx.x == 0 && bad) c.status = WST_NOTNSD;
  // column j of L11^{-1} by forward substitution, one thread per column
  double* M = bb.d_work + c.li_off + (int64_t)(j0 / WB) * WB * WB;
  const int j = threadIdx.x;
  if (j < WB) {
    for (int i = 0; i < j; ++i) M[i + WB * j] = 0.0;
    M[j + WB * j] = 1.0 / s[j * (WB + 1) + j];
    for (int i = j + 1; i < WB; ++i) {
      double a = 0.0;
      for (int k = j; k < i; ++k) a -= s[i * (WB + 1) + k] * M[k + WB * j];
      M[i + WB * j] = a / s[i * (WB + 1) + i];
    }
  }
}

// Panel j0, second launch: the panel's rows below the diagonal block,
// L21 = C21 L11^{-T} as a product with the stored inverse, one 64-row tile
// per workgroup.
__global__ __launch_bounds__(WNT) void k_wide_trsm(BuildBatch bb, int j0) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  const int n = c.n, w = c.w, ld = w + 1;
  if (j0 >= n || c.status) return;
  const int nb = min(WB, n - j0);
  const int nrows = min(w, n - j0 - nb);             // rows of L21 that can be nonzero
  const int64_t r0 = j0 + nb + (int64_t)blockIdx.y * WB;
  if ((int)blockIdx.y * WB >= nrows) return;
  double* band = bb.d_work + c.band_off;
  const double* M = bb.d_work + c.li_off + (int64_t)(j0 / WB) * WB * WB;
  __shared__ __align__(16) double la[WB * TLD];
  __shared__ __align__(16) double lb[WB * WB];
  // la[q][row] = C21(r0 + row, j0 + q); lb[q][k] = L11^{-T}(q, k) = M[k + 64 q]
  load_l21(band, ld, w, n, j0, nb, r0, la);
  for (int idx = threadIdx.x; idx < WB * WB; idx += WNT) lb[idx] = M[idx];
  __syncthreads();
  doublex4 acc[4] = {};
  tile_mfma(acc, la, lb, nb);
  __syncthreads();
  tile_stage(acc, la);
  __syncthreads();
  for (int idx = threadIdx.x; idx < WB * WB; idx += WNT) {
    const int rr = idx % WB, k = idx / WB;
    const int64_t r = r0 + rr;
    if (k < nb && rr < nrows - (int)blockIdx.y * WB && r - (j0 + k) <= w) band[(int64_t)(j0 + k) * ld + (r - j0 - k)] = la[k * TLD + rr];
  }
}

// Trailing update of panel j0: C22 -= L21 L21^T over the lower band window
// [s0, s0 + W)^2, s0 = j0 + nb, W = min(w, n - s0); blockIdx.y enumerates
// the window's lower 64 x 64 tiles (ti >= tj).
__global__ __launch_bounds__(WNT) void k_wide_update(BuildBatch bb, int j0) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  const int n = c.n, w = c.w, ld = w + 1;
  if (j0 >= n || c.status) return;
  const int nb = min(WB, n - j0);
  const int64_t s0 = j0 + nb;
  const int W = min((int64_t)w, n - s0);
  if (W <= 0) return;
  const int t = blockIdx.y;
  const int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  const int tj = t - ti * (ti + 1) / 2;
  if (ti * WB >= W || tj > ti) return;
  double* band = bb.d_work + c.band_off;
  __shared__ __align__(16) double la[WB * TLD];
  __shared__ __align__(16) double lb[WB * WB];
  const int64_t r0 = s0 + (int64_t)ti * WB, q0 = s0 + (int64_t)tj * WB;
  load_l21(band, ld, w, n, j0, nb, r0, la);
  load_l21(band, ld, w, n, j0, nb, q0, lb);
  __syncthreads();
  doublex4 acc[4] = {};
  tile_mfma(acc, la, lb, nb);
  __syncthreads();
  tile_stage(acc, la);
  __syncthreads();
  for (int idx = threadIdx.x; idx < WB * WB; idx += WNT) {
    const int rr = idx % WB, cq = idx / WB;
    const int64_t r = r0 + rr, cc = q0 + cq;
    if (r < s0 + W && cc < s0 + W && r >= cc) band[cc * ld + (r - cc)] -= la[cq * TLD + rr];
  }
}

// ---------------------------------------------------------------------------
// shifted solves X = (A + sB)^{-1} B q_j = -C^{-1} B q_j, b right-hand sides
// (column-major n x b in the A V region of the workspace)
// ---------------------------------------------------------------------------

// T = B q_j (one thread per row, all columns)
__global__ __launch_bounds__(WNT) void k_wide_solve_start(BuildBatch bb, int j) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (c.status || j + 1 >= c.m) return;
  const int n = c.n, b = c.b;
  const int r = blockIdx.y * WNT + threadIdx.x;
  if (r >= n) return;
  const double* q = bb.d_work + c.v_off + (int64_t)j * b * n;
  double* T = bb.d_work + c.av_off;
  const double bd = bb.d_bdiag[c.b_off + r];
  for (int col = 0; col < b; ++col) T[r + (int64_t)col * n] = bd * q[r + (int64_t)col * n];
}

// X = -T
__global__ __launch_bounds__(WNT) void k_wide_solve_end(BuildBatch bb, int j) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (c.status || j + 1 >= c.m) return;
  const int n = c.n, b = c.b;
  const int r = blockIdx.y * WNT + threadIdx.x;
  if (r >= n) return;
  const double* T = bb.d_work + c.av_off;
  double* X = bb.d_work + c.x_off;
  for (int col = 0; col < b; ++col) X[r + (int64_t)col * n] = -T[r + (int64_t)col * n];
}

// Forward, panel j0, columns [c0, c0 + 64): Y1 = L11^{-1} T1 in place, as a
// product with the stored inverse.
__global__ __launch_bounds__(WNT) void k_wide_fwd_diag(BuildBatch bb, int j, int j0) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (c.status || j + 1 >= c.m) return;
  const int n = c.n, b = c.b;
  if (j0 >= n) return;
  const int c0 = blockIdx.y * WB;
  if (c0 >= b) return;
  const int nb = min(WB, n - j0);
  const double* M = bb.d_work + c.li_off + (int64_t)(j0 / WB) * WB * WB;
  double* T = bb.d_work + c.av_off;
  __shared__ __align__(16) double sa[WB * TLD];
  __shared__ __align__(16) double sb[WB * WB];
  // sa[q][k] = L11^{-1}(k, q) = M[k + 64 q]; sb[q][col] = T1(q, c0 + col)
  for (int idx = threadIdx.x; idx < WB * WB; idx += WNT) {
    sa[idx] = M[idx];
    const int q = idx % WB, cc = idx / WB;
    sb[q * WB + cc] = (q < nb && c0 + cc < b) ? T[j0 + q + (int64_t)(c0 + cc) * n] : 0.0;
  }
  __syncthreads();
  doublex4 acc[4] = {};
  tile_mfma(acc, sa, sb, nb);
  __syncthreads();
  tile_stage(acc, sa);
  __syncthreads();
  for (int idx = threadIdx.x; idx < WB * WB; idx += WNT) {
    const int k = idx % WB, cc = idx / WB;
    if (k < nb && c0 + cc < b) T[j0 + k + (int64_t)(c0 + cc) * n] = sa[cc * TLD + k];
  }
}

// Forward, panel j0: T2 -= L21 Y1 for the rows [s0, s0 + W) below the panel;
// blockIdx.y = row tile + nrt * column tile.
__global__ __launch_bounds__(WNT) void k_wide_fwd_update(BuildBatch bb, int j, int j0, int nrt) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (c.status || j + 1 >= c.m) return;
  const int n = c.n, w = c.w, ld = w + 1, b = c.b;
  if (j0 >= n) return;
  const int nb = min(WB, n - j0);
  const int64_t s0 = j0 + nb;
  const int W = min((int64_t)w, n - s0);
  const int ti = blockIdx.y % nrt, tj = blockIdx.y / nrt;
  if (W <= 0 || ti * WB >= W || tj * WB >= b) return;
  const double* band = bb.d_work + c.band_off;
  double* T = bb.d_work + c.av_off;
  __shared__ __align__(16) double la[WB * TLD];
  __shared__ __align__(16) double yb[WB * WB];
  const int64_t r0 = s0 + (int64_t)ti * WB;
  const int c0 = tj * WB;
  load_l21(band, ld, w, n, j0, nb, r0, la);
  for (int idx = threadIdx.x; idx < WB * WB; idx += WNT) {
    const int k = idx % WB, cc = idx / WB;      // yb[k][col] = Y1[k][c0 + col], k fastest (contiguous in T)
    yb[k * WB + cc] = (k < nb && c0 + cc < b) ? T[j0 + k + (int64_t)(c0 + cc) * n] : 0.0;
  }
  __syncthreads();
  doublex4 acc[4] = {};
  tile_mfma(acc, la, yb, nb);
  __syncthreads();
  tile_stage(acc, la);
  __syncthreads();
  for (int idx = threadIdx.x; idx < WB * WB; idx += WNT) {
    const int rr = idx % WB, cq = idx / WB;
    const int64_t r = r0 + rr;
    const int cc = c0 + cq;
    if (r < s0 + W && cc < b) T[r + (int64_t)cc * n] -= la[cq * TLD + rr];
  }
}

// Backward, panel j0, columns [c0, c0 + 64): X1 = L11^{-T} (Y1 - L21^T X2)
// in place, X2 = the solved rows [s0, s0 + W) below the panel.
__global__ __launch_bounds__(WNT) void k_wide_bwd(BuildBatch bb, int j, int j0) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (c.status || j + 1 >= c.m) return;
  const int n = c.n, w = c.w, ld = w + 1, b = c.b;
  if (j0 >= n) return;
  const int c0 = blockIdx.y * WB;
  if (c0 >= b) return;
  const int nb = min(WB, n - j0);
  const int64_t s0 = j0 + nb;
  const int W = (int)max((int64_t)0, min((int64_t)w, n - s0));
  const double* band = bb.d_work + c.band_off;
  double* T = bb.d_work + c.av_off;
  __shared__ __align__(16) double la[WB * TLD];  // la[row][k] chunk of L21 (as [K = rows][64 = k])
  __shared__ __align__(16) double xb[WB * WB];   // xb[row][col] chunk of X2
  // acc[k][col] = sum over the window rows r of L21[r][k] X2[r][col]
  doublex4 acc[4] = {};
  for (int rc = 0; rc < W; rc += WB) {
    const int64_t r0 = s0 + rc;
    // rows fastest across the threads: contiguous in the band and in T
    for (int idx = threadIdx.x; idx < WB * WB; idx += WNT) {
      const int rr = idx % WB, q = idx / WB;
      la[rr * WB + q] = (q < nb && rc + rr < W) ? band_at(band, ld, w, n, r0 + rr, j0 + q) : 0.0;
      xb[rr * WB + q] = (rc + rr < W && c0 + q < b) ? T[r0 + rr + (int64_t)(c0 + q) * n] : 0.0;
    }
    __syncthreads();
    tile_mfma(acc, la, xb, min(WB, W - rc));
    __syncthreads();
  }
  // right-hand side of the diagonal solve in LDS (xb as rhs[q][col])
  tile_stage(acc, la);
  __syncthreads();
  for (int idx = threadIdx.x; idx < WB * WB; idx += WNT) {
    const int k = idx % WB, cc = idx / WB;
    xb[k * WB + cc] = (k < nb && c0 + cc < b) ? T[j0 + k + (int64_t)(c0 + cc) * n] - la[cc * TLD + k] : 0.0;
  }
  // X1 = L11^{-T} rhs: la[q][k] = L11^{-T}(k, q) = L11^{-1}(q, k) = M[q + 64 k]
  const double* M = bb.d_work + c.li_off + (int64_t)(j0 / WB) * WB * WB;
  __syncthreads();                               // every thread is done reading the staged tile
  for (int idx = threadIdx.x; idx < WB * WB; idx += WNT) {
    const int q = idx % WB, k = idx / WB;
    la[q * WB + k] = M[q + WB * k];
  }
  __syncthreads();
  doublex4 x[4] = {};
  tile_mfma(x, la, xb, nb);
  __syncthreads();
  tile_stage(x, la);
  __syncthreads();
  for (int idx = threadIdx.x; idx < WB * WB; idx += WNT) {
    const int k = idx % WB, cc = idx / WB;
    if (k < nb && c0 + cc < b) T[j0 + k + (int64_t)(c0 + cc) * n] = la[cc * TLD + k];
  }
}

// ---------------------------------------------------------------------------
// tall-skinny dense steps of the blocked build (n of a cell in the tens of
// thousands): Gram products as partial sums over chunks of TS_ROWS rows
// summed in a fixed order, and row-parallel updates, so each step of the
// rational Krylov basis (B-weighted CGS2, normalisation) and of the
// projection A^m = V^T A V runs on many workgroups per cell
// ---------------------------------------------------------------------------

// operands of a Gram product A^T diag(d) B for a cell (column-major, ld n)
struct TsOps {
  const double* A;
  const double* B;
  const double* d;     // row weights or nullptr
  int p, q;            // columns of A and B
  double* dst;         // reduced product, p x q, leading dimension p
  bool sym;            // symmetrise the reduced product
};

__device__ inline bool ts_ops(const BuildBatch& bb, const BuildCell& c, int mode, int j, TsOps& o) {
  const int n = c.n, b = c.b, mb = c.m * c.b;
  double* wk = bb.d_work;
  o.d = nullptr;
  o.sym = false;
  if (mode == TS_CGS) {             // coefficients V[:, 0:jb]^T B X
    if (j == 0 || j >= c.m) return false;
    o.A = wk + c.v_off; o.B = wk + c.x_off; o.d = bb.d_bdiag + c.b_off;
    o.p = j * b; o.q = b; o.dst = wk + c.s_off;
  } else if (mode == TS_NORM) {     // Gram X^T B X
    if (j >= c.m) return false;
    o.A = wk + c.x_off; o.B = wk + c.x_off; o.d = bb.d_bdiag + c.b_off;
    o.p = b; o.q = b; o.dst = wk + c.s_off; o.sym = true;
  } else {                          // A^m = V^T (A V)
    o.A = wk + c.v_off; o.B = wk + c.av_off;
    o.p = mb; o.q = mb; o.dst = wk + c.am_off; o.sym = true;
  }
  (void)n;
  return true;
}

// Partial Gram product of rows [ch TS_ROWS, (ch + 1) TS_ROWS) for output
// tile blockIdx.z (64 x 64 tiles of the p x q product, ntj tiles per row of
// tiles); written to the cell's partials region, chunk after chunk.
__global__ __launch_bounds__(WNT) void k_ts_gram(BuildBatch bb, int mode, int j, int ntj) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (c.status) return;
  TsOps o;
  if (!ts_ops(bb, c, mode, j, o)) return;
  const int n = c.n;
  const int r0 = blockIdx.y * TS_ROWS;
  if (r0 >= n) return;
  const int r1 = min(n, r0 + TS_ROWS);
  const int ti = blockIdx.z / ntj, tj = blockIdx.z % ntj;
  if (ti * WB >= o.p || tj * WB >= o.q) return;
  __shared__ __align__(16) double sa[WB * TLD];
  __shared__ __align__(16) double sb[WB * WB];
  doublex4 acc[4] = {};
  for (int rb = r0; rb < r1; rb += WB) {
    const int nr = min(WB, r1 - rb);
    // sa[row][i] = A[rb + row][ti 64 + i], sb[row][jj] = d B[rb + row][tj 64 + jj]
    for (int idx = threadIdx.x; idx < WB * WB; idx += WNT) {
      const int row = idx % WB, col = idx / WB;
      const int64_t r = rb + row;
      const int ia = ti * WB + col, ib = tj * WB + col;
      sa[row * WB + col] = (row < nr && ia < o.p) ? o.A[r + (int64_t)ia * n] : 0.0;
      const double dv = (row < nr && o.d) ? o.d[r] : 1.0;
      sb[row * WB + col] = (row < nr && ib < o.q) ? dv * o.B[r + (int64_t)ib * n] : 0.0;
    }
    __syncthreads();
    tile_mfma(acc, sa, sb, nr);
    __syncthreads();
  }
  double* P = bb.d_work + c.p_off + (int64_t)blockIdx.y * o.p * o.q;
  tile_stage(acc, sa);
  __syncthreads();
  for (int idx = threadIdx.x; idx < WB * WB; idx += WNT) {
    const int i = idx % WB, jj = idx / WB;
    const int gi = ti * WB + i, gj = tj * WB + jj;
    if (gi < o.p && gj < o.q) P[gi + (int64_t)gj * o.p] = sa[jj * TLD + i];
  }
}

// Sum of the partial products in chunk order (symmetrised for the Gram
// matrices) into the destination.
__global__ __launch_bounds__(WNT) void k_ts_reduce(BuildBatch bb, int mode, int j) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (c.status) return;
  TsOps o;
  if (!ts_ops(bb, c, mode, j, o)) return;
  const int64_t e = (int64_t)blockIdx.y * WNT + threadIdx.x;
  const int64_t pq = (int64_t)o.p * o.q;
  if (e >= pq) return;
  const int i = (int)(e % o.p), jj = (int)(e / o.p);
  const int nch = (c.n + TS_ROWS - 1) / TS_ROWS;
  const double* P = bb.d_work + c.p_off;
  double s = 0.0, t = 0.0;
  for (int ch = 0; ch < nch; ++ch) {
    s += P[ch * pq + e];
    if (o.sym) t += P[ch * pq + jj + (int64_t)i * o.p];
  }
  o.dst[e] = o.sym ? 0.5 * (s + t) : s;
}

// X -= V[:, 0:jb] coef (coef jb x b from the reduced CGS product), 64 x 64
// tiles of X.
__global__ __launch_bounds__(WNT) void k_ts_update(BuildBatch bb, int j) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (c.status || j == 0 || j >= c.m) return;
  const int n = c.n, b = c.b, jb = j * b;
  const int r0 = blockIdx.y * WB, c0 = blockIdx.z * WB;
  if (r0 >= n || c0 >= b) return;
  const double* V = bb.d_work + c.v_off;
  const double* coef = bb.d_work + c.s_off;
  double* X = bb.d_work + c.x_off;
  __shared__ __align__(16) double sa[WB * TLD];
  __shared__ __align__(16) double sb[WB * WB];
  doublex4 acc[4] = {};
  for (int k0 = 0; k0 < jb; k0 += WB) {
    const int nk = min(WB, jb - k0);
    for (int idx = threadIdx.x; idx < WB * WB; idx += WNT) {
      const int row = idx % WB, k = idx / WB;          // sa[k][row] = V[r0 + row][k0 + k]
      sa[k * WB + row] = (k < nk && r0 + row < n) ? V[r0 + row + (int64_t)(k0 + k) * n] : 0.0;
      const int kk = idx % WB, col = idx / WB;         // sb[k][col] = coef[k0 + k][c0 + col]
      sb[kk * WB + col] = (kk < nk && c0 + col < b) ? coef[k0 + kk + (int64_t)(c0 + col) * jb] : 0.0;
    }
    __syncthreads();
    tile_mfma(acc, sa, sb, nk);
    __syncthreads();
  }
  tile_stage(acc, sa);
  __syncthreads();
  for (int idx = threadIdx.x; idx < WB * WB; idx += WNT) {
    const int rr = idx % WB, cq = idx / WB;
    const int r = r0 + rr, cc = c0 + cq;
    if (r < n && cc < b) X[r + (int64_t)cc * n] -= sa[cq * TLD + rr];
  }
}

// q_j = X L^{-T} into block j of V (L: the lower Cholesky factor of the
// Gram matrix, b x b at s_off), one thread per row of 64 rows per
// workgroup, each row in an LDS column of its own.
__global__ __launch_bounds__(WB) void k_ts_trsm_rows(BuildBatch bb, int j) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (c.status || j >= c.m) return;
  const int n = c.n, b = c.b;
  const int r = blockIdx.y * WB + threadIdx.x;
  if ((int)blockIdx.y * WB >= n) return;
  extern __shared__ double xr[];                     // xr[l][thread]
  const double* X = bb.d_work + c.x_off;
  const double* L = bb.d_work + c.s_off;
  double* q = bb.d_work + c.v_off + (int64_t)j * b * n;
  if (r >= n) return;
  double* x = xr + threadIdx.x;
  for (int l = 0; l < b; ++l) x[l * WB] = X[r + (int64_t)l * n];
  for (int jj = 0; jj < b; ++jj) {
    double sacc = x[jj * WB];
    for (int l = 0; l < jj; ++l) sacc -= x[l * WB] * L[jj + (int64_t)l * b];
    x[jj * WB] = sacc / L[jj + (int64_t)jj * b];
  }
  for (int l = 0; l < b; ++l) q[r + (int64_t)l * n] = x[l * WB];
}

// A V (local CSR) into the A V region, one thread per row.
__global__ __launch_bounds__(WNT) void k_ts_spmm(BuildBatch bb) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (c.status) return;
  const int n = c.n, mb = c.m * c.b;
  const int r = blockIdx.y * WNT + threadIdx.x;
  if (r >= n) return;
  const int32_t* rp = bb.d_rowptr + c.rp_off;
  const int32_t* col = bb.d_col + c.csr_off;
  const double* a = bb.d_a + c.csr_off;
  const double* V = bb.d_work + c.v_off;
  double* AV = bb.d_work + c.av_off;
  constexpr int NZ = 8;
  const int k0 = rp[r], nk = rp[r + 1] - k0;
  int ci[NZ];
  double av[NZ];
#pragma unroll
  for (int k = 0; k < NZ; ++k) {
    ci[k] = k < nk ? col[k0 + k] : r;
    av[k] = k < nk ? a[k0 + k] : 0.0;
  }
  for (int cc = 0; cc < mb; ++cc) {
    const double* Vc = V + (int64_t)cc * n;
    double sacc = 0.0;
#pragma unroll
    for (int k = 0; k < NZ; ++k) sacc += av[k] * Vc[ci[k]];
    for (int k = k0 + NZ; k < k0 + nk; ++k) sacc += a[k] * Vc[col[k]];
    AV[r + (int64_t)cc * n] = sacc;
  }
}

hipError_t launch_ts_gram(const BuildBatch& bb, int mode, int j, hipStream_t st) {
  const int mb = bb.max_m * bb.max_b;
  const int p = mode == TS_PROJ ? mb : (mode == TS_CGS ? j * bb.max_b : bb.max_b);
  const int q = mode == TS_PROJ ? mb : bb.max_b;
  if (p == 0) return hipSuccess;
  const int nti = (p + WB - 1) / WB, ntj = (q + WB - 1) / WB;
  const dim3 grid(bb.ncell, (bb.max_n + TS_ROWS - 1) / TS_ROWS, nti * ntj);
  hipLaunchKernelGGL(k_ts_gram, grid, dim3(WNT), 0, st, bb, mode, j, ntj);
  const int64_t pq = (int64_t)p * q;
  hipLaunchKernelGGL(k_ts_reduce, dim3(bb.ncell, (unsigned)((pq + WNT - 1) / WNT)), dim3(WNT), 0, st, bb, mode, j);
  return hipGetLastError();
}

hipError_t launch_ts_update(const BuildBatch& bb, int j, hipStream_t st) {
  hipLaunchKernelGGL(k_ts_update, dim3(bb.ncell, (bb.max_n + WB - 1) / WB, (bb.max_b + WB - 1) / WB), dim3(WNT), 0,
                     st, bb, j);
  return hipGetLastError();
}

hipError_t launch_ts_trsm_rows(const BuildBatch& bb, int j, hipStream_t st) {
  const size_t lds = (size_t)WB * bb.max_b * sizeof(double);
  hipLaunchKernelGGL(k_ts_trsm_rows, dim3(bb.ncell, (bb.max_n + WB - 1) / WB), dim3(WB), lds, st, bb, j);
  return hipGetLastError();
}

hipError_t launch_ts_spmm(const BuildBatch& bb, hipStream_t st) {
  hipLaunchKernelGGL(k_ts_spmm, dim3(bb.ncell, (bb.max_n + WNT - 1) / WNT), dim3(WNT), 0, st, bb);
  return hipGetLastError();
}

bool build_is_wide(const BuildBatch& bb, int force) {
  if (force == 1) return true;
  if (force == 2) return false;
  return bb.max_w > WIDE_MIN_W;
}

hipError_t launch_wide_chol(const BuildBatch& bb, hipStream_t st) {
  const int nc = bb.ncell;
  hipLaunchKernelGGL(k_wide_assemble, dim3(nc, (bb.max_n + WNT - 1) / WNT), dim3(WNT), 0, st, bb);
  const int rt = (bb.max_w + WB - 1) / WB;                    // row tiles of a panel's L21
  const int T = (bb.max_w + WB - 1) / WB;                      // tile rows of a trailing window
  const int ntile = T * (T + 1) / 2;
  for (int j0 = 0; j0 < bb.max_n; j0 += WB) {
    hipLaunchKernelGGL(k_wide_potrf, dim3(nc), dim3(WNT), 0, st, bb, j0);
    if (rt > 0) hipLaunchKernelGGL(k_wide_trsm, dim3(nc, rt), dim3(WNT), 0, st, bb, j0);
    if (ntile > 0) hipLaunchKernelGGL(k_wide_update, dim3(nc, ntile), dim3(WNT), 0, st, bb, j0);
  }
  return hipGetLastError();
}

hipError_t launch_wide_solve(const BuildBatch& bb, int j, hipStream_t st) {
  const int nc = bb.ncell;
  const dim3 rows(nc, (bb.max_n + WNT - 1) / WNT);
  const int ct = (bb.max_b + WB - 1) / WB;
  const int nrt = std::max((bb.max_w + WB - 1) / WB, 1);
  hipLaunchKernelGGL(k_wide_solve_start, rows, dim3(WNT), 0, st, bb, j);
  for (int j0 = 0; j0 < bb.max_n; j0 += WB) {
    hipLaunchKernelGGL(k_wide_fwd_diag, dim3(nc, ct), dim3(WNT), 0, st, bb, j, j0);
    hipLaunchKernelGGL(k_wide_fwd_update, dim3(nc, nrt * ct), dim3(WNT), 0, st, bb, j, j0, nrt);
  }
  const int last = (bb.max_n - 1) / WB * WB;
  for (int j0 = last; j0 >= 0; j0 -= WB) hipLaunchKernelGGL(k_wide_bwd, dim3(nc, ct), dim3(WNT), 0, st, bb, j, j0);
  hipLaunchKernelGGL(k_wide_solve_end, rows, dim3(WNT), 0, st, bb, j);
  return hipGetLastError();
}

}  // namespace sfrom_impl
