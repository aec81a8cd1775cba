// Off-line stage on the GPU (Alg. alg1red stage 1), double precision.
//
// Every kernel runs one 256-thread workgroup per coarse cell of the batch;
// cells are independent (Sec. 4.2: no data exchange between cells), so the
// batch is the unit of parallelism. Per cell, with C = -(A_i + s B_i) (SPD):
//
//   K1  banded Cholesky C = L L^T (lexicographic local order, bandwidth w)
//   K2  rational block Krylov (eq. npks): X_1 = B^{-1} W; for each block,
//       B-weighted classical Gram-Schmidt against all previous blocks,
//       applied twice; R^T R = X^T B X (Cholesky; a tiny pivot ratio means
//       the block lost rank, Assumption 1); q_j = X R^{-1};
//       X_{j+1} = (A + sB)^{-1} B q_j = -C^{-1} B q_j (two band solves)
//   K3  projection A^m = V^T A V (eq. tfprj); B^m = I because V is
//       B-orthonormal, and S^m = V^T W = [R_1; 0; ...] because X_1 = q_1 R_1
//   K4  block Lanczos on (A^m, I) from S^m (App. C): Q_1 = E_1, beta_1 = R_1,
//       Z = A^m Q_k - Q_k alpha_k - Q_{k-1} beta_k^T, reorthogonalised twice,
//       Q_{k+1} beta_{k+1} = Z by Cholesky-QR applied twice
//   K5  S-fraction (eq. GammaTrans with G_1 = beta_1^T,
//       G^k = -G_k^{-T} alpha_k G_k^{-1} - G^{k-1},
//       G_{k+1} = (G_k^T G^k)^{-1} beta_{k+1}^T), SPD checks of the pivots.
//
// All dense matrices are column-major in a per-cell double workspace.

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cmath>

#include "sfrom_internal.h"

namespace sfrom_impl {

#define NT 256

enum {
  ST_OK = 0,
  ST_NOTNSD = 1,     // band Cholesky pivot <= 0
  ST_BREAKDOWN = 2,  // Krylov / Lanczos rank loss
  ST_NOTSPD = 3,     // S-fraction pivot not SPD
  ST_NONFINITE = 4
};

// ---------------------------------------------------------------------------
// workgroup-cooperative dense helpers
// ---------------------------------------------------------------------------

// C = alpha op(A) op(B) + beta C, M x N, inner K. op(A)(i,k) = TA ? A[k+i*lda]
// : A[i+k*lda]; op(B)(k,j) = TB ? B[j+k*ldb] : B[k+j*ldb]. 64x64 output tiles,
// 4x4 per thread, K staged through LDS in chunks of 16; the next chunk's
// HBM loads are issued into registers before the current chunk's products,
// so their latency overlaps the arithmetic. C must not alias A, B.
// K-chunk tiles of wg_gemm, one pair shared by all its instantiations
__shared__ double g_gemm_as[16][65];
__shared__ double g_gemm_bs[16][65];

template <bool TA, bool TB>
__device__ void wg_gemm(int M, int N, int K, double alpha, const double* __restrict__ A, int lda,
                        const double* __restrict__ B, int ldb, double beta, double* C, int ldc) {
  auto& As = g_gemm_as;
  auto& Bs = g_gemm_bs;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  // element q of this thread's share of a chunk: A(ii, kk) and B(kb, jj)
  int ii[4], kk[4], jj[4], kb[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + NT * q;
    if (!TA) { ii[q] = e & 63; kk[q] = e >> 6; } else { kk[q] = e & 15; ii[q] = e >> 4; }
    if (!TB) { kb[q] = e & 15; jj[q] = e >> 4; } else { jj[q] = e & 63; kb[q] = e >> 6; }
  }
  for (int i0 = 0; i0 < M; i0 += 64) {
    for (int j0 = 0; j0 < N; j0 += 64) {
      double pa[4], pb[4];
      auto gload = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = i0 + ii[q], k = k0 + kk[q];
          pa[q] = (i < M && k < K) ? (TA ? A[k + (int64_t)i * lda] : A[i + (int64_t)k * lda]) : 0.0;
          const int j = j0 + jj[q], k2 = k0 + kb[q];
          pb[q] = (j < N && k2 < K) ? (TB ? B[j + (int64_t)k2 * ldb] : B[k2 + (int64_t)j * ldb]) : 0.0;
        }
      };
      double acc[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
      gload(0);
      for (int k0 = 0; k0 < K; k0 += 16) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          As[kk[q]][ii[q]] = pa[q];
          Bs[kb[q]][jj[q]] = pb[q];
        }
        __syncthreads();
        if (k0 + 16 < K) gload(k0 + 16);
#pragma unroll 4
        for (int k = 0; k < 16; ++k) {
          double a[4], b[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) a[r] = As[k][tx + 16 * r];
#pragma unroll
          for (int c = 0; c < 4; ++c) b[c] = Bs[k][ty + 16 * c];
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + tx + 16 * r;
        if (i >= M) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int j = j0 + ty + 16 * c;
          if (j >= N) continue;
          double* p = C + i + (int64_t)j * ldc;
          *p = (beta == 0.0) ? alpha * acc[r][c] : alpha * acc[r][c] + beta * (*p);
        }
      }
    }
  }
  __syncthreads();
}

// Y = A X for a cell's CSR operator A (n x n, local row starts) and n x ncol
// column-major X, Y (leading dimension n). One thread per row: a row of at
// most SPMM_NZ nonzeros is held in registers while the columns are swept
// (padding entries add exactly zero), longer rows use the plain loop.
constexpr int SPMM_NZ = 8;
__device__ void wg_spmm_csr(int n, int ncol, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const double* __restrict__ a, const double* __restrict__ X, double* __restrict__ Y) {
  for (int r = threadIdx.x; r < n; r += NT) {
    const int k0 = rp[r], nk = rp[r + 1] - k0;
    if (nk <= SPMM_NZ) {
      int ci[SPMM_NZ];
      double av[SPMM_NZ];
#pragma unroll
      for (int k = 0; k < SPMM_NZ; ++k) {
        ci[k] = k < nk ? col[k0 + k] : r;
        av[k] = k < nk ? a[k0 + k] : 0.0;
      }
      for (int cc = 0; cc < ncol; ++cc) {
        const double* Xc = X + (int64_t)cc * n;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < SPMM_NZ; ++k) s += av[k] * Xc[ci[k]];
        Y[r + (int64_t)cc * n] = s;
      }
    } else {
      for (int cc = 0; cc < ncol; ++cc) {
        double s = 0.0;
        for (int k = k0; k < k0 + nk; ++k) s += a[k] * X[col[k] + (int64_t)cc * n];
        Y[r + (int64_t)cc * n] = s;
      }
    }
  }
}

// Y = diag(d) X for n x ncol column-major X, Y (leading dimension n).
__device__ void wg_scale_rows(int n, int ncol, const double* __restrict__ d, const double* __restrict__ X,
                              double* __restrict__ Y) {
  for (int r = threadIdx.x; r < n; r += NT) {
    const double dr = d[r];
    for (int cc = 0; cc < ncol; ++cc) Y[r + (int64_t)cc * n] = dr * X[r + (int64_t)cc * n];
  }
}

// In-place lower Cholesky of an n x n SPD matrix (global memory). Returns the
// ratio min/max of the pivots' square roots, or -1 if a pivot is not
// positive and finite.
__device__ double wg_potrf_global(int n, double* A, int lda) {
  __shared__ double s_piv;
  __shared__ double s_min, s_max;
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  if (tid == 0) { s_bad = 0; s_min = 1e300; s_max = 0.0; }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      const double d = A[j + (int64_t)j * lda];
      if (!(d > 0.0) || !isfinite(d)) { s_bad = 1; s_piv = 1.0; }
      else {
        s_piv = sqrt(d);
        s_min = fmin(s_min, s_piv);
        s_max = fmax(s_max, s_piv);
      }
      A[j + (int64_t)j * lda] = s_piv;
    }
    __syncthreads();
    const double inv = 1.0 / s_piv;
    for (int i = j + 1 + tid; i < n; i += NT) A[i + (int64_t)j * lda] *= inv;
    __syncthreads();
    const int t = n - j - 1;
    for (int idx = tid; idx < t * t; idx += NT) {
      const int i = j + 1 + idx % t;
      const int k = j + 1 + idx / t;
      if (i >= k) A[i + (int64_t)k * lda] -= A[i + (int64_t)j * lda] * A[k + (int64_t)j * lda];
    }
    __syncthreads();
  }
  const double r = s_bad ? -1.0 : s_min / s_max;
  __syncthreads();
  return r;
}

// X (rows x n) <- X L^{-T} for lower L (n x n): solves q L^T = x row-wise.
__device__ void wg_trsm_right_lt_global(int rows, int n, const double* L, int ldl, double* X, int ldx) {
  for (int r = threadIdx.x; r < rows; r += NT) {
    for (int j = 0; j < n; ++j) {
      double s = X[r + (int64_t)j * ldx];
      for (int l = 0; l < j; ++l) s -= X[r + (int64_t)l * ldx] * L[j + (int64_t)l * ldl];
      X[r + (int64_t)j * ldx] = s / L[j + (int64_t)j * ldl];
    }
  }
  __syncthreads();
}

// Small factors (n <= SMALL_N) are factored and applied from LDS. One
// file-scope matrix buffer is shared by both helpers, so a kernel that uses
// them holds it once.
constexpr int SMALL_N = 64;
constexpr int SMALL_LD = SMALL_N + 1;
__shared__ double g_small[SMALL_N * SMALL_LD];

// wg_potrf for n <= SMALL_N: A copied to LDS (column-major), the same
// right-looking steps with one wave per updated column, the factor written
// back. Same return value.
__device__ double wg_potrf_lds(int n, double* A, int lda) {
  __shared__ double s_min, s_max;
  __shared__ int s_bad;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  double* S = g_small;
  for (int idx = tid; idx < n * n; idx += NT) {
    const int i = idx % n, k = idx / n;
    S[i + k * SMALL_LD] = A[i + (int64_t)k * lda];
  }
  if (tid == 0) { s_bad = 0; s_min = 1e300; s_max = 0.0; }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double d = S[j + j * SMALL_LD];
    const bool ok = d > 0.0 && isfinite(d);
    const double piv = ok ? sqrt(d) : 1.0;
    const double inv = 1.0 / piv;
    if (tid > j && tid < n) S[tid + j * SMALL_LD] *= inv;
    if (tid == 0) {
      if (!ok) s_bad = 1;
      else { s_min = fmin(s_min, piv); s_max = fmax(s_max, piv); }
    }
    __syncthreads();
    for (int k = j + 1 + wv; k < n; k += NT / 64) {
      const double lk = S[k + j * SMALL_LD];
      for (int i = k + lane; i < n; i += 64) S[i + k * SMALL_LD] -= S[i + j * SMALL_LD] * lk;
    }
    if (tid == 0) S[j + j * SMALL_LD] = piv;
    __syncthreads();
  }
  for (int idx = tid; idx < n * n; idx += NT) {
    const int i = idx % n, k = idx / n;
    A[i + (int64_t)k * lda] = S[i + k * SMALL_LD];
  }
  const double r = s_bad ? -1.0 : s_min / s_max;
  __syncthreads();
  return r;
}

// wg_trsm_right_lt for n <= SMALL_N: L staged in LDS (column-major), each
// row of X solved in blocks of 16 unknowns held in registers; earlier
// blocks' solved values are read back once per block.
__device__ void wg_trsm_right_lt_lds(int rows, int n, const double* L, int ldl, double* X, int ldx) {
  constexpr int NBK = 16;
  double* S = g_small;
  for (int idx = threadIdx.x; idx < n * n; idx += NT) {
    const int j = idx % n, l = idx / n;
    S[j + l * SMALL_LD] = (l <= j) ? L[j + (int64_t)l * ldl] : 0.0;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < rows; r += NT) {
    for (int j0 = 0; j0 < n; j0 += NBK) {
      double x[NBK];
#pragma unroll
      for (int q = 0; q < NBK; ++q) x[q] = (j0 + q < n) ? X[r + (int64_t)(j0 + q) * ldx] : 0.0;
      for (int l = 0; l < j0; ++l) {
        const double xl = X[r + (int64_t)l * ldx];
#pragma unroll
        for (int q = 0; q < NBK; ++q) x[q] -= xl * S[j0 + q + l * SMALL_LD];
      }
#pragma unroll
      for (int q = 0; q < NBK; ++q) {
        if (j0 + q < n) {
          double s = x[q];
#pragma unroll
          for (int p = 0; p < q; ++p) s -= x[p] * S[j0 + q + (j0 + p) * SMALL_LD];
          x[q] = s / S[j0 + q + (j0 + q) * SMALL_LD];
        }
      }
#pragma unroll
      for (int q = 0; q < NBK; ++q)
        if (j0 + q < n) X[r + (int64_t)(j0 + q) * ldx] = x[q];
    }
  }
  __syncthreads();
}

__device__ double wg_potrf(int n, double* A, int lda) {
  return n <= SMALL_N ? wg_potrf_lds(n, A, lda) : wg_potrf_global(n, A, lda);
}
__device__ void wg_trsm_right_lt(int rows, int n, const double* L, int ldl, double* X, int ldx) {
  if (n <= SMALL_N) wg_trsm_right_lt_lds(rows, n, L, ldl, X, ldx);
  else wg_trsm_right_lt_global(rows, n, L, ldl, X, ldx);
}

// Ainv = A^{-1} (n x n) by Gauss-Jordan with partial pivoting; W is n x n
// scratch (destroyed), fac is n doubles scratch. Returns 0 if singular.
__device__ int wg_inverse(int n, const double* A, int lda, double* Ainv, int ldi, double* W,
                          double* fac) {
  __shared__ int s_p;
  __shared__ int s_ok;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < n * n; idx += NT) {
    const int i = idx % n, j = idx / n;
    W[i + (int64_t)j * n] = A[i + (int64_t)j * lda];
    Ainv[i + (int64_t)j * ldi] = (i == j) ? 1.0 : 0.0;
  }
  if (tid == 0) s_ok = 1;
  __syncthreads();
  const int wv = tid >> 6, lane = tid & 63;
  for (int j = 0; j < n; ++j) {
    if (wv == 0) {
      // pivot: the largest magnitude in column j at or below row j, the
      // lowest row among equal magnitudes (one wave, shuffle reduction)
      int p = j;
      double best = -1.0;
      for (int i = j + lane; i < n; i += 64) {
        const double v = fabs(W[i + (int64_t)j * n]);
        if (v > best) { best = v; p = i; }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const int op = __shfl_xor(p, o);
        if (ob > best || (ob == best && op < p)) { best = ob; p = op; }
      }
      if (lane == 0) {
        if (!(best > 0.0)) s_ok = 0;
        s_p = p;
      }
    }
    __syncthreads();
    const int p = s_p;
    if (p != j) {
      for (int c = tid; c < n; c += NT) {
        double t = W[j + (int64_t)c * n]; W[j + (int64_t)c * n] = W[p + (int64_t)c * n]; W[p + (int64_t)c * n] = t;
        t = Ainv[j + (int64_t)c * ldi]; Ainv[j + (int64_t)c * ldi] = Ainv[p + (int64_t)c * ldi]; Ainv[p + (int64_t)c * ldi] = t;
      }
    }
    __syncthreads();
    const double piv = W[j + (int64_t)j * n];
    const double ip = (piv != 0.0) ? 1.0 / piv : 0.0;
    for (int c = tid; c < n; c += NT) {
      W[j + (int64_t)c * n] *= ip;
      Ainv[j + (int64_t)c * ldi] *= ip;
    }
    __syncthreads();
    for (int i = tid; i < n; i += NT) fac[i] = (i == j) ? 0.0 : W[i + (int64_t)j * n];
    __syncthreads();
    // eliminate column j from every other row: one wave per column c,
    // lanes along the rows
    for (int c = wv; c < n; c += NT / 64) {
      const double wj = W[j + (int64_t)c * n], aj = Ainv[j + (int64_t)c * ldi];
      for (int i = lane; i < n; i += 64) {
        const double f = fac[i];
        if (f != 0.0) {
          W[i + (int64_t)c * n] -= f * wj;
          Ainv[i + (int64_t)c * ldi] -= f * aj;
        }
      }
    }
    __syncthreads();
  }
  const int ok = s_ok;
  __syncthreads();
  return ok;
}

__device__ void wg_symmetrize(int n, double* A, int lda) {
  for (int idx = threadIdx.x; idx < n * n; idx += NT) {
    const int i = idx % n, j = idx / n;
    if (i < j) {
      const double v = 0.5 * (A[i + (int64_t)j * lda] + A[j + (int64_t)i * lda]);
      A[i + (int64_t)j * lda] = v;
      A[j + (int64_t)i * lda] = v;
    }
  }
  __syncthreads();
}

__device__ void wg_copy(int rows, int cols, const double* A, int lda, double* B, int ldb) {
  for (int idx = threadIdx.x; idx < rows * cols; idx += NT) {
    const int i = idx % rows, j = idx / rows;
    B[i + (int64_t)j * ldb] = A[i + (int64_t)j * lda];
  }
  __syncthreads();
}

// B = A^T (n x n, distinct storage)
__device__ void wg_transpose(int n, const double* A, int lda, double* B, int ldb) {
  for (int idx = threadIdx.x; idx < n * n; idx += NT) {
    const int i = idx % n, j = idx / n;
    B[j + (int64_t)i * ldb] = A[i + (int64_t)j * lda];
  }
  __syncthreads();
}

// X (rows x n) <- X L^{-1} for lower L (n x n): solves q L = x row-wise,
// last column first.
__device__ void wg_trsm_right_l(int rows, int n, const double* L, int ldl, double* X, int ldx) {
  for (int r = threadIdx.x; r < rows; r += NT) {
    for (int j = n - 1; j >= 0; --j) {
      double s = X[r + (int64_t)j * ldx];
      for (int l = j + 1; l < n; ++l) s -= X[r + (int64_t)l * ldx] * L[l + (int64_t)j * ldl];
      X[r + (int64_t)j * ldx] = s / L[j + (int64_t)j * ldl];
    }
  }
  __syncthreads();
}

// 1 if every diagonal entry of the n x n matrix is nonzero and finite
__device__ int wg_diag_ok(int n, const double* A, int lda) {
  __shared__ int s_ok;
  if (threadIdx.x == 0) s_ok = 1;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += NT) {
    const double d = A[i + (int64_t)i * lda];
    if (!(d != 0.0) || !isfinite(d)) s_ok = 0;
  }
  __syncthreads();
  const int ok = s_ok;
  __syncthreads();
  return ok;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

struct KArgs {
  BuildBatch bb;
};

__device__ inline bool cell_failed(const BuildCell& c) { return c.status != ST_OK; }

// K1: assemble the band of C = -(A_i + s B_i) and factor it.
__global__ __launch_bounds__(NT) void k_band_chol(BuildBatch bb) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  const int n = c.n, w = c.w, ld = w + 1;
  double* band = bb.d_work + c.band_off;
  const int32_t* rp = bb.d_rowptr + c.rp_off;
  const int32_t* col = bb.d_col + c.csr_off;
  const double* a = bb.d_a + c.csr_off;
  const double* bd = bb.d_bdiag + c.b_off;
  for (int64_t idx = threadIdx.x; idx < (int64_t)n * ld; idx += NT) band[idx] = 0.0;
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += NT) {
    for (int k = rp[r]; k < rp[r + 1]; ++k) {
      const int cc = col[k];
      if (r >= cc) band[(int64_t)cc * ld + (r - cc)] = -(a[k] + (r == cc ? bb.shift * bd[r] : 0.0));
    }
  }
  __syncthreads();
  __shared__ double s_piv;
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double* cj = band + (int64_t)j * ld;
    if (threadIdx.x == 0) {
      const double d = cj[0];
      if (!(d > 0.0) || !isfinite(d)) { s_bad = 1; s_piv = 1.0; } else s_piv = sqrt(d);
      cj[0] = s_piv;
    }
    __syncthreads();
    const int lim = min(w, n - 1 - j);
    const double inv = 1.0 / s_piv;
    for (int d = 1 + threadIdx.x; d <= lim; d += NT) cj[d] *= inv;
    __syncthreads();
    for (int idx = threadIdx.x; idx < lim * lim; idx += NT) {
      const int d1 = idx / lim + 1, d2 = idx % lim + 1;
      if (d2 >= d1) band[(int64_t)(j + d1) * ld + (d2 - d1)] -= cj[d2] * cj[d1];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && s_bad) c.status = ST_NOTNSD;
}

// K2 start: X = B^{-1} W (W = P^Gamma S_i, scattered from the piece bases).
__global__ __launch_bounds__(NT) void k_krylov_start(BuildBatch bb) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (cell_failed(c)) return;
  const int n = c.n, b = c.b;
  double* X = bb.d_work + c.x_off;
  for (int64_t idx = threadIdx.x; idx < (int64_t)n * b; idx += NT) X[idx] = 0.0;
  __syncthreads();
  const double* bd = bb.d_bdiag + c.b_off;
  for (int k = threadIdx.x; k < c.nw; k += NT) {
    const int64_t e = c.w_off + k;
    const int row = bb.d_wrow[e], col0 = bb.d_wcol[e], bp = bb.d_wbp[e], kp = bb.d_wkp[e];
    const double* s = bb.d_S + bb.d_wsoff[e];
    const double ib = 1.0 / bd[row];
    for (int l = 0; l < bp; ++l) X[row + (int64_t)(col0 + l) * n] = s[(int64_t)l * kp] * ib;
  }
}

// B-weighted block classical Gram-Schmidt of X against V[:, 0:jb], twice.
__global__ __launch_bounds__(NT) void k_cgs2(BuildBatch bb, int j) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (cell_failed(c) || j >= c.m || j == 0) return;
  const int n = c.n, b = c.b, jb = j * b;
  double* X = bb.d_work + c.x_off;
  double* V = bb.d_work + c.v_off;
  double* BX = bb.d_work + c.av_off;            // n x b scratch
  double* coef = bb.d_work + c.s_off;           // jb x b scratch
  const double* bd = bb.d_bdiag + c.b_off;
  for (int pass = 0; pass < 2; ++pass) {
    wg_scale_rows(n, b, bd, X, BX);
    __syncthreads();
    wg_gemm<true, false>(jb, b, n, 1.0, V, n, BX, n, 0.0, coef, jb);
    wg_gemm<false, false>(n, b, jb, -1.0, V, n, coef, jb, 1.0, X, n);
  }
}

// Normalise block j: R^T R = X^T B X, q_j = X R^{-1} -> V[:, j b : (j+1) b].
__global__ __launch_bounds__(NT) void k_normalize(BuildBatch bb, int j) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (cell_failed(c) || j >= c.m) return;
  const int n = c.n, b = c.b;
  double* X = bb.d_work + c.x_off;
  double* V = bb.d_work + c.v_off;
  double* BX = bb.d_work + c.av_off;
  double* gram = bb.d_work + c.s_off;
  const double* bd = bb.d_bdiag + c.b_off;
  wg_scale_rows(n, b, bd, X, BX);
  __syncthreads();
  wg_gemm<true, false>(b, b, n, 1.0, X, n, BX, n, 0.0, gram, b);
  wg_symmetrize(b, gram, b);
  const double ratio = wg_potrf(b, gram, b);          // gram <- L (lower)
  if (!(ratio > 1e-10)) {
    if (threadIdx.x == 0) { c.status = ST_BREAKDOWN; c.fail_block = j + 1; }
    return;
  }
  // R_j = L^T (upper), kept for beta_1 = R_1
  double* R = bb.d_work + c.r_off + (int64_t)j * b * b;
  for (int idx = threadIdx.x; idx < b * b; idx += NT) {
    const int r = idx % b, cc = idx / b;
    R[r + (int64_t)cc * b] = (r <= cc) ? gram[cc + (int64_t)r * b] : 0.0;
  }
  double* q = V + (int64_t)j * b * n;
  wg_copy(n, b, X, n, q, n);
  wg_trsm_right_lt(n, b, gram, b, q, n);
}

// Blocked build, normalisation of block j after the Gram matrix X^T B X has
// been reduced into the small workspace: Cholesky R^T R of it (rank check as
// k_normalize) and R_j kept; q_j = X R^{-1} follows row-parallel.
__global__ __launch_bounds__(NT) void k_ts_chol(BuildBatch bb, int j) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (cell_failed(c) || j >= c.m) return;
  const int b = c.b;
  double* gram = bb.d_work + c.s_off;
  const double ratio = wg_potrf(b, gram, b);          // gram <- L (lower)
  if (!(ratio > 1e-10)) {
    if (threadIdx.x == 0) { c.status = ST_BREAKDOWN; c.fail_block = j + 1; }
    return;
  }
  double* R = bb.d_work + c.r_off + (int64_t)j * b * b;
  for (int idx = threadIdx.x; idx < b * b; idx += NT) {
    const int r = idx % b, cc = idx / b;
    R[r + (int64_t)cc * b] = (r <= cc) ? gram[cc + (int64_t)r * b] : 0.0;
  }
}

// X = (A + sB)^{-1} B q_j = -C^{-1} (B q_j) with the banded factor.
// Solves (L L^T) x = t for one right-hand side per lane: L is the band
// Cholesky factor (column-major band, column c holding L[c..c+w][c]) and t
// is column `col` of the row-major n x b array T, overwritten by x. Each
// lane touches only its own column, so no barrier is needed; the band
// entries are wave-uniform (scalar loads). When `win` is given it holds
// (w + 1) x b doubles in LDS: a ring of the last w + 1 solved rows, so the
// w neighbours of a row are read from LDS instead of from T.
__device__ void lane_band_solve(const double* __restrict__ band, int ld, int w, int n, int b, double* T, int col,
                                double* win) {
  const int W = w + 1;
  // forward: L y = t, y[r] = (t[r] - sum_d L[r][r-d] y[r-d]) / L[r][r]
  int head = 0;                                    // r mod W
  for (int r = 0; r < n; ++r) {
    double acc = T[(int64_t)r * b + col];
    const int lim = min(w, r);
    if (win) {
      int idx = head;
#pragma unroll 4
      for (int d = 1; d <= lim; ++d) {
        idx = (idx == 0) ? W - 1 : idx - 1;
        acc -= band[(int64_t)(r - d) * ld + d] * win[idx * b + col];
      }
    } else {
#pragma unroll 4
      for (int d = 1; d <= lim; ++d) acc -= band[(int64_t)(r - d) * ld + d] * T[(int64_t)(r - d) * b + col];
    }
    const double y = acc / band[(int64_t)r * ld];
    T[(int64_t)r * b + col] = y;
    if (win) win[head * b + col] = y;
    head = (head + 1 == W) ? 0 : head + 1;
  }
  // backward: L^T x = y, x[r] = (y[r] - sum_d L[r+d][r] x[r+d]) / L[r][r]
  head = (n - 1) % W;                              // r mod W
  for (int r = n - 1; r >= 0; --r) {
    const double* cr = band + (int64_t)r * ld;
    double acc = T[(int64_t)r * b + col];
    const int lim = min(w, n - 1 - r);
    if (win) {
      int idx = head;
#pragma unroll 4
      for (int d = 1; d <= lim; ++d) {
        idx = (idx + 1 == W) ? 0 : idx + 1;
        acc -= cr[d] * win[idx * b + col];
      }
    } else {
#pragma unroll 4
      for (int d = 1; d <= lim; ++d) acc -= cr[d] * T[(int64_t)(r + d) * b + col];
    }
    const double x = acc / cr[0];
    T[(int64_t)r * b + col] = x;
    if (win) win[head * b + col] = x;
    head = (head == 0) ? W - 1 : head - 1;
  }
}

// Workgroup form of the same solve with the band column staged in LDS:
// every thread calls it; thread `col` < b owns right-hand side col. The
// forward sweep is right-looking: the LDS ring `win` accumulates the
// updates -sum_c L[r][c] y[c] of the next w rows, and once y[r] is known
// column r of L (read contiguously) updates them. The backward sweep is
// left-looking with four partial sums. Global reads on the sweep's critical
// path (the next band column, the next right-hand side) are issued one row
// ahead, so their latency overlaps the row's arithmetic. win holds
// (w + 1) x b doubles, colbuf w + 1 doubles.
__device__ void wg_band_solve(const double* __restrict__ band, int ld, int w, int n, int b, double* T,
                              double* win, double* colbuf) {
  const int W = w + 1;
  const int col = threadIdx.x, nt = blockDim.x;
  const bool own = col < b;
  // band column r of L (entries 0..min(w, n-1-r)): the first 4 nt entries
  // travel through registers (fetched a row ahead), any further ones are
  // copied when staged
  auto fetch = [&](int r, double (&c)[4]) {
    const int lim = min(w, n - 1 - r);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = col + i * nt;
      c[i] = (k <= lim) ? band[(int64_t)r * ld + k] : 0.0;
    }
  };
  auto stage = [&](int r, const double (&c)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (col + i * nt <= w) colbuf[col + i * nt] = c[i];
    const int lim = min(w, n - 1 - r);
    for (int k = col + 4 * nt; k <= lim; k += nt) colbuf[k] = band[(int64_t)r * ld + k];
  };
  if (own)
    for (int q = 0; q < W; ++q) win[q * b + col] = 0.0;
  double c[4];
  fetch(0, c);
  stage(0, c);
  double t_next = own ? T[col] : 0.0;
  __syncthreads();
  int head = 0;
  for (int r = 0; r < n; ++r) {
    const int lim = min(w, n - 1 - r);
    if (r + 1 < n) fetch(r + 1, c);
    if (own) {
      const double t_r = t_next;
      if (r + 1 < n) t_next = T[(int64_t)(r + 1) * b + col];
      const double y = (t_r + win[head * b + col]) / colbuf[0];
      T[(int64_t)r * b + col] = y;
      int idx = head;
      for (int d = 1; d <= lim; ++d) {
        idx = (idx + 1 == W) ? 0 : idx + 1;
        win[idx * b + col] -= colbuf[d] * y;
      }
      win[head * b + col] = 0.0;                 // the slot now collects row r + W
    }
    head = (head + 1 == W) ? 0 : head + 1;
    __syncthreads();
    if (r + 1 < n) stage(r + 1, c);
    __syncthreads();
  }
  head = (n - 1) % W;
  fetch(n - 1, c);
  __syncthreads();
  stage(n - 1, c);
  double y_next = own ? T[(int64_t)(n - 1) * b + col] : 0.0;
  __syncthreads();
  for (int r = n - 1; r >= 0; --r) {
    const int lim = min(w, n - 1 - r);
    if (r > 0) fetch(r - 1, c);
    if (own) {
      const double y_r = y_next;
      if (r > 0) y_next = T[(int64_t)(r - 1) * b + col];
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int idx = head;
      int d = 1;
      for (; d + 3 <= lim; d += 4) {
        idx = (idx + 1 == W) ? 0 : idx + 1;
        a0 += colbuf[d] * win[idx * b + col];
        idx = (idx + 1 == W) ? 0 : idx + 1;
        a1 += colbuf[d + 1] * win[idx * b + col];
        idx = (idx + 1 == W) ? 0 : idx + 1;
        a2 += colbuf[d + 2] * win[idx * b + col];
        idx = (idx + 1 == W) ? 0 : idx + 1;
        a3 += colbuf[d + 3] * win[idx * b + col];
      }
      for (; d <= lim; ++d) {
        idx = (idx + 1 == W) ? 0 : idx + 1;
        a0 += colbuf[d] * win[idx * b + col];
      }
      const double x = (y_r - ((a0 + a1) + (a2 + a3))) / colbuf[0];
      T[(int64_t)r * b + col] = x;
      win[head * b + col] = x;
    }
    head = (head == 0) ? W - 1 : head - 1;
    __syncthreads();
    if (r > 0) stage(r - 1, c);
    __syncthreads();
  }
}

// Register form of the same solve for a single wave and half bandwidth
// w <= W: lane `col` keeps its right-hand side's window in registers (the
// partial sums of the next W rows while sweeping forward, the last W
// solved values while sweeping backward), updated in place with
// compile-time indices, so a row costs W fused multiply-adds and no LDS
// traffic beyond the broadcast band column. The column is double-buffered
// in LDS (colbuf holds 2 (W + 1) doubles, entries beyond the band zero) and
// fetched from HBM a row ahead, so each row needs one barrier.
template <int W>
__device__ void reg_band_solve(const double* __restrict__ band, int ld, int w, int n, int b, double* T,
                               double* colbuf) {
  constexpr int NB = W + 1;
  constexpr int KF = (NB + 63) / 64;    // column entries per lane
  const int col = threadIdx.x;
  const bool own = col < b;
  auto fetch = [&](int r, double (&c)[KF]) {
    const int lim = min(w, n - 1 - r);
#pragma unroll
    for (int i = 0; i < KF; ++i) {
      const int k = col + 64 * i;
      c[i] = (k <= lim) ? band[(int64_t)r * ld + k] : 0.0;
    }
  };
  auto stage = [&](double* dst, const double (&c)[KF]) {
#pragma unroll
    for (int i = 0; i < KF; ++i)
      if (col + 64 * i < NB) dst[col + 64 * i] = c[i];
  };
  double c[KF];
  fetch(0, c);
  stage(colbuf, c);
  double acc[W];
#pragma unroll
  for (int j = 0; j < W; ++j) acc[j] = 0.0;
  double t_next = own ? T[col] : 0.0;
  __syncthreads();
  for (int r = 0; r < n; ++r) {
    const double* cur = colbuf + (r & 1) * NB;
    if (r + 1 < n) fetch(r + 1, c);
    if (own) {
      const double t_r = t_next;
      if (r + 1 < n) t_next = T[(int64_t)(r + 1) * b + col];
      const double y = (t_r + acc[0]) / cur[0];
      T[(int64_t)r * b + col] = y;
      // acc[j] now collects row r + 1 + j
#pragma unroll
      for (int j = 0; j + 1 < W; ++j) acc[j] = fma(-cur[j + 1], y, acc[j + 1]);
      acc[W - 1] = -cur[W] * y;
    }
    if (r + 1 < n) stage(colbuf + ((r + 1) & 1) * NB, c);
    __syncthreads();
  }
  // backward sweep: xw[j] holds x[r + 1 + j]
  double xw[W];
#pragma unroll
  for (int j = 0; j < W; ++j) xw[j] = 0.0;
  fetch(n - 1, c);
  stage(colbuf + ((n - 1) & 1) * NB, c);
  double y_next = own ? T[(int64_t)(n - 1) * b + col] : 0.0;
  __syncthreads();
  for (int r = n - 1; r >= 0; --r) {
    const double* cur = colbuf + (r & 1) * NB;
    if (r > 0) fetch(r - 1, c);
    if (own) {
      const double y_r = y_next;
      if (r > 0) y_next = T[(int64_t)(r - 1) * b + col];
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
      for (int j = 0; j < W; j += 4) {
        s0 = fma(cur[j + 1], xw[j], s0);
        if (j + 1 < W) s1 = fma(cur[j + 2], xw[j + 1], s1);
        if (j + 2 < W) s2 = fma(cur[j + 3], xw[j + 2], s2);
        if (j + 3 < W) s3 = fma(cur[j + 4], xw[j + 3], s3);
      }
      const double x = (y_r - ((s0 + s1) + (s2 + s3))) / cur[0];
      T[(int64_t)r * b + col] = x;
#pragma unroll
      for (int j = W - 1; j > 0; --j) xw[j] = xw[j - 1];
      xw[0] = x;
    }
    if (r > 0) stage(colbuf + ((r - 1) & 1) * NB, c);
    __syncthreads();
  }
}

// Half bandwidths served by the register solve (one instantiation each).
constexpr int REG_SOLVE_W[] = {32, 64, 88};

// LDS bytes of the solve's window and band column for a batch (0: the
// per-lane solve from T)
inline size_t solve_window_bytes(const BuildBatch& bb) {
  const size_t bytes = (size_t)(bb.max_w + 1) * (bb.max_b + 1) * sizeof(double);
  return bytes <= 64 * 1024 ? bytes : 0;
}

// X = (A + s B)^{-1} B q_j = -C^{-1} B q_j with C = -(A + sB) = L L^T (the
// band factor); one lane per column of the block, row-major staging in the
// free A V region.
__global__ __launch_bounds__(NT) void k_shift_solve(BuildBatch bb, int j, int use_win) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (cell_failed(c) || j + 1 >= c.m) return;
  const int n = c.n, b = c.b, w = c.w, ld = w + 1;
  const double* band = bb.d_work + c.band_off;
  double* X = bb.d_work + c.x_off;
  double* T = bb.d_work + c.av_off;
  const double* q = bb.d_work + c.v_off + (int64_t)j * b * n;
  const double* bd = bb.d_bdiag + c.b_off;
  extern __shared__ double sw_win[];
  for (int col = threadIdx.x; col < b; col += blockDim.x)
    for (int r = 0; r < n; ++r) T[(int64_t)r * b + col] = bd[r] * q[r + (int64_t)col * n];
  if (use_win && b <= (int)blockDim.x) {
    wg_band_solve(band, ld, w, n, b, T, sw_win, sw_win + (int64_t)(w + 1) * b);
  } else {
    for (int col = threadIdx.x; col < b; col += blockDim.x) lane_band_solve(band, ld, w, n, b, T, col, nullptr);
  }
  for (int col = threadIdx.x; col < b; col += blockDim.x)
    for (int r = 0; r < n; ++r) X[r + (int64_t)col * n] = -T[(int64_t)r * b + col];
}

// The same solve with the register window (one wave, b <= 64, w <= W).
template <int W>
__global__ __launch_bounds__(64) void k_shift_solve_reg(BuildBatch bb, int j) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (cell_failed(c) || j + 1 >= c.m) return;
  const int n = c.n, b = c.b, w = c.w, ld = w + 1;
  const double* band = bb.d_work + c.band_off;
  double* X = bb.d_work + c.x_off;
  double* T = bb.d_work + c.av_off;
  const double* q = bb.d_work + c.v_off + (int64_t)j * b * n;
  const double* bd = bb.d_bdiag + c.b_off;
  __shared__ double colbuf[2 * (W + 1)];
  const int col = threadIdx.x;
  if (col < b)
    for (int r = 0; r < n; ++r) T[(int64_t)r * b + col] = bd[r] * q[r + (int64_t)col * n];
  reg_band_solve<W>(band, ld, w, n, b, T, colbuf);
  if (col < b)
    for (int r = 0; r < n; ++r) X[r + (int64_t)col * n] = -T[(int64_t)r * b + col];
}

// K3: A V (local CSR) then A^m = V^T (A V), symmetrised.
__global__ __launch_bounds__(NT) void k_project(BuildBatch bb) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (cell_failed(c)) return;
  const int n = c.n, mb = c.m * c.b;
  const double* V = bb.d_work + c.v_off;
  double* AV = bb.d_work + c.av_off;
  double* Am = bb.d_work + c.am_off;
  const int32_t* rp = bb.d_rowptr + c.rp_off;
  const int32_t* col = bb.d_col + c.csr_off;
  const double* a = bb.d_a + c.csr_off;
  wg_spmm_csr(n, mb, rp, col, a, V, AV);
  __syncthreads();
  wg_gemm<true, false>(mb, mb, n, 1.0, V, n, AV, n, 0.0, Am, mb);
  wg_symmetrize(mb, Am, mb);
}

// K4: block Lanczos on (A^m, I) from S^m = E_1 R_1.
// Work layout in the av region (free after K3): AQ (mb x b), Z (mb x b),
// coef (mb x b), gram (b x b); alphas/betas at s_off: alpha_k then beta_k.
// 3 waves per SIMD: a few spilled registers buy a third resident workgroup
// per CU for this chain of small dependent products
__global__ __launch_bounds__(NT, 3) void k_lanczos(BuildBatch bb) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (cell_failed(c)) return;
  const int b = c.b, m = c.m, mb = m * b;
  const double* Am = bb.d_work + c.am_off;
  double* Q = bb.d_work + c.q_off;
  double* AQ = bb.d_work + c.av_off;
  double* Z = AQ + (int64_t)mb * b;
  double* coef = Z + (int64_t)mb * b;
  double* gram = coef + (int64_t)mb * b;
  double* gram2 = gram + (int64_t)b * b;
  double* alpha = bb.d_work + c.s_off;                 // m b^2
  double* beta = alpha + (int64_t)m * b * b;           // m b^2 (beta_1 .. beta_m)
  const double* R1 = bb.d_work + c.r_off;
  // Q_1 = E_1, beta_1 = R_1
  for (int64_t idx = threadIdx.x; idx < (int64_t)mb * b; idx += NT) {
    const int i = idx % mb, j = idx / mb;
    Q[idx] = (i == j) ? 1.0 : 0.0;
  }
  wg_copy(b, b, R1, b, beta, b);
  for (int k = 0; k < m; ++k) {
    const double* Qk = Q + (int64_t)k * b * mb;
    double* ak = alpha + (int64_t)k * b * b;
    wg_gemm<false, false>(mb, b, mb, 1.0, Am, mb, Qk, mb, 0.0, AQ, mb);
    wg_gemm<true, false>(b, b, mb, 1.0, Qk, mb, AQ, mb, 0.0, ak, b);
    wg_symmetrize(b, ak, b);
    if (k == m - 1) break;
    wg_copy(mb, b, AQ, mb, Z, mb);
    wg_gemm<false, false>(mb, b, b, -1.0, Qk, mb, ak, b, 1.0, Z, mb);
    if (k > 0) {
      const double* bk = beta + (int64_t)k * b * b;
      wg_gemm<false, true>(mb, b, b, -1.0, Q + (int64_t)(k - 1) * b * mb, mb, bk, b, 1.0, Z, mb);
    }
    const int kb = (k + 1) * b;
    for (int pass = 0; pass < 2; ++pass) {
      wg_gemm<true, false>(kb, b, mb, 1.0, Q, mb, Z, mb, 0.0, coef, kb);
      wg_gemm<false, false>(mb, b, kb, -1.0, Q, mb, coef, kb, 1.0, Z, mb);
    }
    // Cholesky-QR, twice: Z = Q_{k+1} beta_{k+1}
    double* bn = beta + (int64_t)(k + 1) * b * b;
    wg_gemm<true, false>(b, b, mb, 1.0, Z, mb, Z, mb, 0.0, gram, b);
    wg_symmetrize(b, gram, b);
    double ratio = wg_potrf(b, gram, b);
    if (!(ratio > 1e-10)) { if (threadIdx.x == 0) { c.status = ST_BREAKDOWN; c.fail_block = k + 2; } return; }
    wg_trsm_right_lt(mb, b, gram, b, Z, mb);
    wg_gemm<true, false>(b, b, mb, 1.0, Z, mb, Z, mb, 0.0, gram2, b);
    wg_symmetrize(b, gram2, b);
    ratio = wg_potrf(b, gram2, b);
    if (!(ratio > 1e-6)) { if (threadIdx.x == 0) { c.status = ST_BREAKDOWN; c.fail_block = k + 2; } return; }
    wg_trsm_right_lt(mb, b, gram2, b, Z, mb);
    // beta = L2^T L1^T (upper)
    for (int idx = threadIdx.x; idx < b * b; idx += NT) {
      const int r = idx % b, cc = idx / b;
      double s = 0.0;
      for (int l = r; l <= cc; ++l) s += gram2[l + (int64_t)r * b] * gram[cc + (int64_t)l * b];
      bn[r + (int64_t)cc * b] = (r <= cc) ? s : 0.0;
    }
    wg_copy(mb, b, Z, mb, Q + (int64_t)(k + 1) * b * mb, mb);
  }
}

// K5: S-fraction blocks from (alpha_k, beta_k) (eq. GammaTrans, corrected).
// Output at out_off: Ghat^1..Ghat^m then G^1..G^m.
// No general inverse is formed: with H_k = G_k^{-T},
//   H_1 = beta_1^{-1} (beta_1 upper triangular, G_1 = beta_1^T),
//   Ghat^k = G_k G_k^T,  G^k = -H_k (alpha_k H_k^T) - G^{k-1},
//   G_{k+1} = (G_k^T G^k)^{-1} beta_{k+1}^T = (G^k)^{-1} H_k beta_{k+1}^T
//     (a Cholesky solve with the factor of G^k that the SPD check computes),
//   H_{k+1} = (G_{k+1}^{-1})^T = G^k G_k beta_{k+1}^{-1}
//     (a triangular solve), so every step is a product or a triangular solve.
// 3 waves per SIMD: a few spilled registers buy a third resident workgroup
// per CU for this chain of small dependent products
__global__ __launch_bounds__(NT, 3) void k_sfraction(BuildBatch bb) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (cell_failed(c)) return;
  const int b = c.b, m = c.m;
  const int64_t bb2 = (int64_t)b * b;
  const double* alpha = bb.d_work + c.s_off;
  const double* beta = alpha + m * bb2;
  double* out = bb.d_work + c.out_off;
  double* Ghat = out;
  double* G = out + m * bb2;
  // scratch in the av region: Gk, H (= G_k^{-T}), T1, Y, P, Bt, ch
  double* base = bb.d_work + c.av_off;
  double* Gk = base;
  double* H = Gk + bb2;
  double* T1 = H + bb2;
  double* Y = T1 + bb2;
  double* P = Y + bb2;
  double* Bt = P + bb2;
  double* ch = Bt + bb2;
  // G_1 = beta_1^T; H_1 = I beta_1^{-1} (right solve with beta_1^T as L^T)
  wg_transpose(b, beta, b, Gk, b);
  if (!wg_diag_ok(b, Gk, b)) { if (threadIdx.x == 0) c.status = ST_NOTSPD; return; }
  for (int idx = threadIdx.x; idx < b * b; idx += NT) H[idx] = (idx % b == idx / b) ? 1.0 : 0.0;
  __syncthreads();
  wg_trsm_right_lt(b, b, Gk, b, H, b);
  for (int k = 0; k < m; ++k) {
    double* Gh = Ghat + k * bb2;
    double* Gc = G + k * bb2;
    wg_gemm<false, true>(b, b, b, 1.0, Gk, b, Gk, b, 0.0, Gh, b);
    wg_symmetrize(b, Gh, b);
    wg_gemm<false, true>(b, b, b, 1.0, alpha + k * bb2, b, H, b, 0.0, T1, b);
    if (k > 0) wg_copy(b, b, G + (k - 1) * bb2, b, Gc, b);
    wg_gemm<false, false>(b, b, b, -1.0, H, b, T1, b, (k > 0) ? -1.0 : 0.0, Gc, b);
    wg_symmetrize(b, Gc, b);
    // SPD checks of the pivots (eq. S-fraction); the deepest G^m of a
    // floating cell is only semidefinite to rounding and is not checked.
    wg_copy(b, b, Gh, b, ch, b);
    double r1 = wg_potrf(b, ch, b);
    double r2 = 1.0;
    if (k < m - 1) {
      wg_copy(b, b, Gc, b, ch, b);
      r2 = wg_potrf(b, ch, b);      // ch: lower Cholesky factor L of G^k
    }
    if (!(r1 > 0.0) || !(r2 > 0.0)) { if (threadIdx.x == 0) c.status = ST_NOTSPD; return; }
    if (k < m - 1) {
      const double* bn = beta + (k + 1) * bb2;
      wg_transpose(b, bn, b, Bt, b);                                   // beta_{k+1}^T, lower
      if (!wg_diag_ok(b, Bt, b)) { if (threadIdx.x == 0) c.status = ST_NOTSPD; return; }
      // Y = H_k beta_{k+1}^T; G_{k+1}^T = Y^T L^{-T} L^{-1}
      wg_gemm<false, false>(b, b, b, 1.0, H, b, Bt, b, 0.0, Y, b);
      wg_transpose(b, Y, b, T1, b);
      wg_trsm_right_lt(b, b, ch, b, T1, b);
      wg_trsm_right_l(b, b, ch, b, T1, b);
      // P = G^k G_k, then H_{k+1} = P beta_{k+1}^{-1}
      wg_gemm<false, false>(b, b, b, 1.0, Gc, b, Gk, b, 0.0, P, b);
      wg_trsm_right_lt(b, b, Bt, b, P, b);
      wg_transpose(b, T1, b, Gk, b);
      wg_copy(b, b, P, b, H, b);
    }
  }
  // finite check
  __shared__ int s_nf;
  if (threadIdx.x == 0) s_nf = 0;
  __syncthreads();
  for (int64_t idx = threadIdx.x; idx < 2 * m * bb2; idx += NT)
    if (!isfinite(out[idx])) s_nf = 1;
  __syncthreads();
  if (threadIdx.x == 0 && s_nf) c.status = ST_NONFINITE;
}

// The same factorisation with the active part of the band in LDS: the
// w + 1 columns j .. j + w that step j reads or updates sit in a ring of
// slots (column c in slot c mod (w + 1), band offsets contiguous), so the
// rank-1 update is LDS arithmetic (one wave per updated column, lanes along
// it) and HBM sees each column once in each direction: column j leaves for
// the factor after its step and column j + w + 1, fetched into registers
// during the step, takes its slot. Every thread computes the pivot itself,
// so a step needs three barriers. Dynamic LDS: (w + 1)^2 doubles.
__global__ __launch_bounds__(NT) void k_band_chol_win(BuildBatch bb) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  const int n = c.n, w = c.w, W1 = w + 1, ld = w + 1;
  double* band = bb.d_work + c.band_off;
  const int32_t* rp = bb.d_rowptr + c.rp_off;
  const int32_t* col = bb.d_col + c.csr_off;
  const double* a = bb.d_a + c.csr_off;
  const double* bd = bb.d_bdiag + c.b_off;
  extern __shared__ double win[];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  for (int64_t idx = tid; idx < (int64_t)n * ld; idx += NT) band[idx] = 0.0;
  __syncthreads();
  for (int r = tid; r < n; r += NT) {
    for (int k = rp[r]; k < rp[r + 1]; ++k) {
      const int cc = col[k];
      if (r >= cc) band[(int64_t)cc * ld + (r - cc)] = -(a[k] + (r == cc ? bb.shift * bd[r] : 0.0));
    }
  }
  __syncthreads();
  for (int idx = tid; idx < min(W1, n) * W1; idx += NT) win[idx] = band[idx];
  __shared__ int s_bad;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double* cj = win + (j % W1) * W1;
    const bool refill = j + W1 < n;
    const double pre = (refill && tid < W1) ? band[(int64_t)(j + W1) * ld + tid] : 0.0;
    const double d = cj[0];
    const bool ok = d > 0.0 && isfinite(d);
    const double piv = ok ? sqrt(d) : 1.0;
    const double inv = 1.0 / piv;
    const int lim = min(w, n - 1 - j);
    if (tid >= 1 && tid <= lim) cj[tid] *= inv;
    if (tid == 0 && !ok) s_bad = 1;
    __syncthreads();
    for (int d1 = 1 + wv; d1 <= lim; d1 += NT / 64) {
      double* cd = win + ((j + d1) % W1) * W1;
      const double v1 = cj[d1];
      for (int e = lane; e <= lim - d1; e += 64) cd[e] -= cj[d1 + e] * v1;
    }
    __syncthreads();
    if (tid < W1) {
      band[(int64_t)j * ld + tid] = tid == 0 ? piv : cj[tid];
      if (refill) cj[tid] = pre;
    }
    __syncthreads();
  }
  if (tid == 0 && s_bad) c.status = ST_NOTNSD;
}

// LDS bytes of the windowed factorisation for a batch (0: use k_band_chol)
inline size_t chol_window_bytes(const BuildBatch& bb) {
  const size_t bytes = (size_t)(bb.max_w + 1) * (bb.max_w + 1) * sizeof(double);
  return (bb.max_w + 1 <= NT && bytes <= 64 * 1024) ? bytes : 0;
}

// Blocked build of a batch with wide bands: the same steps as launch_build
// with the band factorisation, the shifted solves and the tall-skinny
// products of the Krylov basis and of the projection spread over many
// workgroups per cell; block Lanczos and the S-fraction (m b x m b dense
// work) stay one workgroup per cell.
static hipError_t launch_build_wide(const BuildBatch& bb, hipStream_t st) {
  const dim3 grid(bb.ncell), block(NT);
  hipError_t e = launch_wide_chol(bb, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_krylov_start, grid, block, 0, st, bb);
  for (int j = 0; j < bb.max_m; ++j) {
    if (j > 0)
      for (int pass = 0; pass < 2; ++pass) {
        if ((e = launch_ts_gram(bb, TS_CGS, j, st)) != hipSuccess) return e;
        if ((e = launch_ts_update(bb, j, st)) != hipSuccess) return e;
      }
    if ((e = launch_ts_gram(bb, TS_NORM, j, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ts_chol, grid, block, 0, st, bb, j);
    if ((e = launch_ts_trsm_rows(bb, j, st)) != hipSuccess) return e;
    if (j + 1 < bb.max_m && (e = launch_wide_solve(bb, j, st)) != hipSuccess) return e;
  }
  if ((e = launch_ts_spmm(bb, st)) != hipSuccess) return e;
  if ((e = launch_ts_gram(bb, TS_PROJ, 0, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_lanczos, grid, block, 0, st, bb);
  hipLaunchKernelGGL(k_sfraction, grid, block, 0, st, bb);
  return hipGetLastError();
}

hipError_t launch_build(const BuildBatch& bb, hipStream_t st) {
  const dim3 grid(bb.ncell), block(NT);
  const bool wide = build_is_wide(bb, bb.wide_mode);
  if (wide) return launch_build_wide(bb, st);
  const size_t cw = chol_window_bytes(bb);
  if (cw) {
    hipLaunchKernelGGL(k_band_chol_win, grid, block, cw, st, bb);
  } else {
    hipLaunchKernelGGL(k_band_chol, grid, block, 0, st, bb);
  }
  hipLaunchKernelGGL(k_krylov_start, grid, block, 0, st, bb);
  for (int j = 0; j < bb.max_m; ++j) {
    hipLaunchKernelGGL(k_cgs2, grid, block, 0, st, bb, j);
    hipLaunchKernelGGL(k_normalize, grid, block, 0, st, bb, j);
    // one lane per right-hand side: the window in registers when one wave
    // holds every right-hand side and the band fits a register window, else
    // in LDS
    if (j + 1 < bb.max_m) {
      int regw = 0;
      if (bb.max_b <= 64)
        for (int W : REG_SOLVE_W)
          if (!regw && bb.max_w <= W) regw = W;
      if (regw == REG_SOLVE_W[0]) {
        hipLaunchKernelGGL(k_shift_solve_reg<REG_SOLVE_W[0]>, grid, dim3(64), 0, st, bb, j);
      } else if (regw == REG_SOLVE_W[1]) {
        hipLaunchKernelGGL(k_shift_solve_reg<REG_SOLVE_W[1]>, grid, dim3(64), 0, st, bb, j);
      } else if (regw == REG_SOLVE_W[2]) {
        hipLaunchKernelGGL(k_shift_solve_reg<REG_SOLVE_W[2]>, grid, dim3(64), 0, st, bb, j);
      } else {
        const size_t wb = solve_window_bytes(bb);
        hipLaunchKernelGGL(k_shift_solve, grid, dim3(std::min(NT, (bb.max_b + 63) / 64 * 64)), wb, st, bb, j,
                           wb > 0 ? 1 : 0);
      }
    }
  }
  hipLaunchKernelGGL(k_project, grid, block, 0, st, bb);
  hipLaunchKernelGGL(k_lanczos, grid, block, 0, st, bb);
  hipLaunchKernelGGL(k_sfraction, grid, block, 0, st, bb);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// packing into the on-line layout and piece masses
// ---------------------------------------------------------------------------

template <typename T>
__device__ inline T cvt(double v);
template <>
__device__ inline double cvt<double>(double v) { return v; }
template <>
__device__ inline float cvt<float>(double v) { return (float)v; }
template <>
__device__ inline __hip_bfloat16 cvt<__hip_bfloat16>(double v) { return __float2bfloat16((float)v); }

// On-line blocks of a cell: the three-point scheme with its hidden layers
// in the variables V^k = G_k^{-1} U^k (unit mass) is block tridiagonal with
// D_0 = -G^1, C_0 = G^1 G_2 = G_1^{-T} beta_2^T = beta_1^{-1} beta_2^T, and
// for l >= 1 D_l = -G_l^T (G^l + G^{l-1}) G_l = alpha_l and
// C_l = G_l^T G^l G_{l+1} = beta_{l+1}^T (both by eq. GammaTrans; layers
// counted from 0). They are stored as D_0, C_0, D_1, ..., D_{m-1}, each b
// rows of stride ld (row-major, zero padded). The FP64 S-fraction blocks are
// kept as well (export, piece masses, spectral bound).
template <typename T>
__global__ __launch_bounds__(NT) void k_pack(BuildCell* bc, double* work, const OnlineCell* oc, T* blocks,
                                             double* rom64, const int64_t* rom64_off) {
  BuildCell& c = bc[blockIdx.x];
  const OnlineCell& o = oc[blockIdx.x];
  const int b = c.b, m = c.m;
  const int64_t bb2 = (int64_t)b * b;
  const double* src = work + c.out_off;
  double* r64 = rom64 + rom64_off[blockIdx.x];
  for (int64_t idx = threadIdx.x; idx < 2 * m * bb2; idx += NT) r64[idx] = src[idx];
  if (cell_failed(c)) return;
  const double* alpha = work + c.s_off;
  const double* beta = alpha + m * bb2;
  double* C0 = work + c.av_off;
  if (m > 1) {
    double* binv = C0 + bb2;
    double* Wk = binv + bb2;
    double* fac = Wk + bb2;
    if (!wg_inverse(b, beta, b, binv, b, Wk, fac)) {
      if (threadIdx.x == 0) c.status = ST_NOTSPD;
      return;
    }
    wg_gemm<false, true>(b, b, b, 1.0, binv, b, beta + bb2, b, 0.0, C0, b);
  }
  const double* G1 = src + m * bb2;
  T* dst = blocks + o.blk_off;
  const int ld = o.ld;
  const int64_t bsz = (int64_t)b * ld;
  for (int64_t idx = threadIdx.x; idx < (2 * m - 1) * bsz; idx += NT) {
    const int j = (int)(idx / bsz);
    const int r = (int)((idx % bsz) / ld), cc = (int)(idx % ld);
    const int l = j >> 1;
    double v = 0.0;
    if (cc < b) {
      if ((j & 1) == 0) {
        const double* M = (l == 0) ? G1 : alpha + l * bb2;
        v = 0.5 * (M[r + (int64_t)cc * b] + M[cc + (int64_t)r * b]);
        if (l == 0) v = -v;
      } else {
        v = (l == 0) ? C0[r + (int64_t)cc * b] : beta[(l + 1) * bb2 + cc + (int64_t)r * b];
      }
    }
    dst[idx] = cvt<T>(v);
  }
}

hipError_t launch_pack(int32_t ncell, BuildCell* d_bcells, double* d_work,
                       const OnlineCell* d_ocells, int32_t prec, void* d_blocks, double* d_rom64,
                       const int64_t* d_rom64_off, hipStream_t st) {
  const dim3 grid(ncell), block(NT);
  if (prec == SFROM_F64)
    hipLaunchKernelGGL(k_pack<double>, grid, block, 0, st, d_bcells, d_work, d_ocells, (double*)d_blocks, d_rom64, d_rom64_off);
  else if (prec == SFROM_F32)
    hipLaunchKernelGGL(k_pack<float>, grid, block, 0, st, d_bcells, d_work, d_ocells, (float*)d_blocks, d_rom64, d_rom64_off);
  else
    hipLaunchKernelGGL(k_pack<__hip_bfloat16>, grid, block, 0, st, d_bcells, d_work, d_ocells, (__hip_bfloat16*)d_blocks, d_rom64, d_rom64_off);
  return hipGetLastError();
}

// M_p = sum_{cells c owning p} ([Ghat_c^1]_pp)^{-1}; store M_p^{-1}. One
// thread per piece (b_p is small: a face or edge basis); the three b_p x b_p
// work matrices live in global scratch at 3 * minv_off.
template <typename T>
__global__ void k_piece_mass(MassArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.npiece) return;
  const OnlinePiece pc = a.d_pieces[p];
  const int bp = pc.b;
  double* M = a.d_scratch + 3 * pc.minv_off;
  double* Wm = M + bp * bp;
  double* Inv = Wm + bp * bp;
  for (int i = 0; i < bp * bp; ++i) M[i] = 0.0;
  for (int e = 0; e < pc.ncell; ++e) {
    const int cell = a.d_inc_cell[pc.inc_off + e];
    const int col0 = a.d_inc_col[pc.inc_off + e];
    const int b = a.d_cells[cell].b;
    const double* G1 = a.d_rom64 + a.d_rom64_off[cell];   // Ghat^1 of the cell
    for (int j = 0; j < bp; ++j)
      for (int i = 0; i < bp; ++i) Wm[i + j * bp] = G1[(col0 + i) + (int64_t)(col0 + j) * b];
    // invert the small SPD block by Gauss-Jordan
    for (int i = 0; i < bp * bp; ++i) Inv[i] = 0.0;
    for (int i = 0; i < bp; ++i) Inv[i + i * bp] = 1.0;
    int ok = 1;
    for (int j = 0; j < bp; ++j) {
      int piv = j;
      for (int i = j + 1; i < bp; ++i) if (fabs(Wm[i + j * bp]) > fabs(Wm[piv + j * bp])) piv = i;
      if (!(fabs(Wm[piv + j * bp]) > 0.0)) { ok = 0; break; }
      if (piv != j)
        for (int cc = 0; cc < bp; ++cc) {
          double t = Wm[j + cc * bp]; Wm[j + cc * bp] = Wm[piv + cc * bp]; Wm[piv + cc * bp] = t;
          t = Inv[j + cc * bp]; Inv[j + cc * bp] = Inv[piv + cc * bp]; Inv[piv + cc * bp] = t;
        }
      const double ip = 1.0 / Wm[j + j * bp];
      for (int cc = 0; cc < bp; ++cc) { Wm[j + cc * bp] *= ip; Inv[j + cc * bp] *= ip; }
      for (int i = 0; i < bp; ++i) {
        if (i == j) continue;
        const double f = Wm[i + j * bp];
        if (f == 0.0) continue;
        for (int cc = 0; cc < bp; ++cc) { Wm[i + cc * bp] -= f * Wm[j + cc * bp]; Inv[i + cc * bp] -= f * Inv[j + cc * bp]; }
      }
    }
    if (!ok) { a.d_status[p] = 1; return; }
    for (int i = 0; i < bp * bp; ++i) M[i] += Inv[i];
  }
  // M_p^{-1}
  for (int i = 0; i < bp * bp; ++i) { Wm[i] = 0.5 * (M[i] + M[(i % bp) * bp + i / bp]); Inv[i] = 0.0; }
  for (int i = 0; i < bp; ++i) Inv[i + i * bp] = 1.0;
  for (int j = 0; j < bp; ++j) {
    int piv = j;
    for (int i = j + 1; i < bp; ++i) if (fabs(Wm[i + j * bp]) > fabs(Wm[piv + j * bp])) piv = i;
    if (!(fabs(Wm[piv + j * bp]) > 0.0)) { a.d_status[p] = 1; return; }
    if (piv != j)
      for (int cc = 0; cc < bp; ++cc) {
        double t = Wm[j + cc * bp]; Wm[j + cc * bp] = Wm[piv + cc * bp]; Wm[piv + cc * bp] = t;
        t = Inv[j + cc * bp]; Inv[j + cc * bp] = Inv[piv + cc * bp]; Inv[piv + cc * bp] = t;
      }
    const double ip = 1.0 / Wm[j + j * bp];
    for (int cc = 0; cc < bp; ++cc) { Wm[j + cc * bp] *= ip; Inv[j + cc * bp] *= ip; }
    for (int i = 0; i < bp; ++i) {
      if (i == j) continue;
      const double f = Wm[i + j * bp];
      if (f == 0.0) continue;
      for (int cc = 0; cc < bp; ++cc) { Wm[i + cc * bp] -= f * Wm[j + cc * bp]; Inv[i + cc * bp] -= f * Inv[j + cc * bp]; }
    }
  }
  T* out = (T*)a.d_minv + pc.minv_off;
  for (int i = 0; i < bp * bp; ++i) out[i] = cvt<T>(0.5 * (Inv[i] + Inv[(i % bp) * bp + i / bp]));
  a.d_status[p] = 0;
}

hipError_t launch_piece_mass(const MassArgs& a, hipStream_t st) {
  const int tpb = 64;
  const dim3 grid((a.npiece + tpb - 1) / tpb), block(tpb);
  // masses are kept in float for BF16 (only the blocks are bfloat16)
  if (a.prec == SFROM_F64)
    hipLaunchKernelGGL(k_piece_mass<double>, grid, block, 0, st, a);
  else
    hipLaunchKernelGGL(k_piece_mass<float>, grid, block, 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Learned off-line stage: S-fraction from predicted Cholesky factors, the
// transfer-function fallback test, and factor targets of built cells.
// Workspace regions of a cell (see the build's layout): out = S-fraction
// (Ghat^1..m, G^1..m), av = scratch, am = on-line blocks in FP64 (D_0, C_0,
// ..., D_{m-1}, column-major b x b), r = (Ghat^1)^{-1}, q = R factors or
// the dense ROM matrix, s = transfer functions, v = A X or Z, x = X.
// ---------------------------------------------------------------------------

// Lower Cholesky factor stored as the row-major lower triangle of a b x b
// matrix: element (i, j), j <= i, at i (i + 1) / 2 + j.
__device__ inline int tri_index(int i, int j) { return i * (i + 1) / 2 + j; }

// S-fraction of a candidate cell: layer 1 in closed form from B, W and A
// (Ghat^1 = W^T B^{-1} W, G^1 = -(Ghat^1)^{-1} X^T A X (Ghat^1)^{-1},
// X = B^{-1} W, which k_krylov_start has written), layers 2..m from the
// predicted factors as L L^T + eps I (eps = 1e-10 tr / b), so every pivot is
// SPD by construction.
__global__ __launch_bounds__(NT) void k_learned_sfraction(BuildBatch bb, const float* __restrict__ y, int P) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (cell_failed(c)) return;
  const int n = c.n, b = c.b, m = c.m;
  const int64_t bb2 = (int64_t)b * b;
  const double* X = bb.d_work + c.x_off;
  const double* bd = bb.d_bdiag + c.b_off;
  double* AX = bb.d_work + c.v_off;
  double* out = bb.d_work + c.out_off;
  double* Gh = out;
  double* G = out + m * bb2;
  double* T = bb.d_work + c.av_off;
  double* T2 = T + bb2;
  double* Gi = T2 + bb2;
  double* Wk = Gi + bb2;
  double* fac = Wk + bb2;
  const int32_t* rp = bb.d_rowptr + c.rp_off;
  const int32_t* col = bb.d_col + c.csr_off;
  const double* a = bb.d_a + c.csr_off;
  // Ghat^1 = X^T B X
  for (int idx = threadIdx.x; idx < b * b; idx += NT) {
    const int i = idx % b, j = idx / b;
    double acc = 0.0;
    for (int r = 0; r < n; ++r) acc += X[r + (int64_t)i * n] * bd[r] * X[r + (int64_t)j * n];
    Gh[idx] = acc;
  }
  // A X
  for (int64_t idx = threadIdx.x; idx < (int64_t)n * b; idx += NT) {
    const int r = (int)(idx % n), j = (int)(idx / n);
    double acc = 0.0;
    for (int k = rp[r]; k < rp[r + 1]; ++k) acc += a[k] * X[col[k] + (int64_t)j * n];
    AX[idx] = acc;
  }
  __syncthreads();
  wg_symmetrize(b, Gh, b);
  wg_gemm<true, false>(b, b, n, 1.0, X, n, AX, n, 0.0, T, b);          // X^T A X
  if (!wg_inverse(b, Gh, b, Gi, b, Wk, fac)) { if (threadIdx.x == 0) c.status = ST_NOTSPD; return; }
  wg_gemm<false, false>(b, b, b, 1.0, T, b, Gi, b, 0.0, T2, b);
  wg_gemm<false, false>(b, b, b, -1.0, Gi, b, T2, b, 0.0, G, b);
  wg_symmetrize(b, G, b);
  // deep layers from the factors
  const float* yc = y + (int64_t)blockIdx.x * P;
  const int nt = b * (b + 1) / 2;
  for (int k = 1; k < m; ++k) {
    for (int which = 0; which < 2; ++which) {
      const float* f = yc + (int64_t)(2 * (k - 1) + which) * nt;
      for (int idx = threadIdx.x; idx < b * b; idx += NT) {
        const int i = idx % b, j = idx / b;
        T[idx] = (j <= i) ? (double)f[tri_index(i, j)] : 0.0;
      }
      __syncthreads();
      double* M = (which == 0 ? Gh : G) + k * bb2;
      wg_gemm<false, true>(b, b, b, 1.0, T, b, T, b, 0.0, M, b);
      __shared__ double s_tr;
      if (threadIdx.x == 0) {
        double tr = 0.0;
        for (int i = 0; i < b; ++i) tr += M[i + (int64_t)i * b];
        s_tr = tr;
      }
      __syncthreads();
      const double eps = 1e-10 * s_tr / b;
      for (int i = threadIdx.x; i < b; i += NT) M[i + (int64_t)i * b] += eps;
      __syncthreads();
      wg_symmetrize(b, M, b);
    }
  }
}

// On-line blocks in FP64 of a cell whose S-fraction is in `out`, with
// R_k = chol(Ghat^k) (k >= 2) as the change of variables of the hidden
// layers: D_0 = -G^1, C_0 = G^1 R_2, D_l = -R_l^T (G^l + G^{l-1}) R_l,
// C_l = R_l^T G^l R_{l+1}; also (Ghat^1)^{-1} for the transfer function.
__global__ __launch_bounds__(NT) void k_sfraction_to_normal(BuildBatch bb) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (cell_failed(c)) return;
  const int b = c.b, m = c.m;
  const int64_t bb2 = (int64_t)b * b;
  const double* Gh = bb.d_work + c.out_off;
  const double* G = Gh + m * bb2;
  double* R = bb.d_work + c.q_off;          // R_1..R_{m-1} (0-based layers)
  double* blk = bb.d_work + c.am_off;
  double* T = bb.d_work + c.av_off;
  double* T2 = T + bb2;
  double* Wk = T2 + bb2;
  double* fac = Wk + bb2;
  double* Gi = bb.d_work + c.r_off;
  if (!wg_inverse(b, Gh, b, Gi, b, Wk, fac)) { if (threadIdx.x == 0) c.status = ST_NOTSPD; return; }
  for (int k = 1; k < m; ++k) {
    double* Rk = R + (k - 1) * bb2;
    wg_copy(b, b, Gh + k * bb2, b, Rk, b);
    if (!(wg_potrf(b, Rk, b) > 0.0)) { if (threadIdx.x == 0) c.status = ST_NOTSPD; return; }
    for (int idx = threadIdx.x; idx < b * b; idx += NT) {
      const int i = idx % b, j = idx / b;
      if (i < j) Rk[idx] = 0.0;
    }
    __syncthreads();
  }
  for (int l = 0; l < m; ++l) {
    double* D = blk + 2 * l * bb2;
    if (l == 0) {
      for (int idx = threadIdx.x; idx < b * b; idx += NT) D[idx] = -G[idx];
      __syncthreads();
    } else {
      const double* Rl = R + (l - 1) * bb2;
      for (int idx = threadIdx.x; idx < b * b; idx += NT) T[idx] = G[l * bb2 + idx] + G[(l - 1) * bb2 + idx];
      __syncthreads();
      wg_gemm<false, false>(b, b, b, 1.0, T, b, Rl, b, 0.0, T2, b);
      wg_gemm<true, false>(b, b, b, -1.0, Rl, b, T2, b, 0.0, D, b);
      wg_symmetrize(b, D, b);
    }
    if (l + 1 < m) {
      double* Cb = blk + (2 * l + 1) * bb2;
      const double* Rn = R + l * bb2;
      wg_gemm<false, false>(b, b, b, 1.0, G + l * bb2, b, Rn, b, 0.0, T2, b);
      if (l == 0) wg_copy(b, b, T2, b, Cb, b);
      else wg_gemm<true, false>(b, b, b, 1.0, R + (l - 1) * bb2, b, T2, b, 0.0, Cb, b);
    }
  }
}

// Exact cell transfer function F(z) = W^T (A + z B)^{-1} W from the band
// factor of -(A + z B) that k_band_chol left (shift z < 0); F goes to s.
__global__ __launch_bounds__(NT) void k_tf_exact(BuildBatch bb, int use_win) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (cell_failed(c)) return;
  const int n = c.n, b = c.b, w = c.w, ld = w + 1;
  const double* band = bb.d_work + c.band_off;
  double* Wd = bb.d_work + c.v_off;
  double* T = bb.d_work + c.av_off;
  double* F = bb.d_work + c.s_off;
  for (int64_t idx = threadIdx.x; idx < (int64_t)n * b; idx += NT) Wd[idx] = 0.0;
  __syncthreads();
  for (int k = threadIdx.x; k < c.nw; k += NT) {
    const int64_t e = c.w_off + k;
    const int row = bb.d_wrow[e], col0 = bb.d_wcol[e], bp = bb.d_wbp[e], kp = bb.d_wkp[e];
    const double* sp = bb.d_S + bb.d_wsoff[e];
    for (int l = 0; l < bp; ++l) Wd[row + (int64_t)(col0 + l) * n] = sp[(int64_t)l * kp];
  }
  __syncthreads();
  extern __shared__ double tf_win[];
  for (int col = threadIdx.x; col < b; col += NT)
    for (int r = 0; r < n; ++r) T[(int64_t)r * b + col] = Wd[r + (int64_t)col * n];
  if (use_win && b <= NT) {
    wg_band_solve(band, ld, w, n, b, T, tf_win, tf_win + (int64_t)(w + 1) * b);
  } else {
    for (int col = threadIdx.x; col < b; col += NT) lane_band_solve(band, ld, w, n, b, T, col, nullptr);
  }
  __syncthreads();
  // (A + z B)^{-1} = -(L L^T)^{-1}; T is row-major n x b
  wg_gemm<true, true>(b, b, n, -1.0, Wd, n, T, b, 0.0, F, b);
}

// ROM transfer function U^1(z) = E_1^T (L' + z D')^{-1} E_1 of the on-line
// blocks (D' = blkdiag((Ghat^1)^{-1}, I, ..., I)) via the Cholesky factor of
// M = -(L' + z D') (SPD for z < 0): U^1 = -Z^T Z with Z = chol(M)^{-1} E_1.
// mis[cell] = max(mis, ||U^1 - F||_F / ||F||_F).
__global__ __launch_bounds__(NT) void k_tf_rom(BuildBatch bb, double z, double* __restrict__ mis) {
  BuildCell& c = bb.d_cells[blockIdx.x];
  if (cell_failed(c)) return;
  const int b = c.b, m = c.m, mb = m * b;
  const int64_t bb2 = (int64_t)b * b;
  const double* blk = bb.d_work + c.am_off;
  const double* Gi = bb.d_work + c.r_off;
  double* M = bb.d_work + c.q_off;
  double* Z = bb.d_work + c.v_off;
  const double* F = bb.d_work + c.s_off;
  double* U = bb.d_work + c.s_off + bb2;
  for (int64_t idx = threadIdx.x; idx < (int64_t)mb * mb; idx += NT) {
    const int i = (int)(idx % mb), j = (int)(idx / mb);
    const int li = i / b, lj = j / b, ri = i % b, rj = j % b;
    double v = 0.0;
    if (li == lj) {
      v = -blk[2 * li * bb2 + ri + (int64_t)rj * b];
      if (li == 0) v -= z * Gi[ri + (int64_t)rj * b];
      else if (ri == rj) v -= z;
    } else if (lj == li + 1) {
      v = -blk[(2 * li + 1) * bb2 + ri + (int64_t)rj * b];           // -C_li
    } else if (li == lj + 1) {
      v = -blk[(2 * lj + 1) * bb2 + rj + (int64_t)ri * b];           // -C_lj^T
    }
    M[idx] = v;
  }
  __syncthreads();
  if (!(wg_potrf(mb, M, mb) > 0.0)) {
    if (threadIdx.x == 0) mis[blockIdx.x] = 1e300;
    return;
  }
  for (int64_t idx = threadIdx.x; idx < (int64_t)mb * b; idx += NT) {
    const int i = (int)(idx % mb), j = (int)(idx / mb);
    Z[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < mb; ++j) {
    const double ip = 1.0 / M[j + (int64_t)j * mb];
    for (int cc = threadIdx.x; cc < b; cc += NT) Z[j + (int64_t)cc * mb] *= ip;
    __syncthreads();
    for (int idx = threadIdx.x; idx < (mb - 1 - j) * b; idx += NT) {
      const int i = j + 1 + idx % (mb - 1 - j), cc = idx / (mb - 1 - j);
      Z[i + (int64_t)cc * mb] -= M[i + (int64_t)j * mb] * Z[j + (int64_t)cc * mb];
    }
    __syncthreads();
  }
  wg_gemm<true, false>(b, b, mb, -1.0, Z, mb, Z, mb, 0.0, U, b);
  __shared__ double s_num[NT], s_den[NT];
  double num = 0.0, den = 0.0;
  for (int idx = threadIdx.x; idx < b * b; idx += NT) {
    const double d = U[idx] - F[idx];
    num += d * d;
    den += F[idx] * F[idx];
  }
  s_num[threadIdx.x] = num;
  s_den[threadIdx.x] = den;
  __syncthreads();
  for (int st = NT / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      s_num[threadIdx.x] += s_num[threadIdx.x + st];
      s_den[threadIdx.x] += s_den[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double r = sqrt(s_num[0] / s_den[0]);
    mis[blockIdx.x] = fmax(mis[blockIdx.x], (r == r) ? r : 1e300);
  }
}

// Copies the S-fraction to rom64 and packs the FP64 on-line blocks of the
// cells with take[cell] != 0 into the on-line layout (row-major b x ld,
// diagonal blocks symmetrised).
template <typename T>
__global__ __launch_bounds__(NT) void k_pack_normal(const BuildCell* bc, const double* work, const OnlineCell* oc,
                                                    const int32_t* take, T* blocks, double* rom64,
                                                    const int64_t* rom64_off) {
  const BuildCell& c = bc[blockIdx.x];
  if (!take[blockIdx.x] || c.status != ST_OK) return;
  const OnlineCell& o = oc[blockIdx.x];
  const int b = c.b, m = c.m;
  const int64_t bb2 = (int64_t)b * b;
  const double* src = work + c.out_off;
  double* r64 = rom64 + rom64_off[blockIdx.x];
  for (int64_t idx = threadIdx.x; idx < 2 * m * bb2; idx += NT) r64[idx] = src[idx];
  const double* blk = work + c.am_off;
  T* dst = blocks + o.blk_off;
  const int ld = o.ld;
  const int64_t bsz = (int64_t)b * ld;
  for (int64_t idx = threadIdx.x; idx < (2 * m - 1) * bsz; idx += NT) {
    const int j = (int)(idx / bsz);
    const int r = (int)((idx % bsz) / ld), cc = (int)(idx % ld);
    double v = 0.0;
    if (cc < b) {
      const double* B = blk + j * bb2;
      v = (j & 1) ? B[r + (int64_t)cc * b] : 0.5 * (B[r + (int64_t)cc * b] + B[cc + (int64_t)r * b]);
    }
    dst[idx] = cvt<T>(v);
  }
}

// Targets of built cells: rows of the lower Cholesky factors of Ghat^k and
// G^k + eps I (eps = 1e-10 tr(G^k) / b), k = 2..m, one cell per workgroup;
// scratch holds b^2 doubles per cell.
__global__ __launch_bounds__(NT) void k_factor_targets(const double* rom64, const int64_t* rom64_off,
                                                       const int32_t* cells, int b, int m, double* scratch,
                                                       float* out, int P, int32_t* bad) {
  const int i = cells[blockIdx.x];
  const int64_t bb2 = (int64_t)b * b;
  const double* Gh = rom64 + rom64_off[i];
  const double* G = Gh + m * bb2;
  double* T = scratch + (int64_t)blockIdx.x * bb2;
  float* o = out + (int64_t)blockIdx.x * P;
  const int nt = b * (b + 1) / 2;
  for (int k = 1; k < m; ++k) {
    for (int which = 0; which < 2; ++which) {
      const double* M = (which == 0 ? Gh : G) + k * bb2;
      __shared__ double s_tr;
      if (threadIdx.x == 0) {
        double tr = 0.0;
        for (int q = 0; q < b; ++q) tr += M[q + (int64_t)q * b];
        s_tr = tr;
      }
      __syncthreads();
      const double eps = (which == 1) ? 1e-10 * s_tr / b : 0.0;
      for (int idx = threadIdx.x; idx < b * b; idx += NT) T[idx] = M[idx] + ((idx % b == idx / b) ? eps : 0.0);
      __syncthreads();
      if (!(wg_potrf(b, T, b) > 0.0)) { if (threadIdx.x == 0) bad[blockIdx.x] = 1; return; }
      float* f = o + (int64_t)(2 * (k - 1) + which) * nt;
      for (int idx = threadIdx.x; idx < nt; idx += NT) {
        // row-major lower triangle: idx -> (r, q)
        int r = (int)((sqrt(8.0 * idx + 1.0) - 1.0) / 2.0);
        while (r * (r + 1) / 2 > idx) --r;
        while ((r + 1) * (r + 2) / 2 <= idx) ++r;
        const int q = idx - r * (r + 1) / 2;
        f[idx] = (float)T[r + (int64_t)q * b];
      }
      __syncthreads();
    }
  }
}

hipError_t launch_learned_check(const BuildBatch& bb, const float* y, int P, const double* z, int nz, double* mis,
                                hipStream_t st) {
  const dim3 grid(bb.ncell), block(NT);
  hipLaunchKernelGGL(k_krylov_start, grid, block, 0, st, bb);
  hipLaunchKernelGGL(k_learned_sfraction, grid, block, 0, st, bb, y, P);
  hipLaunchKernelGGL(k_sfraction_to_normal, grid, block, 0, st, bb);
  for (int j = 0; j < nz; ++j) {
    BuildBatch bz = bb;
    bz.shift = z[j];
    const size_t cw = chol_window_bytes(bz);
    if (cw) hipLaunchKernelGGL(k_band_chol_win, grid, block, cw, st, bz);
    else hipLaunchKernelGGL(k_band_chol, grid, block, 0, st, bz);
    const size_t wb = solve_window_bytes(bz);
    hipLaunchKernelGGL(k_tf_exact, grid, block, wb, st, bz, wb > 0 ? 1 : 0);
    hipLaunchKernelGGL(k_tf_rom, grid, block, 0, st, bz, z[j], mis);
  }
  return hipGetLastError();
}

hipError_t launch_pack_normal(int32_t ncell, const BuildCell* d_bcells, const double* d_work,
                              const OnlineCell* d_ocells, const int32_t* d_take, int32_t prec, void* d_blocks,
                              double* d_rom64, const int64_t* d_rom64_off, hipStream_t st) {
  const dim3 grid(ncell), block(NT);
  if (prec == SFROM_F64)
    hipLaunchKernelGGL(k_pack_normal<double>, grid, block, 0, st, d_bcells, d_work, d_ocells, d_take, (double*)d_blocks, d_rom64, d_rom64_off);
  else if (prec == SFROM_F32)
    hipLaunchKernelGGL(k_pack_normal<float>, grid, block, 0, st, d_bcells, d_work, d_ocells, d_take, (float*)d_blocks, d_rom64, d_rom64_off);
  else
    hipLaunchKernelGGL(k_pack_normal<__hip_bfloat16>, grid, block, 0, st, d_bcells, d_work, d_ocells, d_take, (__hip_bfloat16*)d_blocks, d_rom64, d_rom64_off);
  return hipGetLastError();
}

hipError_t launch_factor_targets(const double* d_rom64, const int64_t* d_rom64_off, const int32_t* d_cells, int n,
                                 int b, int m, double* d_scratch, float* d_out, int P, int32_t* d_bad,
                                 hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_factor_targets, dim3(n), dim3(NT), 0, st, d_rom64, d_rom64_off, d_cells, b, m, d_scratch,
                     d_out, P, d_bad);
  return hipGetLastError();
}

}  // namespace sfrom_impl
