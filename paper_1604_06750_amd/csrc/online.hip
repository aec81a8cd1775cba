// On-line stage (Alg. alg1red stage 2): one explicit leapfrog step of the
// coupled S-fraction ROM for a batch of sources.
//
// Unknowns: reduced piece dofs y_p (the conjugated boundary values of
// eq. contred) and each cell's hidden layers U^2..U^m. With U^1 the cell's
// piece dofs gathered in the column order of its boundary basis and
// U^{m+1} = 0, the step is
//
//   cell phase   Phi^k = G^k (U^{k+1} - U^k),                k = 1..m
//                U^k <- 2U^k - U^k_old + dt^2 Ghat^k (Phi^k - Phi^{k-1}),
//                                                           k = 2..m
//                (eq. intrtstep_td; Alg. alg1red step 2.2)
//   piece phase  r_p = sum over the cells owning p of their Phi^1 slice
//                      + w^n g_p                            (step 2.1)
//                y_p <- 2y_p - y_p,old + dt^2 M_p^{-1} r_p   (eq. bdrytstep,
//                M_p = sum_i [(Ghat_i^1)^{-1}]_pp; step 2.3)
//   receivers    trace = sum_p q_p^T y_p                     (eq. solatrec)
//
// State rows hold n_s sources contiguously ([row][source]). The exchange
// between the two phases goes through the Phi^1 scratch in HBM, summed in a
// fixed order (no atomics), so results are deterministic.

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include "sfrom_internal.h"

namespace sfrom_impl {

template <typename TB, typename TA>
__device__ inline TA ld_block(const TB* p);
template <>
__device__ inline double ld_block<double, double>(const double* p) { return *p; }
template <>
__device__ inline float ld_block<float, float>(const float* p) { return *p; }
template <>
__device__ inline float ld_block<__hip_bfloat16, float>(const __hip_bfloat16* p) {
  return __bfloat162float(*p);
}

constexpr int CELL_NT = 256;

// Cell phase. grid = (n_cells, ceil(n_s / nst)); dynamic LDS holds U and Phi
// for the workgroup's source tile: 2 * max_m * max_b * nst accumulators.
template <typename T, typename TB, typename TA>
__global__ __launch_bounds__(CELL_NT) void k_cell_phase(StepArgs a, int nst) {
  extern __shared__ unsigned char smem_raw[];
  TA* U = reinterpret_cast<TA*>(smem_raw);
  TA* P = U + (int64_t)a.max_m * a.max_b * nst;
  const OnlineCell c = a.d_cells[blockIdx.x];
  const int m = c.m, b = c.b, ns = a.ns;
  const int s0 = blockIdx.y * nst;
  const int nsl = min(nst, ns - s0);
  const int lay = b * nst;
  const T* ycur = reinterpret_cast<const T*>(a.y_cur);
  const T* hcur = reinterpret_cast<const T*>(a.h_cur);
  T* hold = reinterpret_cast<T*>(a.h_old);
  T* phi = reinterpret_cast<T*>(a.phi);
  const int32_t* gat = a.d_gather + c.u1_off;
  for (int idx = threadIdx.x; idx < lay; idx += CELL_NT) {
    const int r = idx / nst, s = idx % nst;
    U[idx] = (s < nsl) ? (TA)ycur[(int64_t)gat[r] * ns + s0 + s] : (TA)0;
  }
  for (int k = 1; k < m; ++k) {
    const int64_t row0 = c.hid_off + (int64_t)(k - 1) * b;
    for (int idx = threadIdx.x; idx < lay; idx += CELL_NT) {
      const int r = idx / nst, s = idx % nst;
      U[k * lay + idx] = (s < nsl) ? (TA)hcur[(row0 + r) * ns + s0 + s] : (TA)0;
    }
  }
  __syncthreads();
  const TB* blk = reinterpret_cast<const TB*>(a.d_blocks) + c.blk_off;
  // fluxes Phi^k = G^k (U^{k+1} - U^k)
  for (int idx = threadIdx.x; idx < m * lay; idx += CELL_NT) {
    const int k = idx / lay, rem = idx % lay;
    const int r = rem / nst, s = rem % nst;
    const TB* G = blk + (int64_t)k * b * b + (int64_t)r * b;
    const TA* Uk = U + k * lay + s;
    const TA* Un = U + (k + 1) * lay + s;
    TA acc = 0;
    if (k + 1 < m) {
      for (int cc = 0; cc < b; ++cc) acc += ld_block<TB, TA>(G + cc) * (Un[cc * nst] - Uk[cc * nst]);
    } else {
      for (int cc = 0; cc < b; ++cc) acc -= ld_block<TB, TA>(G + cc) * Uk[cc * nst];
    }
    P[idx] = acc;
  }
  __syncthreads();
  // hidden layers
  const TA dt2 = (TA)a.dt2;
  for (int idx = threadIdx.x; idx < (m - 1) * lay; idx += CELL_NT) {
    const int k = 1 + idx / lay, rem = idx % lay;
    const int r = rem / nst, s = rem % nst;
    const TB* Gh = blk + (int64_t)m * b * b + (int64_t)(k - 1) * b * b + (int64_t)r * b;
    const TA* Pk = P + k * lay + s;
    const TA* Pm = P + (k - 1) * lay + s;
    TA acc = 0;
    for (int cc = 0; cc < b; ++cc) acc += ld_block<TB, TA>(Gh + cc) * (Pk[cc * nst] - Pm[cc * nst]);
    if (s < nsl) {
      const int64_t h = (c.hid_off + (int64_t)(k - 1) * b + r) * ns + s0 + s;
      hold[h] = (T)((TA)2 * U[k * lay + rem] - (TA)hold[h] + dt2 * acc);
    }
  }
  for (int idx = threadIdx.x; idx < lay; idx += CELL_NT) {
    const int r = idx / nst, s = idx % nst;
    if (s < nsl) phi[(c.u1_off + r) * ns + s0 + s] = (T)P[idx];
  }
}

constexpr int MAX_BP = 32;

// Piece phase: one thread per (piece, source).
template <typename T, typename TA>
__global__ __launch_bounds__(256) void k_piece_phase(StepArgs a) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)a.npiece * a.ns) return;
  const int p = (int)(gid / a.ns), s = (int)(gid % a.ns);
  const OnlinePiece pc = a.d_pieces[p];
  const int bp = pc.b, ns = a.ns;
  const T* phi = reinterpret_cast<const T*>(a.phi);
  const T* ycur = reinterpret_cast<const T*>(a.y_cur);
  T* yold = reinterpret_cast<T*>(a.y_old);
  const TA* minv = reinterpret_cast<const TA*>(a.d_minv) + pc.minv_off;
  const TA wn = (TA)a.w[a.step];
  TA r[MAX_BP];
  for (int j = 0; j < bp; ++j) {
    TA acc = 0;
    for (int e = 0; e < pc.ncell; ++e) acc += (TA)phi[(a.d_inc[pc.inc_off + e] + j) * ns + s];
    if (pc.src_off >= 0) acc += wn * (TA)reinterpret_cast<const T*>(a.d_src)[(pc.src_off + j) * ns + s];
    r[j] = acc;
  }
  const TA dt2 = (TA)a.dt2;
  for (int i = 0; i < bp; ++i) {
    TA acc = 0;
    for (int j = 0; j < bp; ++j) acc += minv[i + j * bp] * r[j];
    const int64_t q = (pc.dof_off + i) * ns + s;
    yold[q] = (T)((TA)2 * (TA)ycur[q] - (TA)yold[q] + dt2 * acc);
  }
}

// Receivers: one thread per (receiver, source) over the new piece state.
template <typename T, typename TA>
__global__ __launch_bounds__(256) void k_receivers(StepArgs a) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)a.nrec * a.ns) return;
  const int r = (int)(gid / a.ns), s = (int)(gid % a.ns);
  const T* y = reinterpret_cast<const T*>(a.y_old);   // holds level n+1 now
  TA acc = 0;
  for (int64_t k = a.d_rptr[r]; k < a.d_rptr[r + 1]; ++k) acc += (TA)a.d_rval[k] * (TA)y[a.d_rrow[k] * a.ns + s];
  reinterpret_cast<T*>(a.traces)[(a.trace_step * a.nrec + r) * a.ns + s] = (T)acc;
}

int cell_tile(const StepArgs& a, size_t acc_bytes) {
  // largest power-of-two source tile (<= 64) whose LDS fits in 64 KiB
  int nst = 64;
  while (nst > 1 && 2 * (size_t)a.max_m * a.max_b * nst * acc_bytes > 65536) nst /= 2;
  if (nst > a.ns) {
    int t = 1;
    while (t < a.ns) t *= 2;
    nst = t;
  }
  return nst;
}

template <typename T, typename TB, typename TA>
static hipError_t cell_impl(const StepArgs& a, hipStream_t st) {
  const int nst = cell_tile(a, sizeof(TA));
  const size_t lds = 2 * (size_t)a.max_m * a.max_b * nst * sizeof(TA);
  const dim3 g1(a.ncell, (a.ns + nst - 1) / nst);
  hipLaunchKernelGGL((k_cell_phase<T, TB, TA>), g1, dim3(CELL_NT), lds, st, a, nst);
  return hipGetLastError();
}

template <typename T, typename TA>
static hipError_t piece_impl(const StepArgs& a, hipStream_t st) {
  const int64_t np = (int64_t)a.npiece * a.ns;
  hipLaunchKernelGGL((k_piece_phase<T, TA>), dim3((np + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T, typename TA>
static hipError_t rec_impl(const StepArgs& a, hipStream_t st) {
  if (a.nrec > 0) {
    const int64_t nr = (int64_t)a.nrec * a.ns;
    hipLaunchKernelGGL((k_receivers<T, TA>), dim3((nr + 255) / 256), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_cell_phase(const StepArgs& a, hipStream_t st) {
  if (a.prec == SFROM_F64) return cell_impl<double, double, double>(a, st);
  if (a.prec == SFROM_F32) return cell_impl<float, float, float>(a, st);
  return cell_impl<float, __hip_bfloat16, float>(a, st);
}

hipError_t launch_piece_phase(const StepArgs& a, hipStream_t st) {
  if (a.prec == SFROM_F64) return piece_impl<double, double>(a, st);
  return piece_impl<float, float>(a, st);
}

hipError_t launch_receivers(const StepArgs& a, hipStream_t st) {
  if (a.prec == SFROM_F64) return rec_impl<double, double>(a, st);
  return rec_impl<float, float>(a, st);
}

hipError_t launch_online_step(const StepArgs& a, hipStream_t st) {
  hipError_t e = launch_cell_phase(a, st);
  if (e != hipSuccess) return e;
  e = launch_piece_phase(a, st);
  if (e != hipSuccess) return e;
  return launch_receivers(a, st);
}

}  // namespace sfrom_impl
