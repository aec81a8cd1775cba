// Fine-grid leapfrog comparator (Sec. 1, eq. wave_fll):
//   u^{n+1} = 2u^n - u^{n-1} + dt^2 B^{-1} (A u^n + w^n g),
// for a batch of sources, with A in CSR and the state stored [node][source].
// A wavefront covers consecutive sources of one row when n_s >= 64, so the
// row's CSR entries are uniform across the wave and the state accesses are
// contiguous.

#include <hip/hip_runtime.h>

#include "sfrom_internal.h"

namespace sfrom_impl {

// One thread per (group of FR consecutive rows, source). Every thread first
// reads the CSR entries of its rows (up to FMAXNZ per row, predicated), then
// issues all neighbour loads, then accumulates, so each thread has dozens of
// independent loads in flight instead of a chain of dependent ones. When
// n_s is a multiple of 64 a wavefront covers whole rows and the row indices
// are made wave-uniform, which turns the CSR reads into scalar loads.
// Workgroups are dealt to the 8 XCDs round-robin; the id is remapped so that
// each XCD sweeps one contiguous slab of rows, keeping the neighbour rows of
// a 7-point operator in that XCD's L2.
constexpr int FR = 4;
constexpr int FNT = 256;
constexpr int FMAXNZ = 8;

template <typename T, bool UNI>
__global__ __launch_bounds__(FNT) void k_fine_step(FineArgs a, int64_t nblk) {
  const int64_t per = (nblk + 7) / 8;
  const int64_t lb = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (lb >= nblk) return;
  const int ns = a.ns;
  const int64_t gid = lb * FNT + threadIdx.x;
  const int64_t ngrp = (a.n + FR - 1) / FR;
  int64_t grp;
  int s;
  if constexpr (UNI) {
    // wave-uniform group index: 64 consecutive sources of one row group
    const int64_t wv = gid >> 6;
    const int per_grp = ns >> 6;
    grp = (int64_t)__builtin_amdgcn_readfirstlane((int)(wv / per_grp));
    s = (int)((wv % per_grp) << 6) + (threadIdx.x & 63);
  } else {
    grp = gid / ns;
    s = (int)(gid - grp * ns);
  }
  if (grp >= ngrp) return;
  const T* __restrict__ av = reinterpret_cast<const T*>(a.a);
  const T* __restrict__ u = reinterpret_cast<const T*>(a.u_cur);
  T* __restrict__ uo = reinterpret_cast<T*>(a.u_old);
  const T* __restrict__ binv = reinterpret_cast<const T*>(a.binv);
  const T dt2 = (T)a.dt2;
  int64_t r0[FR], r1[FR];
#pragma unroll
  for (int q = 0; q < FR; ++q) {
    const int64_t row = grp * FR + q;
    const int64_t rc = min(row, a.n - 1);
    const int64_t b0 = a.rowptr[rc], b1 = a.rowptr[rc + 1];
    r0[q] = b0;
    r1[q] = (row < a.n) ? b1 : b0;      // rows past the end are empty
  }
  // All loads below are unconditional from clamped (always valid) addresses,
  // with the unused values masked afterwards, so that the compiler issues
  // them back to back instead of one guarded branch at a time.
  const int64_t nnz = a.rowptr[a.n];
  int cl[FR][FMAXNZ];
  T va[FR][FMAXNZ];
#pragma unroll
  for (int q = 0; q < FR; ++q)
#pragma unroll
    for (int e = 0; e < FMAXNZ; ++e) {
      const int64_t k = min(r0[q] + e, nnz - 1);
      cl[q][e] = a.col[k];
      va[q][e] = av[k];
    }
  T acc[FR], uc[FR], ol[FR], bi[FR];
#pragma unroll
  for (int q = 0; q < FR; ++q) {
    const int64_t row = min(grp * FR + q, a.n - 1);
    T x[FMAXNZ];
#pragma unroll
    for (int e = 0; e < FMAXNZ; ++e) x[e] = u[(int64_t)cl[q][e] * ns + s];
    uc[q] = u[row * ns + s];
    ol[q] = uo[row * ns + s];
    bi[q] = binv[row];
    acc[q] = 0;
#pragma unroll
    for (int e = 0; e < FMAXNZ; ++e) acc[q] += (r0[q] + e < r1[q]) ? va[q][e] * x[e] : (T)0;
  }
#pragma unroll
  for (int q = 0; q < FR; ++q)
    for (int64_t k = r0[q] + FMAXNZ; k < r1[q]; ++k) acc[q] += av[k] * u[(int64_t)a.col[k] * ns + s];
#pragma unroll
  for (int q = 0; q < FR; ++q) {
    const int64_t row = grp * FR + q;
    if (row < a.n) uo[row * ns + s] = (T)2 * uc[q] - ol[q] + dt2 * bi[q] * acc[q];
  }
}

// Cartesian 7-point form: neighbour addresses are computed from the node
// index (clamped at the walls, where the coefficient is zero), so every load
// of a thread is independent of every other. The 8 coefficients of a node
// are wave-uniform when n_s is a multiple of 64.
template <typename T, bool UNI>
__global__ __launch_bounds__(FNT) void k_fine_stencil(FineArgs a, int64_t nblk) {
  const int64_t per = (nblk + 7) / 8;
  const int64_t lb = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (lb >= nblk) return;
  const int ns = a.ns;
  const int64_t gid = lb * FNT + threadIdx.x;
  const int64_t ngrp = (a.n + FR - 1) / FR;
  int64_t grp;
  int s;
  if constexpr (UNI) {
    const int64_t wv = gid >> 6;
    const int per_grp = ns >> 6;
    grp = (int64_t)__builtin_amdgcn_readfirstlane((int)(wv / per_grp));
    s = (int)((wv % per_grp) << 6) + (threadIdx.x & 63);
  } else {
    grp = gid / ns;
    s = (int)(gid - grp * ns);
  }
  if (grp >= ngrp) return;
  const T* __restrict__ cf = reinterpret_cast<const T*>(a.stencil);
  const T* __restrict__ u = reinterpret_cast<const T*>(a.u_cur);
  T* __restrict__ uo = reinterpret_cast<T*>(a.u_old);
  const int64_t sx = 1, sy = a.ux, sz = (int64_t)a.ux * a.uy;
  const T dt2 = (T)a.dt2;
  T res[FR];
#pragma unroll
  for (int q = 0; q < FR; ++q) {
    const int64_t node = min(grp * FR + q, a.n - 1);
    const T* c = cf + node * 8;
    const int64_t nb[6] = {max(node - sx, (int64_t)0), min(node + sx, a.n - 1), max(node - sy, (int64_t)0),
                           min(node + sy, a.n - 1), max(node - sz, (int64_t)0), min(node + sz, a.n - 1)};
    T x[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) x[e] = u[nb[e] * ns + s];
    const T uc = u[node * ns + s];
    const T ol = uo[node * ns + s];
    T acc = c[6] * uc;
#pragma unroll
    for (int e = 0; e < 6; ++e) acc += c[e] * x[e];
    res[q] = (T)2 * uc - ol + dt2 * c[7] * acc;
  }
#pragma unroll
  for (int q = 0; q < FR; ++q) {
    const int64_t node = grp * FR + q;
    if (node < a.n) uo[node * ns + s] = res[q];
  }
}

template <typename T>
__global__ void k_fine_src(FineArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nsrc_entries) return;
  const int64_t row = a.src_row[e];
  const int s = a.src_col[e];
  T* uo = reinterpret_cast<T*>(a.u_old);
  const T binv = reinterpret_cast<const T*>(a.binv)[row];
  uo[row * a.ns + s] += (T)a.dt2 * binv * (T)(a.w[a.step] * a.src_val[e]);
}

template <typename T>
__global__ void k_fine_rec(FineArgs a) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)a.nrec * a.ns) return;
  const int r = (int)(gid / a.ns), s = (int)(gid % a.ns);
  const T* u = reinterpret_cast<const T*>(a.u_old);   // level n+1
  T acc = 0;
  for (int64_t k = a.rec_ptr[r]; k < a.rec_ptr[r + 1]; ++k) acc += (T)a.rec_val[k] * u[a.rec_row[k] * a.ns + s];
  reinterpret_cast<T*>(a.traces)[(a.trace_step * a.nrec + r) * a.ns + s] = acc;
}

template <typename T>
static hipError_t fine_impl(const FineArgs& a, hipStream_t st) {
  const int64_t tot = (a.n + FR - 1) / FR * a.ns;
  const int64_t nblk = (tot + FNT - 1) / FNT;
  const int64_t grid = (nblk + 7) / 8 * 8;
  if (a.stencil) {
    if (a.ns % 64 == 0) hipLaunchKernelGGL((k_fine_stencil<T, true>), dim3(grid), dim3(FNT), 0, st, a, nblk);
    else hipLaunchKernelGGL((k_fine_stencil<T, false>), dim3(grid), dim3(FNT), 0, st, a, nblk);
  } else if (a.ns % 64 == 0) {
    hipLaunchKernelGGL((k_fine_step<T, true>), dim3(grid), dim3(FNT), 0, st, a, nblk);
  } else {
    hipLaunchKernelGGL((k_fine_step<T, false>), dim3(grid), dim3(FNT), 0, st, a, nblk);
  }
  if (a.nsrc_entries > 0)
    hipLaunchKernelGGL(k_fine_src<T>, dim3((a.nsrc_entries + 255) / 256), dim3(256), 0, st, a);
  if (a.nrec > 0) {
    const int64_t nr = (int64_t)a.nrec * a.ns;
    hipLaunchKernelGGL(k_fine_rec<T>, dim3((nr + 255) / 256), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_fine_step(const FineArgs& a, hipStream_t st) {
  return (a.prec == SFROM_F64) ? fine_impl<double>(a, st) : fine_impl<float>(a, st);
}

}  // namespace sfrom_impl
