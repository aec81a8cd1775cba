// Fine-grid leapfrog comparator (Sec. 1, eq. wave_fll):
//   u^{n+1} = 2u^n - u^{n-1} + dt^2 B^{-1} (A u^n + w^n g),
// for a batch of sources, with A in CSR and the state stored [node][source].
// A wavefront covers consecutive sources of one row when n_s >= 64, so the
// row's CSR entries are uniform across the wave and the state accesses are
// contiguous.

#include <hip/hip_runtime.h>

#include "sfrom_internal.h"

namespace sfrom_impl {

template <typename T>
__global__ __launch_bounds__(256) void k_fine_step(FineArgs a) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= a.n * a.ns) return;
  const int64_t row = gid / a.ns;
  const int s = (int)(gid % a.ns);
  const T* av = reinterpret_cast<const T*>(a.a);
  const T* u = reinterpret_cast<const T*>(a.u_cur);
  T* uo = reinterpret_cast<T*>(a.u_old);
  T acc = 0;
  for (int64_t k = a.rowptr[row]; k < a.rowptr[row + 1]; ++k) acc += av[k] * u[(int64_t)a.col[k] * a.ns + s];
  const T binv = reinterpret_cast<const T*>(a.binv)[row];
  uo[gid] = (T)2 * u[gid] - uo[gid] + (T)a.dt2 * binv * acc;
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
  const int64_t tot = a.n * a.ns;
  hipLaunchKernelGGL(k_fine_step<T>, dim3((tot + 255) / 256), dim3(256), 0, st, a);
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
