// Fine-grid leapfrog comparator (Sec. 1, eq. wave_fll):
//   u^{n+1} = 2u^n - u^{n-1} + dt^2 B^{-1} (A u^n + w^n g),
// for a batch of sources, with A in CSR and the state stored [node][source].
// A wavefront covers consecutive sources of one row when n_s >= 64, so the
// row's CSR entries are uniform across the wave and the state accesses are
// contiguous.

#include <hip/hip_runtime.h>

#include <algorithm>

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

// Traces of level `lv` (a state array) for trace step ts, one thread per
// (receiver, source), r_gid counting from 0.
template <typename T>
__device__ inline void fine_receiver(const FineArgs& a, const T* __restrict__ lv, int64_t ts, int64_t r_gid) {
  if (r_gid >= (int64_t)a.nrec * a.ns) return;
  const int r = (int)(r_gid / a.ns), s = (int)(r_gid % a.ns);
  T acc = 0;
  for (int64_t k = a.rec_ptr[r]; k < a.rec_ptr[r + 1]; ++k) acc += (T)a.rec_val[k] * lv[a.rec_row[k] * a.ns + s];
  reinterpret_cast<T*>(a.traces)[(ts * a.nrec + r) * a.ns + s] = acc;
}

// Cartesian 7-point step with 2.5D blocking, for n_s a multiple of 64. A
// workgroup owns a TX x TY tile of (x, y) columns and one group of 64
// sources (lane = source), and marches a segment of z planes; wave w owns
// tile row w (TX consecutive columns). The values of its columns at planes
// z - 1, z and z + 1 stay in registers, so along z every state value is
// read from HBM once; the +-y neighbours and the row ends come from an LDS
// copy of plane z (the tile plus its one-node ring, which the waves load
// from the neighbouring tiles). Loads of plane z + 2, of the ring of plane
// z + 1 and of the next plane's old values, coefficients and source
// indices are issued one plane ahead. A row's coefficients (8 per node)
// are one coalesced load, broadcast to the lanes through LDS. A point
// source at a node adds w^n g to its flux (source rows of dense values,
// index per node). The old level is streamed with non-temporal loads and
// stores, so that the current level's planes, which neighbouring tiles
// re-read as their rings, stay in L2. The state, coefficient and
// source-index arrays are
// padded by FINE_PAD nodes, so a row's loads are issued unconditionally
// and the values of columns beyond the grid are dropped. The workgroups
// after the tiles compute the traces of the level that this launch reads
// (the previous step's output), so the step is one launch.
template <typename T, int TX, int TY>
__global__ __launch_bounds__(64 * TY) void k_fine_25d(FineArgs a, int ntx, int nty, int zseg, int nzs,
                                                      int64_t ntile, int64_t tile_grid) {
  if ((int64_t)blockIdx.x >= tile_grid) {
    if (a.trace_step > 0)
      fine_receiver<T>(a, reinterpret_cast<const T*>(a.u_cur), a.trace_step - 1,
                       ((int64_t)blockIdx.x - tile_grid) * blockDim.x + threadIdx.x);
    return;
  }
  // workgroups are dealt to the 8 XCDs round-robin: each XCD gets a
  // contiguous range of tiles, so neighbouring tiles (whose rows form each
  // other's rings) share that XCD's L2
  const int64_t per = tile_grid / 8;
  const int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t >= ntile) return;
  extern __shared__ __align__(16) unsigned char f25_raw[];
  T* pl = reinterpret_cast<T*>(f25_raw);
  constexpr int PX = TX + 2, PY = TY + 2, NPL = PX * PY * 64, PLANE = NPL + TY * TX * 8;
  constexpr int NH = 2 * (TX + TY), NHW = NH / TY;   // ring nodes, per wave
  static_assert(NH % TY == 0 && TX * 8 == 64, "8 columns per row, ring split evenly over the waves");
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tx = (int)(t % ntx);
  int64_t rr = t / ntx;
  const int ty = (int)(rr % nty);
  rr /= nty;
  const int zs = (int)(rr % nzs);
  const int sg = (int)(rr / nzs);
  const int ux = a.ux, uy = a.uy, uz = a.uz, ns = a.ns;
  const int x0 = tx * TX, y0 = ty * TY, y = y0 + w;
  const int zb = zs * zseg, ze = min(zb + zseg, uz);
  // lane's source column in every state array
  const T* __restrict__ u = reinterpret_cast<const T*>(a.u_cur) + sg * 64 + lane;
  T* __restrict__ uo = reinterpret_cast<T*>(a.u_old) + sg * 64 + lane;
  const T* __restrict__ cf = reinterpret_cast<const T*>(a.stencil);
  const T* __restrict__ gs = reinterpret_cast<const T*>(a.src_dense) + sg * 64 + lane;
  const T dt2 = (T)a.dt2;
  const int ncol = min(TX, ux - x0);                 // columns of the tile inside the grid
  const bool rowok = y < uy;
  const int yc = min(y, uy - 1);
  // first node of this wave's row in plane z (z clamped into the grid)
  auto row0 = [&](int z) -> int64_t { return x0 + (int64_t)ux * (yc + (int64_t)uy * min(max(z, 0), uz - 1)); };
  // the row's TX values of plane z, zero off the grid
  auto ld_cols = [&](int z, T (&v)[TX]) {
    const T* p = u + row0(z) * ns;
    const bool ok = rowok && z >= 0 && z < uz;
#pragma unroll
    for (int i = 0; i < TX; ++i) {
      const T x = p[(int64_t)i * ns];
      v[i] = (ok && i < ncol) ? x : (T)0;
    }
  };
  // ring node j of this wave: left and right columns, then bottom and top
  // rows (tile coordinates)
  int hx[NHW], hy[NHW];
#pragma unroll
  for (int j = 0; j < NHW; ++j) {
    const int q = w + j * TY;
    if (q < TY) { hx[j] = -1; hy[j] = q; }
    else if (q < 2 * TY) { hx[j] = TX; hy[j] = q - TY; }
    else if (q < 2 * TY + TX) { hx[j] = q - 2 * TY; hy[j] = -1; }
    else { hx[j] = q - 2 * TY - TX; hy[j] = TY; }
  }
  auto ld_ring = [&](int z, T (&v)[NHW]) {
#pragma unroll
    for (int j = 0; j < NHW; ++j) {
      const int xx = x0 + hx[j], yy = y0 + hy[j];
      const bool ok = xx >= 0 && xx < ux && yy >= 0 && yy < uy && z >= 0 && z < uz;
      const int64_t nd = ok ? xx + (int64_t)ux * (yy + (int64_t)uy * z) : 0;
      const T x = u[nd * ns];
      v[j] = ok ? x : (T)0;
    }
  };
  // per-row data of plane z: the row's 64 coefficients (one per lane), old
  // values, source index (lanes < TX)
  auto ld_row = [&](int z, T& c, T (&o)[TX], int& sidx) {
    const int64_t r0 = row0(z);
    c = cf[r0 * 8 + lane];
    const T* p = uo + r0 * ns;
#pragma unroll
    for (int i = 0; i < TX; ++i) o[i] = __builtin_nontemporal_load(p + (int64_t)i * ns);
    sidx = a.src_idx[r0 + (lane & (TX - 1))];
  };
  T zm[TX], zc[TX], zp[TX], zq[TX], hz[NHW], hn[NHW], oc[TX], on[TX];
  T cc, cn;
  int sc, sn;
  ld_cols(zb - 1, zm);
  ld_cols(zb, zc);
  ld_cols(zb + 1, zp);
  ld_ring(zb, hz);
  ld_row(zb, cc, oc, sc);
  const T wn = (T)a.w[a.step];
  for (int z = zb; z < ze; ++z) {
    // loads one plane ahead
    ld_cols(z + 2, zq);
    ld_ring(z + 1, hn);
    ld_row(min(z + 1, ze - 1), cn, on, sn);
    // plane z and the row's coefficients into LDS
    T* P = pl + (z & 1) * PLANE;
    T* C = P + NPL + w * TX * 8;
#pragma unroll
    for (int i = 0; i < TX; ++i) P[((w + 1) * PX + i + 1) * 64 + lane] = zc[i];
#pragma unroll
    for (int j = 0; j < NHW; ++j) P[((hy[j] + 1) * PX + hx[j] + 1) * 64 + lane] = hz[j];
    C[lane] = cc;
    __syncthreads();
    if (rowok) {
      T* po = uo + row0(z) * ns;
#pragma unroll
      for (int i = 0; i < TX; ++i) {
        if (i >= ncol) break;
        T c[8];   // same LDS address in every lane: a broadcast read
#pragma unroll
        for (int k = 0; k < 8; ++k) c[k] = C[i * 8 + k];
        const T xm = (i > 0) ? zc[i - 1] : P[((w + 1) * PX) * 64 + lane];
        const T xp = (i < TX - 1) ? zc[i + 1] : P[((w + 1) * PX + TX + 1) * 64 + lane];
        const T ym = P[(w * PX + i + 1) * 64 + lane];
        const T yp = P[((w + 2) * PX + i + 1) * 64 + lane];
        T acc = c[6] * zc[i];
        acc += c[0] * xm;
        acc += c[1] * xp;
        acc += c[2] * ym;
        acc += c[3] * yp;
        acc += c[4] * zm[i];
        acc += c[5] * zp[i];
        const int si = __builtin_amdgcn_readlane(sc, i);
        if (si >= 0) acc += wn * gs[(int64_t)si * ns];
        __builtin_nontemporal_store((T)2 * zc[i] - oc[i] + dt2 * c[7] * acc, po + (int64_t)i * ns);
      }
    }
#pragma unroll
    for (int i = 0; i < TX; ++i) { zm[i] = zc[i]; zc[i] = zp[i]; zp[i] = zq[i]; oc[i] = on[i]; }
#pragma unroll
    for (int j = 0; j < NHW; ++j) hz[j] = hn[j];
    cc = cn;
    sc = sn;
  }
}

// Traces of the final level of a run of k_fine_25d launches.
template <typename T>
__global__ void k_fine_rec_level(FineArgs a) {
  fine_receiver<T>(a, reinterpret_cast<const T*>(a.u_cur), a.trace_step, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
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

// 2.5D tiles of 8 x 8 columns: two LDS planes of (TX + 2)(TY + 2) nodes x
// 64 sources plus the tile's coefficients (float: 3 workgroups per CU)
template <typename T>
struct Tile25 {
  static constexpr int TX = 8, TY = 8;
};

template <typename T>
static hipError_t fine_25d_impl(const FineArgs& a, hipStream_t st) {
  constexpr int TX = Tile25<T>::TX, TY = Tile25<T>::TY;
  const int ntx = (a.ux + TX - 1) / TX, nty = (a.uy + TY - 1) / TY, nsg = a.ns / 64;
  const int64_t cols = (int64_t)ntx * nty * nsg;
  // z segments: about 1024 workgroups in all, each segment at least 8 planes
  int nzs = (int)std::min<int64_t>(std::max<int64_t>((1024 + cols - 1) / cols, 1), (a.uz + 7) / 8);
  nzs = std::max(nzs, 1);
  const int zseg = (a.uz + nzs - 1) / nzs;
  nzs = (a.uz + zseg - 1) / zseg;
  const int64_t ntile = cols * nzs;
  const int64_t tile_grid = (ntile + 7) / 8 * 8;
  const int64_t nrt = (a.trace_step > 0) ? (int64_t)a.nrec * a.ns : 0;
  const int64_t rgrid = (nrt + 64 * TY - 1) / (64 * TY);
  const size_t lds = (size_t)2 * ((TX + 2) * (TY + 2) * 64 + TY * TX * 8) * sizeof(T);
  static_assert(TX <= FINE_PAD, "arrays are padded by FINE_PAD nodes");
  hipLaunchKernelGGL((k_fine_25d<T, TX, TY>), dim3(tile_grid + rgrid), dim3(64 * TY), lds, st, a, ntx, nty, zseg, nzs,
                     ntile, tile_grid);
  return hipGetLastError();
}

template <typename T>
static hipError_t fine_rec_level_impl(const FineArgs& a, hipStream_t st) {
  const int64_t nr = (int64_t)a.nrec * a.ns;
  if (nr > 0) hipLaunchKernelGGL(k_fine_rec_level<T>, dim3((nr + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

bool fine_uses_25d(const FineArgs& a) { return a.stencil != nullptr && a.ns % 64 == 0 && a.src_dense_ok; }

hipError_t launch_fine_rec_level(const FineArgs& a, hipStream_t st) {
  return (a.prec == SFROM_F64) ? fine_rec_level_impl<double>(a, st) : fine_rec_level_impl<float>(a, st);
}

template <typename T>
static hipError_t fine_impl(const FineArgs& a, hipStream_t st) {
  if (fine_uses_25d(a)) return fine_25d_impl<T>(a, st);
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
