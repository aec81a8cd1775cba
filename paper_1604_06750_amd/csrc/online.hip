// On-line stage (Alg. alg1red stage 2): one explicit leapfrog step of the
// coupled S-fraction ROM for a batch of sources.
//
// Unknowns: reduced piece dofs y_p (the conjugated boundary values of
// eq. contred) and each cell's hidden layers. The S-fraction's three-point
// scheme (eqs. GammaU1st, GammaUrem, intrtstep_td) is stepped after the
// change of variables U^k = G_k V^k (k >= 2) of its hidden layers, where
// Ghat^k = G_k G_k^T is the factor of the recursion of eq. GammaTrans. In
// these variables the hidden layers have unit mass and the cell operator is
// block tridiagonal with blocks
//   D_0 = -G^1,   C_0 = G^1 G_2,
//   D_l = -G_l^T (G^l + G^{l-1}) G_l,  C_l = G_l^T G^l G_{l+1}   (l >= 1,
// layers counted from 0), i.e. the Lanczos blocks alpha, beta^T of the cell.
// The form is exactly equivalent, and its blocks are bounded by the
// largest frequency of the cell, while the blocks G^k and Ghat^k of deep
// layers can be near singular; rounding D and C to FP32 or BF16 therefore
// perturbs the spectrum by a unit roundoff of its largest eigenvalue only.
// With X_0 = U^1 (the cell's piece dofs, gathered in the column order of its
// boundary basis) and X_l = V^{l+1}:
//
//   cell phase   a_l = C_{l-1}^T X_{l-1} + D_l X_l + C_l X_{l+1}
//                Phi^1 = a_0 (the flux G^1 (U^2 - U^1) into the pieces),
//                X_l <- 2X_l - X_l,old + dt^2 a_l,  l >= 1
//                (Alg. alg1red, stage 2: the cells' hidden layers)
//   piece phase  r_p = sum over the cells owning p of their Phi^1 slice
//                      + w^n g_p                            (the exchange)
//                y_p <- 2y_p - y_p,old + dt^2 M_p^{-1} r_p   (eq. bdrytstep,
//                M_p = sum_i [(Ghat_i^1)^{-1}]_pp)
//   receivers    trace = sum_p q_p^T y_p                     (eq. solatrec)
//
// Blocks of a cell are stored in the order D_0, C_0, D_1, C_1, ..., D_{m-1},
// each b rows of stride ld (row-major, zero padded). State rows hold n_s
// sources contiguously ([row][source]). The exchange between the two
// phases goes through the Phi^1 scratch in HBM, summed in a fixed order (no
// atomics), so results are deterministic.

#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <algorithm>
#include <type_traits>

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

// Cell phase. grid = (n_cells, ceil(n_s / nst)); dynamic LDS holds the
// cell's layers X_0..X_{m-1} for the workgroup's source tile (max_m * max_b
// * nst values of the accumulation type).
template <typename T, typename TB, typename TA>
__global__ __launch_bounds__(CELL_NT) void k_cell_phase(StepArgs a, int nst) {
  extern __shared__ unsigned char smem_raw[];
  TA* X = reinterpret_cast<TA*>(smem_raw);
  const OnlineCell c = a.d_cells[a.d_cell_list ? a.d_cell_list[blockIdx.x] : (int)blockIdx.x];
  const int m = c.m, b = c.b, ld = c.ld, ns = a.ns;
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
    X[idx] = (s < nsl) ? (TA)ycur[(int64_t)gat[r] * ns + s0 + s] : (TA)0;
  }
  for (int k = 1; k < m; ++k) {
    const T* hl = hcur + (c.hid_off + (int64_t)(k - 1) * ld) * ns;
    for (int idx = threadIdx.x; idx < lay; idx += CELL_NT) {
      const int r = idx % b, s = idx / b;
      X[k * lay + r * nst + s] = (s < nsl) ? (TA)hl[(int64_t)(s0 + s) * ld + r] : (TA)0;
    }
  }
  __syncthreads();
  const TB* blk = reinterpret_cast<const TB*>(a.d_blocks) + c.blk_off;
  const int64_t bsz = (int64_t)b * ld;
  const TA dt2 = (TA)a.dt2;
  for (int idx = threadIdx.x; idx < m * lay; idx += CELL_NT) {
    const int l = idx / lay, rem = idx % lay;
    const int r = rem % b, s = rem / b;     // consecutive threads: consecutive rows
    const TA* xs = X + s;
    TA acc = 0;
    const TB* D = blk + 2 * l * bsz + (int64_t)r * ld;
    for (int cc = 0; cc < b; ++cc) acc += ld_block<TB, TA>(D + cc) * xs[l * lay + cc * nst];
    if (l > 0) {   // C_{l-1}^T X_{l-1}: column r of C_{l-1}
      const TB* Cp = blk + (2 * l - 1) * bsz + r;
      for (int cc = 0; cc < b; ++cc) acc += ld_block<TB, TA>(Cp + (int64_t)cc * ld) * xs[(l - 1) * lay + cc * nst];
    }
    if (l + 1 < m) {   // C_l X_{l+1}
      const TB* Cn = blk + (2 * l + 1) * bsz + (int64_t)r * ld;
      for (int cc = 0; cc < b; ++cc) acc += ld_block<TB, TA>(Cn + cc) * xs[(l + 1) * lay + cc * nst];
    }
    if (s < nsl) {
      if (l == 0) {
        phi[(c.u1_off + r) * ns + s0 + s] = (T)acc;
      } else {
        const int64_t h = (c.hid_off + (int64_t)(l - 1) * ld) * ns + (int64_t)(s0 + s) * ld + r;
        hold[h] = (T)((TA)2 * X[l * lay + r * nst + s] - (TA)hold[h] + dt2 * acc);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Cell phase on the matrix cores (float state; float or bfloat16 blocks).
//
// One workgroup per (cell, tile of 16*CT sources); wave w owns rows
// [16w, 16w+16) of every layer. The cell's blocks are consumed as one
// stream of 16-column chunks: for layer l the strips C_{l-1}^T, D_l, C_l
// (block 2l+t-1 for t = 0, 1, 2; t = 0 absent for l = 0, t = 2 for
// l = m-1), each nch = ceil(b/16) chunks. Every wave keeps the next R
// chunks of its strip in flight in a register ring, across strip and layer
// boundaries, so the A operand is read from HBM once per source tile
// without holding whole strips in registers. Inside a chunk, lane group
// g = lane/16 supplies k = 16 ch + 4 g + j to MFMA step j: each lane reads
// its A values as one vector from the row-major block (four scalars from
// one column for the transposed C_{l-1}) and its B values as one float4
// from the transposed LDS tile.
//
// LDS: three transposed layer tiles [16*CT columns][kp], kp = 16*NCH + 4,
// used as a ring: X_{l-1}, X_l, X_{l+1} during layer l; X_{l+2} is loaded
// into registers during layer l and stored over X_{l-1} after it. The
// hidden layers are stored source-major (ld floats per source, zero
// padded), so a thread moves four rows of one source with one float4.
// ---------------------------------------------------------------------------

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

// Precision modes of the matrix-core cell phase: 0 = FP32 blocks and state,
// 1 = BF16 blocks with FP32 accumulation and state, 2 = FP64.
template <int PM>
struct Prec;
template <>
struct Prec<0> {
  using T = float; using TB = float; using V4 = float4; using ACC = floatx4;
};
template <>
struct Prec<1> {
  using T = float; using TB = __hip_bfloat16; using V4 = float4; using ACC = floatx4;
};
template <>
struct Prec<2> {
  using T = double; using TB = double; using V4 = double4; using ACC = doublex4;
};
template <typename V4, typename T>
__device__ inline V4 mk4(T a, T b, T c, T d) {
  V4 v;
  v.x = a; v.y = b; v.z = c; v.w = d;
  return v;
}

__device__ inline short f2bf(float f) {
  // round to nearest even (the state is finite; NaN propagates as NaN)
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

template <int PM>
struct AFrag;
template <>
struct AFrag<0> {
  float4 v;
  __device__ void load(const float* p) { v = *reinterpret_cast<const float4*>(p); }
  // A[i][k..k+3] = C[k..k+3][i] of a row-major block with row stride ld,
  // rows >= nrow read as zero
  __device__ void load_t(const float* base, int ld, int k, int i, int nrow) {
    v.x = (k < nrow) ? base[(int64_t)k * ld + i] : 0.f;
    v.y = (k + 1 < nrow) ? base[(int64_t)(k + 1) * ld + i] : 0.f;
    v.z = (k + 2 < nrow) ? base[(int64_t)(k + 2) * ld + i] : 0.f;
    v.w = (k + 3 < nrow) ? base[(int64_t)(k + 3) * ld + i] : 0.f;
  }
  __device__ void zero() { v = make_float4(0.f, 0.f, 0.f, 0.f); }
};
template <>
struct AFrag<2> {
  double4 v;
  __device__ void load(const double* p) {
    const double2* q = reinterpret_cast<const double2*>(p);
    const double2 a = q[0], b = q[1];
    v.x = a.x; v.y = a.y; v.z = b.x; v.w = b.y;
  }
  __device__ void load_t(const double* base, int ld, int k, int i, int nrow) {
    v.x = (k < nrow) ? base[(int64_t)k * ld + i] : 0.0;
    v.y = (k + 1 < nrow) ? base[(int64_t)(k + 1) * ld + i] : 0.0;
    v.z = (k + 2 < nrow) ? base[(int64_t)(k + 2) * ld + i] : 0.0;
    v.w = (k + 3 < nrow) ? base[(int64_t)(k + 3) * ld + i] : 0.0;
  }
  __device__ void zero() { v.x = v.y = v.z = v.w = 0.0; }
};
template <>
struct AFrag<1> {
  shortx4 v;
  __device__ void load(const __hip_bfloat16* p) { v = *reinterpret_cast<const shortx4*>(p); }
  __device__ void load_t(const __hip_bfloat16* base_, int ld, int k, int i, int nrow) {
    const short* base = reinterpret_cast<const short*>(base_);
    v.x = (k < nrow) ? base[(int64_t)k * ld + i] : (short)0;
    v.y = (k + 1 < nrow) ? base[(int64_t)(k + 1) * ld + i] : (short)0;
    v.z = (k + 2 < nrow) ? base[(int64_t)(k + 2) * ld + i] : (short)0;
    v.w = (k + 3 < nrow) ? base[(int64_t)(k + 3) * ld + i] : (short)0;
  }
  __device__ void zero() { v = shortx4{0, 0, 0, 0}; }
};

// B fragments of chunk ch: column tile ct reads its 4 consecutive k of the
// transposed LDS tile Bt
template <int CT, typename V4, typename T>
__device__ inline void load_b(V4 (&bv)[CT], const T* Bt, int kp, int ch, int g, int li) {
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) bv[ct] = *reinterpret_cast<const V4*>(Bt + (ct * 16 + li) * kp + ch * 16 + g * 4);
}

// acc[ct] += A chunk x B chunk for column tile ct, reading that tile's B
// fragment from LDS just before its products (fewer live registers; the
// dependent products of one tile are interleaved with other waves')
template <int CT, int PM>
__device__ inline void mma_chunk_lean(typename Prec<PM>::ACC (&acc)[CT], const AFrag<PM>& A,
                                      const typename Prec<PM>::T* Bt, int kp, int ch, int g, int li) {
  using V4 = typename Prec<PM>::V4;
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const V4 bv = *reinterpret_cast<const V4*>(Bt + (ct * 16 + li) * kp + ch * 16 + g * 4);
    if constexpr (PM == 0) {
      acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.v.x, bv.x, acc[ct], 0, 0, 0);
      acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.v.y, bv.y, acc[ct], 0, 0, 0);
      acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.v.z, bv.z, acc[ct], 0, 0, 0);
      acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.v.w, bv.w, acc[ct], 0, 0, 0);
    } else if constexpr (PM == 2) {
      acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(A.v.x, bv.x, acc[ct], 0, 0, 0);
      acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(A.v.y, bv.y, acc[ct], 0, 0, 0);
      acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(A.v.z, bv.z, acc[ct], 0, 0, 0);
      acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(A.v.w, bv.w, acc[ct], 0, 0, 0);
    } else {
      const shortx4 bb = shortx4{f2bf(bv.x), f2bf(bv.y), f2bf(bv.z), f2bf(bv.w)};
      acc[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A.v, bb, acc[ct], 0, 0, 0);
    }
  }
}

// acc[ct] += A chunk x B chunk (column tile ct)
template <int CT, int PM>
__device__ inline void mma_chunk(typename Prec<PM>::ACC (&acc)[CT], const AFrag<PM>& A,
                                 const typename Prec<PM>::V4 (&bv)[CT]) {
  // consecutive MFMAs go to independent accumulators (column tiles)
  if constexpr (PM == 0) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.v.x, bv[ct].x, acc[ct], 0, 0, 0);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.v.y, bv[ct].y, acc[ct], 0, 0, 0);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.v.z, bv[ct].z, acc[ct], 0, 0, 0);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.v.w, bv[ct].w, acc[ct], 0, 0, 0);
  } else if constexpr (PM == 2) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(A.v.x, bv[ct].x, acc[ct], 0, 0, 0);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(A.v.y, bv[ct].y, acc[ct], 0, 0, 0);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(A.v.z, bv[ct].z, acc[ct], 0, 0, 0);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(A.v.w, bv[ct].w, acc[ct], 0, 0, 0);
  } else {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const shortx4 bb = shortx4{f2bf(bv[ct].x), f2bf(bv[ct].y), f2bf(bv[ct].z), f2bf(bv[ct].w)};
      acc[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A.v, bb, acc[ct], 0, 0, 0);
    }
  }
}

// Position in the chunk stream of a cell: strip (layer l, kind t) and chunk ch.
struct StripPos {
  int l, t, ch;
};
// First strip of the stream (D_0).
__device__ inline StripPos stream_begin() { return StripPos{0, 1, 0}; }
// Advances to the next chunk; false past the end of the stream.
__device__ inline bool stream_next(StripPos& p, int m, int nch) {
  if (++p.ch < nch) return true;
  p.ch = 0;
  ++p.t;
  if (p.t == 3 || (p.t == 2 && p.l == m - 1)) { ++p.l; p.t = 0; }
  return p.l < m;
}
__device__ inline bool last_chunk_of_layer(const StripPos& p, int m, int nch) {
  return p.ch == nch - 1 && (p.t == 2 || (p.t == 1 && p.l == m - 1));
}

// One (cell, source tile) work item `bid` of the cell phase, by one
// workgroup of 64 NCH threads with the layer tiles in `lds_raw`.
template <int NCH, int CT, int R, bool HO, int TS, bool LEAN, int PM>
__device__ inline void cell_mfma_body(const StepArgs& a, int kp, int ntile, int bid, unsigned char* lds_raw) {
  using T = typename Prec<PM>::T;
  using TB = typename Prec<PM>::TB;
  using V4 = typename Prec<PM>::V4;
  using ACC = typename Prec<PM>::ACC;
  constexpr int NS = 16 * CT;
  T* lds = reinterpret_cast<T*>(lds_raw);
  // Workgroups are dealt to the 8 XCDs round-robin; the source tiles of one
  // cell are placed 8 workgroup ids apart so that they land on the same XCD
  // close in time and share its L2 copy of the cell's blocks.
  int cell, tile;
  {
    const int grp = bid / (8 * ntile), r = bid % (8 * ntile);
    tile = r / 8;
    cell = grp * 8 + r % 8;
    if (cell >= a.nlist) return;
    if (a.d_cell_list) cell = a.d_cell_list[cell];
  }
  const OnlineCell c = a.d_cells[cell];
  const int m = c.m, b = c.b, ld = c.ld, ns = a.ns;
  const int s0 = tile * NS;
  const int nsl = min(NS, ns - s0);
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, g = l >> 4, li = l & 15;
  const int nch = (b + 15) >> 4;
  const bool active = w < nch;
  const int arow = w * 16 + li;
  const T* __restrict__ ycur = reinterpret_cast<const T*>(a.y_cur);
  const T* __restrict__ hcur = reinterpret_cast<const T*>(a.h_cur);
  T* __restrict__ hold = reinterpret_cast<T*>(a.h_old);
  T* __restrict__ phi = reinterpret_cast<T*>(a.phi);
  const int32_t* __restrict__ gat = a.d_gather + c.u1_off;
  const TB* __restrict__ blk = reinterpret_cast<const TB*>(a.d_blocks) + c.blk_off;
  const int64_t bsz = (int64_t)b * ld;
  const T dt2 = (T)a.dt2;
  const int tsz = NS * kp;
  // hidden layer j >= 1 of this cell, first source of the tile
  auto hrow = [&](auto* base, int j) { return base + (c.hid_off + (int64_t)(j - 1) * ld) * ns + (int64_t)s0 * ld; };

  auto load_chunk = [&](AFrag<PM>& A, const StripPos& p) {
    const TB* base = blk + (int64_t)(2 * p.l + p.t - 1) * bsz;
    const int kk = p.ch * 16 + g * 4;
    if (!active || arow >= b) A.zero();
    else if (p.t == 0) A.load_t(base, ld, kk, arow, b);
    else if (kk < ld) A.load(base + (int64_t)arow * ld + kk);
    else A.zero();
  };
  // layer items of this thread: item i covers column icol_i and rows
  // 4 q_i .. 4 q_i + 3 of a transposed tile; NS * 4 * NCH items over
  // 64 * NCH threads is CT items per thread.
  int icol[CT], iq[CT];
  bool iok[CT];
#pragma unroll
  for (int i = 0; i < CT; ++i) {
    const int item = tid + i * 64 * NCH;
    iq[i] = item % (4 * NCH);
    icol[i] = item / (4 * NCH);
    iok[i] = iq[i] < 4 * nch && 4 * iq[i] < ld && icol[i] < nsl;
  }
  // X_0 values of the thread's items, gathered from the piece dofs (zero
  // outside the cell or the tile). All index loads are issued before any
  // value load, at clamped in-bounds addresses, so the gather costs two
  // memory round trips rather than one per element.
  auto load_x0 = [&](V4 (&v)[CT]) {
    int32_t gi[CT][4];
#pragma unroll
    for (int i = 0; i < CT; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) gi[i][e] = gat[min(4 * iq[i] + e, b - 1)];
#pragma unroll
    for (int i = 0; i < CT; ++i) {
      const int64_t sc = s0 + min(icol[i], nsl - 1);
      T x[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const T y = ycur[(int64_t)gi[i][e] * ns + sc];
        x[e] = (iok[i] && 4 * iq[i] + e < b) ? y : (T)0;
      }
      v[i] = mk4<V4, T>(x[0], x[1], x[2], x[3]);
    }
  };
  // X_j, j >= 1, of the thread's items (zero outside the cell or the tile)
  auto load_hidden = [&](V4 (&v)[CT], int j) {
    const T* src = hrow(hcur, j);
#pragma unroll
    for (int i = 0; i < CT; ++i)
      v[i] = iok[i] ? *reinterpret_cast<const V4*>(src + (int64_t)icol[i] * ld + 4 * iq[i]) : mk4<V4, T>(0, 0, 0, 0);
  };
  auto store_layer = [&](const V4 (&v)[CT], int j) {
    T* tile = lds + (j % TS) * tsz;
#pragma unroll
    for (int i = 0; i < CT; ++i)
      if (iq[i] < 4 * NCH) *reinterpret_cast<V4*>(tile + icol[i] * kp + 4 * iq[i]) = v[i];
  };
  // previous-level values of the layer's outputs owned by this lane
  auto load_old = [&](V4 (&o)[CT], int j) {
    const int row0 = w * 16 + 4 * g;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int col = ct * 16 + li;
      o[ct] = (active && row0 < b && col < nsl)
                  ? *reinterpret_cast<const V4*>(hrow(hold, j) + (int64_t)col * ld + row0)
                  : mk4<V4, T>(0, 0, 0, 0);
    }
  };

  V4 xn[CT];
  {
    load_x0(xn);
    store_layer(xn, 0);
    if (m > 1) {
      load_hidden(xn, 1);
      store_layer(xn, 1);
    }
    if (!(LEAN && TS == 2) && m > 2) load_hidden(xn, 2);
  }
  // the ring: chunk stream positions q .. q+R-1
  AFrag<PM> ring[R];
  StripPos pf = stream_begin();   // next chunk to fetch
  bool pf_ok = true;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    if (pf_ok) {
      load_chunk(ring[u], pf);
      pf_ok = stream_next(pf, m, nch);
    } else {
      ring[u].zero();
    }
  }
  __syncthreads();
  StripPos p = stream_begin();    // chunk consumed next
  V4 ho[CT];
  ACC acc[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) acc[ct] = ACC{0, 0, 0, 0};
  bool more = true;
  while (more) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      if (more) {
        const AFrag<PM> cur = ring[u];
        if (pf_ok) {
          load_chunk(ring[u], pf);
          pf_ok = stream_next(pf, m, nch);
        }
        const int ly = p.l;
        if (active) {
          const T* Bt = lds + ((ly + p.t + TS - 1) % TS) * tsz;
          if constexpr (LEAN) {
            mma_chunk_lean<CT, PM>(acc, cur, Bt, kp, p.ch, g, li);
          } else {
            V4 bv[CT];
            load_b<CT>(bv, Bt, kp, p.ch, g, li);
            mma_chunk<CT, PM>(acc, cur, bv);
          }
        }
        if (HO && PM != 2 && p.ch == 0 && p.t == (ly == 0 ? 1 : 0) && ly >= 1) load_old(ho, ly);
        if (TS == 2 && p.t == 0 && p.ch == nch - 1 && ly + 1 < m) {
          // two tiles: X_{ly+1} replaces X_{ly-1} once every wave is done
          // with C_{ly-1}^T X_{ly-1}
          if (LEAN) load_hidden(xn, ly + 1);
          __syncthreads();
          store_layer(xn, ly + 1);
          __syncthreads();
          if (!LEAN && ly + 2 < m) load_hidden(xn, ly + 2);
        }
        if (last_chunk_of_layer(p, m, nch)) {
          if (!HO && ly >= 1 && PM != 2) load_old(ho, ly);
          if constexpr (PM == 2) {
            // the FP64 product leaves rows 16 w + g + 4 r of column li in
            // register r (the FP32 one rows 16 w + 4 g + r), so the epilogue
            // moves single elements
            if (active) {
              const T* Tl = lds + (ly % TS) * tsz;
#pragma unroll
              for (int ct = 0; ct < CT; ++ct) {
                const int col = ct * 16 + li;
                if (col >= nsl) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                  const int row = w * 16 + g + 4 * r;
                  if (row >= b) continue;
                  if (ly == 0) {
                    phi[(c.u1_off + row) * ns + s0 + col] = acc[ct][r];
                  } else {
                    T* hp = hrow(hold, ly) + (int64_t)col * ld + row;
                    *hp = (T)2 * Tl[col * kp + row] - *hp + dt2 * acc[ct][r];
                  }
                }
              }
            }
          } else if (active) {
            const T* Tl = lds + (ly % TS) * tsz;
            const int row0 = w * 16 + 4 * g;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              const int col = ct * 16 + li;
              if (row0 < b && col < nsl) {
                if (ly == 0) {
#pragma unroll
                  for (int r = 0; r < 4; ++r)
                    if (row0 + r < b) phi[(c.u1_off + row0 + r) * ns + s0 + col] = acc[ct][r];
                } else {
                  const V4 xc = *reinterpret_cast<const V4*>(Tl + col * kp + row0);
                  V4 o;
                  o.x = (T)2 * xc.x - ho[ct].x + dt2 * acc[ct][0];
                  o.y = (T)2 * xc.y - ho[ct].y + dt2 * acc[ct][1];
                  o.z = (T)2 * xc.z - ho[ct].z + dt2 * acc[ct][2];
                  o.w = (T)2 * xc.w - ho[ct].w + dt2 * acc[ct][3];
                  *reinterpret_cast<V4*>(hrow(hold, ly) + (int64_t)col * ld + row0) = o;
                }
              }
            }
          }
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) acc[ct] = ACC{0, 0, 0, 0};
          if (TS == 3 && ly + 2 < m) {
            __syncthreads();                     // every wave is done with X_{ly-1}
            store_layer(xn, ly + 2);
            __syncthreads();
            if (ly + 3 < m) load_hidden(xn, ly + 3);
          }
        }
        more = stream_next(p, m, nch);
      }
    }
  }
}

template <int NCH, int CT, int R, bool HO, int TS, int MINW, bool LEAN, int PM>
__global__ __launch_bounds__(64 * NCH, MINW) void k_cell_mfma(StepArgs a, int kp, int ntile) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  cell_mfma_body<NCH, CT, R, HO, TS, LEAN, PM>(a, kp, ntile, blockIdx.x, lds_raw);
}

template <int NCH, int CT, int R, bool HO, int TS, int MINW, bool LEAN, int PM>
static void launch_mfma(const StepArgs& a, hipStream_t st) {
  constexpr int NS = 16 * CT;
  const int kp = 16 * NCH + 4;
  const size_t lds = (size_t)TS * NS * kp * sizeof(typename Prec<PM>::T);
  const int ntile = (a.ns + NS - 1) / NS;
  const int groups = (a.nlist + 7) / 8;
  hipLaunchKernelGGL((k_cell_mfma<NCH, CT, R, HO, TS, MINW, LEAN, PM>), dim3(groups * 8 * ntile), dim3(64 * NCH), lds,
                     st, a, kp, ntile);
}

constexpr int LDS_BYTES = 160 * 1024;

// LDS bytes of TS layer tiles of NS sources at NCH strips, ES-byte elements
constexpr int tile_bytes(int NCH, int TS, int NS, int ES) { return TS * NS * (16 * NCH + 4) * ES; }

// waves per SIMD that the LDS admits for workgroups of NCH waves
constexpr int lds_waves(int NCH, int bytes) {
  const int wgs = LDS_BYTES / bytes;
  const int w = (wgs * NCH + 3) / 4;
  return w < 1 ? 1 : (w > 8 ? 8 : w);
}

template <int NCH, int PM>
static void launch_variant(const StepArgs& a, int variant, hipStream_t st) {
  constexpr int ES = sizeof(typename Prec<PM>::T);
  constexpr int B3 = tile_bytes(NCH, 3, 64, ES), B2 = tile_bytes(NCH, 2, 64, ES);
  // the fallback: 32-source tile, three layer tiles when they fit, else two
  constexpr int TS32 = tile_bytes(NCH, 3, 32, ES) <= LDS_BYTES ? 3 : 2;
  if ((variant == 0 && B3 > LDS_BYTES) || ((variant == 1 || variant == 2) && B2 > LDS_BYTES)) variant = 3;
  switch (variant) {
    case 5:
      // 16-source tiles: four times the workgroups of variant 0, for
      // partitions with few (large) cells
      launch_mfma<NCH, 1, 4, PM != 2, 3, lds_waves(NCH, tile_bytes(NCH, 3, 16, ES)), false, PM>(a, st);
      break;
    case 0:
      if constexpr (B3 <= LDS_BYTES) launch_mfma<NCH, 4, 4, false, 3, lds_waves(NCH, B3), false, PM>(a, st);
      break;
    case 1:
      if constexpr (B2 <= LDS_BYTES) launch_mfma<NCH, 4, 4, false, 2, lds_waves(NCH, B2), false, PM>(a, st);
      break;
    case 2:
      if constexpr (B2 <= LDS_BYTES) launch_mfma<NCH, 4, 4, false, 2, lds_waves(NCH, B2), true, PM>(a, st);
      break;
    default: launch_mfma<NCH, 2, 4, PM != 2, TS32, 1, false, PM>(a, st); break;
  }
}

template <int PM>
static hipError_t mfma_dispatch(const StepArgs& a, int variant, hipStream_t st) {
  const int need = (a.max_b + 15) / 16;
  if (need <= 4) launch_variant<4, PM>(a, variant, st);
  else if (need <= 6) launch_variant<6, PM>(a, variant, st);
  else if (need <= 7) launch_variant<7, PM>(a, variant, st);
  else if (need <= 8) launch_variant<8, PM>(a, variant, st);
  else if (need <= 9) launch_variant<9, PM>(a, variant, st);
  else if (need <= 10) launch_variant<10, PM>(a, variant, st);
  else if (need <= 12) launch_variant<12, PM>(a, variant, st);
  else if (need <= 16) launch_variant<16, PM>(a, variant, st);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// Piece phase: one thread per (piece, source). A wavefront holds one piece
// when n_s >= 64; pieces are faces (2 cells), edge lines (4) or corner points
// (8), so the body is instantiated per incidence count NC and every load of
// the incident fluxes is unconditional. The piece's dofs are held in
// registers (loops unrolled to MAXB with predication on b_p).
template <typename T, typename TA, int MAXB, int NC>
__device__ inline void piece_body(const StepArgs& a, const OnlinePiece& pc, int s) {
  const int bp = pc.b, ns = a.ns;
  const T* __restrict__ phi = reinterpret_cast<const T*>(a.phi);
  const T* __restrict__ ycur = reinterpret_cast<const T*>(a.y_cur);
  T* __restrict__ yold = reinterpret_cast<T*>(a.y_old);
  const TA* __restrict__ minv = reinterpret_cast<const TA*>(a.d_minv) + pc.minv_off;
  int64_t base[NC];
#pragma unroll
  for (int e = 0; e < NC; ++e) base[e] = a.d_inc[pc.inc_off + e] * ns + s;
  // Every load of the piece is issued before any value is used: rows
  // j >= b_p read row b_p - 1 (in bounds) and are dropped afterwards, so the
  // loads need no branches and share one memory round trip.
  T f[MAXB][NC], yc[MAXB], yo[MAXB];
#pragma unroll
  for (int j = 0; j < MAXB; ++j) {
    const int jr = min(j, bp - 1);
#pragma unroll
    for (int e = 0; e < NC; ++e) f[j][e] = phi[base[e] + (int64_t)jr * ns];
    const int64_t q = (pc.dof_off + jr) * ns + s;
    yc[j] = ycur[q];
    yo[j] = yold[q];
  }
  TA r[MAXB];
#pragma unroll
  for (int j = 0; j < MAXB; ++j) {
    TA acc = 0;
#pragma unroll
    for (int e = 0; e < NC; ++e) acc += (TA)f[j][e];
    r[j] = (j < bp) ? acc : (TA)0;
  }
  if (pc.src_off >= 0) {
    const T* src = reinterpret_cast<const T*>(a.d_src) + pc.src_off * ns + s;
    const TA wn = (TA)a.w[a.step];
    T g[MAXB];
#pragma unroll
    for (int j = 0; j < MAXB; ++j) g[j] = src[(int64_t)min(j, bp - 1) * ns];
#pragma unroll
    for (int j = 0; j < MAXB; ++j)
      if (j < bp) r[j] += wn * (TA)g[j];
  }
  const TA dt2 = (TA)a.dt2;
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    TA acc = 0;
#pragma unroll
    for (int j = 0; j < MAXB; ++j) acc += minv[min(i, bp - 1) + min(j, bp - 1) * bp] * r[j];
    if (i < bp) {
      const int64_t q = (pc.dof_off + i) * ns + s;
      yold[q] = (T)((TA)2 * (TA)yc[i] - (TA)yo[i] + dt2 * acc);
    }
  }
}

// Traces of the receivers that read piece p, for source s, from the piece's
// new state that this thread has just stored (same sum order as
// k_receivers, so the traces are the same).
template <typename T, typename TA>
__device__ inline void piece_receivers(const StepArgs& a, int p, int s) {
  const T* y = reinterpret_cast<const T*>(a.y_old);   // holds level n+1 now
  const int e0 = a.d_prec_ptr[p], e1 = a.d_prec_ptr[p + 1];
  for (int e = e0; e < e1; ++e) {
    const int r = a.d_prec_list[e];
    TA acc = 0;
    for (int64_t k = a.d_rptr[r]; k < a.d_rptr[r + 1]; ++k) acc += (TA)a.d_rval[k] * (TA)y[a.d_rrow[k] * a.ns + s];
    reinterpret_cast<T*>(a.traces)[(a.trace_step * a.nrec + r) * a.ns + s] = (T)acc;
  }
}

// Work item gid = (piece, source) of the piece phase. With `uni` (n_s a
// multiple of 64 and 64 consecutive items per wavefront) a wavefront holds one
// piece, so its descriptor, incidence list and inverse mass are read through
// the scalar cache.
template <typename T, typename TA, int MAXB>
__device__ inline void piece_item(const StepArgs& a, int64_t gid, bool uni) {
  if (gid >= (int64_t)a.npiece * a.ns) return;
  int p = (int)(gid / a.ns);
  const int s = (int)(gid % a.ns);
  if (uni) p = __builtin_amdgcn_readfirstlane(p);
  const OnlinePiece pc = a.d_pieces[p];
  // the unrolled bodies hold NC x rows flux values in registers: edge lines
  // (4 cells) up to 9 rows, corner points (8 cells) up to 4; wider pieces of
  // those kinds take the generic loop below
  constexpr int CAP4 = MAXB < 9 ? MAXB : 9, CAP8 = MAXB < 4 ? MAXB : 4;
  const int kind = (pc.ncell == 2) ? 2 : (pc.ncell == 4 && pc.b <= CAP4) ? 4 : (pc.ncell == 8 && pc.b <= CAP8) ? 8 : 0;
  switch (kind) {
    case 2: piece_body<T, TA, MAXB, 2>(a, pc, s); break;
    case 4: piece_body<T, TA, CAP4, 4>(a, pc, s); break;
    case 8: piece_body<T, TA, CAP8, 8>(a, pc, s); break;
    default: {
      // generic incidence count (partitions that are not Cartesian)
      const int bp = pc.b, ns = a.ns;
      const T* phi = reinterpret_cast<const T*>(a.phi);
      const T* ycur = reinterpret_cast<const T*>(a.y_cur);
      T* yold = reinterpret_cast<T*>(a.y_old);
      const TA* minv = reinterpret_cast<const TA*>(a.d_minv) + pc.minv_off;
      TA r[MAXB];
#pragma unroll
      for (int j = 0; j < MAXB; ++j) {
        TA acc = 0;
        if (j < bp) {
          for (int e = 0; e < pc.ncell; ++e) acc += (TA)phi[(a.d_inc[pc.inc_off + e] + j) * ns + s];
          if (pc.src_off >= 0) acc += (TA)a.w[a.step] * (TA)reinterpret_cast<const T*>(a.d_src)[(pc.src_off + j) * ns + s];
        }
        r[j] = acc;
      }
#pragma unroll
      for (int i = 0; i < MAXB; ++i) {
        if (i < bp) {
          TA acc = 0;
#pragma unroll
          for (int j = 0; j < MAXB; ++j)
            if (j < bp) acc += minv[i + j * bp] * r[j];
          const int64_t q = (pc.dof_off + i) * ns + s;
          yold[q] = (T)((TA)2 * (TA)ycur[q] - (TA)yold[q] + (TA)a.dt2 * acc);
        }
      }
    }
  }
  if (a.d_prec_ptr) piece_receivers<T, TA>(a, p, s);
}

template <typename T, typename TA, int MAXB, bool UNI>
__global__ __launch_bounds__(256) void k_piece_phase(StepArgs a) {
  piece_item<T, TA, MAXB>(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, UNI);
}

// Work item gid = (receiver, source) of the receivers: the new piece state.
template <typename T, typename TA>
__device__ inline void receiver_item(const StepArgs& a, int64_t gid) {
  if (gid >= (int64_t)a.nrec * a.ns) return;
  const int r = (int)(gid / a.ns), s = (int)(gid % a.ns);
  const T* y = reinterpret_cast<const T*>(a.y_old);   // holds level n+1 now
  TA acc = 0;
  for (int64_t k = a.d_rptr[r]; k < a.d_rptr[r + 1]; ++k) acc += (TA)a.d_rval[k] * (TA)y[a.d_rrow[k] * a.ns + s];
  reinterpret_cast<T*>(a.traces)[(a.trace_step * a.nrec + r) * a.ns + s] = (T)acc;
}

template <typename T, typename TA>
__global__ __launch_bounds__(256) void k_receivers(StepArgs a) {
  receiver_item<T, TA>(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Persistent on-line kernel: one cooperative launch runs many leapfrog steps.
// Each step: the cell phase over all (cell, 64-source tile) items, strided
// over the resident workgroups (with the receivers of the previous step when
// they are not fused), a grid barrier, the piece phase over all (piece,
// source) items, a grid barrier. The launch is cooperative, so every
// workgroup is resident and every thread reaches every barrier.
// ---------------------------------------------------------------------------

template <int NCH, int PM, int MAXB, int TS, int MINW, bool LEAN>
__global__ __launch_bounds__(64 * NCH, MINW) void k_persistent(StepArgs a, int kp, int ntile, PersistArgs pa) {
  using T = typename Prec<PM>::T;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const int ncb = ((a.nlist + 7) / 8) * 8 * ntile;
  const int64_t npi = (int64_t)a.npiece * a.ns, nri = (int64_t)a.nrec * a.ns;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool uni = a.ns % 64 == 0;
  StepArgs b = a;
  for (int64_t s = 0; s < pa.n_steps; ++s) {
    const int cur = (pa.cur0 + (int)(s & 1)) & 1;
    b.y_cur = pa.y[cur]; b.y_old = pa.y[1 - cur];
    b.h_cur = pa.h[cur]; b.h_old = pa.h[1 - cur];
    b.step = s; b.trace_step = s;
    if (!pa.rec_fused && s > 0) {
      // the previous step's new level is this step's current level
      StepArgs r = b;
      r.y_old = b.y_cur;
      r.trace_step = s - 1;
      for (int64_t gid = g0; gid < nri; gid += stride) receiver_item<T, T>(r, gid);
    }
    for (int bid = blockIdx.x; bid < ncb; bid += gridDim.x) {
      cell_mfma_body<NCH, 4, 4, false, TS, LEAN, PM>(b, kp, ntile, bid, lds_raw);
      __syncthreads();   // the next item rewrites the layer tiles
    }
    grid.sync();
    for (int64_t gid = g0; gid < npi; gid += stride) piece_item<T, T, MAXB>(b, gid, uni);
    grid.sync();
  }
  if (!pa.rec_fused && pa.n_steps > 0) {
    StepArgs r = b;   // b.y_old holds the last step's new level
    for (int64_t gid = g0; gid < nri; gid += stride) receiver_item<T, T>(r, gid);
  }
}

template <int NCH, int PM, int MAXB>
static hipError_t launch_persistent_t(const StepArgs& a, const PersistArgs& pa, hipStream_t st) {
  constexpr int ES = sizeof(typename Prec<PM>::T);
  constexpr int B3 = tile_bytes(NCH, 3, 64, ES), B2 = tile_bytes(NCH, 2, 64, ES);
  static_assert(B2 <= LDS_BYTES, "two layer tiles must fit");
  constexpr int TS = B3 <= LDS_BYTES ? 3 : 2;
  constexpr int MINW = lds_waves(NCH, TS == 3 ? B3 : B2);
  constexpr bool LEAN = TS == 2;
  const void* fn = reinterpret_cast<const void*>(&k_persistent<NCH, PM, MAXB, TS, MINW, LEAN>);
  const int kp = 16 * NCH + 4;
  const size_t lds = (size_t)TS * 64 * kp * ES;
  const int ntile = (a.ns + 63) / 64;
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * NCH, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const int grid = per_cu * prop.multiProcessorCount;
  StepArgs a1 = a;
  PersistArgs p1 = pa;
  int kp1 = kp, nt1 = ntile;
  void* args[] = {&a1, &kp1, &nt1, &p1};
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(64 * NCH), args, (unsigned)lds, st);
}

template <int NCH, int PM>
static hipError_t persistent_bp(const StepArgs& a, const PersistArgs& pa, hipStream_t st) {
  if (a.max_bp <= 4) return launch_persistent_t<NCH, PM, 4>(a, pa, st);
  if (a.max_bp <= 9) return launch_persistent_t<NCH, PM, 9>(a, pa, st);
  return launch_persistent_t<NCH, PM, 16>(a, pa, st);
}

template <int PM>
static hipError_t persistent_nch(const StepArgs& a, const PersistArgs& pa, hipStream_t st) {
  const int need = (a.max_b + 15) / 16;
  if (need <= 4) return persistent_bp<4, PM>(a, pa, st);
  if (need <= 7) return persistent_bp<7, PM>(a, pa, st);
  return persistent_bp<9, PM>(a, pa, st);
}

bool persistent_supported(const StepArgs& a) {
  return (a.prec == SFROM_F32 || a.prec == SFROM_F64) && a.max_b <= 144 && a.max_bp <= 16 && a.ns > 0;
}

hipError_t launch_persistent(const StepArgs& a, const PersistArgs& pa, hipStream_t st) {
  if (!persistent_supported(a)) return hipErrorInvalidValue;
  if (a.prec == SFROM_F64) return persistent_nch<2>(a, pa, st);
  return persistent_nch<0>(a, pa, st);
}


int cell_tile(const StepArgs& a, size_t acc_bytes) {
  // largest power-of-two source tile (<= 64) whose LDS fits in 64 KiB
  int nst = 64;
  while (nst > 1 && (size_t)a.max_m * a.max_b * nst * acc_bytes > 65536) nst /= 2;
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
  const size_t lds = (size_t)a.max_m * a.max_b * nst * sizeof(TA);
  const dim3 g1(a.nlist, (a.ns + nst - 1) / nst);
  hipLaunchKernelGGL((k_cell_phase<T, TB, TA>), g1, dim3(CELL_NT), lds, st, a, nst);
  return hipGetLastError();
}

template <typename T, typename TA>
static hipError_t piece_impl(const StepArgs& a, hipStream_t st) {
  const int64_t np = (int64_t)a.npiece * a.ns;
  const dim3 g((np + 255) / 256), b(256);
  if (a.ns % 64 == 0) {
    if (a.max_bp <= 4) hipLaunchKernelGGL((k_piece_phase<T, TA, 4, true>), g, b, 0, st, a);
    else if (a.max_bp <= 9) hipLaunchKernelGGL((k_piece_phase<T, TA, 9, true>), g, b, 0, st, a);
    else if (a.max_bp <= 16) hipLaunchKernelGGL((k_piece_phase<T, TA, 16, true>), g, b, 0, st, a);
    else hipLaunchKernelGGL((k_piece_phase<T, TA, 32, true>), g, b, 0, st, a);
  } else {
    if (a.max_bp <= 4) hipLaunchKernelGGL((k_piece_phase<T, TA, 4, false>), g, b, 0, st, a);
    else if (a.max_bp <= 9) hipLaunchKernelGGL((k_piece_phase<T, TA, 9, false>), g, b, 0, st, a);
    else if (a.max_bp <= 16) hipLaunchKernelGGL((k_piece_phase<T, TA, 16, false>), g, b, 0, st, a);
    else hipLaunchKernelGGL((k_piece_phase<T, TA, 32, false>), g, b, 0, st, a);
  }
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

int cell_variants(const StepArgs& a) { return a.max_b > 256 ? 1 : 6; }

hipError_t launch_cell_phase(const StepArgs& a, hipStream_t st) {
  // variants 0..3: matrix-core kernel (FP32, BF16 blocks or FP64) with 4
  // chunks in flight and the register budget of the waves the LDS admits
  // (source tile 64 with three layer tiles; two tiles; two tiles with
  // per-tile B reads and the next layer read at its store; source tile 32);
  // 4: the scalar kernel; 5: matrix cores with 16-source tiles
  if (a.max_b > 256 || a.cell_variant == 4) {
    if (a.prec == SFROM_F64) return cell_impl<double, double, double>(a, st);
    if (a.prec == SFROM_F32) return cell_impl<float, float, float>(a, st);
    return cell_impl<float, __hip_bfloat16, float>(a, st);
  }
  if (a.prec == SFROM_F32) return mfma_dispatch<0>(a, a.cell_variant, st);
  if (a.prec == SFROM_F64) return mfma_dispatch<2>(a, a.cell_variant, st);
  return mfma_dispatch<1>(a, a.cell_variant, st);
}

hipError_t launch_piece_phase(const StepArgs& a, hipStream_t st) {
  if (a.prec == SFROM_F64) return piece_impl<double, double>(a, st);
  return piece_impl<float, float>(a, st);
}

hipError_t launch_receivers(const StepArgs& a, hipStream_t st) {
  if (a.prec == SFROM_F64) return rec_impl<double, double>(a, st);
  return rec_impl<float, float>(a, st);
}

// Correction at the corner-set nodes (App. D), in three short kernels so
// that no thread walks a long chain of dependent loads. Kernel 1: one thread
// per (copy, source) writes the copy's value u_t = S_p(row, :) y_p into delta.
template <typename T>
__global__ __launch_bounds__(256) void k_corner_value(CornerArgs c) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= c.ncopy * c.ns) return;
  const int t = (int)(gid / c.ns), s = (int)(gid % c.ns);
  const int ns = c.ns;
  const T* __restrict__ row = reinterpret_cast<const T*>(c.srow) + c.soff[t];
  const T* __restrict__ yp = reinterpret_cast<const T*>(c.y) + c.hdof[t] * ns + s;
  const int bp = c.hbp[t];
  T u0 = 0, u1 = 0;
  int j = 0;
  for (; j + 1 < bp; j += 2) {
    u0 += row[j] * yp[(int64_t)j * ns];
    u1 += row[j + 1] * yp[(int64_t)(j + 1) * ns];
  }
  if (j < bp) u0 += row[j] * yp[(int64_t)j * ns];
  reinterpret_cast<T*>(c.delta)[(int64_t)t * ns + s] = u0 + u1;
}

// Kernel 2: one thread per (removed node, source) replaces its copies'
// values by delta_t = sum_t' w_t' u_t' - u_t.
template <typename T>
__global__ __launch_bounds__(256) void k_corner_delta(CornerArgs c) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)c.ncorner * c.ns) return;
  const int k = (int)(gid / c.ns), s = (int)(gid % c.ns);
  const int ns = c.ns;
  const T* __restrict__ hw = reinterpret_cast<const T*>(c.hw);
  T* __restrict__ delta = reinterpret_cast<T*>(c.delta);
  T ubar = 0;
  for (int t = c.hptr[k]; t < c.hptr[k + 1]; ++t) ubar += hw[t] * delta[(int64_t)t * ns + s];
  for (int t = c.hptr[k]; t < c.hptr[k + 1]; ++t) delta[(int64_t)t * ns + s] = ubar - delta[(int64_t)t * ns + s];
}

// Kernel 3: one thread per (dof row of a piece holding copies, source); every
// copy lies in exactly one piece, so each dof row is written by one thread.
template <typename T>
__global__ __launch_bounds__(256) void k_corner_apply(CornerArgs c) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)c.nrow * c.ns) return;
  const int r = (int)(gid / c.ns), s = (int)(gid % c.ns);
  const int ns = c.ns;
  const int q = c.rowq[r], j = c.rowj[r];
  T* __restrict__ y = reinterpret_cast<T*>(c.y);
  const T* __restrict__ srow = reinterpret_cast<const T*>(c.srow);
  const T* __restrict__ delta = reinterpret_cast<const T*>(c.delta);
  T a0 = 0, a1 = 0;
  int e = c.pptr[q];
  const int e1 = c.pptr[q + 1];
  for (; e + 1 < e1; e += 2) {
    const int t0 = c.plist[e], t1 = c.plist[e + 1];
    a0 += srow[c.soff[t0] + j] * delta[(int64_t)t0 * ns + s];
    a1 += srow[c.soff[t1] + j] * delta[(int64_t)t1 * ns + s];
  }
  if (e < e1) {
    const int t0 = c.plist[e];
    a0 += srow[c.soff[t0] + j] * delta[(int64_t)t0 * ns + s];
  }
  y[(c.pdof[q] + j) * ns + s] += a0 + a1;
}

template <typename T>
static hipError_t corner_impl(const CornerArgs& c, hipStream_t st) {
  const int64_t n0 = c.ncopy * c.ns, n1 = (int64_t)c.ncorner * c.ns, n2 = (int64_t)c.nrow * c.ns;
  if (n0 > 0) hipLaunchKernelGGL((k_corner_value<T>), dim3((unsigned)((n0 + 255) / 256)), dim3(256), 0, st, c);
  if (n1 > 0) hipLaunchKernelGGL((k_corner_delta<T>), dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, c);
  if (n2 > 0) hipLaunchKernelGGL((k_corner_apply<T>), dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, c);
  return hipGetLastError();
}

hipError_t launch_corner_correction(const CornerArgs& c, hipStream_t st) {
  if (c.prec == SFROM_F64) return corner_impl<double>(c, st);
  return corner_impl<float>(c, st);
}

// Sets *flag when any of the n state values is NaN or infinite (leap-frog
// divergence). The flag is written with a vector atomic by one lane per wave.
template <typename T>
__global__ __launch_bounds__(256) void k_nonfinite(const T* __restrict__ x, int64_t n, int32_t* flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = (double)x[i];
    bad |= !(v - v == 0.0);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// Writes zero to one int32 (a kernel, not a memset, so that callers which
// capture the run into a graph record no memset node).
__global__ void k_zero_flag(int32_t* flag) { *flag = 0; }

hipError_t launch_zero_flag(int32_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(1), 0, st, flag);
  return hipGetLastError();
}

hipError_t launch_nonfinite(const void* x, int64_t n, int prec, int32_t* flag, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>(2048, (n + 255) / 256);
  if (prec == SFROM_F64)
    hipLaunchKernelGGL(k_nonfinite<double>, dim3(grid), dim3(256), 0, st, (const double*)x, n, flag);
  else
    hipLaunchKernelGGL(k_nonfinite<float>, dim3(grid), dim3(256), 0, st, (const float*)x, n, flag);
  return hipGetLastError();
}

hipError_t launch_online_step(const StepArgs& a, hipStream_t st) {
  hipError_t e = launch_cell_phase(a, st);
  if (e != hipSuccess) return e;
  e = launch_piece_phase(a, st);
  if (e != hipSuccess) return e;
  return launch_receivers(a, st);
}

}  // namespace sfrom_impl
