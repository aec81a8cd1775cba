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
    const TB* G = blk + (int64_t)k * b * c.ld + (int64_t)r * c.ld;
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
    const TB* Gh = blk + (int64_t)(m + k - 1) * b * c.ld + (int64_t)r * c.ld;
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

// ---------------------------------------------------------------------------
// Cell phase on the matrix cores (float state; float or bfloat16 blocks).
//
// One workgroup per (cell, tile of 16*CT sources); wave w owns rows
// [16w, 16w+16) of every b x b block product, so a block is streamed from
// HBM once per source tile and each wave holds its 16-row strip of the
// block in registers (NCH float4 per lane). The K dimension is traversed in
// chunks of 16 with a permuted order: inside a chunk, lane group g = lane/16
// supplies k = 16 ch + 4 g + j to MFMA step j, so each lane fetches its A
// values as one float4 from the row-major (symmetric) block and its B values
// as one float4 from the transposed LDS tile. The strip of the next block is
// prefetched while the current product runs.
//
// LDS: Dt = (U^{k+1} - U^k)^T and Et = (Phi^k - Phi^{k-1})^T, each
// [16*CT columns][kp], kp = 16*NCH + 4. The fluxes of the previous layer
// stay in registers.
// ---------------------------------------------------------------------------

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

__device__ inline short f2bf(float f) {
  // round to nearest even (the state is finite; NaN propagates as NaN)
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

template <bool BF16>
struct AFrag;
template <>
struct AFrag<false> {
  float4 v;
  __device__ void load(const float* p) { v = *reinterpret_cast<const float4*>(p); }
  __device__ void zero() { v = make_float4(0.f, 0.f, 0.f, 0.f); }
};
template <>
struct AFrag<true> {
  shortx4 v;
  __device__ void load(const __hip_bfloat16* p) { v = *reinterpret_cast<const shortx4*>(p); }
  __device__ void zero() { v = shortx4{0, 0, 0, 0}; }
};

template <int NCH, int CT, bool BF16>
__device__ inline void mfma_strip(floatx4 (&acc)[CT], const AFrag<BF16> (&A)[NCH], const float* Bt, int kp,
                                  int nch, int g, int li) {
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    if (ch < nch) {
      float4 bv[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
        bv[ct] = *reinterpret_cast<const float4*>(Bt + (ct * 16 + li) * kp + ch * 16 + g * 4);
      // consecutive MFMAs go to independent accumulators (column tiles)
      if constexpr (!BF16) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[ch].v.x, bv[ct].x, acc[ct], 0, 0, 0);
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[ch].v.y, bv[ct].y, acc[ct], 0, 0, 0);
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[ch].v.z, bv[ct].z, acc[ct], 0, 0, 0);
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[ch].v.w, bv[ct].w, acc[ct], 0, 0, 0);
      } else {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const shortx4 bb = shortx4{f2bf(bv[ct].x), f2bf(bv[ct].y), f2bf(bv[ct].z), f2bf(bv[ct].w)};
          acc[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[ch].v, bb, acc[ct], 0, 0, 0);
        }
      }
    }
  }
}

template <int NCH, int CT, bool PF, bool BF16>
__global__ __launch_bounds__(64 * NCH) void k_cell_mfma(StepArgs a, int kp, int ntile) {
  using TB = typename std::conditional<BF16, __hip_bfloat16, float>::type;
  constexpr int NS = 16 * CT;
  extern __shared__ float lds[];
  float* Dt = lds;
  float* Et = lds + NS * kp;
  // Workgroups are dealt to the 8 XCDs round-robin; the source tiles of one
  // cell are placed 8 workgroup ids apart so that they land on the same XCD
  // close in time and share its L2 copy of the cell's blocks.
  int cell, tile;
  {
    const int bid = blockIdx.x;
    const int grp = bid / (8 * ntile), r = bid % (8 * ntile);
    tile = r / 8;
    cell = grp * 8 + r % 8;
    if (cell >= a.ncell) return;
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
  const float* __restrict__ ycur = reinterpret_cast<const float*>(a.y_cur);
  const float* __restrict__ hcur = reinterpret_cast<const float*>(a.h_cur);
  float* __restrict__ hold = reinterpret_cast<float*>(a.h_old);
  float* __restrict__ phi = reinterpret_cast<float*>(a.phi);
  const int32_t* __restrict__ gat = a.d_gather + c.u1_off;
  const TB* __restrict__ blk = reinterpret_cast<const TB*>(a.d_blocks) + c.blk_off;
  const int64_t bsz = (int64_t)b * ld;
  const float dt2 = (float)a.dt2;

  AFrag<BF16> Acur[NCH], Anxt[PF ? NCH : 1];
  auto load_strip = [&](auto& A, const TB* base) {
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int kk = ch * 16 + g * 4;
      if (active && ch < nch && arow < b && kk < ld) A[ch].load(base + (int64_t)arow * ld + kk);
      else A[ch].zero();
    }
  };
  auto copy_strip = [&]() {
    if constexpr (PF) {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) Acur[ch] = Anxt[ch];
    }
  };
  // Delta items of this thread: item i covers column col_i and rows
  // 4 q_i .. 4 q_i + 3 of the transposed tile; NS * 4 * NCH items over
  // 64 * NCH threads is CT items per thread.
  int icol[CT], iq[CT];
  bool iok[CT];
#pragma unroll
  for (int i = 0; i < CT; ++i) {
    const int item = tid + i * 64 * NCH;
    icol[i] = item % NS;
    iq[i] = item / NS;
    iok[i] = iq[i] < 4 * nch;
  }
  // U^j values of the thread's items (zero outside the cell or the tile)
  auto load_layer = [&](float4 (&v)[CT], int j) {
#pragma unroll
    for (int i = 0; i < CT; ++i) {
      float x[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int kk = 4 * iq[i] + e;
        float t = 0.f;
        if (j < m && iok[i] && kk < b && icol[i] < nsl) {
          if (j == 0) t = ycur[(int64_t)gat[kk] * ns + s0 + icol[i]];
          else t = hcur[(c.hid_off + (int64_t)(j - 1) * b + kk) * ns + s0 + icol[i]];
        }
        x[e] = t;
      }
      v[i] = make_float4(x[0], x[1], x[2], x[3]);
    }
  };

  float4 UA[CT], UB[CT];
  load_layer(UA, 0);
  load_layer(UB, 1);
  load_strip(Acur, blk);                       // G^1
  floatx4 prev[CT];
  for (int k = 0; k < m; ++k) {
    // Dt = (U^{k+1} - U^k)^T; U^{m+1} = 0 (load_layer returns zeros for j >= m)
#pragma unroll
    for (int i = 0; i < CT; ++i) {
      if (iok[i]) {
        const float4 d = make_float4(UB[i].x - UA[i].x, UB[i].y - UA[i].y, UB[i].z - UA[i].z, UB[i].w - UA[i].w);
        *reinterpret_cast<float4*>(Dt + icol[i] * kp + 4 * iq[i]) = d;
      }
      UA[i] = UB[i];
    }
    if (k + 2 <= m) load_layer(UB, k + 2);     // in flight during this layer's products
    __syncthreads();
    if (PF) {
      if (k >= 1) load_strip(Anxt, blk + (int64_t)(m + k - 1) * bsz);
      else if (m > 1) load_strip(Anxt, blk + bsz);
    }
    floatx4 acc[CT];
    if (active) mfma_strip<NCH, CT, BF16>(acc, Acur, Dt, kp, nch, g, li);
    // operands of the hidden-layer update, loaded before the second product
    float hc[CT][4], ho[CT][4];
    if (k >= 1 && active) {
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = w * 16 + 4 * g + r, col = ct * 16 + li;
          const bool ok = row < b && col < nsl;
          const int64_t hi = (c.hid_off + (int64_t)(k - 1) * b + row) * ns + s0 + col;
          hc[ct][r] = ok ? hcur[hi] : 0.f;
          ho[ct][r] = ok ? hold[hi] : 0.f;
        }
    }
    if (active) {
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int col = ct * 16 + li;
        if (k == 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = w * 16 + 4 * g + r;
            if (row < b && col < nsl) phi[(c.u1_off + row) * ns + s0 + col] = acc[ct][r];
          }
        } else {
          const floatx4 e = acc[ct] - prev[ct];
          *reinterpret_cast<float4*>(Et + col * kp + w * 16 + 4 * g) = make_float4(e[0], e[1], e[2], e[3]);
        }
        prev[ct] = acc[ct];
      }
    }
    __syncthreads();
    if (PF) copy_strip();
    else if (k >= 1) load_strip(Acur, blk + (int64_t)(m + k - 1) * bsz);
    else if (m > 1) load_strip(Acur, blk + bsz);
    if (k >= 1) {
      if (PF && k + 1 < m) load_strip(Anxt, blk + (int64_t)(k + 1) * bsz);
      floatx4 acc2[CT];
      if (active) {
        mfma_strip<NCH, CT, BF16>(acc2, Acur, Et, kp, nch, g, li);
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const int col = ct * 16 + li;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = w * 16 + 4 * g + r;
            if (row < b && col < nsl) {
              const int64_t hi = (c.hid_off + (int64_t)(k - 1) * b + row) * ns + s0 + col;
              hold[hi] = 2.f * hc[ct][r] - ho[ct][r] + dt2 * acc2[ct][r];
            }
          }
        }
      }
      if (PF) copy_strip();
      else if (k + 1 < m) load_strip(Acur, blk + (int64_t)(k + 1) * bsz);
    }
  }
}

// ---------------------------------------------------------------------------
// Streaming variant of the matrix-core cell phase: NW = ceil(nch / TPW)
// waves per workgroup, each owning TPW 16-row tiles and streaming its A
// fragments from HBM through a register ring of RING chunks. Registers and
// LDS per workgroup are small, so several cells are in flight per CU and the
// latency of one cell's loads is hidden behind another cell's products.
// ---------------------------------------------------------------------------
template <int TPW, int CT, bool BF16>
__global__ __launch_bounds__(256) void k_cell_stream(StepArgs a, int kp, int ntile) {
  using TB = typename std::conditional<BF16, __hip_bfloat16, float>::type;
  constexpr int NS = 16 * CT;
  constexpr int RING = 4;
  extern __shared__ float lds[];
  float* Dt = lds;
  float* Et = lds + NS * kp;
  int cell, tile;
  {
    const int bid = blockIdx.x;
    const int grp = bid / (8 * ntile), r = bid % (8 * ntile);
    tile = r / 8;
    cell = grp * 8 + r % 8;
    if (cell >= a.ncell) return;
  }
  const OnlineCell c = a.d_cells[cell];
  const int m = c.m, b = c.b, ld = c.ld, ns = a.ns;
  const int s0 = tile * NS;
  const int nsl = min(NS, ns - s0);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int nw = nthr >> 6;
  const int w = tid >> 6, l = tid & 63, g = l >> 4, li = l & 15;
  const int nch = (b + 15) >> 4;
  const float* __restrict__ ycur = reinterpret_cast<const float*>(a.y_cur);
  const float* __restrict__ hcur = reinterpret_cast<const float*>(a.h_cur);
  float* __restrict__ hold = reinterpret_cast<float*>(a.h_old);
  float* __restrict__ phi = reinterpret_cast<float*>(a.phi);
  const int32_t* __restrict__ gat = a.d_gather + c.u1_off;
  const TB* __restrict__ blk = reinterpret_cast<const TB*>(a.d_blocks) + c.blk_off;
  const int64_t bsz = (int64_t)b * ld;
  const float dt2 = (float)a.dt2;

  // product of the wave's row tiles of block `base` with the transposed LDS
  // tile Bt; results in acc[t][ct]
  auto product = [&](floatx4 (&acc)[TPW][CT], const TB* base, const float* Bt) {
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[t][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
      const int rt = w + t * nw;
      if (rt >= nch) continue;
      const int row = rt * 16 + li;
      const bool rok = row < b;
      const TB* rp = base + (int64_t)(rok ? row : 0) * ld;
      AFrag<BF16> ring[RING];
#pragma unroll
      for (int u = 0; u < RING; ++u) {
        const int kk = u * 16 + g * 4;
        if (u < nch && rok && kk < ld) ring[u].load(rp + kk); else ring[u].zero();
      }
      for (int ch0 = 0; ch0 < nch; ch0 += RING) {
#pragma unroll
        for (int u = 0; u < RING; ++u) {
          const int ch = ch0 + u;
          if (ch < nch) {
            const AFrag<BF16> av = ring[u];
            const int kn = (ch + RING) * 16 + g * 4;
            if (ch + RING < nch && rok && kn < ld) ring[u].load(rp + kn); else ring[u].zero();
            float4 bv[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
              bv[ct] = *reinterpret_cast<const float4*>(Bt + (ct * 16 + li) * kp + ch * 16 + g * 4);
            if constexpr (!BF16) {
#pragma unroll
              for (int ct = 0; ct < CT; ++ct) acc[t][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.v.x, bv[ct].x, acc[t][ct], 0, 0, 0);
#pragma unroll
              for (int ct = 0; ct < CT; ++ct) acc[t][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.v.y, bv[ct].y, acc[t][ct], 0, 0, 0);
#pragma unroll
              for (int ct = 0; ct < CT; ++ct) acc[t][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.v.z, bv[ct].z, acc[t][ct], 0, 0, 0);
#pragma unroll
              for (int ct = 0; ct < CT; ++ct) acc[t][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.v.w, bv[ct].w, acc[t][ct], 0, 0, 0);
            } else {
#pragma unroll
              for (int ct = 0; ct < CT; ++ct) {
                const shortx4 bb = shortx4{f2bf(bv[ct].x), f2bf(bv[ct].y), f2bf(bv[ct].z), f2bf(bv[ct].w)};
                acc[t][ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av.v, bb, acc[t][ct], 0, 0, 0);
              }
            }
          }
        }
      }
    }
  };

  floatx4 prev[TPW][CT];
  for (int k = 0; k < m; ++k) {
    // Dt = (U^{k+1} - U^k)^T, zero padded to 16 nch rows and NS columns
    for (int t = tid; t < NS * 4 * nch; t += nthr) {
      const int col = t % NS, q = t / NS;
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int kk = 4 * q + e;
        float d = 0.f;
        if (kk < b && col < nsl) {
          const float un = (k + 1 < m) ? hcur[(c.hid_off + (int64_t)k * b + kk) * ns + s0 + col] : 0.f;
          const float uc = (k == 0) ? ycur[(int64_t)gat[kk] * ns + s0 + col]
                                    : hcur[(c.hid_off + (int64_t)(k - 1) * b + kk) * ns + s0 + col];
          d = un - uc;
        }
        v[e] = d;
      }
      *reinterpret_cast<float4*>(Dt + col * kp + 4 * q) = make_float4(v[0], v[1], v[2], v[3]);
    }
    __syncthreads();
    floatx4 acc[TPW][CT];
    product(acc, blk + (int64_t)k * bsz, Dt);
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int rt = w + t * nw;
      if (rt >= nch) continue;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int col = ct * 16 + li;
        if (k == 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = rt * 16 + 4 * g + r;
            if (row < b && col < nsl) phi[(c.u1_off + row) * ns + s0 + col] = acc[t][ct][r];
          }
        } else {
          const floatx4 e = acc[t][ct] - prev[t][ct];
          *reinterpret_cast<float4*>(Et + col * kp + rt * 16 + 4 * g) = make_float4(e[0], e[1], e[2], e[3]);
        }
        prev[t][ct] = acc[t][ct];
      }
    }
    __syncthreads();
    if (k >= 1) {
      floatx4 acc2[TPW][CT];
      product(acc2, blk + (int64_t)(m + k - 1) * bsz, Et);
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int rt = w + t * nw;
        if (rt >= nch) continue;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const int col = ct * 16 + li;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = rt * 16 + 4 * g + r;
            if (row < b && col < nsl) {
              const int64_t hi = (c.hid_off + (int64_t)(k - 1) * b + row) * ns + s0 + col;
              hold[hi] = 2.f * hcur[hi] - hold[hi] + dt2 * acc2[t][ct][r];
            }
          }
        }
      }
    }
    // Dt is rewritten at the next layer only after every wave has finished
    // reading it (the barrier above), and Et only after the next barrier
  }
}

template <int TPW, int CT, bool BF16>
static void launch_stream(const StepArgs& a, hipStream_t st) {
  constexpr int NS = 16 * CT;
  const int nchmax = (a.max_b + 15) / 16;
  const int kp = 16 * nchmax + 4;
  const int nw = (nchmax + TPW - 1) / TPW;
  const size_t lds = 2 * (size_t)NS * kp * sizeof(float);
  const int ntile = (a.ns + NS - 1) / NS;
  const int groups = (a.ncell + 7) / 8;
  hipLaunchKernelGGL((k_cell_stream<TPW, CT, BF16>), dim3(groups * 8 * ntile), dim3(64 * nw), lds, st, a, kp, ntile);
}

template <int NCH, int CT, bool PF, bool BF16>
static void launch_mfma(const StepArgs& a, hipStream_t st) {
  constexpr int NS = 16 * CT;
  const int kp = 16 * NCH + 4;
  const size_t lds = 2 * (size_t)NS * kp * sizeof(float);
  const int ntile = (a.ns + NS - 1) / NS;
  const int groups = (a.ncell + 7) / 8;
  hipLaunchKernelGGL((k_cell_mfma<NCH, CT, PF, BF16>), dim3(groups * 8 * ntile), dim3(64 * NCH), lds, st, a, kp,
                     ntile);
}

template <int NCH, bool BF16>
static void launch_variant(const StepArgs& a, int variant, hipStream_t st) {
  switch (variant) {
    case 0: launch_mfma<NCH, 4, true, BF16>(a, st); break;
    case 1: launch_mfma<NCH, 4, false, BF16>(a, st); break;
    case 2: launch_mfma<NCH, 2, true, BF16>(a, st); break;
    default: launch_mfma<NCH, 2, false, BF16>(a, st); break;
  }
}

template <bool BF16>
static hipError_t mfma_dispatch(const StepArgs& a, int variant, hipStream_t st) {
  const int need = (a.max_b + 15) / 16;
  if (variant >= 4) {
    if ((need + 1) / 2 > 4 && variant < 6) variant += 2;   // keep <= 4 waves per group
    switch (variant) {
      case 4: launch_stream<2, 1, BF16>(a, st); break;
      case 5: launch_stream<2, 2, BF16>(a, st); break;
      case 6: launch_stream<3, 1, BF16>(a, st); break;
      default: launch_stream<3, 2, BF16>(a, st); break;
    }
    return hipGetLastError();
  }
  if (need <= 4) launch_variant<4, BF16>(a, variant, st);
  else if (need <= 6) launch_variant<6, BF16>(a, variant, st);
  else if (need <= 7) launch_variant<7, BF16>(a, variant, st);
  else if (need <= 8) launch_variant<8, BF16>(a, variant, st);
  else if (need <= 9) launch_variant<9, BF16>(a, variant, st);
  else if (need <= 10) launch_variant<10, BF16>(a, variant, st);
  else if (need <= 12) launch_variant<12, BF16>(a, variant, st);
  else if (need <= 16) launch_variant<16, BF16>(a, variant, st);
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
  TA r[MAXB];
#pragma unroll
  for (int j = 0; j < MAXB; ++j) {
    TA acc = 0;
    if (j < bp) {
#pragma unroll
      for (int e = 0; e < NC; ++e) acc += (TA)phi[base[e] + (int64_t)j * ns];
    }
    r[j] = acc;
  }
  if (pc.src_off >= 0) {
    const T* src = reinterpret_cast<const T*>(a.d_src) + pc.src_off * ns + s;
    const TA wn = (TA)a.w[a.step];
#pragma unroll
    for (int j = 0; j < MAXB; ++j)
      if (j < bp) r[j] += wn * (TA)src[(int64_t)j * ns];
  }
  const TA dt2 = (TA)a.dt2;
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    if (i < bp) {
      TA acc = 0;
#pragma unroll
      for (int j = 0; j < MAXB; ++j)
        if (j < bp) acc += minv[i + j * bp] * r[j];
      const int64_t q = (pc.dof_off + i) * ns + s;
      yold[q] = (T)((TA)2 * (TA)ycur[q] - (TA)yold[q] + dt2 * acc);
    }
  }
}

template <typename T, typename TA, int MAXB>
__global__ __launch_bounds__(256) void k_piece_phase(StepArgs a) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)a.npiece * a.ns) return;
  const int p = (int)(gid / a.ns), s = (int)(gid % a.ns);
  const OnlinePiece pc = a.d_pieces[p];
  switch (pc.ncell) {
    case 2: piece_body<T, TA, MAXB, 2>(a, pc, s); break;
    case 4: piece_body<T, TA, (MAXB < 9 ? MAXB : 9), 4>(a, pc, s); break;
    case 8: piece_body<T, TA, (MAXB < 4 ? MAXB : 4), 8>(a, pc, s); break;
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
  const dim3 g((np + 255) / 256), b(256);
  if (a.max_bp <= 4) hipLaunchKernelGGL((k_piece_phase<T, TA, 4>), g, b, 0, st, a);
  else if (a.max_bp <= 9) hipLaunchKernelGGL((k_piece_phase<T, TA, 9>), g, b, 0, st, a);
  else if (a.max_bp <= 16) hipLaunchKernelGGL((k_piece_phase<T, TA, 16>), g, b, 0, st, a);
  else hipLaunchKernelGGL((k_piece_phase<T, TA, 32>), g, b, 0, st, a);
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

int cell_variants(const StepArgs& a) { return (a.prec == SFROM_F64 || a.max_b > 256) ? 1 : 9; }

hipError_t launch_cell_phase(const StepArgs& a, hipStream_t st) {
  // variants 0..3: matrix-core kernel with one wave per row strip (source
  // tile 64/32, with/without strip prefetch); 4..7: streaming matrix-core
  // kernel (2 or 3 row tiles per wave, source tile 16/32); 8 (and FP64): the
  // scalar kernel
  if (a.prec == SFROM_F64 || a.max_b > 256 || a.cell_variant >= 8) {
    if (a.prec == SFROM_F64) return cell_impl<double, double, double>(a, st);
    if (a.prec == SFROM_F32) return cell_impl<float, float, float>(a, st);
    return cell_impl<float, __hip_bfloat16, float>(a, st);
  }
  if (a.prec == SFROM_F32) return mfma_dispatch<false>(a, a.cell_variant, st);
  return mfma_dispatch<true>(a, a.cell_variant, st);
}

hipError_t launch_piece_phase(const StepArgs& a, hipStream_t st) {
  if (a.prec == SFROM_F64) return piece_impl<double, double>(a, st);
  return piece_impl<float, float>(a, st);
}

hipError_t launch_receivers(const StepArgs& a, hipStream_t st) {
  if (a.prec == SFROM_F64) return rec_impl<double, double>(a, st);
  return rec_impl<float, float>(a, st);
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
