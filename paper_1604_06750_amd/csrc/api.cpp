// Host side of libsfrom: argument validation, partition bookkeeping, device
// memory, orchestration of the off-line build and of the on-line and
// fine-grid time loops. All arithmetic of the method runs in the HIP
// kernels; the host only validates, packs and launches.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sfrom_internal.h"

using namespace sfrom_impl;

// Receivers per piece up to which the piece phase computes the traces.
constexpr int MAX_FUSED_RECEIVERS = 8;

// Device memory of sfrom_run_noalloc, for callers that cannot allocate: the
// non-finite flag (first 256 bytes) and the Phi^1 exchange buffer of the
// on-line step. A file-scope array, so each GPU the library runs on holds
// one copy until the process ends; all calls on one GPU share it.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(256) << 20;
constexpr size_t NOALLOC_FLAG_BYTES = 256;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of `scratch` on each GPU (host code must not use the
// array's name, which is a host-side stand-in). Set once per device by
// sfrom_create with that device current.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

hipError_t init_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

struct Fail {
  int code;
};

// In-place lower Cholesky factor of a column-major n x n SPD matrix (upper
// triangle zeroed); false if a pivot is not positive.
bool host_cholesky(int n, double* A) {
  for (int j = 0; j < n; ++j) {
    double d = A[j + (int64_t)j * n];
    for (int k = 0; k < j; ++k) d -= A[j + (int64_t)k * n] * A[j + (int64_t)k * n];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    d = std::sqrt(d);
    A[j + (int64_t)j * n] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = A[i + (int64_t)j * n];
      for (int k = 0; k < j; ++k) v -= A[i + (int64_t)k * n] * A[j + (int64_t)k * n];
      A[i + (int64_t)j * n] = v / d;
    }
    for (int i = 0; i < j; ++i) A[i + (int64_t)j * n] = 0.0;
  }
  return true;
}

int set_err(sfrom_t* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess) {                                                             \
      h->err = std::string("HIP error in ") + #expr + ": " + hipGetErrorString(_e);     \
      throw Fail{_e == hipErrorOutOfMemory ? SFROM_ENOMEM : SFROM_EDEVICE};            \
    }                                                                                   \
  } while (0)

#define REQUIRE(cond, code, msg)          \
  do {                                    \
    if (!(cond)) {                        \
      h->err = (msg);                     \
      throw Fail{code};                   \
    }                                     \
  } while (0)

template <typename T>
void dfree(T*& p) {
  if (p) hipFree((void*)p);
  p = nullptr;
}

template <typename T>
T* dalloc(sfrom_t* h, size_t count) {
  if (count == 0) count = 1;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, count * sizeof(T));
  if (e != hipSuccess) {
    h->err = "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed: " + hipGetErrorString(e);
    throw Fail{SFROM_ENOMEM};
  }
  return reinterpret_cast<T*>(p);
}

template <typename T>
T* dupload(sfrom_t* h, const std::vector<T>& v) {
  T* p = dalloc<T>(h, v.size());
  if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}

size_t prec_bytes(int prec) { return prec == SFROM_F64 ? 8 : 4; }        // state / masses
size_t block_bytes(int prec) { return prec == SFROM_F64 ? 8 : (prec == SFROM_F32 ? 4 : 2); }

// Forgets the captured run: its kernels hold device pointers that the
// caller's next set-up may free.
void drop_graph(sfrom_t* h) {
  if (h->graph_exec) { hipGraphExecDestroy(h->graph_exec); h->graph_exec = nullptr; }
  h->graph_key.clear();
}

void free_corner_stage(sfrom_t* h) {
  auto& cs = h->cstage;
  dfree(cs.d_hptr); dfree(cs.d_hbp); dfree(cs.d_pptr); dfree(cs.d_plist); dfree(cs.d_pbp);
  dfree(cs.d_rowq); dfree(cs.d_rowj);
  dfree(cs.d_hdof); dfree(cs.d_soff); dfree(cs.d_pdof);
  dfree(cs.d_srow); dfree(cs.d_hw); dfree(cs.d_delta);
  cs.ready = false;
  cs.delta_ns = -1;
}

void free_rom(sfrom_t* h) {
  if (h->device < 0) { h->built = false; return; }
  drop_graph(h);
  dfree(h->d_blocks); dfree(h->d_minv); dfree(h->d_rom64); dfree(h->d_rom64_off);
  dfree(h->d_ocells); dfree(h->d_opieces); dfree(h->d_gather); dfree(h->d_inc);
  dfree(h->d_inc_cell); dfree(h->d_inc_col);
  dfree(h->d_src); dfree(h->d_rptr); dfree(h->d_rrow); dfree(h->d_rval);
  dfree(h->d_prec_ptr); dfree(h->d_prec_list);
  h->rec_fused = false;
  dfree(h->d_y[0]); dfree(h->d_y[1]); dfree(h->d_h[0]); dfree(h->d_h[1]); dfree(h->d_phi); dfree(h->d_flag);
  for (auto& bk : h->buckets) dfree(bk.d_list);
  h->buckets.clear();
  free_corner_stage(h);
  h->built = false;
  h->rom_imported = false;
  h->lam_rom = -1.0;
  h->state_ns = -1;
  h->steps_done = 0;
  h->src_dirty = h->rec_dirty = true;
}

void free_fine(sfrom_t* h) {
  dfree(h->d_stencil);
  dfree(h->d_frowptr); dfree(h->d_fcol); dfree(h->d_fa); dfree(h->d_fbinv);
  dfree(h->d_u[0]); dfree(h->d_u[1]);
  dfree(h->d_fsrc_row); dfree(h->d_fsrc_col); dfree(h->d_fsrc_val);
  dfree(h->d_fsrc_idx); dfree(h->d_fsrc_dense); h->fsrc_dense_prec = -1;
  dfree(h->d_frec_ptr); dfree(h->d_frec_row); dfree(h->d_frec_val);
  h->fine_prec = -1; h->fine_ns = -1; h->fine_io_dirty = true;
}

void free_stage(sfrom_t* h) {
  auto& st = h->stage;
  if (h->device >= 0) {
    dfree(st.d_rowptr); dfree(st.d_col); dfree(st.d_a); dfree(st.d_bdiag);
    dfree(st.d_wrow); dfree(st.d_wcol); dfree(st.d_wsoff); dfree(st.d_wbp); dfree(st.d_wkp); dfree(st.d_S);
  }
  st = sfrom::CellStage();
}

void free_all(sfrom_t* h) {
  if (h->device < 0) return;
  free_stage(h);
  if (h->capture_stream) { hipStreamDestroy(h->capture_stream); h->capture_stream = nullptr; }
  for (int k = 0; k < 4; ++k)
    for (auto& pr : h->ev_pending[k]) { h->ev_pool.push_back(pr.first); h->ev_pool.push_back(pr.second); }
  for (auto e : h->ev_pool) hipEventDestroy(e);
  h->ev_pool.clear();
  for (int k = 0; k < 4; ++k) h->ev_pending[k].clear();
  free_rom(h);
  free_fine(h);
  dfree(h->d_w);
  h->d_w_cap = 0;
}

// ---------------------------------------------------------------------------
// optional per-kernel event timing
// ---------------------------------------------------------------------------

hipEvent_t take_event(sfrom_t* h) {
  if (!h->ev_pool.empty()) {
    hipEvent_t e = h->ev_pool.back();
    h->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  return e;
}

// `sample` selects the steps whose launches are timed (one step in
// h->prof_every while profiling)
template <typename F>
void timed(sfrom_t* h, int kid, bool sample, F&& launch) {
  if (!h->profiling || !sample) {
    HIPCHK(launch());
    return;
  }
  hipEvent_t a = take_event(h), b = take_event(h);
  HIPCHK(hipEventRecord(a, h->stream));
  HIPCHK(launch());
  HIPCHK(hipEventRecord(b, h->stream));
  h->ev_pending[kid].push_back({a, b});
}

void collect_events(sfrom_t* h) {
  bool any = false;
  for (int k = 0; k < 4; ++k) any |= !h->ev_pending[k].empty();
  if (!any) return;
  HIPCHK(hipStreamSynchronize(h->stream));
  for (int k = 0; k < 4; ++k) {
    for (auto& pr : h->ev_pending[k]) {
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
      h->prof_ms[k] += ms;
      h->prof_n[k] += 1;
      h->ev_pool.push_back(pr.first);
      h->ev_pool.push_back(pr.second);
    }
    h->ev_pending[k].clear();
  }
}

// ---------------------------------------------------------------------------
// partition bookkeeping
// ---------------------------------------------------------------------------

void finalize_partition(sfrom_t* h) {
  if (h->part_ready) return;
  REQUIRE(h->n > 0, SFROM_ESTATE, "no pencil: call sfrom_set_pencil or sfrom_setup_voxel_acoustic first");
  const int nc = (int)h->cells.size(), np = (int)h->pieces.size();
  REQUIRE(nc >= 1, SFROM_ESTATE, "no cells defined");
  for (int i = 0; i < nc; ++i) REQUIRE(h->cells[i].defined, SFROM_ESTATE, "cell " + std::to_string(i) + " not defined");
  for (int p = 0; p < np; ++p) REQUIRE(h->pieces[p].defined, SFROM_ESTATE, "piece " + std::to_string(p) + " not defined");
  const int64_t n = h->n;
  std::vector<int32_t> cnt(n, 0);
  for (auto& c : h->cells)
    for (int64_t g : c.gnode) cnt[g]++;
  for (int64_t g = 0; g < n; ++g)
    REQUIRE(cnt[g] >= 1, SFROM_ESPLIT, "node " + std::to_string(g) + " belongs to no cell");
  h->piece_of_node.assign(n, -1);
  h->pos_in_piece.assign(n, -1);
  for (int p = 0; p < np; ++p) {
    const auto& pc = h->pieces[p];
    for (size_t k = 0; k < pc.gnode.size(); ++k) {
      const int64_t g = pc.gnode[k];
      REQUIRE(h->piece_of_node[g] < 0, SFROM_EINVAL, "node " + std::to_string(g) + " in two pieces");
      REQUIRE(cnt[g] >= 2, SFROM_EINVAL, "piece " + std::to_string(p) + " contains node " + std::to_string(g) + " that is not shared by two cells");
      h->piece_of_node[g] = p;
      h->pos_in_piece[g] = (int32_t)k;
    }
  }
  for (int64_t g = 0; g < n; ++g)
    REQUIRE(cnt[g] < 2 || h->piece_of_node[g] >= 0, SFROM_EINVAL, "skeleton node " + std::to_string(g) + " is in no piece");
  // incident cells of every piece: cells containing its nodes (all nodes must agree)
  std::vector<std::vector<int32_t>> node_cells_first(np);
  std::vector<int32_t> hits(np, 0);
  h->piece_cells.assign(np, {});
  for (int i = 0; i < nc; ++i) {
    std::map<int32_t, int32_t> count;
    for (int64_t g : h->cells[i].gnode) {
      const int32_t p = h->piece_of_node[g];
      if (p >= 0) count[p]++;
    }
    for (auto& kv : count) {
      REQUIRE(kv.second == (int32_t)h->pieces[kv.first].gnode.size(), SFROM_EINVAL,
              "cell " + std::to_string(i) + " holds only part of piece " + std::to_string(kv.first));
      h->piece_cells[kv.first].push_back(i);
    }
  }
  h->cell_pieces.assign(nc, {});
  h->cell_piece_col.assign(nc, {});
  h->cell_b.assign(nc, 0);
  for (int p = 0; p < np; ++p) {
    REQUIRE(h->piece_cells[p].size() >= 2, SFROM_EINVAL, "piece " + std::to_string(p) + " is not shared by two cells");
    for (int32_t c : h->piece_cells[p]) h->cell_pieces[c].push_back(p);
  }
  for (int i = 0; i < nc; ++i) {
    std::sort(h->cell_pieces[i].begin(), h->cell_pieces[i].end());
    int32_t col = 0;
    for (int32_t p : h->cell_pieces[i]) {
      h->cell_piece_col[i].push_back(col);
      col += h->pieces[p].b;
    }
    h->cell_b[i] = col;
    REQUIRE(col > 0, SFROM_EINVAL, "cell " + std::to_string(i) + " has no skeleton pieces");
  }
  h->piece_dof_off.assign(np + 1, 0);
  for (int p = 0; p < np; ++p) h->piece_dof_off[p + 1] = h->piece_dof_off[p] + h->pieces[p].b;
  // splitting check (eq. splitN_c): sum_i P_i A_i P_i^T = A, sum_i P_i B_i P_i^T = B
  std::vector<double> asum(h->a.size(), 0.0), bsum(n, 0.0);
  double amax = 0.0, bmax = 0.0;
  for (double v : h->a) amax = std::max(amax, std::fabs(v));
  for (double v : h->b) bmax = std::max(bmax, std::fabs(v));
  for (int i = 0; i < nc; ++i) {
    const auto& c = h->cells[i];
    for (int r = 0; r < c.n; ++r) {
      const int64_t gr = c.gnode[r];
      bsum[gr] += c.b[r];
      const int32_t* cb = h->col.data() + h->rowptr[gr];
      const int32_t* ce = h->col.data() + h->rowptr[gr + 1];
      for (int k = c.rowptr[r]; k < c.rowptr[r + 1]; ++k) {
        const int64_t gc = c.gnode[c.col[k]];
        const int32_t* it = std::lower_bound(cb, ce, (int32_t)gc);
        if (it == ce || *it != gc) {
          REQUIRE(c.a[k] == 0.0, SFROM_ESPLIT, "cell " + std::to_string(i) + " has an entry outside the pattern of A");
          continue;
        }
        asum[it - h->col.data()] += c.a[k];
      }
    }
  }
  for (size_t k = 0; k < asum.size(); ++k)
    REQUIRE(std::fabs(asum[k] - h->a[k]) <= 1e-12 * amax, SFROM_ESPLIT, "sum of cell operators differs from A at entry " + std::to_string(k));
  for (int64_t g = 0; g < n; ++g)
    REQUIRE(std::fabs(bsum[g] - h->b[g]) <= 1e-12 * bmax, SFROM_ESPLIT, "sum of cell masses differs from B at node " + std::to_string(g));
  // Gershgorin bound of each cell's pencil: every eigenvalue of
  // B_i^{-1}(-A_i) lies in a disc around a diagonal entry of radius the
  // row's off-diagonal absolute sum
  double lam = 0.0;
  for (const auto& c : h->cells)
    for (int r = 0; r < c.n; ++r) {
      double s = 0.0;
      for (int k = c.rowptr[r]; k < c.rowptr[r + 1]; ++k) s += std::fabs(c.a[k]);
      lam = std::max(lam, s / c.b[r]);
    }
  h->lam_cells = lam;
  h->part_ready = true;
}

// restriction of sparse columns to the skeleton pieces (Sec. 6: reduced
// inputs g_ij = S_ij^T g restricted to Gamma_ij)
void make_columns(sfrom_t* h, Columns& out, int32_t count, const int64_t* colptr, const int64_t* row,
                  const double* val, int project) {
  Columns c;
  c.count = count;
  c.colptr.push_back(0);
  c.rptr.push_back(0);
  for (int j = 0; j < count; ++j) {
    std::map<int32_t, std::vector<double>> coef;   // piece -> S_p^T g
    for (int64_t k = colptr[j]; k < colptr[j + 1]; ++k) {
      const int64_t g = row[k];
      REQUIRE(g >= 0 && g < h->n, SFROM_EINVAL, "column row index out of range");
      REQUIRE(std::isfinite(val[k]), SFROM_ENONFINITE, "non-finite column value");
      if (val[k] == 0.0) continue;
      const int32_t p = h->piece_of_node[g];
      REQUIRE(p >= 0, SFROM_ESUPPORT, "column " + std::to_string(j) + " has a nonzero at node " + std::to_string(g) + " off the skeleton (eq. gsupport)");
      const auto& pc = h->pieces[p];
      auto& cv = coef[p];
      if (cv.empty()) cv.assign(pc.b, 0.0);
      const int32_t pos = h->pos_in_piece[g];
      const int64_t kp = (int64_t)pc.gnode.size();
      for (int l = 0; l < pc.b; ++l) cv[l] += pc.S[pos + l * kp] * val[k];
    }
    if (project) {
      std::vector<std::pair<int64_t, double>> ent;
      for (auto& kv : coef) {
        const auto& pc = h->pieces[kv.first];
        const int64_t kp = (int64_t)pc.gnode.size();
        for (int64_t r = 0; r < kp; ++r) {
          double s = 0.0;
          for (int l = 0; l < pc.b; ++l) s += pc.S[r + l * kp] * kv.second[l];
          if (s != 0.0) ent.push_back({pc.gnode[r], s});
        }
      }
      std::sort(ent.begin(), ent.end());
      for (auto& e : ent) { c.row.push_back(e.first); c.val.push_back(e.second); }
    } else {
      for (int64_t k = colptr[j]; k < colptr[j + 1]; ++k) {
        if (val[k] == 0.0) continue;
        c.row.push_back(row[k]);
        c.val.push_back(val[k]);
      }
    }
    c.colptr.push_back((int64_t)c.row.size());
    for (auto& kv : coef) {
      c.rpiece.push_back(kv.first);
      c.rcoff.push_back((int64_t)c.rcoef.size());
      c.rcoef.insert(c.rcoef.end(), kv.second.begin(), kv.second.end());
    }
    c.rptr.push_back((int64_t)c.rpiece.size());
  }
  out = std::move(c);
}

// ---------------------------------------------------------------------------
// off-line build
// ---------------------------------------------------------------------------

// Host-side state of one build: per-cell workspace layout and limits.
struct BuildCtx {
  std::vector<BuildCell> bcells;   // workspace offsets relative to the cell's own slice
  std::vector<int64_t> wsize;      // doubles of workspace per cell
  int max_m = 0, max_b = 0, max_n = 0;
};

// Uploads the build's inputs (cell operators A_i and B_i, the skeleton rows
// of each W_i = P_i^T P^Gamma S and the piece bases S_p) once per partition.
void stage_cells(sfrom_t* h) {
  auto& st = h->stage;
  if (st.ready) return;
  free_stage(h);
  const int nc = (int)h->cells.size(), np = (int)h->pieces.size();
  st.soff.resize(np);
  int64_t ns = 0;
  for (int p = 0; p < np; ++p) { st.soff[p] = ns; ns += (int64_t)h->pieces[p].S.size(); }
  std::vector<double> S((size_t)ns);
  for (int p = 0; p < np; ++p) std::copy(h->pieces[p].S.begin(), h->pieces[p].S.end(), S.begin() + st.soff[p]);
  int64_t nrp = 0, nnz = 0, nb = 0, nwr = 0;
  st.rp_off.resize(nc); st.csr_off.resize(nc); st.b_off.resize(nc); st.w_off.resize(nc);
  st.nw.assign(nc, 0); st.bw.assign(nc, 0);
  for (int i = 0; i < nc; ++i) {
    const CellDef& c = h->cells[i];
    st.rp_off[i] = nrp; st.csr_off[i] = nnz; st.b_off[i] = nb; st.w_off[i] = nwr;
    nrp += c.n + 1; nnz += (int64_t)c.col.size(); nb += c.n;
    int nw = 0, w = 0;
    for (int r = 0; r < c.n; ++r) {
      if (h->piece_of_node[c.gnode[r]] >= 0) ++nw;
      for (int k = c.rowptr[r]; k < c.rowptr[r + 1]; ++k) w = std::max(w, std::abs(r - c.col[k]));
    }
    st.nw[i] = nw; st.bw[i] = w;
    nwr += nw;
  }
  std::vector<int32_t> rowptr((size_t)nrp), col((size_t)nnz), wrow((size_t)nwr), wcol((size_t)nwr), wbp((size_t)nwr),
      wkp((size_t)nwr);
  std::vector<double> av((size_t)nnz), bd((size_t)nb);
  std::vector<int64_t> wsoff((size_t)nwr);
  std::vector<int32_t> pcol(np, -1);
  for (int i = 0; i < nc; ++i) {
    const CellDef& c = h->cells[i];
    std::copy(c.rowptr.begin(), c.rowptr.end(), rowptr.begin() + st.rp_off[i]);
    std::copy(c.col.begin(), c.col.end(), col.begin() + st.csr_off[i]);
    std::copy(c.a.begin(), c.a.end(), av.begin() + st.csr_off[i]);
    std::copy(c.b.begin(), c.b.end(), bd.begin() + st.b_off[i]);
    for (size_t q = 0; q < h->cell_pieces[i].size(); ++q) pcol[h->cell_pieces[i][q]] = h->cell_piece_col[i][q];
    int64_t t = st.w_off[i];
    for (int r = 0; r < c.n; ++r) {
      const int32_t p = h->piece_of_node[c.gnode[r]];
      if (p < 0) continue;
      wrow[t] = r;
      wcol[t] = pcol[p];
      wsoff[t] = st.soff[p] + h->pos_in_piece[c.gnode[r]];
      wbp[t] = h->pieces[p].b;
      wkp[t] = (int32_t)h->pieces[p].gnode.size();
      ++t;
    }
    for (int32_t p : h->cell_pieces[i]) pcol[p] = -1;
  }
  st.d_rowptr = dupload(h, rowptr); st.d_col = dupload(h, col); st.d_a = dupload(h, av); st.d_bdiag = dupload(h, bd);
  st.d_wrow = dupload(h, wrow); st.d_wcol = dupload(h, wcol); st.d_wsoff = dupload(h, wsoff);
  st.d_wbp = dupload(h, wbp); st.d_wkp = dupload(h, wkp); st.d_S = dupload(h, S);
  st.ready = true;
}

void build_layout(sfrom_t* h, const sfrom_build_opts* o, BuildCtx& ctx) {
  REQUIRE(o != nullptr, SFROM_EINVAL, "null build options");
  REQUIRE(h->device >= 0, SFROM_EDEVICE, "host-only handle: no device for the build");
  finalize_partition(h);
  const int nc = (int)h->cells.size(), np = (int)h->pieces.size();
  REQUIRE(o->shift < 0.0 && std::isfinite(o->shift), SFROM_EINVAL, "shift must be negative (Sec. 4.2)");
  REQUIRE(o->online_prec >= SFROM_F64 && o->online_prec <= SFROM_BF16, SFROM_EINVAL, "bad on-line precision");
  free_rom(h);
  h->prec = o->online_prec;
  h->shift = o->shift;
  h->cell_m.assign(nc, o->m);
  if (o->m_per_cell)
    for (int i = 0; i < nc; ++i) h->cell_m[i] = o->m_per_cell[i];
  for (int p = 0; p < np; ++p)
    REQUIRE(h->pieces[p].b <= 32, SFROM_EINVAL, "piece " + std::to_string(p) + ": at most 32 basis vectors per piece");
  int max_m = 0, max_b = 0, max_n = 0;
  for (int i = 0; i < nc; ++i) {
    REQUIRE(h->cell_m[i] >= 1, SFROM_EINVAL, "m must be >= 1");
    REQUIRE((int64_t)h->cell_m[i] * h->cell_b[i] <= h->cells[i].n, SFROM_EBREAKDOWN,
            "cell " + std::to_string(i) + ": m b_i exceeds the cell size (Assumption 1)");
    max_m = std::max(max_m, h->cell_m[i]);
    max_b = std::max(max_b, h->cell_b[i]);
    max_n = std::max(max_n, h->cells[i].n);
  }
  // ---- on-line layout -------------------------------------------------------
  h->ocells.resize(nc);
  std::vector<int32_t> gather;
  int64_t blk = 0, hid = 0, hdofs = 0, u1 = 0, r64 = 0;
  h->rom64_off.resize(nc);
  for (int i = 0; i < nc; ++i) {
    OnlineCell& oc = h->ocells[i];
    oc.m = h->cell_m[i];
    oc.b = h->cell_b[i];
    oc.ld = (oc.b + 3) / 4 * 4;
    oc.pad_ = 0;
    oc.blk_off = blk;
    oc.hid_off = hid;
    oc.u1_off = u1;
    blk += (int64_t)(2 * oc.m - 1) * oc.b * oc.ld;
    hid += (int64_t)(oc.m - 1) * oc.ld;
    hdofs += (int64_t)(oc.m - 1) * oc.b;
    u1 += oc.b;
    h->rom64_off[i] = r64;
    r64 += (int64_t)2 * oc.m * oc.b * oc.b;
    for (size_t q = 0; q < h->cell_pieces[i].size(); ++q) {
      const int32_t p = h->cell_pieces[i][q];
      for (int l = 0; l < h->pieces[p].b; ++l) gather.push_back((int32_t)(h->piece_dof_off[p] + l));
    }
  }
  h->n_hidden_dofs = hdofs;
  h->n_hidden_rows = hid;
  h->block_elems = blk;
  h->opieces.resize(np);
  std::vector<int64_t> inc;
  std::vector<int32_t> inc_cell, inc_col;
  int64_t moff = 0;
  for (int p = 0; p < np; ++p) {
    OnlinePiece& op = h->opieces[p];
    op.b = h->pieces[p].b;
    op.ncell = (int32_t)h->piece_cells[p].size();
    op.dof_off = h->piece_dof_off[p];
    op.inc_off = (int64_t)inc.size();
    op.minv_off = moff;
    op.src_off = -1;
    moff += (int64_t)op.b * op.b;
    for (int32_t c : h->piece_cells[p]) {
      const auto& cp = h->cell_pieces[c];
      const size_t q = std::lower_bound(cp.begin(), cp.end(), p) - cp.begin();
      inc.push_back(h->ocells[c].u1_off + h->cell_piece_col[c][q]);
      inc_cell.push_back(c);
      inc_col.push_back(h->cell_piece_col[c][q]);
    }
  }
  h->d_ocells = dupload(h, h->ocells);
  h->d_opieces = dupload(h, h->opieces);
  h->d_gather = dupload(h, gather);
  h->d_inc = dupload(h, inc);
  h->d_inc_cell = dupload(h, inc_cell);
  h->d_inc_col = dupload(h, inc_col);
  h->d_blocks = dalloc<unsigned char>(h, (size_t)blk * block_bytes(h->prec));
  h->d_minv = dalloc<unsigned char>(h, (size_t)moff * prec_bytes(h->prec));
  h->d_rom64 = dalloc<double>(h, (size_t)r64);
  h->d_rom64_off = dupload(h, h->rom64_off);
  stage_cells(h);
  // ---- per-cell workspace sizes -----------------------------------------------
  std::vector<BuildCell>& bcells = ctx.bcells;
  std::vector<int64_t>& wsize = ctx.wsize;
  // the blocked build (any cell wider than WIDE_MIN_W, or forced) needs a
  // region for partial Gram products in every cell of a batch
  int max_w = 0;
  for (int i = 0; i < nc; ++i) max_w = std::max(max_w, h->stage.bw[i]);
  const bool any_wide = h->wide_mode == 1 || (h->wide_mode == 0 && max_w > WIDE_MIN_W);
  bcells.assign(nc, BuildCell{});
  wsize.assign(nc, 0);
  for (int i = 0; i < nc; ++i) {
    const CellDef& c = h->cells[i];
    BuildCell& bc = bcells[i];
    bc.n = c.n; bc.b = h->cell_b[i]; bc.m = h->cell_m[i]; bc.nnz = (int32_t)c.a.size();
    const int w = h->stage.bw[i];
    bc.w = w;
    const int64_t n = c.n, b = bc.b, mb = (int64_t)bc.m * b;
    int64_t off = 0;
    bc.band_off = off; off += n * (w + 1);
    bc.v_off = off; off += n * mb;
    bc.x_off = off; off += n * b;
    bc.av_off = off; off += std::max({n * mb, 3 * mb * b + 2 * b * b, 8 * b * b + b, n * b});
    bc.am_off = off; off += mb * mb;
    bc.q_off = off; off += mb * mb;
    bc.s_off = off; off += std::max(2 * mb * b, mb * b);
    bc.r_off = off; off += mb * b;
    bc.out_off = off; off += 2 * mb * b;
    bc.p_off = off;
    if (any_wide) off += ts_partials(n, bc.m, b);
    bc.li_off = off;
    if (any_wide) off += (n + 63) / 64 * 64 * 64;
    bc.status = 0;
    wsize[i] = off;
  }
  ctx.max_m = max_m; ctx.max_b = max_b; ctx.max_n = max_n;
  // cell-phase buckets: cells grouped by the strip count of the matrix-core
  // kernel instantiation they need (4, 6, 7, 8, 9, 10, 12, 16 strips)
  auto inst = [](int b) {
    const int q = (b + 15) / 16;
    return q <= 4 ? 4 : q <= 6 ? 6 : q <= 10 ? q : q <= 12 ? 12 : 16;
  };
  std::map<int, std::vector<int32_t>> groups;
  for (int i = 0; i < nc; ++i) groups[inst(h->cell_b[i])].push_back(i);
  for (auto& kv : groups) {
    sfrom::CellBucket bk;
    bk.count = (int32_t)kv.second.size();
    for (int32_t i : kv.second) {
      bk.max_b = std::max(bk.max_b, h->cell_b[i]);
      bk.max_m = std::max(bk.max_m, h->cell_m[i]);
    }
    bk.d_list = dupload(h, kv.second);
    h->buckets.push_back(bk);
  }
}

// Runs `body` on batches of the listed cells: uploads each batch's cell
// operators, skeleton maps and workspace descriptors, so that body(bb, ids)
// can launch per-cell kernels (blockIdx.x = position in `ids`).
template <class F>
void for_batches(sfrom_t* h, const sfrom_build_opts* o, BuildCtx& ctx, const std::vector<int32_t>& list, F&& body) {
  if (list.empty()) return;
  // workspace budget: up to 128 GiB (HBM holds 288 GB; large cells need
  // about 0.6 GB each, and fewer batches mean fewer, fuller launches), at
  // most half of the memory that is free now
  size_t free_b = 0, total_b = 0;
  HIPCHK(hipMemGetInfo(&free_b, &total_b));
  const int64_t budget = std::max<int64_t>((int64_t)1 << 30, std::min<int64_t>((int64_t)128 << 30, (int64_t)(free_b / 2)));
  int64_t wmax = 0;
  for (int32_t i : list) wmax = std::max(wmax, ctx.wsize[i]);
  int per_batch = o->cells_per_batch > 0 ? o->cells_per_batch : (int)list.size();
  per_batch = (int)std::max<int64_t>(1, std::min<int64_t>(per_batch, budget / (wmax * 8)));
  double* d_work = dalloc<double>(h, (size_t)(wmax * per_batch));
  BuildCell* d_bc = dalloc<BuildCell>(h, per_batch);
  try {
    for (size_t c0 = 0; c0 < list.size(); c0 += per_batch) {
      const int cnt = (int)std::min<size_t>(per_batch, list.size() - c0);
      std::vector<int32_t> ids(list.begin() + c0, list.begin() + c0 + cnt);
      const auto& st = h->stage;
      std::vector<BuildCell> bcb(cnt);
      int64_t woff = 0;
      for (int t = 0; t < cnt; ++t) {
        const int i = ids[t];
        BuildCell& bc = bcb[t];
        bc = ctx.bcells[i];
        bc.rp_off = st.rp_off[i];
        bc.csr_off = st.csr_off[i];
        bc.b_off = st.b_off[i];
        bc.w_off = st.w_off[i];
        bc.nw = st.nw[i];
        // rebase workspace offsets into this batch's work array
        const int64_t base = woff;
        bc.band_off += base; bc.v_off += base; bc.x_off += base; bc.av_off += base;
        bc.am_off += base; bc.q_off += base; bc.s_off += base; bc.r_off += base; bc.out_off += base;
        bc.p_off += base; bc.li_off += base;
        woff += ctx.wsize[i];
      }
      HIPCHK(hipMemcpy(d_bc, bcb.data(), cnt * sizeof(BuildCell), hipMemcpyHostToDevice));
      BuildBatch bb;
      bb.ncell = cnt;
      bb.max_m = ctx.max_m; bb.max_b = ctx.max_b; bb.max_n = ctx.max_n;
      bb.max_w = 0;
      for (const BuildCell& x : bcb) bb.max_w = std::max(bb.max_w, x.w);
      bb.shift = o->shift;
      bb.wide_mode = h->wide_mode;
      bb.d_cells = d_bc;
      bb.d_rowptr = st.d_rowptr; bb.d_col = st.d_col; bb.d_a = st.d_a; bb.d_bdiag = st.d_bdiag;
      bb.d_wrow = st.d_wrow; bb.d_wcol = st.d_wcol; bb.d_wsoff = st.d_wsoff; bb.d_wbp = st.d_wbp; bb.d_wkp = st.d_wkp;
      bb.d_S = st.d_S;
      bb.d_work = d_work;
      body(bb, ids);
    }
  } catch (...) {
    dfree(d_work); dfree(d_bc);
    throw;
  }
  dfree(d_work); dfree(d_bc);
}

// Status of the batch's cells after the build kernels; throws the first
// failure (freeing the partial ROM).
void check_batch_status(sfrom_t* h, const BuildBatch& bb, const std::vector<int32_t>& ids) {
  std::vector<BuildCell> bcb(ids.size());
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipMemcpy(bcb.data(), bb.d_cells, ids.size() * sizeof(BuildCell), hipMemcpyDeviceToHost));
  h->breakdowns.clear();
  for (size_t t = 0; t < ids.size(); ++t)
    if (bcb[t].status == 2) h->breakdowns.push_back({ids[t], bcb[t].fail_block});
  for (size_t t = 0; t < ids.size(); ++t) {
    const int st = bcb[t].status;
    if (st == 0) continue;
    const std::string cell = "cell " + std::to_string(ids[t]) + ": ";
    free_rom(h);
    if (st == 1) { h->err = cell + "-(A_i + s B_i) is not positive definite (A_i not <= 0)"; throw Fail{SFROM_ENOTNSD}; }
    if (st == 2) {
      h->err = cell + "Krylov/Lanczos block " + std::to_string(bcb[t].fail_block) + " lost rank (Assumption 1)";
      throw Fail{SFROM_EBREAKDOWN};
    }
    if (st == 3) { h->err = cell + "S-fraction pivot not SPD (Assumption 2)"; throw Fail{SFROM_ENOTSPD}; }
    h->err = cell + "non-finite S-fraction"; throw Fail{SFROM_ENONFINITE};
  }
}

// Plain block-Lanczos build (Alg. alg1red stage 1) of the listed cells.
void build_lanczos(sfrom_t* h, const sfrom_build_opts* o, BuildCtx& ctx, const std::vector<int32_t>& list) {
  for_batches(h, o, ctx, list, [&](BuildBatch& bb, const std::vector<int32_t>& ids) {
    std::vector<OnlineCell> ocb(ids.size());
    std::vector<int64_t> r64b(ids.size());
    for (size_t t = 0; t < ids.size(); ++t) { ocb[t] = h->ocells[ids[t]]; r64b[t] = h->rom64_off[ids[t]]; }
    OnlineCell* d_ocb = dupload(h, ocb);
    int64_t* d_r64b = dupload(h, r64b);
    HIPCHK(launch_build(bb, h->stream));
    HIPCHK(launch_pack((int32_t)ids.size(), bb.d_cells, bb.d_work, d_ocb, h->prec, h->d_blocks, h->d_rom64, d_r64b,
                       h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    dfree(d_ocb); dfree(d_r64b);
    check_batch_status(h, bb, ids);
  });
}

// Build with the learned stage for the candidate cells (see sfrom.h).
void build_learned(sfrom_t* h, const sfrom_build_opts* o, sfrom_surrogate* sur, int n, const int32_t* cells,
                   const float* x, double omega_max, double tol, int32_t* accepted, double* mismatch) {
  auto t0 = std::chrono::steady_clock::now();
  REQUIRE(sur != nullptr && n >= 0 && (n == 0 || (cells && x && accepted)), SFROM_EINVAL, "bad learned-build arguments");
  REQUIRE(omega_max > 0.0 && std::isfinite(omega_max) && tol > 0.0, SFROM_EINVAL, "omega_max and tol must be positive");
  BuildCtx ctx;
  build_layout(h, o, ctx);
  const int nc = (int)h->cells.size();
  const int P = surrogate_outputs(sur);
  std::vector<char> is_cand(nc, 0);
  std::vector<int32_t> cand(cells, cells + n);
  int b0 = -1, m0 = -1;
  for (int32_t id : cand) {
    REQUIRE(id >= 0 && id < nc && !is_cand[id], SFROM_EINVAL, "bad or repeated candidate cell");
    is_cand[id] = 1;
    if (b0 < 0) { b0 = h->cell_b[id]; m0 = h->cell_m[id]; }
    REQUIRE(h->cell_b[id] == b0 && h->cell_m[id] == m0, SFROM_EINVAL, "candidate cells must share b and m");
  }
  if (n > 0) {
    REQUIRE(m0 >= 2 && (int64_t)(m0 - 1) * b0 * (b0 + 1) == P, SFROM_EINVAL,
            "network outputs do not match the candidates' (m, b)");
  }
  std::vector<double> z(16);
  for (int j = 0; j < 16; ++j) {
    const double sg = (j + 0.5) * omega_max / 16.0;
    z[j] = -sg * sg;
  }
  std::vector<double> mis(n, 0.0);
  std::vector<int32_t> acc(n, 0);
  float* d_y = nullptr;
  try {
    if (n > 0) {
      d_y = dalloc<float>(h, (size_t)n * P);
      HIPCHK(hipStreamSynchronize(h->stream));
      HIPCHK(surrogate_predict(sur, x, n, d_y));
      HIPCHK(hipDeviceSynchronize());
    }
    size_t done = 0;
    for_batches(h, o, ctx, cand, [&](BuildBatch& bb, const std::vector<int32_t>& ids) {
      const size_t pos0 = done;
      done += ids.size();
      double* d_mis = dalloc<double>(h, ids.size());
      HIPCHK(hipMemsetAsync(d_mis, 0, ids.size() * sizeof(double), h->stream));
      HIPCHK(launch_learned_check(bb, d_y + pos0 * P, P, z.data(), 16, d_mis, h->stream));
      std::vector<double> mb(ids.size());
      std::vector<BuildCell> bcb(ids.size());
      HIPCHK(hipMemcpyAsync(mb.data(), d_mis, ids.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(hipMemcpyAsync(bcb.data(), bb.d_cells, ids.size() * sizeof(BuildCell), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      std::vector<int32_t> take(ids.size());
      std::vector<OnlineCell> ocb(ids.size());
      std::vector<int64_t> r64b(ids.size());
      for (size_t t = 0; t < ids.size(); ++t) {
        const bool ok = bcb[t].status == 0 && mb[t] <= tol;
        take[t] = ok ? 1 : 0;
        mis[pos0 + t] = bcb[t].status == 0 ? mb[t] : 1e300;
        acc[pos0 + t] = take[t];
        ocb[t] = h->ocells[ids[t]];
        r64b[t] = h->rom64_off[ids[t]];
      }
      int32_t* d_take = dupload(h, take);
      OnlineCell* d_ocb = dupload(h, ocb);
      int64_t* d_r64b = dupload(h, r64b);
      HIPCHK(launch_pack_normal((int32_t)ids.size(), bb.d_cells, bb.d_work, d_ocb, d_take, h->prec, h->d_blocks,
                                h->d_rom64, d_r64b, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      dfree(d_take); dfree(d_ocb); dfree(d_r64b); dfree(d_mis);
    });
    std::vector<int32_t> rest;
    for (int i = 0; i < nc; ++i)
      if (!is_cand[i]) rest.push_back(i);
    for (int t = 0; t < n; ++t)
      if (!acc[t]) rest.push_back(cand[t]);
    std::sort(rest.begin(), rest.end());
    build_lanczos(h, o, ctx, rest);
  } catch (...) {
    dfree(d_y);
    throw;
  }
  dfree(d_y);
  for (int t = 0; t < n; ++t) {
    accepted[t] = acc[t];
    if (mismatch) mismatch[t] = mis[t];
  }
  h->built = true;
  h->masses_dirty = true;
  h->src_dirty = h->rec_dirty = true;
  auto t1 = std::chrono::steady_clock::now();
  h->build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
}

// Factor-vector targets of built cells (see sfrom.h).
void factor_targets(sfrom_t* h, int n, const int32_t* cells, float* t) {
  REQUIRE(h->built, SFROM_ESTATE, "no ROM: build first");
  REQUIRE(n > 0 && cells && t, SFROM_EINVAL, "bad target arguments");
  const int nc = (int)h->ocells.size();
  int b0 = -1, m0 = -1;
  for (int k = 0; k < n; ++k) {
    REQUIRE(cells[k] >= 0 && cells[k] < nc, SFROM_EINVAL, "bad cell id");
    const OnlineCell& oc = h->ocells[cells[k]];
    if (b0 < 0) { b0 = oc.b; m0 = oc.m; }
    REQUIRE(oc.b == b0 && oc.m == m0, SFROM_EINVAL, "cells must share b and m");
  }
  REQUIRE(m0 >= 2, SFROM_EINVAL, "targets need m >= 2");
  const int P = (m0 - 1) * b0 * (b0 + 1);
  std::vector<int32_t> ids(cells, cells + n);
  int32_t* d_ids = dupload(h, ids);
  double* d_scr = dalloc<double>(h, (size_t)n * b0 * b0);
  std::vector<int32_t> bad(n, 0);
  int32_t* d_bad = dupload(h, bad);
  const hipError_t e = launch_factor_targets(h->d_rom64, h->d_rom64_off, d_ids, n, b0, m0, d_scr, t, P, d_bad,
                                             h->stream);
  if (e == hipSuccess) hipMemcpyAsync(bad.data(), d_bad, n * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream);
  hipStreamSynchronize(h->stream);
  dfree(d_ids); dfree(d_scr); dfree(d_bad);
  HIPCHK(e);
  for (int k = 0; k < n; ++k)
    REQUIRE(!bad[k], SFROM_ENOTSPD, "cell " + std::to_string(cells[k]) + ": a deep block is not positive definite");
}

void build(sfrom_t* h, const sfrom_build_opts* o) {
  auto t0 = std::chrono::steady_clock::now();
  REQUIRE(o != nullptr, SFROM_EINVAL, "null build options");
  const int nc = (int)h->cells.size();
  std::vector<int32_t> m_cell(nc, o->m);
  if (o->m_per_cell) std::copy(o->m_per_cell, o->m_per_cell + nc, m_cell.begin());
  sfrom_build_opts oo = *o;
  oo.m_per_cell = m_cell.data();
  std::vector<int32_t> all(nc);
  for (int i = 0; i < nc; ++i) all[i] = i;
  for (;;) {
    BuildCtx ctx;
    try {
      build_layout(h, &oo, ctx);
      build_lanczos(h, &oo, ctx, all);
      break;
    } catch (const Fail& f) {
      // with the policy on, cells whose block k >= 2 lost rank drop to
      // m_i = k - 1 and the build starts again (each retry lowers some m_i)
      if (f.code != SFROM_EBREAKDOWN || !h->reduce_m_on_breakdown || h->breakdowns.empty()) throw;
      for (const auto& bd : h->breakdowns) {
        const int cell = bd.first, k = bd.second;
        if (k < 2 || k - 1 >= m_cell[cell]) throw;
        m_cell[cell] = k - 1;
      }
      h->breakdowns.clear();
    }
  }
  h->built = true;
  h->masses_dirty = true;
  h->src_dirty = h->rec_dirty = true;
  auto t1 = std::chrono::steady_clock::now();
  h->build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
}

void update_masses(sfrom_t* h) {
  if (!h->masses_dirty) return;
  const int np = (int)h->pieces.size();
  int64_t moff = 0;
  for (auto& op : h->opieces) moff += (int64_t)op.b * op.b;
  int32_t* d_st = dalloc<int32_t>(h, np);
  double* d_scr = dalloc<double>(h, (size_t)3 * moff);
  MassArgs ma;
  ma.npiece = np;
  ma.d_pieces = h->d_opieces;
  ma.d_inc_cell = h->d_inc_cell;
  ma.d_inc_col = h->d_inc_col;
  ma.d_cells = h->d_ocells;
  ma.d_rom64 = h->d_rom64;
  ma.d_rom64_off = h->d_rom64_off;
  ma.prec = h->prec;
  ma.d_minv = h->d_minv;
  ma.d_status = d_st;
  ma.d_scratch = d_scr;
  HIPCHK(launch_piece_mass(ma, h->stream));
  std::vector<int32_t> st(np);
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipMemcpy(st.data(), d_st, np * sizeof(int32_t), hipMemcpyDeviceToHost));
  dfree(d_st); dfree(d_scr);
  for (int p = 0; p < np; ++p)
    REQUIRE(st[p] == 0, SFROM_ENOTSPD, "piece " + std::to_string(p) + ": singular interface mass");
  h->masses_dirty = false;
}

// Bytes of one level of the piece state and of the hidden state for the
// current state width.
size_t ystate_bytes(const sfrom_t* h, int ns) { return (size_t)h->piece_dof_off.back() * ns * prec_bytes(h->prec); }
size_t hstate_bytes(const sfrom_t* h, int ns) {
  return (size_t)std::max<int64_t>(h->n_hidden_rows, 1) * ns * prec_bytes(h->prec);
}

// Zeroes both levels of the ROM state (eq. initial: u = 0 for t <= 0).
void zero_state(sfrom_t* h) {
  h->steps_done = 0;
  h->cur = 0;
  if (h->state_ns < 0) return;
  for (int k = 0; k < 2; ++k) {
    HIPCHK(hipMemsetAsync(h->d_y[k], 0, ystate_bytes(h, h->state_ns), h->stream));
    HIPCHK(hipMemsetAsync(h->d_h[k], 0, hstate_bytes(h, h->state_ns), h->stream));
  }
}

// (Re)allocates the ROM state and the Phi^1 exchange buffer for n_s sources
// and zeroes the state. A captured run refers to the old buffers, so it is
// dropped first.
void alloc_state(sfrom_t* h, int ns) {
  drop_graph(h);
  int64_t nu1 = 0;
  for (auto& oc : h->ocells) nu1 += oc.b;
  for (int k = 0; k < 2; ++k) {
    dfree(h->d_y[k]); dfree(h->d_h[k]);
    h->d_y[k] = dalloc<unsigned char>(h, ystate_bytes(h, ns));
    h->d_h[k] = dalloc<unsigned char>(h, hstate_bytes(h, ns));
  }
  dfree(h->d_phi);
  h->d_phi = dalloc<unsigned char>(h, (size_t)nu1 * ns * prec_bytes(h->prec));
  h->state_ns = ns;
  zero_state(h);
}

// ROM-side device inputs/outputs and state for n_s sources
// Device arrays of the App. D correction from the corner map and the built
// ROM's piece bases: per copy its piece's dof rows and its basis row, per
// piece holding copies the list of its copies.
void stage_corners(sfrom_t* h) {
  auto& cs = h->cstage;
  const auto& cm = h->cmap;
  REQUIRE(!cm.corner.empty(), SFROM_ESTATE, "no corner set was removed: call sfrom_remove_corner_set");
  const int64_t nc = (int64_t)cm.hnode.size();
  REQUIRE(nc < ((int64_t)1 << 31), SFROM_EINVAL, "too many hanging nodes");
  std::vector<int32_t> hptr(cm.hptr.begin(), cm.hptr.end()), hbp(nc);
  std::vector<int64_t> hdof(nc), soff(nc);
  std::vector<double> srow, hw(nc);
  std::vector<std::vector<int32_t>> by_piece(h->pieces.size());
  for (int64_t t = 0; t < nc; ++t) {
    const int64_t l = cm.hnode[t];
    REQUIRE(l >= 0 && l < h->n, SFROM_ESTATE, "corner map does not match the pencil");
    const int32_t p = h->piece_of_node[l];
    REQUIRE(p >= 0, SFROM_ESTATE, "a hanging node lies in no piece");
    const sfrom_impl::PieceDef& pd = h->pieces[p];
    const int64_t kp = (int64_t)pd.gnode.size();
    const int64_t r = h->pos_in_piece[l];
    hdof[t] = h->piece_dof_off[p];
    hbp[t] = pd.b;
    soff[t] = (int64_t)srow.size();
    for (int j = 0; j < pd.b; ++j) srow.push_back(pd.S[r + j * kp]);
    hw[t] = cm.hweight[t];
    by_piece[p].push_back((int32_t)t);
  }
  std::vector<int32_t> pptr{0}, plist, pbp, rowq, rowj;
  std::vector<int64_t> pdof;
  for (size_t p = 0; p < by_piece.size(); ++p) {
    if (by_piece[p].empty()) continue;
    for (int32_t t : by_piece[p]) plist.push_back(t);
    for (int j = 0; j < h->pieces[p].b; ++j) {
      rowq.push_back((int32_t)pdof.size());
      rowj.push_back(j);
    }
    pptr.push_back((int32_t)plist.size());
    pdof.push_back(h->piece_dof_off[p]);
    pbp.push_back(h->pieces[p].b);
  }
  free_corner_stage(h);
  cs.ncorner = (int32_t)cm.corner.size();
  cs.npiece = (int32_t)pdof.size();
  cs.nrow = (int32_t)rowq.size();
  cs.ncopy = nc;
  cs.d_rowq = dupload(h, rowq); cs.d_rowj = dupload(h, rowj);
  cs.d_hptr = dupload(h, hptr); cs.d_hbp = dupload(h, hbp); cs.d_hdof = dupload(h, hdof);
  cs.d_soff = dupload(h, soff);
  cs.d_pptr = dupload(h, pptr); cs.d_plist = dupload(h, plist); cs.d_pdof = dupload(h, pdof);
  cs.d_pbp = dupload(h, pbp);
  if (srow.empty()) srow.push_back(0.0);
  if (h->prec == SFROM_F64) {
    cs.d_srow = dupload(h, srow);
    cs.d_hw = dupload(h, hw);
  } else {
    std::vector<float> f(srow.begin(), srow.end()), g(hw.begin(), hw.end());
    cs.d_srow = dupload(h, f);
    cs.d_hw = dupload(h, g);
  }
  cs.ready = true;
}

void prepare_online(sfrom_t* h) {
  const int ns = h->src.count;
  REQUIRE(ns > 0, SFROM_ESTATE, "no sources: call sfrom_set_sources");
  const size_t eb = prec_bytes(h->prec);
  if (h->corner_corr) {
    if (!h->cstage.ready) {
      drop_graph(h);
      stage_corners(h);
    }
    if (h->cstage.delta_ns != ns) {
      drop_graph(h);
      dfree(h->cstage.d_delta);
      h->cstage.d_delta = dalloc<unsigned char>(h, (size_t)std::max<int64_t>(h->cstage.ncopy, 1) * ns * eb);
      h->cstage.delta_ns = ns;
    }
  }
  if (h->src_dirty) {
    drop_graph(h);   // the captured run reads the source arrays replaced here
    // dense reduced sources for pieces that carry a source
    std::vector<int64_t> srow(h->pieces.size(), -1);
    int64_t rows = 0;
    for (size_t k = 0; k < h->src.rpiece.size(); ++k) {
      const int32_t p = h->src.rpiece[k];
      if (srow[p] < 0) { srow[p] = rows; rows += h->pieces[p].b; }
    }
    std::vector<double> dense((size_t)std::max<int64_t>(rows, 1) * ns, 0.0);
    for (int j = 0; j < ns; ++j)
      for (int64_t k = h->src.rptr[j]; k < h->src.rptr[j + 1]; ++k) {
        const int32_t p = h->src.rpiece[k];
        for (int l = 0; l < h->pieces[p].b; ++l) dense[(srow[p] + l) * ns + j] += h->src.rcoef[h->src.rcoff[k] + l];
      }
    dfree(h->d_src);
    if (h->prec == SFROM_F64) {
      h->d_src = dupload(h, dense);
    } else {
      std::vector<float> f(dense.begin(), dense.end());
      h->d_src = dupload(h, f);
    }
    for (size_t p = 0; p < h->pieces.size(); ++p) h->opieces[p].src_off = srow[p];
    HIPCHK(hipMemcpy(h->d_opieces, h->opieces.data(), h->opieces.size() * sizeof(OnlinePiece), hipMemcpyHostToDevice));
    h->src_dirty = false;
  }
  if (h->rec_dirty) {
    drop_graph(h);   // and the receiver arrays replaced here
    std::vector<int64_t> rptr(1, 0), rrow;
    std::vector<double> rval;
    for (int r = 0; r < h->rec.count; ++r) {
      for (int64_t k = h->rec.rptr[r]; k < h->rec.rptr[r + 1]; ++k) {
        const int32_t p = h->rec.rpiece[k];
        for (int l = 0; l < h->pieces[p].b; ++l) {
          rrow.push_back(h->piece_dof_off[p] + l);
          rval.push_back(h->rec.rcoef[h->rec.rcoff[k] + l]);
        }
      }
      rptr.push_back((int64_t)rrow.size());
    }
    dfree(h->d_rptr); dfree(h->d_rrow); dfree(h->d_rval);
    h->d_rptr = dupload(h, rptr);
    h->d_rrow = dupload(h, rrow);
    h->d_rval = dupload(h, rval);
    // receivers that each read exactly one piece are computed by the piece
    // phase (per-piece receiver lists); otherwise the receivers kernel runs
    dfree(h->d_prec_ptr); dfree(h->d_prec_list);
    h->rec_fused = h->rec.count > 0;
    for (int r = 0; r < h->rec.count && h->rec_fused; ++r) h->rec_fused = h->rec.rptr[r + 1] - h->rec.rptr[r] == 1;
    if (h->rec_fused) {
      const int np = (int)h->pieces.size();
      std::vector<int32_t> pptr(np + 1, 0), plist(h->rec.count);
      for (int r = 0; r < h->rec.count; ++r) pptr[h->rec.rpiece[h->rec.rptr[r]] + 1]++;
      // a piece-phase thread computes its piece's receivers one after the
      // other: with many receivers on one piece (few, large pieces) the
      // separate receivers kernel, one thread per receiver, is faster
      h->rec_fused = *std::max_element(pptr.begin(), pptr.end()) <= MAX_FUSED_RECEIVERS;
    }
    // with the corner correction the traces are read after it, by the
    // receivers kernel
    if (h->corner_corr) h->rec_fused = false;
    if (h->rec_fused) {
      const int np = (int)h->pieces.size();
      std::vector<int32_t> pptr(np + 1, 0), plist(h->rec.count);
      for (int r = 0; r < h->rec.count; ++r) pptr[h->rec.rpiece[h->rec.rptr[r]] + 1]++;
      for (int p = 0; p < np; ++p) pptr[p + 1] += pptr[p];
      std::vector<int32_t> fill(pptr.begin(), pptr.end() - 1);
      for (int r = 0; r < h->rec.count; ++r) plist[fill[h->rec.rpiece[h->rec.rptr[r]]]++] = r;
      h->d_prec_ptr = dupload(h, pptr);
      h->d_prec_list = dupload(h, plist);
    }
    h->rec_dirty = false;
  }
  if (h->state_ns != ns) alloc_state(h, ns);
}

// Autotuner of the cell phase: on the first run for a given (precision,
// max b, max m, n_s), every kernel variant is timed over a few launches on
// scratch copies of the state (the real state is not touched) and the
// fastest is kept for the life of the handle.
int autotune_cell(sfrom_t* h, StepArgs a, bool noalloc = false) {
  if (h->pinned_variant >= 0) {
    h->tuned_variant = std::min(h->pinned_variant, cell_variants(a) - 1);
    return h->tuned_variant;
  }
  const auto key = std::make_tuple(a.prec, a.max_b, a.max_m, a.ns);
  auto it = h->tuned.find(key);
  if (it != h->tuned.end()) return it->second;
  REQUIRE(!noalloc, SFROM_ESTATE, "the cell-phase kernel is not tuned for these sizes: call sfrom_run once first");
  const int nv = cell_variants(a);
  if (nv <= 1) { h->tuned[key] = 0; return 0; }
  const size_t eb = prec_bytes(h->prec);
  const int64_t npd = h->piece_dof_off.back();
  int64_t nu1 = 0;
  for (auto& oc : h->ocells) nu1 += oc.b;
  const size_t ybytes = (size_t)npd * a.ns * eb;
  const size_t hbytes = (size_t)std::max<int64_t>(h->n_hidden_rows, 1) * a.ns * eb;
  const size_t pbytes = (size_t)nu1 * a.ns * eb;
  void* sy = dalloc<unsigned char>(h, ybytes);
  void* sh0 = dalloc<unsigned char>(h, hbytes);
  void* sh1 = dalloc<unsigned char>(h, hbytes);
  void* sp = dalloc<unsigned char>(h, pbytes);
  HIPCHK(hipMemcpyAsync(sy, h->d_y[h->cur], ybytes, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(sh0, h->d_h[h->cur], hbytes, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(sh1, h->d_h[1 - h->cur], hbytes, hipMemcpyDeviceToDevice, h->stream));
  a.y_cur = sy; a.h_cur = sh0; a.h_old = sh1; a.phi = sp;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int best = 0;
  float best_ms = 1e30f;
  for (int v = 0; v < nv; ++v) {
    a.cell_variant = v;
    HIPCHK(launch_cell_phase(a, h->stream));      // warm-up (code object load)
    HIPCHK(hipEventRecord(e0, h->stream));
    const int reps = 4;
    for (int r = 0; r < reps; ++r) HIPCHK(launch_cell_phase(a, h->stream));
    HIPCHK(hipEventRecord(e1, h->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) { best_ms = ms; best = v; }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  dfree(sy); dfree(sh0); dfree(sh1); dfree(sp);
  h->tuned[key] = best;
  h->tuned_variant = best;
  h->tuned_ms = best_ms / 4;
  return best;
}

const double* stage_w(sfrom_t* h, int64_t n_steps, const double* w, int w_on_device) {
  if (w_on_device) return w;
  if (h->d_w_cap < n_steps) {
    dfree(h->d_w);
    h->d_w = dalloc<double>(h, n_steps);
    h->d_w_cap = n_steps;
  }
  HIPCHK(hipMemcpyAsync(h->d_w, w, n_steps * sizeof(double), hipMemcpyHostToDevice, h->stream));
  return h->d_w;
}

double rom_lambda_exact(sfrom_t* h);

// Leapfrog stability (Remark MFEM: the explicit scheme is stable for
// dt^2 lambda_max < 4). The cheap sufficient test uses the cells' Gershgorin
// bound (valid for blocks built from the cells' pencils); only when it fails,
// or for imported blocks, is the ROM's own largest eigenvalue computed.
void check_cfl(sfrom_t* h, double dt, bool noalloc = false) {
  const double d2 = dt * dt;
  if (!h->rom_imported && h->lam_cells > 0.0 && d2 * h->lam_cells < 4.0) return;
  REQUIRE(!noalloc || h->lam_rom >= 0.0, SFROM_ESTATE,
          "the ROM's largest eigenvalue is needed for this dt: call sfrom_rom_lambda_max or sfrom_run first");
  const double lam = rom_lambda_exact(h);
  char msg[160];
  std::snprintf(msg, sizeof msg, "dt = %.6g exceeds the leapfrog stability limit 2/sqrt(lambda_max) = %.6g of the ROM",
                dt, 2.0 / std::sqrt(lam));
  REQUIRE(d2 * lam < 4.0, SFROM_ECFL, msg);
}

// With `noalloc` (sfrom_run_noalloc) the run allocates no device memory:
// w and traces are device pointers, the handle must already be prepared
// for its sources, receivers and ROM (a previous sfrom_run), and the Phi^1
// exchange buffer and the non-finite flag live in `scratch`; the run is
// enqueued eagerly (no graph capture) and without profiling events.
void run(sfrom_t* h, int64_t n_steps, double dt, const double* w, int w_on_device, void* traces, int traces_on_device,
         bool noalloc = false) {
  REQUIRE(h->device >= 0, SFROM_EDEVICE, "host-only handle");
  REQUIRE(h->built, SFROM_ESTATE, "no ROM: call sfrom_build first");
  REQUIRE(n_steps >= 0, SFROM_EINVAL, "n_steps < 0");
  REQUIRE(dt > 0.0 && std::isfinite(dt), SFROM_EINVAL, "dt must be positive");
  REQUIRE(w != nullptr || n_steps == 0, SFROM_EINVAL, "null wavelet");
  if (!w_on_device)
    for (int64_t k = 0; k < n_steps; ++k)
      REQUIRE(std::isfinite(w[k]), SFROM_ENONFINITE, "wavelet sample " + std::to_string(k) + " is not finite");
  void* noalloc_base = nullptr;
  if (noalloc) {
    REQUIRE(w_on_device && traces_on_device, SFROM_EINVAL, "sfrom_run_noalloc takes device pointers only");
    REQUIRE(!h->corner_corr, SFROM_ESTATE, "sfrom_run_noalloc does not apply the corner correction: disable it");
    REQUIRE(!h->masses_dirty && !h->src_dirty && !h->rec_dirty && h->state_ns == h->src.count && h->src.count > 0,
            SFROM_ESTATE,
            "the on-line stage is not prepared for the current ROM, sources and receivers: call sfrom_run once first");
    int64_t nu1 = 0;
    for (auto& oc : h->ocells) nu1 += oc.b;
    const size_t need = NOALLOC_FLAG_BYTES + (size_t)nu1 * h->src.count * prec_bytes(h->prec);
    REQUIRE(need <= NOALLOC_SCRATCH_BYTES, SFROM_EINVAL,
            "sfrom_run_noalloc needs " + std::to_string(need) + " bytes of scratch, more than its maximum of " +
                std::to_string(NOALLOC_SCRATCH_BYTES) + " (use sfrom_run, or fewer sources)");
    REQUIRE(h->device < MAX_DEVICES && g_scratch_ptr[h->device], SFROM_EDEVICE, "no scratch address for this device");
    noalloc_base = g_scratch_ptr[h->device];
  }
  update_masses(h);
  if (n_steps > 0) check_cfl(h, dt, noalloc);
  prepare_online(h);
  const int ns = h->src.count, nr = h->rec.count;
  const size_t eb = prec_bytes(h->prec);
  const size_t tbytes = (size_t)n_steps * nr * ns * eb;
  void* d_tr = traces;
  bool own = false;
  if (!traces_on_device && tbytes > 0) { d_tr = dalloc<unsigned char>(h, tbytes); own = true; }
  const double* d_w = stage_w(h, n_steps, w, w_on_device);
  const bool profiling = h->profiling && !noalloc;
  StepArgs a;
  a.ncell = (int32_t)h->ocells.size();
  a.npiece = (int32_t)h->opieces.size();
  a.ns = ns; a.nrec = nr; a.prec = h->prec;
  a.max_b = 0; a.max_m = 0;
  for (auto& oc : h->ocells) { a.max_b = std::max(a.max_b, oc.b); a.max_m = std::max(a.max_m, oc.m); }
  a.max_bp = 0;
  for (auto& op : h->opieces) { a.max_bp = std::max(a.max_bp, op.b); REQUIRE(op.ncell <= 8, SFROM_EINVAL, "a piece is shared by more than 8 cells"); }
  a.dt2 = dt * dt;
  a.d_cells = h->d_ocells; a.d_pieces = h->d_opieces; a.d_gather = h->d_gather; a.d_inc = h->d_inc;
  a.d_blocks = h->d_blocks; a.d_minv = h->d_minv; a.d_src = h->d_src;
  a.phi = noalloc ? static_cast<unsigned char*>(noalloc_base) + NOALLOC_FLAG_BYTES : h->d_phi;
  a.w = d_w;
  a.d_rptr = h->d_rptr; a.d_rrow = h->d_rrow; a.d_rval = h->d_rval;
  a.d_prec_ptr = h->rec_fused ? h->d_prec_ptr : nullptr;
  a.d_prec_list = h->rec_fused ? h->d_prec_list : nullptr;
  a.traces = d_tr;
  a.d_cell_list = nullptr;
  a.nlist = a.ncell;
  // persistent mode: one cooperative launch for all n_steps steps
  const bool persist = h->persistent && n_steps > 0 && !noalloc;
  if (persist) {
    REQUIRE(persistent_supported(a), SFROM_EINVAL,
            "the persistent kernel takes FP32 or FP64 on-line blocks, b_i <= 144 and b_p <= 16");
    REQUIRE(!h->corner_corr, SFROM_ESTATE, "the persistent kernel does not apply the corner correction");
  }
  // one cell-phase launch per bucket of cells with the same strip count
  // (matrix-core precisions), each with its own autotuned variant
  const bool use_buckets = a.prec != SFROM_F64 && a.max_b <= 256 && h->buckets.size() > 1;
  std::vector<StepArgs> ba;
  if (use_buckets) {
    int largest = 0;
    for (size_t k = 0; k < h->buckets.size(); ++k) {
      auto& bk = h->buckets[k];
      StepArgs ab = a;
      ab.d_cell_list = bk.d_list;
      ab.nlist = bk.count;
      ab.max_b = bk.max_b;
      ab.max_m = bk.max_m;
      bk.variant = ab.cell_variant = autotune_cell(h, ab, noalloc);
      ba.push_back(ab);
      if (bk.count > h->buckets[largest].count) largest = (int)k;
    }
    h->tuned_variant = h->buckets[largest].variant;
    a.cell_variant = h->tuned_variant;
  } else {
    a.cell_variant = autotune_cell(h, a, noalloc);
  }
  auto cell_phase = [&](const StepArgs& x, hipStream_t st) -> hipError_t {
    if (!use_buckets) return launch_cell_phase(x, st);
    for (StepArgs ab : ba) {
      ab.y_cur = x.y_cur; ab.y_old = x.y_old; ab.h_cur = x.h_cur; ab.h_old = x.h_old;
      ab.step = x.step; ab.trace_step = x.trace_step;
      const hipError_t e = launch_cell_phase(ab, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  CornerArgs ca{};
  if (h->corner_corr) {
    const auto& cs = h->cstage;
    ca.ncorner = cs.ncorner; ca.npiece = cs.npiece; ca.nrow = cs.nrow; ca.ns = ns; ca.prec = h->prec;
    ca.ncopy = cs.ncopy;
    ca.rowq = cs.d_rowq; ca.rowj = cs.d_rowj;
    ca.hptr = cs.d_hptr; ca.hdof = cs.d_hdof; ca.hbp = cs.d_hbp; ca.soff = cs.d_soff;
    ca.srow = cs.d_srow; ca.hw = cs.d_hw;
    ca.pptr = cs.d_pptr; ca.plist = cs.d_plist; ca.pdof = cs.d_pdof; ca.pbp = cs.d_pbp;
    ca.delta = cs.d_delta;
  }
  const bool graph = h->use_graph && !h->profiling && n_steps > 0 && !noalloc && !persist;
  std::vector<int64_t> key;
  if (graph) {
    double dtv = dt;
    int64_t dbits;
    std::memcpy(&dbits, &dtv, 8);
    key = {n_steps, dbits, (int64_t)(intptr_t)d_w, (int64_t)(intptr_t)d_tr, (int64_t)h->cur,
           (int64_t)(intptr_t)h->d_y[0], (int64_t)(intptr_t)h->d_y[1], (int64_t)(intptr_t)h->d_h[0],
           (int64_t)(intptr_t)h->d_h[1], (int64_t)(intptr_t)h->d_phi, (int64_t)(intptr_t)h->d_minv,
           (int64_t)(intptr_t)h->d_src, (int64_t)(intptr_t)h->d_rval,
           (int64_t)ns, (int64_t)nr, (int64_t)a.cell_variant, (int64_t)(intptr_t)h->d_blocks};
    for (const StepArgs& ab : ba) key.push_back(ab.cell_variant);
    key.push_back(h->corner_corr ? (int64_t)(intptr_t)h->cstage.d_delta : 0);
    if (h->graph_exec && key == h->graph_key) {
      HIPCHK(hipGraphLaunch(h->graph_exec, h->stream));
      h->graph_launches++;
      if (n_steps % 2) h->cur = 1 - h->cur;
      goto done;
    }
    if (h->graph_exec) { hipGraphExecDestroy(h->graph_exec); h->graph_exec = nullptr; }
    // capture on a private stream (the null stream cannot be captured); the
    // graph is launched on the handle's stream, which orders it after all
    // work already enqueued there
    if (!h->capture_stream) HIPCHK(hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
  }
  {
  hipStream_t ls = graph ? h->capture_stream : h->stream;
  {
    const int cur0 = h->cur;
    int cur = cur0;
    if (persist) {
      PersistArgs pa{};
      pa.n_steps = n_steps;
      pa.cur0 = cur0;
      pa.rec_fused = h->rec_fused ? 1 : 0;
      pa.y[0] = h->d_y[0]; pa.y[1] = h->d_y[1];
      pa.h[0] = h->d_h[0]; pa.h[1] = h->d_h[1];
      HIPCHK(launch_persistent(a, pa, ls));
      cur = (cur0 + (int)(n_steps & 1)) & 1;
    }
    for (int64_t s = 0; s < n_steps && !persist; ++s) {
      a.y_cur = h->d_y[cur]; a.y_old = h->d_y[1 - cur];
      a.h_cur = h->d_h[cur]; a.h_old = h->d_h[1 - cur];
      a.step = s; a.trace_step = s;
      const bool sample = profiling && s % h->prof_every == 0;
      timed(h, 0, sample, [&] { return cell_phase(a, ls); });
      timed(h, 1, sample, [&] { return launch_piece_phase(a, ls); });
      if (h->corner_corr) {
        ca.y = a.y_old;   // level n + 1
        HIPCHK(launch_corner_correction(ca, ls));
      }
      if (!h->rec_fused) timed(h, 2, sample, [&] { return launch_receivers(a, ls); });
      cur = 1 - cur;
      if (profiling && ((s + 1) % 1024) == 0) collect_events(h);
    }
    if (graph) {
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamEndCapture(h->capture_stream, &g));
      hipGraphExec_t ex = nullptr;
      const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      HIPCHK(e);
      h->graph_exec = ex;
      h->graph_key = key;
      HIPCHK(hipGraphLaunch(h->graph_exec, h->stream));
      h->graph_launches++;
    }
    h->cur = cur;
  }
  }
done:
  h->steps_done += n_steps;
  if (own) {
    HIPCHK(hipMemcpyAsync(traces, d_tr, tbytes, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    dfree(d_tr);
  }
  if (n_steps > 0) {
    // a reduced-precision ROM can lose the stability of the leap-frog scheme
    // (rounded blocks of a deep layer need not stay definite); report it
    // instead of returning garbage
    int32_t* d_flag = static_cast<int32_t*>(noalloc_base);
    if (!noalloc) {
      if (!h->d_flag) h->d_flag = dalloc<int32_t>(h, 1);
      d_flag = h->d_flag;
    }
    HIPCHK(launch_zero_flag(d_flag, h->stream));
    const int64_t npd = h->piece_dof_off.back();
    HIPCHK(launch_nonfinite(h->d_y[h->cur], npd * ns, h->prec, d_flag, h->stream));
    HIPCHK(launch_nonfinite(h->d_h[h->cur], h->n_hidden_rows * ns, h->prec, d_flag, h->stream));
    int32_t flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    REQUIRE(flag == 0, SFROM_ENONFINITE,
            "the ROM state became non-finite: the scheme is unstable for this dt in this storage precision");
  }
}

// ---------------------------------------------------------------------------
// fine-grid comparator
// ---------------------------------------------------------------------------

void prepare_fine(sfrom_t* h, int prec) {
  REQUIRE(h->device >= 0, SFROM_EDEVICE, "host-only handle");
  REQUIRE(h->n > 0, SFROM_ESTATE, "no pencil");
  REQUIRE(prec == SFROM_F64 || prec == SFROM_F32, SFROM_EINVAL, "fine-grid precision must be F64 or F32");
  const int ns = h->src.count;
  REQUIRE(ns > 0, SFROM_ESTATE, "no sources: call sfrom_set_sources");
  const size_t eb = prec_bytes(prec);
  if (h->fine_prec != prec) {
    dfree(h->d_frowptr); dfree(h->d_fcol); dfree(h->d_fa); dfree(h->d_fbinv);
    h->d_frowptr = dupload(h, h->rowptr);
    h->d_fcol = dupload(h, h->col);
    std::vector<double> binv(h->n);
    for (int64_t i = 0; i < h->n; ++i) binv[i] = 1.0 / h->b[i];
    if (prec == SFROM_F64) {
      h->d_fa = dupload(h, h->a);
      h->d_fbinv = dupload(h, binv);
    } else {
      std::vector<float> af(h->a.begin(), h->a.end()), bf(binv.begin(), binv.end());
      h->d_fa = dupload(h, af);
      h->d_fbinv = dupload(h, bf);
    }
    dfree(h->d_stencil);
    if (!h->stencil.empty()) {
      // padded by FINE_PAD nodes of zero coefficients (unconditional row loads)
      if (prec == SFROM_F64) {
        std::vector<double> sd(h->stencil);
        sd.resize(sd.size() + (size_t)FINE_PAD * 8, 0.0);
        h->d_stencil = dupload(h, sd);
      } else {
        std::vector<float> sf(h->stencil.begin(), h->stencil.end());
        sf.resize(sf.size() + (size_t)FINE_PAD * 8, 0.0f);
        h->d_stencil = dupload(h, sf);
      }
    }
    h->fine_prec = prec;
    h->fine_ns = -1;
  }
  if (h->fine_io_dirty) {
    std::vector<int64_t> srow;
    std::vector<int32_t> scol;
    std::vector<double> sval;
    for (int j = 0; j < ns; ++j)
      for (int64_t k = h->src.colptr[j]; k < h->src.colptr[j + 1]; ++k) {
        srow.push_back(h->src.row[k]); scol.push_back(j); sval.push_back(h->src.val[k]);
      }
    dfree(h->d_fsrc_row); dfree(h->d_fsrc_col); dfree(h->d_fsrc_val);
    h->d_fsrc_row = dupload(h, srow);
    h->d_fsrc_col = dupload(h, scol);
    h->d_fsrc_val = dupload(h, sval);
    h->fsrc_n = (int64_t)srow.size();
    dfree(h->d_frec_ptr); dfree(h->d_frec_row); dfree(h->d_frec_val);
    h->d_frec_ptr = dupload(h, h->rec.colptr.empty() ? std::vector<int64_t>(1, 0) : h->rec.colptr);
    h->d_frec_row = dupload(h, h->rec.row);
    h->d_frec_val = dupload(h, h->rec.val);
    h->fine_io_dirty = false;
    dfree(h->d_fsrc_idx); dfree(h->d_fsrc_dense); h->fsrc_dense_prec = -1;
  }
  if (!h->stencil.empty() && h->fsrc_dense_prec != prec) {
    // point sources of the Cartesian kernel: a dense row of n_s values per
    // node that carries a source entry
    std::vector<int32_t> idx(h->n + FINE_PAD, -1);
    int32_t rows = 0;
    for (int j = 0; j < ns; ++j)
      for (int64_t k = h->src.colptr[j]; k < h->src.colptr[j + 1]; ++k)
        if (idx[h->src.row[k]] < 0) idx[h->src.row[k]] = rows++;
    std::vector<double> dense((size_t)std::max(rows, 1) * ns, 0.0);
    for (int j = 0; j < ns; ++j)
      for (int64_t k = h->src.colptr[j]; k < h->src.colptr[j + 1]; ++k)
        dense[(size_t)idx[h->src.row[k]] * ns + j] += h->src.val[k];
    dfree(h->d_fsrc_idx); dfree(h->d_fsrc_dense);
    h->d_fsrc_idx = dupload(h, idx);
    if (prec == SFROM_F64) {
      h->d_fsrc_dense = dupload(h, dense);
    } else {
      std::vector<float> f(dense.begin(), dense.end());
      h->d_fsrc_dense = dupload(h, f);
    }
    h->fsrc_dense_prec = prec;
  }
  if (h->fine_ns != ns) {
    for (int k = 0; k < 2; ++k) {
      dfree(h->d_u[k]);
      // FINE_PAD nodes of padding for the Cartesian kernel's row loads
      h->d_u[k] = dalloc<unsigned char>(h, (size_t)(h->n + FINE_PAD) * ns * eb);
      HIPCHK(hipMemsetAsync(h->d_u[k], 0, (size_t)(h->n + FINE_PAD) * ns * eb, h->stream));
    }
    h->fine_ns = ns;
    h->fcur = 0;
  }
}

void fine_run(sfrom_t* h, int64_t n_steps, double dt, const double* w, int w_on_device, void* traces,
              int traces_on_device, int prec) {
  REQUIRE(n_steps >= 0, SFROM_EINVAL, "n_steps < 0");
  REQUIRE(dt > 0.0 && std::isfinite(dt), SFROM_EINVAL, "dt must be positive");
  prepare_fine(h, prec);
  const int ns = h->src.count, nr = h->rec.count;
  const size_t eb = prec_bytes(prec);
  const size_t tbytes = (size_t)n_steps * nr * ns * eb;
  void* d_tr = traces;
  bool own = false;
  if (!traces_on_device && tbytes > 0) { d_tr = dalloc<unsigned char>(h, tbytes); own = true; }
  const double* d_w = stage_w(h, n_steps, w, w_on_device);
  FineArgs a;
  a.n = h->n; a.ns = ns; a.nrec = nr; a.prec = prec; a.dt2 = dt * dt;
  a.rowptr = h->d_frowptr; a.col = h->d_fcol; a.a = h->d_fa; a.binv = h->d_fbinv;
  a.stencil = h->d_stencil;
  a.ux = h->grid_u[0]; a.uy = h->grid_u[1]; a.uz = h->grid_u[2];
  a.w = d_w;
  a.nsrc_entries = h->fsrc_n; a.src_row = h->d_fsrc_row; a.src_col = h->d_fsrc_col; a.src_val = h->d_fsrc_val;
  a.rec_ptr = h->d_frec_ptr; a.rec_row = h->d_frec_row; a.rec_val = h->d_frec_val;
  a.traces = d_tr;
  a.src_idx = h->d_fsrc_idx;
  a.src_dense = h->d_fsrc_dense;
  a.src_dense_ok = (h->d_fsrc_idx != nullptr && h->fsrc_dense_prec == prec) ? 1 : 0;
  for (int64_t s = 0; s < n_steps; ++s) {
    a.u_cur = h->d_u[h->fcur]; a.u_old = h->d_u[1 - h->fcur];
    a.step = s; a.trace_step = s;
    timed(h, 3, s % h->prof_every == 0, [&] { return launch_fine_step(a, h->stream); });
    h->fcur = 1 - h->fcur;
    if (h->profiling && ((s + 1) % 1024) == 0) collect_events(h);
  }
  if (n_steps > 0 && fine_uses_25d(a)) {
    // each step wrote the traces of the level it read; the last level's
    a.u_cur = h->d_u[h->fcur];
    a.trace_step = n_steps - 1;
    HIPCHK(launch_fine_rec_level(a, h->stream));
  }
  if (own) {
    HIPCHK(hipMemcpyAsync(traces, d_tr, tbytes, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    dfree(d_tr);
  }
}

// Largest eigenvalue of a symmetric operator by Lanczos (no reorthogonalisation:
// the extreme Ritz value converges first and ghost copies do not move it).
template <typename MV>
double lanczos_max(int64_t n, MV matvec, int maxit = 300) {
  std::vector<double> v(n), vp(n, 0.0), wv(n);
  // deterministic start vector
  uint64_t s = 0x9E3779B97F4A7C15ull;
  double nrm = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    s ^= s << 13; s ^= s >> 7; s ^= s << 17;
    v[i] = (double)(s >> 11) / 9007199254740992.0 - 0.5;
    nrm += v[i] * v[i];
  }
  nrm = std::sqrt(nrm);
  for (auto& x : v) x /= nrm;
  std::vector<double> al, be;
  double beta = 0.0, prev = 0.0, lam = 0.0;
  for (int it = 0; it < maxit && it < n; ++it) {
    matvec(v.data(), wv.data());
    double alpha = 0.0;
    for (int64_t i = 0; i < n; ++i) alpha += wv[i] * v[i];
    for (int64_t i = 0; i < n; ++i) wv[i] -= alpha * v[i] + beta * vp[i];
    double bn = 0.0;
    for (int64_t i = 0; i < n; ++i) bn += wv[i] * wv[i];
    bn = std::sqrt(bn);
    al.push_back(alpha);
    // largest eigenvalue of the tridiagonal (al, be) by bisection on the
    // Sturm count of eigenvalues below x
    const int k = (int)al.size();
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < k; ++i) {
      double r = 0.0;
      if (i > 0) r += std::fabs(be[i - 1]);
      if (i + 1 < k) r += std::fabs(be[i]);
      lo = std::min(lo, al[i] - r);
      hi = std::max(hi, al[i] + r);
    }
    for (int rep = 0; rep < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++rep) {
      const double mid = 0.5 * (lo + hi);
      int below = 0;
      double d = 1.0;
      for (int i = 0; i < k; ++i) {
        d = al[i] - mid - (i > 0 ? be[i - 1] * be[i - 1] / d : 0.0);
        if (d == 0.0) d = -1e-300;
        if (d < 0.0) ++below;
      }
      if (below == k) hi = mid; else lo = mid;
    }
    lam = hi;
    if (bn < 1e-14 * std::fabs(lam)) break;
    if (it > 20 && std::fabs(lam - prev) <= 1e-13 * std::fabs(lam)) break;
    prev = lam;
    be.push_back(bn);
    for (int64_t i = 0; i < n; ++i) { vp[i] = v[i]; v[i] = wv[i] / bn; }
    beta = bn;
  }
  return lam;
}


// Largest eigenvalue of the global ROM pencil (-L, D) by Lanczos on the
// host (FP64 blocks as built or imported), cached until the ROM changes.
double rom_lambda_exact(sfrom_t* h) {
  if (h->lam_rom >= 0.0) return h->lam_rom;
  const int nc = (int)h->ocells.size();
  // host copy of the double blocks; operator D^{-1/2}(-L)D^{-1/2} applied in
  // cell-blocked flux form with D = blkdiag(M_p, (Ghat_i^k)^{-1}).
  std::vector<double> r64;
  int64_t tot = 0;
  for (int i = 0; i < nc; ++i) tot += 2LL * h->ocells[i].m * h->ocells[i].b * h->ocells[i].b;
  r64.resize(tot);
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipMemcpy(r64.data(), h->d_rom64, tot * 8, hipMemcpyDeviceToHost));
  const int64_t npd = h->piece_dof_off.back();
  const int64_t ndof = npd + h->n_hidden_dofs;
  std::vector<int64_t> hoff(nc + 1, 0);   // hidden dofs of the cells, unpadded
  for (int i = 0; i < nc; ++i) hoff[i + 1] = hoff[i] + (int64_t)(h->ocells[i].m - 1) * h->ocells[i].b;
  // symmetric square roots of the mass blocks: piece masses M_p and hidden (Ghat^k)^{-1}
  auto symsqrt = [](int n, const double* A, double* out, bool inverse) {
    // Jacobi eigen-decomposition (small n)
    std::vector<double> a(A, A + n * n), v(n * n, 0.0);
    for (int i = 0; i < n; ++i) v[i + i * n] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
      double off = 0.0;
      for (int p = 0; p < n; ++p) for (int q = p + 1; q < n; ++q) off += a[p + q * n] * a[p + q * n];
      if (off < 1e-30) break;
      for (int p = 0; p < n; ++p)
        for (int q = p + 1; q < n; ++q) {
          const double apq = a[p + q * n];
          if (std::fabs(apq) < 1e-300) continue;
          const double th = 0.5 * (a[q + q * n] - a[p + p * n]) / apq;
          const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
          const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
          for (int k = 0; k < n; ++k) {
            const double akp = a[k + p * n], akq = a[k + q * n];
            a[k + p * n] = c * akp - s * akq; a[k + q * n] = s * akp + c * akq;
          }
          for (int k = 0; k < n; ++k) {
            const double apk = a[p + k * n], aqk = a[q + k * n];
            a[p + k * n] = c * apk - s * aqk; a[q + k * n] = s * apk + c * aqk;
          }
          for (int k = 0; k < n; ++k) {
            const double vkp = v[k + p * n], vkq = v[k + q * n];
            v[k + p * n] = c * vkp - s * vkq; v[k + q * n] = s * vkp + c * vkq;
          }
        }
    }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) {
          const double ev = std::max(a[k + k * n], 1e-300);
          s += v[i + k * n] * v[j + k * n] * (inverse ? 1.0 / std::sqrt(ev) : std::sqrt(ev));
        }
        out[i + j * n] = s;
      }
  };
  // piece masses M_p = sum_c ([Ghat_c^1]_pp)^{-1}  -> M_p^{-1/2}
  std::vector<std::vector<double>> pm(h->pieces.size());
  for (size_t p = 0; p < h->pieces.size(); ++p) {
    const int bp = h->pieces[p].b;
    std::vector<double> M(bp * bp, 0.0);
    for (int32_t c : h->piece_cells[p]) {
      const auto& cp = h->cell_pieces[c];
      const size_t q = std::lower_bound(cp.begin(), cp.end(), (int32_t)p) - cp.begin();
      const int col0 = h->cell_piece_col[c][q], b = h->ocells[c].b;
      const double* G1 = r64.data() + h->rom64_off[c];
      std::vector<double> blk(bp * bp), inv(bp * bp), tmp(bp * bp);
      for (int j = 0; j < bp; ++j) for (int i = 0; i < bp; ++i) blk[i + j * bp] = G1[(col0 + i) + (int64_t)(col0 + j) * b];
      // inverse via inverse square root squared
      symsqrt(bp, blk.data(), tmp.data(), true);
      for (int i = 0; i < bp; ++i) for (int j = 0; j < bp; ++j) {
        double s = 0.0; for (int k = 0; k < bp; ++k) s += tmp[i + k * bp] * tmp[k + j * bp];
        M[i + j * bp] += s;
      }
    }
    pm[p].resize(bp * bp);
    symsqrt(bp, M.data(), pm[p].data(), true);
  }
  // hidden mass (Ghat^k)^{-1} -> its inverse square root is Ghat^{1/2}
  std::vector<std::vector<double>> hsq(nc);
  for (int i = 0; i < nc; ++i) {
    const int m = h->ocells[i].m, b = h->ocells[i].b;
    hsq[i].resize((size_t)std::max(m - 1, 0) * b * b);
    for (int k = 1; k < m; ++k) symsqrt(b, r64.data() + h->rom64_off[i] + (int64_t)k * b * b, hsq[i].data() + (int64_t)(k - 1) * b * b, false);
  }
  auto apply_msq = [&](const double* x, double* y) {   // y = D^{-1/2} x
    for (size_t p = 0; p < h->pieces.size(); ++p) {
      const int bp = h->pieces[p].b; const int64_t o = h->piece_dof_off[p];
      for (int i = 0; i < bp; ++i) { double s = 0.0; for (int j = 0; j < bp; ++j) s += pm[p][i + j * bp] * x[o + j]; y[o + i] = s; }
    }
    for (int i = 0; i < nc; ++i) {
      const int m = h->ocells[i].m, b = h->ocells[i].b;
      for (int k = 1; k < m; ++k) {
        const int64_t o = npd + hoff[i] + (int64_t)(k - 1) * b;
        const double* S = hsq[i].data() + (int64_t)(k - 1) * b * b;
        for (int r = 0; r < b; ++r) { double s = 0.0; for (int c = 0; c < b; ++c) s += S[r + c * b] * x[o + c]; y[o + r] = s; }
      }
    }
  };
  std::vector<double> t1(ndof), t2(ndof);
  auto mv = [&](const double* x, double* y) {
    apply_msq(x, t1.data());
    std::fill(t2.begin(), t2.end(), 0.0);
    for (int i = 0; i < nc; ++i) {
      const int m = h->ocells[i].m, b = h->ocells[i].b;
      const double* G = r64.data() + h->rom64_off[i] + (int64_t)m * b * b;
      std::vector<int64_t> rows((size_t)m * b);
      int r0 = 0;
      for (size_t q = 0; q < h->cell_pieces[i].size(); ++q) {
        const int32_t p = h->cell_pieces[i][q];
        for (int l = 0; l < h->pieces[p].b; ++l) rows[r0++] = h->piece_dof_off[p] + l;
      }
      for (int k = 1; k < m; ++k) for (int r = 0; r < b; ++r) rows[(size_t)k * b + r] = npd + hoff[i] + (int64_t)(k - 1) * b + r;
      // (-L U)^k = -(Phi^k - Phi^{k-1}), Phi^k = G^k (U^{k+1} - U^k)
      std::vector<double> phi((size_t)m * b);
      for (int k = 0; k < m; ++k)
        for (int r = 0; r < b; ++r) {
          double s = 0.0;
          for (int c = 0; c < b; ++c) {
            const double up = (k + 1 < m) ? t1[rows[(size_t)(k + 1) * b + c]] : 0.0;
            s += G[(int64_t)k * b * b + r + (int64_t)c * b] * (up - t1[rows[(size_t)k * b + c]]);
          }
          phi[(size_t)k * b + r] = s;
        }
      for (int k = 0; k < m; ++k)
        for (int r = 0; r < b; ++r) t2[rows[(size_t)k * b + r]] -= phi[(size_t)k * b + r] - (k > 0 ? phi[(size_t)(k - 1) * b + r] : 0.0);
    }
    apply_msq(t2.data(), y);
  };
  h->lam_rom = lanczos_max(ndof, mv);
  return h->lam_rom;
}


// ---------------------------------------------------------------------------
// ROM and state checkpoint (sfrom_save / sfrom_load)
// ---------------------------------------------------------------------------

constexpr char kMagic[8] = {'S', 'F', 'R', 'O', 'M', 'C', 'K', 'P'};
constexpr int32_t kVersion = 1;

struct File {
  std::FILE* f = nullptr;
  ~File() { if (f) std::fclose(f); }
};

void put(sfrom_t* h, File& F, const void* p, size_t n) {
  REQUIRE(n == 0 || std::fwrite(p, 1, n, F.f) == n, SFROM_EINVAL, "write to the checkpoint file failed");
}
void get(sfrom_t* h, File& F, void* p, size_t n) {
  REQUIRE(n == 0 || std::fread(p, 1, n, F.f) == n, SFROM_EINVAL, "checkpoint file is truncated");
}
template <typename T>
void put_v(sfrom_t* h, File& F, T v) { put(h, F, &v, sizeof v); }
template <typename T>
T get_v(sfrom_t* h, File& F) { T v; get(h, F, &v, sizeof v); return v; }

// device -> file in chunks
void put_dev(sfrom_t* h, File& F, const void* d, size_t n) {
  std::vector<unsigned char> buf(std::min<size_t>(n, (size_t)64 << 20));
  for (size_t o = 0; o < n; o += buf.size()) {
    const size_t k = std::min(buf.size(), n - o);
    HIPCHK(hipMemcpy(buf.data(), (const unsigned char*)d + o, k, hipMemcpyDeviceToHost));
    put(h, F, buf.data(), k);
  }
}
void get_dev(sfrom_t* h, File& F, void* d, size_t n) {
  std::vector<unsigned char> buf(std::min<size_t>(n, (size_t)64 << 20));
  for (size_t o = 0; o < n; o += buf.size()) {
    const size_t k = std::min(buf.size(), n - o);
    get(h, F, buf.data(), k);
    HIPCHK(hipMemcpy((unsigned char*)d + o, buf.data(), k, hipMemcpyHostToDevice));
  }
}

int64_t minv_elems(const sfrom_t* h) {
  int64_t moff = 0;
  for (auto& op : h->opieces) moff += (int64_t)op.b * op.b;
  return moff;
}
int64_t rom64_elems(const sfrom_t* h) {
  int64_t r = 0;
  for (auto& oc : h->ocells) r += 2LL * oc.m * oc.b * oc.b;
  return r;
}

void save_checkpoint(sfrom_t* h, const char* path) {
  REQUIRE(path != nullptr, SFROM_EINVAL, "null path");
  REQUIRE(h->device >= 0, SFROM_EDEVICE, "host-only handle");
  REQUIRE(h->built, SFROM_ESTATE, "no ROM: build or load first");
  update_masses(h);
  HIPCHK(hipStreamSynchronize(h->stream));
  File F;
  F.f = std::fopen(path, "wb");
  REQUIRE(F.f != nullptr, SFROM_EINVAL, std::string("cannot open ") + path + " for writing");
  const int nc = (int)h->cells.size(), np = (int)h->pieces.size();
  put(h, F, kMagic, 8);
  put_v<int32_t>(h, F, kVersion);
  put_v<int32_t>(h, F, nc);
  put_v<int32_t>(h, F, np);
  put_v<int32_t>(h, F, h->prec);
  put_v<double>(h, F, h->shift);
  put_v<int32_t>(h, F, h->rom_imported ? 1 : 0);
  for (int i = 0; i < nc; ++i) { put_v<int32_t>(h, F, h->ocells[i].m); put_v<int32_t>(h, F, h->ocells[i].b); }
  for (int p = 0; p < np; ++p) {
    const auto& pc = h->pieces[p];
    put_v<int32_t>(h, F, pc.b);
    put_v<int64_t>(h, F, (int64_t)pc.gnode.size());
    put(h, F, pc.gnode.data(), pc.gnode.size() * 8);
    put(h, F, pc.S.data(), pc.S.size() * 8);
  }
  put_dev(h, F, h->d_rom64, (size_t)rom64_elems(h) * 8);
  put_dev(h, F, h->d_blocks, (size_t)h->block_elems * block_bytes(h->prec));
  put_dev(h, F, h->d_minv, (size_t)minv_elems(h) * prec_bytes(h->prec));
  put_v<int32_t>(h, F, h->state_ns);
  put_v<int32_t>(h, F, h->cur);
  put_v<int64_t>(h, F, h->steps_done);
  if (h->state_ns > 0)
    for (int k = 0; k < 2; ++k) {
      put_dev(h, F, h->d_y[k], ystate_bytes(h, h->state_ns));
      put_dev(h, F, h->d_h[k], hstate_bytes(h, h->state_ns));
    }
  REQUIRE(std::fflush(F.f) == 0, SFROM_EINVAL, "write to the checkpoint file failed");
}

void load_arrays(sfrom_t* h, File& F);

void load_checkpoint(sfrom_t* h, const char* path) {
  REQUIRE(path != nullptr, SFROM_EINVAL, "null path");
  REQUIRE(h->device >= 0, SFROM_EDEVICE, "host-only handle");
  finalize_partition(h);
  File F;
  F.f = std::fopen(path, "rb");
  REQUIRE(F.f != nullptr, SFROM_EINVAL, std::string("cannot open ") + path);
  char magic[8];
  get(h, F, magic, 8);
  REQUIRE(std::memcmp(magic, kMagic, 8) == 0, SFROM_EINVAL, "not an sfrom checkpoint file");
  const int32_t ver = get_v<int32_t>(h, F);
  REQUIRE(ver == kVersion, SFROM_EINVAL, "unsupported checkpoint version " + std::to_string(ver));
  const int nc = (int)h->cells.size(), np = (int)h->pieces.size();
  REQUIRE(get_v<int32_t>(h, F) == nc && get_v<int32_t>(h, F) == np, SFROM_EINVAL,
          "checkpoint partition differs: cell or piece count");
  const int32_t prec = get_v<int32_t>(h, F);
  REQUIRE(prec >= SFROM_F64 && prec <= SFROM_BF16, SFROM_EINVAL, "bad on-line precision in checkpoint");
  const double shift = get_v<double>(h, F);
  const int32_t imported = get_v<int32_t>(h, F);
  std::vector<int32_t> mpc(nc);
  for (int i = 0; i < nc; ++i) {
    mpc[i] = get_v<int32_t>(h, F);
    const int32_t b = get_v<int32_t>(h, F);
    REQUIRE(b == h->cell_b[i] && mpc[i] >= 1, SFROM_EINVAL,
            "checkpoint partition differs: boundary dimension of cell " + std::to_string(i));
  }
  for (int p = 0; p < np; ++p) {
    const auto& pc = h->pieces[p];
    const int32_t bp = get_v<int32_t>(h, F);
    const int64_t kp = get_v<int64_t>(h, F);
    REQUIRE(bp == pc.b && kp == (int64_t)pc.gnode.size(), SFROM_EINVAL,
            "checkpoint partition differs: piece " + std::to_string(p));
    std::vector<int64_t> g((size_t)kp);
    std::vector<double> S((size_t)kp * bp);
    get(h, F, g.data(), g.size() * 8);
    get(h, F, S.data(), S.size() * 8);
    REQUIRE(g == pc.gnode && S == pc.S, SFROM_EINVAL,
            "checkpoint partition differs: nodes or basis of piece " + std::to_string(p));
  }
  sfrom_build_opts o{};
  o.m = mpc[0];
  o.m_per_cell = mpc.data();
  o.shift = shift;
  o.online_prec = prec;
  BuildCtx ctx;
  build_layout(h, &o, ctx);   // on-line layout and device arrays, no build
  // from here on the previous ROM is gone: a failure leaves no ROM
  h->rom_imported = imported != 0;
  try {
    load_arrays(h, F);
  } catch (const Fail&) {
    free_rom(h);
    throw;
  }
}

void load_arrays(sfrom_t* h, File& F) {
  get_dev(h, F, h->d_rom64, (size_t)rom64_elems(h) * 8);
  get_dev(h, F, h->d_blocks, (size_t)h->block_elems * block_bytes(h->prec));
  get_dev(h, F, h->d_minv, (size_t)minv_elems(h) * prec_bytes(h->prec));
  const int32_t sns = get_v<int32_t>(h, F);
  const int32_t cur = get_v<int32_t>(h, F);
  const int64_t done = get_v<int64_t>(h, F);
  REQUIRE(cur == 0 || cur == 1, SFROM_EINVAL, "bad state level in checkpoint");
  if (sns > 0) {
    alloc_state(h, sns);
    for (int k = 0; k < 2; ++k) {
      get_dev(h, F, h->d_y[k], ystate_bytes(h, sns));
      get_dev(h, F, h->d_h[k], hstate_bytes(h, sns));
    }
  }
  h->cur = cur;
  h->steps_done = done;
  h->masses_dirty = false;
  h->lam_rom = -1.0;
  h->built = true;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

#define API_BEGIN(h)                                          \
  if (!(h)) return SFROM_EINVAL;                              \
  try {                                                       \
    if ((h)->device >= 0) HIPCHK(hipSetDevice((h)->device));
#define API_END(h)                                            \
  }                                                           \
  catch (const Fail& f) { return f.code; }                    \
  catch (const std::bad_alloc&) {                             \
    (h)->err = "host allocation failed";                      \
    return SFROM_ENOMEM;                                      \
  }                                                           \
  catch (...) {                                               \
    (h)->err = "unexpected exception";                        \
    return SFROM_EINVAL;                                      \
  }                                                           \
  (h)->err.clear();                                           \
  return SFROM_OK;

// Why the calling thread's last sfrom_create failed (read through
// sfrom_last_error(NULL)).
thread_local std::string g_create_err = "no failed create on this thread";

int create_fail(const char* what, hipError_t e) {
  g_create_err = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return e == hipErrorOutOfMemory ? SFROM_ENOMEM : SFROM_EDEVICE;
}

extern "C" {

int sfrom_create(sfrom_t** out, int device, void* hip_stream) {
  if (!out) return SFROM_EINVAL;
  *out = nullptr;
  if (device == -1) {   // host-only handle: problem set-up and validation, no device work
    sfrom_t* h = new (std::nothrow) sfrom_t();
    if (!h) return SFROM_ENOMEM;
    h->device = -1;
    *out = h;
    return SFROM_OK;
  }
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return create_fail("hipGetDeviceCount", e);
  if (device < 0 || device >= ndev) {
    g_create_err = "device " + std::to_string(device) + " not in [0, " + std::to_string(ndev) + ")";
    return SFROM_EDEVICE;
  }
  sfrom_t* h = new (std::nothrow) sfrom_t();
  if (!h) return SFROM_ENOMEM;
  h->device = device;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if ((e = hipSetDevice(device)) != hipSuccess) { delete h; return create_fail("hipSetDevice", e); }
  if ((e = init_scratch(device)) != hipSuccess) { delete h; return create_fail("scratch symbol address", e); }
  *out = h;
  return SFROM_OK;
}

void sfrom_destroy(sfrom_t* h) {
  if (!h) return;
  if (h->device < 0) { delete h; return; }
  hipSetDevice(h->device);
  if (h->stream) hipStreamSynchronize(h->stream); else hipDeviceSynchronize();
  free_all(h);
  delete h;
}

const char* sfrom_last_error(const sfrom_t* h) { return h ? h->err.c_str() : g_create_err.c_str(); }

int sfrom_set_pencil(sfrom_t* h, int64_t n, const int64_t* rowptr, const int32_t* col, const double* a,
                     const double* b) {
  API_BEGIN(h)
  REQUIRE(n > 0 && rowptr && col && a && b, SFROM_EINVAL, "bad pencil arguments");
  REQUIRE(n < ((int64_t)1 << 31), SFROM_EINVAL, "n must fit in int32 column indices");
  REQUIRE(rowptr[0] == 0, SFROM_EINVAL, "rowptr[0] must be 0");
  for (int64_t i = 0; i < n; ++i) REQUIRE(rowptr[i + 1] >= rowptr[i], SFROM_EINVAL, "rowptr not monotone");
  const int64_t nnz = rowptr[n];
  for (int64_t i = 0; i < n; ++i) {
    REQUIRE(b[i] > 0.0, std::isfinite(b[i]) ? SFROM_EBPOS : SFROM_ENONFINITE, "B must be diagonal positive (Sec. 1)");
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      REQUIRE(col[k] >= 0 && col[k] < n, SFROM_EINVAL, "column index out of range");
      REQUIRE(k == rowptr[i] || col[k] > col[k - 1], SFROM_EINVAL, "columns must be sorted and unique within a row");
      REQUIRE(std::isfinite(a[k]), SFROM_ENONFINITE, "non-finite entry in A");
    }
  }
  // symmetry: A = A^T
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      const int32_t j = col[k];
      const int32_t* cb = col + rowptr[j];
      const int32_t* ce = col + rowptr[j + 1];
      const int32_t* it = std::lower_bound(cb, ce, (int32_t)i);
      REQUIRE(it != ce && *it == i && a[it - col] == a[k], SFROM_ENOTSYM, "A is not symmetric");
    }
  free_all(h);
  h->n = n;
  h->rowptr.assign(rowptr, rowptr + n + 1);
  h->col.assign(col, col + nnz);
  h->a.assign(a, a + nnz);
  h->b.assign(b, b + n);
  h->cells.clear();
  h->pieces.clear();
  h->part_ready = false;
  free_stage(h);
  h->stencil.clear();
  h->grid_u[0] = h->grid_u[1] = h->grid_u[2] = 0;
  h->src = Columns();
  h->rec = Columns();
  h->cmap = sfrom::CornerMap();
  h->corner_corr = false;
  API_END(h)
}

int sfrom_add_cell(sfrom_t* h, int32_t cell, int32_t n_i, const int64_t* global_node, const int32_t* rowptr_i,
                   const int32_t* col_i, const double* a_i, const double* b_i) {
  API_BEGIN(h)
  REQUIRE(h->n > 0, SFROM_ESTATE, "no pencil");
  REQUIRE(cell >= 0 && n_i > 0 && global_node && rowptr_i && col_i && a_i && b_i, SFROM_EINVAL, "bad cell arguments");
  if ((int)h->cells.size() <= cell) h->cells.resize(cell + 1);
  REQUIRE(!h->cells[cell].defined, SFROM_EINVAL, "cell " + std::to_string(cell) + " defined twice");
  REQUIRE(rowptr_i[0] == 0, SFROM_EINVAL, "rowptr_i[0] must be 0");
  CellDef c;
  c.n = n_i;
  c.gnode.assign(global_node, global_node + n_i);
  std::vector<int64_t> sorted(c.gnode);
  std::sort(sorted.begin(), sorted.end());
  REQUIRE(std::adjacent_find(sorted.begin(), sorted.end()) == sorted.end(), SFROM_EINVAL, "repeated node in cell");
  REQUIRE(sorted.front() >= 0 && sorted.back() < h->n, SFROM_EINVAL, "cell node out of range");
  for (int r = 0; r < n_i; ++r) {
    REQUIRE(rowptr_i[r + 1] >= rowptr_i[r], SFROM_EINVAL, "rowptr_i not monotone");
    REQUIRE(b_i[r] > 0.0, std::isfinite(b_i[r]) ? SFROM_EBPOS : SFROM_ENONFINITE, "B_i must be positive (Sec. 2)");
    for (int k = rowptr_i[r]; k < rowptr_i[r + 1]; ++k) {
      REQUIRE(col_i[k] >= 0 && col_i[k] < n_i, SFROM_EINVAL, "local column out of range");
      REQUIRE(k == rowptr_i[r] || col_i[k] > col_i[k - 1], SFROM_EINVAL, "local columns must be sorted and unique");
      REQUIRE(std::isfinite(a_i[k]), SFROM_ENONFINITE, "non-finite entry in A_i");
    }
  }
  const int nnz = rowptr_i[n_i];
  for (int r = 0; r < n_i; ++r)
    for (int k = rowptr_i[r]; k < rowptr_i[r + 1]; ++k) {
      const int j = col_i[k];
      const int32_t* cb = col_i + rowptr_i[j];
      const int32_t* ce = col_i + rowptr_i[j + 1];
      const int32_t* it = std::lower_bound(cb, ce, r);
      REQUIRE(it != ce && *it == r && a_i[it - col_i] == a_i[k], SFROM_ENOTSYM, "A_i is not symmetric");
    }
  c.rowptr.assign(rowptr_i, rowptr_i + n_i + 1);
  c.col.assign(col_i, col_i + nnz);
  c.a.assign(a_i, a_i + nnz);
  c.b.assign(b_i, b_i + n_i);
  c.defined = true;
  h->cells[cell] = std::move(c);
  h->part_ready = false;
  free_stage(h);
  free_rom(h);
  API_END(h)
}

int sfrom_add_piece(sfrom_t* h, int32_t piece, int32_t k_p, const int64_t* global_node, int32_t b_p,
                    const double* S_p) {
  API_BEGIN(h)
  REQUIRE(h->n > 0, SFROM_ESTATE, "no pencil");
  REQUIRE(piece >= 0 && k_p > 0 && b_p > 0 && b_p <= k_p && global_node && S_p, SFROM_EINVAL, "bad piece arguments");
  if ((int)h->pieces.size() <= piece) h->pieces.resize(piece + 1);
  REQUIRE(!h->pieces[piece].defined, SFROM_EINVAL, "piece " + std::to_string(piece) + " defined twice");
  PieceDef p;
  p.gnode.assign(global_node, global_node + k_p);
  for (int64_t g : p.gnode) REQUIRE(g >= 0 && g < h->n, SFROM_EINVAL, "piece node out of range");
  p.b = b_p;
  p.S.assign(S_p, S_p + (int64_t)k_p * b_p);
  for (int i = 0; i < b_p; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = 0.0;
      for (int r = 0; r < k_p; ++r) s += S_p[r + (int64_t)i * k_p] * S_p[r + (int64_t)j * k_p];
      REQUIRE(std::fabs(s - (i == j ? 1.0 : 0.0)) <= 1e-10, SFROM_EINVAL,
              "piece " + std::to_string(piece) + ": basis is not orthonormal (S_p^T S_p = I)");
    }
  p.defined = true;
  h->pieces[piece] = std::move(p);
  h->part_ready = false;
  free_stage(h);
  free_rom(h);
  API_END(h)
}

int sfrom_build(sfrom_t* h, const sfrom_build_opts* opts) {
  API_BEGIN(h)
  build(h, opts);
  API_END(h)
}

int sfrom_build_learned(sfrom_t* h, const sfrom_build_opts* opts, sfrom_surrogate_t* s, int32_t n,
                        const int32_t* cells, const float* x, double omega_max, double tol,
                        int32_t* accepted, double* mismatch) {
  API_BEGIN(h)
  build_learned(h, opts, s, n, cells, x, omega_max, tol, accepted, mismatch);
  API_END(h)
}

int sfrom_surrogate_targets(sfrom_t* h, int32_t n, const int32_t* cells, float* t) {
  API_BEGIN(h)
  factor_targets(h, n, cells, t);
  API_END(h)
}

int sfrom_import_rom(sfrom_t* h, int32_t cell, int32_t m, int32_t b, const double* Ghat, const double* G) {
  API_BEGIN(h)
  REQUIRE(h->built, SFROM_ESTATE, "no ROM to modify: build first");
  REQUIRE(cell >= 0 && cell < (int)h->ocells.size() && Ghat && G, SFROM_EINVAL, "bad cell");
  const OnlineCell& oc = h->ocells[cell];
  REQUIRE(m == oc.m && b == oc.b, SFROM_EINVAL, "m and b must match the built layout of the cell");
  const int64_t bb2 = (int64_t)b * b;
  std::vector<double> r64(2 * m * bb2);
  for (int64_t k = 0; k < m * bb2; ++k) {
    REQUIRE(std::isfinite(Ghat[k]) && std::isfinite(G[k]), SFROM_ENONFINITE, "non-finite block");
    r64[k] = Ghat[k];
    r64[m * bb2 + k] = G[k];
  }
  for (int k = 0; k < m; ++k)
    for (int i = 0; i < b; ++i)
      for (int j = 0; j < i; ++j) {
        const int64_t u = k * bb2 + i + (int64_t)j * b, v = k * bb2 + j + (int64_t)i * b;
        REQUIRE(Ghat[u] == Ghat[v] && G[u] == G[v], SFROM_ENOTSPD, "blocks must be symmetric");
      }
  HIPCHK(hipMemcpy(h->d_rom64 + h->rom64_off[cell], r64.data(), r64.size() * sizeof(double), hipMemcpyHostToDevice));
  // on-line blocks D_0, C_0, D_1, ..., D_{m-1} (b x ld, row-major, zero
  // padded) in the unit-mass variables V^k = R_k^{-1} U^k of the hidden
  // layers, Ghat^k = R_k R_k^T (Cholesky; R_0 = I): D_0 = -G^1,
  // D_l = -R_l^T (G^l + G^{l-1}) R_l, C_l = R_l^T G^l R_{l+1}
  std::vector<std::vector<double>> R(m);
  for (int k = 1; k < m; ++k) {
    R[k].assign(Ghat + k * bb2, Ghat + (k + 1) * bb2);
    REQUIRE(host_cholesky(b, R[k].data()), SFROM_ENOTSPD, "Ghat^k is not positive definite (eq. S-fraction)");
  }
  // X^T M Y for column-major b x b matrices; X or Y null means the identity
  auto congruence = [&](const double* X, const double* M, const double* Y, std::vector<double>& out) {
    std::vector<double> t(bb2);
    for (int i = 0; i < b; ++i)
      for (int j = 0; j < b; ++j) {
        double acc = 0.0;
        if (!Y) acc = M[i + (int64_t)j * b];
        else
          for (int q = 0; q < b; ++q) acc += M[i + (int64_t)q * b] * Y[q + (int64_t)j * b];
        t[i + (int64_t)j * b] = acc;
      }
    out.assign(bb2, 0.0);
    for (int i = 0; i < b; ++i)
      for (int j = 0; j < b; ++j) {
        double acc = 0.0;
        if (!X) acc = t[i + (int64_t)j * b];
        else
          for (int q = 0; q < b; ++q) acc += X[q + (int64_t)i * b] * t[q + (int64_t)j * b];
        out[i + (int64_t)j * b] = acc;
      }
  };
  const int ld = oc.ld;
  const int64_t bsz = (int64_t)b * ld;
  std::vector<double> blk((2 * m - 1) * bsz, 0.0);
  std::vector<double> M(bb2);
  for (int l = 0; l < m; ++l) {
    std::vector<double> Gs(G + l * bb2, G + (l + 1) * bb2);
    if (l > 0)
      for (int64_t q = 0; q < bb2; ++q) Gs[q] += G[(l - 1) * bb2 + q];
    congruence(l ? R[l].data() : nullptr, Gs.data(), l ? R[l].data() : nullptr, M);
    for (int r = 0; r < b; ++r)
      for (int c = 0; c < b; ++c)
        blk[2 * l * bsz + (int64_t)r * ld + c] = -0.5 * (M[r + (int64_t)c * b] + M[c + (int64_t)r * b]);
    if (l + 1 < m) {
      congruence(l ? R[l].data() : nullptr, G + l * bb2, R[l + 1].data(), M);
      for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) blk[(2 * l + 1) * bsz + (int64_t)r * ld + c] = M[r + (int64_t)c * b];
    }
  }
  const size_t eb = block_bytes(h->prec);
  unsigned char* dst = reinterpret_cast<unsigned char*>(h->d_blocks) + (size_t)oc.blk_off * eb;
  if (h->prec == SFROM_F64) {
    HIPCHK(hipMemcpy(dst, blk.data(), blk.size() * 8, hipMemcpyHostToDevice));
  } else if (h->prec == SFROM_F32) {
    std::vector<float> f(blk.begin(), blk.end());
    HIPCHK(hipMemcpy(dst, f.data(), f.size() * 4, hipMemcpyHostToDevice));
  } else {
    std::vector<uint16_t> bf(blk.size());
    for (size_t k = 0; k < blk.size(); ++k) {
      float f = (float)blk[k];
      uint32_t u;
      std::memcpy(&u, &f, 4);
      u += 0x7FFF + ((u >> 16) & 1);   // round to nearest even
      bf[k] = (uint16_t)(u >> 16);
    }
    HIPCHK(hipMemcpy(dst, bf.data(), bf.size() * 2, hipMemcpyHostToDevice));
  }
  h->masses_dirty = true;
  h->rom_imported = true;   // the cells' Gershgorin bound no longer covers these blocks
  h->lam_rom = -1.0;
  API_END(h)
}

int sfrom_save(sfrom_t* h, const char* path) {
  API_BEGIN(h)
  save_checkpoint(h, path);
  API_END(h)
}

int sfrom_load(sfrom_t* h, const char* path) {
  API_BEGIN(h)
  load_checkpoint(h, path);
  API_END(h)
}

int sfrom_export_rom(sfrom_t* h, int32_t cell, int32_t* m, int32_t* b, double* Ghat, double* G) {
  API_BEGIN(h)
  REQUIRE(h->built, SFROM_ESTATE, "no ROM: build first");
  REQUIRE(cell >= 0 && cell < (int)h->ocells.size() && m && b, SFROM_EINVAL, "bad cell");
  const OnlineCell& oc = h->ocells[cell];
  *m = oc.m;
  *b = oc.b;
  const int64_t bb2 = (int64_t)oc.b * oc.b;
  HIPCHK(hipStreamSynchronize(h->stream));
  if (Ghat) HIPCHK(hipMemcpy(Ghat, h->d_rom64 + h->rom64_off[cell], oc.m * bb2 * 8, hipMemcpyDeviceToHost));
  if (G) HIPCHK(hipMemcpy(G, h->d_rom64 + h->rom64_off[cell] + oc.m * bb2, oc.m * bb2 * 8, hipMemcpyDeviceToHost));
  API_END(h)
}

int sfrom_set_sources(sfrom_t* h, int32_t n_s, const int64_t* colptr, const int64_t* row, const double* val,
                      int32_t project) {
  API_BEGIN(h)
  REQUIRE(n_s > 0 && colptr && (colptr[n_s] == 0 || (row && val)), SFROM_EINVAL, "bad source arguments");
  finalize_partition(h);
  make_columns(h, h->src, n_s, colptr, row, val, project);
  h->src_dirty = true;
  h->fine_io_dirty = true;
  h->state_ns = -1;
  h->fine_ns = -1;
  API_END(h)
}

int sfrom_set_receivers(sfrom_t* h, int32_t n_r, const int64_t* colptr, const int64_t* row, const double* val,
                        int32_t project) {
  API_BEGIN(h)
  REQUIRE(n_r >= 0 && colptr && (colptr[n_r] == 0 || (row && val)), SFROM_EINVAL, "bad receiver arguments");
  finalize_partition(h);
  make_columns(h, h->rec, n_r, colptr, row, val, project);
  h->rec_dirty = true;
  h->fine_io_dirty = true;
  API_END(h)
}

int sfrom_point_columns(sfrom_t* h, int32_t count, const int64_t* node, int64_t* colptr_out, int64_t* row_out,
                        double* val_out) {
  API_BEGIN(h)
  REQUIRE(count >= 0 && node && colptr_out && row_out && val_out, SFROM_EINVAL, "bad arguments");
  finalize_partition(h);
  std::vector<int64_t> cp(count + 1, 0), rw;
  std::vector<double> vl;
  for (int j = 0; j < count; ++j) {
    const int64_t g = node[j];
    REQUIRE(g >= 0 && g < h->n, SFROM_EINVAL, "node out of range");
    const int32_t p = h->piece_of_node[g];
    REQUIRE(p >= 0, SFROM_ESUPPORT, "node " + std::to_string(g) + " is not on the skeleton (eq. gsupport)");
    const auto& pc = h->pieces[p];
    const int64_t kp = (int64_t)pc.gnode.size();
    const int32_t pos = h->pos_in_piece[g];
    for (int64_t r = 0; r < kp; ++r) {
      double s = 0.0;
      for (int l = 0; l < pc.b; ++l) s += pc.S[r + l * kp] * pc.S[pos + l * kp];
      rw.push_back(pc.gnode[r]);
      vl.push_back(s);
    }
    cp[j + 1] = (int64_t)rw.size();
  }
  std::memcpy(colptr_out, cp.data(), cp.size() * 8);
  if (!rw.empty()) {
    std::memcpy(row_out, rw.data(), rw.size() * 8);
    std::memcpy(val_out, vl.data(), vl.size() * 8);
  }
  API_END(h)
}

int sfrom_reset(sfrom_t* h) {
  API_BEGIN(h)
  REQUIRE(h->built, SFROM_ESTATE, "no ROM: build first");
  zero_state(h);
  API_END(h)
}

int sfrom_run(sfrom_t* h, int64_t n_steps, double dt, const double* w, int32_t w_on_device, void* traces,
              int32_t traces_on_device) {
  API_BEGIN(h)
  run(h, n_steps, dt, w, w_on_device, traces, traces_on_device);
  API_END(h)
}

int sfrom_run_noalloc(sfrom_t* h, int64_t n_steps, double dt, const double* w, void* traces) {
  API_BEGIN(h)
  run(h, n_steps, dt, w, 1, traces, 1, true);
  API_END(h)
}

int sfrom_fine_reset(sfrom_t* h) {
  API_BEGIN(h)
  h->fine_ns = -1;
  API_END(h)
}

int sfrom_fine_run(sfrom_t* h, int64_t n_steps, double dt, const double* w, int32_t w_on_device, void* traces,
                   int32_t traces_on_device, int32_t prec) {
  API_BEGIN(h)
  fine_run(h, n_steps, dt, w, w_on_device, traces, traces_on_device, prec);
  API_END(h)
}

int sfrom_fine_lambda_max(sfrom_t* h, double* lambda) {
  API_BEGIN(h)
  REQUIRE(h->n > 0 && lambda, SFROM_ESTATE, "no pencil");
  const int64_t n = h->n;
  std::vector<double> d(n);
  for (int64_t i = 0; i < n; ++i) d[i] = 1.0 / std::sqrt(h->b[i]);
  auto mv = [&](const double* x, double* y) {
    for (int64_t i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int64_t k = h->rowptr[i]; k < h->rowptr[i + 1]; ++k) acc += h->a[k] * d[h->col[k]] * x[h->col[k]];
      y[i] = -d[i] * acc;
    }
  };
  *lambda = lanczos_max(n, mv);
  API_END(h)
}

int sfrom_rom_lambda_max(sfrom_t* h, double* lambda) {
  API_BEGIN(h)
  REQUIRE(h->built && lambda, SFROM_ESTATE, "no ROM: build first");
  *lambda = rom_lambda_exact(h);
  API_END(h)
}

int sfrom_set_graph(sfrom_t* h, int32_t enable) {
  API_BEGIN(h)
  REQUIRE(h->device >= 0, SFROM_EDEVICE, "host-only handle");
  h->use_graph = enable != 0;
  if (!h->use_graph && h->graph_exec) { hipGraphExecDestroy(h->graph_exec); h->graph_exec = nullptr; h->graph_key.clear(); }
  API_END(h)
}

int sfrom_set_corner_correction(sfrom_t* h, int32_t enable) {
  API_BEGIN(h)
  REQUIRE(enable == 0 || enable == 1, SFROM_EINVAL, "enable must be 0 or 1");
  REQUIRE(!enable || !h->cmap.corner.empty(), SFROM_ESTATE, "no corner set was removed: call sfrom_remove_corner_set");
  if ((enable != 0) != h->corner_corr) {
    drop_graph(h);
    h->corner_corr = enable != 0;
    h->rec_dirty = true;
  }
  API_END(h)
}

int sfrom_set_persistent(sfrom_t* h, int32_t enable) {
  API_BEGIN(h)
  REQUIRE(enable == 0 || enable == 1, SFROM_EINVAL, "enable must be 0 or 1");
  if ((enable != 0) != h->persistent) drop_graph(h);
  h->persistent = enable != 0;
  API_END(h)
}

int sfrom_set_breakdown_policy(sfrom_t* h, int32_t reduce_m) {
  API_BEGIN(h)
  REQUIRE(reduce_m == 0 || reduce_m == 1, SFROM_EINVAL, "reduce_m must be 0 or 1");
  h->reduce_m_on_breakdown = reduce_m != 0;
  API_END(h)
}

int sfrom_set_build_path(sfrom_t* h, int32_t mode) {
  API_BEGIN(h)
  REQUIRE(mode >= 0 && mode <= 2, SFROM_EINVAL, "mode must be 0 (automatic), 1 (blocked wide-band) or 2 (per-cell)");
  h->wide_mode = mode;
  API_END(h)
}

int sfrom_set_cell_variant(sfrom_t* h, int32_t variant) {
  API_BEGIN(h)
  REQUIRE(variant >= -1 && variant < 6, SFROM_EINVAL, "variant must be -1 (autotune) or 0..5");
  h->pinned_variant = variant;
  API_END(h)
}

int sfrom_profile(sfrom_t* h, int32_t enable) {
  API_BEGIN(h)
  REQUIRE(h->device >= 0, SFROM_EDEVICE, "host-only handle");
  REQUIRE(enable >= 0, SFROM_EINVAL, "profile interval must be >= 0");
  collect_events(h);
  h->profiling = enable != 0;
  h->prof_every = enable > 1 ? enable : 1;
  API_END(h)
}

int sfrom_profile_read(sfrom_t* h, int32_t kernel, double* total_ms, int64_t* launches) {
  API_BEGIN(h)
  REQUIRE(kernel >= 0 && kernel < 4 && total_ms && launches, SFROM_EINVAL, "bad kernel id");
  if (h->device >= 0) collect_events(h);
  *total_ms = h->prof_ms[kernel];
  *launches = h->prof_n[kernel];
  h->prof_ms[kernel] = 0.0;
  h->prof_n[kernel] = 0;
  API_END(h)
}

int sfrom_get_info(const sfrom_t* hc, sfrom_info* info) {
  if (!hc || !info) return SFROM_EINVAL;
  sfrom_t* h = const_cast<sfrom_t*>(hc);
  std::memset(info, 0, sizeof(*info));
  info->n = h->n;
  info->nnz = h->rowptr.empty() ? 0 : h->rowptr.back();
  info->n_cells = (int32_t)h->cells.size();
  info->n_pieces = (int32_t)h->pieces.size();
  info->n_piece_dofs = h->piece_dof_off.empty() ? 0 : h->piece_dof_off.back();
  info->n_hidden_dofs = h->built ? h->n_hidden_dofs : 0;
  for (int32_t b : h->cell_b) info->max_b = std::max(info->max_b, b);
  for (int32_t m : h->cell_m) info->max_m = std::max(info->max_m, m);
  info->n_sources = h->src.count;
  info->n_receivers = h->rec.count;
  info->built = h->built ? 1 : 0;
  info->online_prec = h->prec;
  info->block_bytes = h->built ? h->block_elems * (int64_t)block_bytes(h->prec) : 0;
  info->build_ms = h->build_ms;
  info->cell_variant = h->tuned_variant;
  info->steps_done = h->steps_done;
  return SFROM_OK;
}

int sfrom_export_pencil(sfrom_t* h, int64_t* rowptr, int32_t* col, double* a, double* b) {
  API_BEGIN(h)
  REQUIRE(h->n > 0, SFROM_ESTATE, "no pencil");
  if (rowptr) std::memcpy(rowptr, h->rowptr.data(), h->rowptr.size() * 8);
  if (col) std::memcpy(col, h->col.data(), h->col.size() * 4);
  if (a) std::memcpy(a, h->a.data(), h->a.size() * 8);
  if (b) std::memcpy(b, h->b.data(), h->b.size() * 8);
  API_END(h)
}

int sfrom_export_cell(sfrom_t* h, int32_t cell, int32_t* n_i, int32_t* nnz_i, int32_t* b_dim, int64_t* global_node,
                      int32_t* rowptr_i, int32_t* col_i, double* a_i, double* b_i) {
  API_BEGIN(h)
  REQUIRE(cell >= 0 && cell < (int)h->cells.size() && h->cells[cell].defined, SFROM_EINVAL, "bad cell");
  finalize_partition(h);
  const CellDef& c = h->cells[cell];
  if (n_i) *n_i = c.n;
  if (nnz_i) *nnz_i = (int32_t)c.a.size();
  if (b_dim) *b_dim = h->cell_b[cell];
  if (global_node) std::memcpy(global_node, c.gnode.data(), c.gnode.size() * 8);
  if (rowptr_i) std::memcpy(rowptr_i, c.rowptr.data(), c.rowptr.size() * 4);
  if (col_i) std::memcpy(col_i, c.col.data(), c.col.size() * 4);
  if (a_i) std::memcpy(a_i, c.a.data(), c.a.size() * 8);
  if (b_i) std::memcpy(b_i, c.b.data(), c.b.size() * 8);
  API_END(h)
}

int sfrom_export_piece(sfrom_t* h, int32_t piece, int32_t* k_p, int32_t* b_p, int64_t* global_node, double* S_p) {
  API_BEGIN(h)
  REQUIRE(piece >= 0 && piece < (int)h->pieces.size() && h->pieces[piece].defined, SFROM_EINVAL, "bad piece");
  const PieceDef& p = h->pieces[piece];
  if (k_p) *k_p = (int32_t)p.gnode.size();
  if (b_p) *b_p = p.b;
  if (global_node) std::memcpy(global_node, p.gnode.data(), p.gnode.size() * 8);
  if (S_p) std::memcpy(S_p, p.S.data(), p.S.size() * 8);
  API_END(h)
}

}  // extern "C"
