// Internal definitions of libsfrom shared by the host C++ and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/sfrom.h"

namespace sfrom_impl {

// ---------------------------------------------------------------------------
// Problem description (host)
// ---------------------------------------------------------------------------

struct CellDef {
  bool defined = false;
  int32_t n = 0;
  std::vector<int64_t> gnode;     // local -> global node
  std::vector<int32_t> rowptr;    // local CSR of A_i
  std::vector<int32_t> col;
  std::vector<double> a;
  std::vector<double> b;          // diag(B_i)
};

struct PieceDef {
  bool defined = false;
  std::vector<int64_t> gnode;     // global nodes, k_p
  int32_t b = 0;                  // basis size b_p
  std::vector<double> S;          // k_p x b_p column-major
};

// Columns (sources or receivers) after restriction to the skeleton.
struct Columns {
  int32_t count = 0;
  std::vector<int64_t> colptr, row;   // fine-grid CSC (possibly projected)
  std::vector<double> val;
  // reduced coefficients: per column, list of (piece, coeff[b_p])
  std::vector<int64_t> rptr;          // per column into rpiece
  std::vector<int32_t> rpiece;
  std::vector<int64_t> rcoff;         // offset into rcoef for each (column, piece)
  std::vector<double> rcoef;
};

// Per-cell descriptor of the off-line workspace (device), all offsets in doubles.
struct BuildCell {
  int32_t n;        // local nodes
  int32_t b;        // boundary dimension
  int32_t m;        // layers
  int32_t w;        // lower bandwidth
  int32_t nnz;      // local CSR nonzeros
  int32_t nw;       // number of skeleton rows (entries of the W map)
  int64_t csr_off;  // into rowptr-free arrays (rowptr stored separately)
  int64_t rp_off;   // into rowptr array (n+1 entries)
  int64_t w_off;    // into the W map arrays
  int64_t b_off;    // into diag(B_i) array
  int64_t band_off; // band storage n*(w+1)
  int64_t v_off;    // V: n x m b
  int64_t x_off;    // X: n x b (work) and B q
  int64_t av_off;   // A V: n x m b (reused as Lanczos work)
  int64_t am_off;   // A^m: (m b)^2
  int64_t q_off;    // Lanczos Q: (m b) x (m b)
  int64_t s_off;    // small work: 8 b^2 + ...
  int64_t r_off;    // R_j factors: m b^2 (R_1 = beta_1)
  int64_t out_off;  // S-fraction output: 2 m b^2 (Ghat^1..m then G^1..m)
  int32_t status;   // per-cell status (written by kernels)
  int32_t fail_block; // on a rank loss: the 1-based Krylov / Lanczos block that lost rank
  int64_t p_off;    // blocked build only: partial Gram products, ceil(n / TS_ROWS) x max((m b)^2, m b^2)
  int64_t li_off;   // blocked build only: inverse of each 64 x 64 diagonal factor block, ceil(n / 64) x 64^2
};

// Per-cell on-line descriptor.
struct OnlineCell {
  int32_t m, b;
  int32_t ld;        // row stride of every stored block (b rounded up to 4, zero padded)
  int32_t pad_;
  int64_t blk_off;   // elements into the block array: D_0, C_0, ..., D_{m-1} (b x ld each)
  int64_t hid_off;   // padded rows into the hidden state: layer l >= 1 of the
                     // cell is an n_s x ld block (source-major, rows b..ld-1
                     // zero) starting at element (hid_off + (l-1) ld) n_s
  int64_t u1_off;    // rows into the gather map / phi scratch (b rows)
};

// Per-piece on-line descriptor.
struct OnlinePiece {
  int32_t b;         // b_p
  int32_t ncell;     // incident cells
  int64_t dof_off;   // rows into the piece state
  int64_t inc_off;   // into the incidence array (phi base rows), ncell entries
  int64_t minv_off;  // elements into M_p^{-1} (b_p x b_p)
  int64_t src_off;   // rows into the dense reduced-source array, -1 if none
};

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files)
// ---------------------------------------------------------------------------

// Off-line build of a batch of cells. Returns hipError_t; per-cell status in
// the device BuildCell array.
struct BuildBatch {
  int32_t ncell;
  int32_t max_m, max_b, max_n;
  int32_t max_w;              // largest band width of the batch's cells
  double shift;
  BuildCell* d_cells;
  const int32_t* d_rowptr;
  const int32_t* d_col;
  const double* d_a;
  const double* d_bdiag;
  const int32_t* d_wrow;      // skeleton rows of the cell
  const int32_t* d_wcol;      // first column of the row's piece block in W
  const int64_t* d_wsoff;     // offset of S_p row for this node (S_p + pos) in d_S
  const int32_t* d_wbp;       // b_p of that piece
  const int32_t* d_wkp;       // k_p (leading dimension of S_p)
  const double* d_S;
  double* d_work;
  int32_t wide_mode;          // 0: blocked wide-band kernels when max_w > WIDE_MIN_W; 1: always; 2: never
};
hipError_t launch_build(const BuildBatch& bb, hipStream_t st);
// Blocked band factorisation and shifted solves over many workgroups per
// cell (wide.hip), used for bands wider than WIDE_MIN_W.
constexpr int WIDE_MIN_W = 128;
// Rows per partial Gram product of the blocked build (a cell's n rows are
// split into ceil(n / TS_ROWS) chunks summed in a fixed order).
constexpr int TS_ROWS = 4096;
inline int64_t ts_partials(int64_t n, int64_t m, int64_t b) {
  const int64_t mb = m * b;
  return ((n + TS_ROWS - 1) / TS_ROWS) * (mb * mb > mb * b ? mb * mb : mb * b);
}
bool build_is_wide(const BuildBatch& bb, int force);
hipError_t launch_wide_chol(const BuildBatch& bb, hipStream_t st);
hipError_t launch_wide_solve(const BuildBatch& bb, int j, hipStream_t st);
// Tall-skinny steps of the blocked build: Gram products A^T diag(d) B
// (mode TS_CGS: V[:, 0:jb]^T B X into the CGS coefficients; TS_NORM: X^T B X
// into the Gram matrix; TS_PROJ: V^T (A V) into A^m), the CGS update
// X -= V coef, q_j = X L^{-T} and the sparse product A V.
enum { TS_CGS = 0, TS_NORM = 1, TS_PROJ = 2 };
hipError_t launch_ts_gram(const BuildBatch& bb, int mode, int j, hipStream_t st);
hipError_t launch_ts_update(const BuildBatch& bb, int j, hipStream_t st);
hipError_t launch_ts_trsm_rows(const BuildBatch& bb, int j, hipStream_t st);
hipError_t launch_ts_spmm(const BuildBatch& bb, hipStream_t st);

// Learned off-line stage (cells of one batch): S-fraction from the
// predicted factors y (one row of P floats per cell), its on-line blocks in
// FP64 and the transfer-function mismatch against the exact cell transfer
// function at the nz points z[] (max into mis[cell], which the caller
// zeroes).
hipError_t launch_learned_check(const BuildBatch& bb, const float* y, int P, const double* z, int nz, double* mis,
                                hipStream_t st);
// Packs the cells with take[cell] != 0 from their FP64 on-line blocks.
hipError_t launch_pack_normal(int32_t ncell, const BuildCell* d_bcells, const double* d_work,
                              const OnlineCell* d_ocells, const int32_t* d_take, int32_t prec, void* d_blocks,
                              double* d_rom64, const int64_t* d_rom64_off, hipStream_t st);
// Cholesky-factor targets (P floats per cell) of built cells.
hipError_t launch_factor_targets(const double* d_rom64, const int64_t* d_rom64_off, const int32_t* d_cells, int n,
                                 int b, int m, double* d_scratch, float* d_out, int P, int32_t* d_bad,
                                 hipStream_t st);

// Pack the double S-fraction of one batch into the on-line layout.
hipError_t launch_pack(int32_t ncell, BuildCell* d_bcells, double* d_work,
                       const OnlineCell* d_ocells, int32_t prec, void* d_blocks,
                       double* d_rom64, const int64_t* d_rom64_off, hipStream_t st);

// Piece masses M_p^{-1} from Ghat^1 of the incident cells.
struct MassArgs {
  int32_t npiece;
  const OnlinePiece* d_pieces;
  const int32_t* d_inc_cell;     // incident cell id per incidence entry
  const int32_t* d_inc_col;      // column offset of the piece inside that cell
  const OnlineCell* d_cells;
  const double* d_rom64;         // per cell Ghat^1..m, G^1..m (double)
  const int64_t* d_rom64_off;
  int32_t prec;
  void* d_minv;                  // output in on-line precision
  int32_t* d_status;             // per piece status
  double* d_scratch;             // 3 * sum_p b_p^2 doubles
};
hipError_t launch_piece_mass(const MassArgs& a, hipStream_t st);

// One on-line leapfrog step.
struct StepArgs {
  int32_t ncell, npiece, ns, nrec;
  int32_t prec;
  int32_t max_b, max_m, max_bp;
  double dt2;
  const OnlineCell* d_cells;
  const OnlinePiece* d_pieces;
  const int32_t* d_gather;       // per cell boundary row -> piece dof row
  const int64_t* d_inc;          // phi base rows per piece incidence
  const void* d_blocks;
  const void* d_minv;
  const void* d_src;             // dense reduced sources of source pieces
  void* y_cur;                   // piece state level n   (read)
  void* y_old;                   // piece state level n-1 (overwritten by n+1)
  void* h_cur;                   // hidden level n
  void* h_old;                   // hidden level n-1 (overwritten by n+1)
  void* phi;                     // phi scratch, sum_i b_i rows
  const double* w;               // device wavelet samples
  int64_t step;                  // index into w
  // receivers (CSR over piece dofs)
  const int64_t* d_rptr;
  const int64_t* d_rrow;
  const double* d_rval;
  void* traces;                  // n_steps x n_rec x ns
  int64_t trace_step;            // which slice to write
  // receivers computed by the piece phase (each receiver reads one piece):
  // receivers d_prec_list[d_prec_ptr[p] .. d_prec_ptr[p+1]) belong to piece
  // p; null when the receivers kernel runs instead
  const int32_t* d_prec_ptr;
  const int32_t* d_prec_list;
  int32_t cell_variant;          // kernel variant of the cell phase (autotuned)
  // cell phase over a subset: cells d_cell_list[0..nlist) (all cells, in
  // order, when d_cell_list is null and nlist == ncell)
  const int32_t* d_cell_list;
  int32_t nlist;
};
hipError_t launch_online_step(const StepArgs& a, hipStream_t st);
// Persistent on-line kernel (one cooperative launch for n_steps steps): the
// two state levels of the piece dofs and hidden layers, the level that holds
// step 0's current state, and whether the piece phase computes the traces.
struct PersistArgs {
  int64_t n_steps;
  int32_t cur0, rec_fused;
  void* y[2];
  void* h[2];
};
// FP32 or FP64, max_b <= 144 and max_bp <= 16
bool persistent_supported(const StepArgs& a);
hipError_t launch_persistent(const StepArgs& a, const PersistArgs& pa, hipStream_t st);
// Correction at the corner-set nodes (App. D) on the piece state y (level
// n + 1, after the piece phase): for corner node k with hanging copies
// t = hptr[k] .. hptr[k+1], u_t = S_p(row of t, :) y_p and
// delta_t = sum_t' w_t' u_t' - u_t (kernels 1 and 2: values per copy, then
// means and differences per removed node); then for each piece q holding
// copies, y_q += sum over its copies t of S_q(row of t, :)^T delta_t
// (kernel 3, one thread per dof row of such a piece and source). Values
// (rows, weights, delta, y) are in the state precision.
struct CornerArgs {
  int32_t ncorner, npiece, nrow, ns, prec;
  int64_t ncopy;
  const int32_t* rowq;    // nrow: piece (index into pptr) of each dof row
  const int32_t* rowj;    // nrow: the row's index j < b_p within its piece
  const int32_t* hptr;    // ncorner + 1
  const int64_t* hdof;    // per copy: first dof row of its piece
  const int32_t* hbp;     // per copy: b_p of its piece
  const int64_t* soff;    // per copy: offset of its basis row in srow
  const void* srow;       // basis rows, b_p values per copy
  const void* hw;         // per copy: weight b'_l / b_k
  const int32_t* pptr;    // npiece + 1: copies of each piece that holds copies
  const int32_t* plist;   // copy ids, ascending within a piece
  const int64_t* pdof;    // per such piece: first dof row
  const int32_t* pbp;     // per such piece: b_p
  void* delta;            // ncopies x ns
  void* y;                // piece state, n_piece_dofs x ns
};
hipError_t launch_corner_correction(const CornerArgs& c, hipStream_t st);
// the three parts of a step, for per-kernel timing
hipError_t launch_cell_phase(const StepArgs& a, hipStream_t st);
hipError_t launch_piece_phase(const StepArgs& a, hipStream_t st);
hipError_t launch_receivers(const StepArgs& a, hipStream_t st);
// Surrogate network (surrogate.hip): number of outputs, and BF16-operand
// prediction of the unnormalised outputs for n inputs (device pointers).
int surrogate_outputs(const sfrom_surrogate* s);
hipError_t surrogate_predict(sfrom_surrogate* s, const float* x, int n, float* out);
// ORs 1 into *flag if any of n state values (double for F64, else float) is
// not finite
hipError_t launch_nonfinite(const void* x, int64_t n, int prec, int32_t* flag, hipStream_t st);
hipError_t launch_zero_flag(int32_t* flag, hipStream_t st);
int cell_variants(const StepArgs& a);

// Fine-grid leapfrog step (CSR).
struct FineArgs {
  int64_t n;
  int32_t ns, nrec, prec;
  double dt2;
  const int64_t* rowptr;
  const int32_t* col;
  const void* a;                 // values in precision prec
  const void* binv;              // 1/b in precision prec
  void* u_cur;
  void* u_old;                   // overwritten by level n+1
  const double* w;
  int64_t step;
  int64_t nsrc_entries;
  const int64_t* src_row;        // source entries (node, source, value)
  const int32_t* src_col;
  const double* src_val;
  const int64_t* rec_ptr;        // receivers CSC over nodes
  const int64_t* rec_row;
  const double* rec_val;
  void* traces;
  int64_t trace_step;
  // Cartesian 7-point form (when stencil != nullptr): unknown grid ux x uy x uz,
  // x fastest, 8 coefficients per node: A to x-, x+, y-, y+, z-, z+, diag, 1/b
  const void* stencil;
  int32_t ux, uy, uz;
  // point sources of the Cartesian form: per node the row of src_dense
  // (n_s values of precision prec) that its flux adds w^n times, or -1
  const int32_t* src_idx;
  const void* src_dense;
  int32_t src_dense_ok;          // src_idx / src_dense are set (2.5D kernel usable)
};
hipError_t launch_fine_step(const FineArgs& a, hipStream_t st);
// The Cartesian step of n_s a multiple of 64 is one launch that also writes
// the traces of the level it reads (trace step - 1); the traces of a run's
// last level then need this launch (u_cur = that level, trace_step).
bool fine_uses_25d(const FineArgs& a);
// Nodes of padding after the fine state (n_s values each), stencil (8
// values each) and source-index (1 each) arrays of the Cartesian kernel.
constexpr int FINE_PAD = 64;
hipError_t launch_fine_rec_level(const FineArgs& a, hipStream_t st);

}  // namespace sfrom_impl

struct sfrom {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;

  // pencil
  int64_t n = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> a, b;

  std::vector<sfrom_impl::CellDef> cells;
  std::vector<sfrom_impl::PieceDef> pieces;

  // derived partition
  bool part_ready = false;
  std::vector<int32_t> piece_of_node;       // n, -1 off skeleton
  std::vector<int32_t> pos_in_piece;        // n
  std::vector<std::vector<int32_t>> cell_pieces;   // ascending piece ids
  std::vector<std::vector<int32_t>> cell_piece_col;// column offset of each piece in W_i
  std::vector<int32_t> cell_b;
  std::vector<std::vector<int32_t>> piece_cells;   // ascending cell ids
  std::vector<int64_t> piece_dof_off;              // n_pieces + 1

  // Cell operators, skeleton maps and piece bases staged in HBM for the
  // off-line build: uploaded once per partition and shared by every build,
  // each cell addressed by its offsets into the concatenated arrays.
  struct CellStage {
    bool ready = false;
    int32_t* d_rowptr = nullptr;   // per cell n_i + 1 local row starts
    int32_t* d_col = nullptr;
    double* d_a = nullptr;
    double* d_bdiag = nullptr;
    int32_t* d_wrow = nullptr;     // skeleton rows of W_i: local row, column, basis entry
    int32_t* d_wcol = nullptr;
    int64_t* d_wsoff = nullptr;
    int32_t* d_wbp = nullptr;
    int32_t* d_wkp = nullptr;
    double* d_S = nullptr;         // piece bases, piece after piece
    std::vector<int64_t> rp_off, csr_off, b_off, w_off;
    std::vector<int32_t> nw, bw;   // skeleton rows and half bandwidth per cell
    std::vector<int64_t> soff;     // offset of each piece basis in d_S
  };
  CellStage stage;
  // Upper bound of the largest eigenvalue of every cell's local pencil
  // (Gershgorin discs of B_i^{-1}(-A_i)); -1 until computed for the current
  // partition. Each cell's S-fraction is a Galerkin projection of that
  // pencil and the global ROM an assembly of the cells' ROMs, so the bound
  // also bounds the ROM's largest eigenvalue (used by the CFL check).
  double lam_cells = -1.0;

  // Corner-set removal (App. B): for each removed node of the pencil before
  // the removal (old numbering, ascending) its hanging copies (new
  // numbering) and their weights b'_l / b_k; old nodes kept map one to one
  struct CornerMap {
    int64_t n_old = 0;
    std::vector<int64_t> new_of_old;   // n_old, -1 at removed nodes
    std::vector<int64_t> corner;       // removed old nodes, ascending
    std::vector<int64_t> hptr;         // corner.size() + 1
    std::vector<int64_t> hnode;        // copies, new numbering
    std::vector<double> hweight;
  };
  CornerMap cmap;
  // on-line steps of a run in one cooperative persistent launch
  bool persistent = false;
  // App. D correction after every on-line step, and its device arrays
  // (staged from the built ROM's piece bases on the first run)
  bool corner_corr = false;
  struct CornerStage {
    bool ready = false;
    int32_t ncorner = 0, npiece = 0, nrow = 0;
    int64_t ncopy = 0;
    int32_t *d_hptr = nullptr, *d_hbp = nullptr, *d_pptr = nullptr, *d_plist = nullptr, *d_pbp = nullptr;
    int32_t *d_rowq = nullptr, *d_rowj = nullptr;
    int64_t *d_hdof = nullptr, *d_soff = nullptr, *d_pdof = nullptr;
    void *d_srow = nullptr, *d_hw = nullptr, *d_delta = nullptr;
    int32_t delta_ns = -1;
  };
  CornerStage cstage;

  // a cell whose rational Krylov or Lanczos block k (>= 2) loses rank is
  // rebuilt with m_i = k - 1 instead of failing the build
  bool reduce_m_on_breakdown = false;
  std::vector<std::pair<int32_t, int32_t>> breakdowns;   // (cell, failing block) of the last failed batch

  // ROM
  bool built = false;
  bool rom_imported = false;   // some cell's blocks came from sfrom_import_rom
  double lam_rom = -1.0;       // largest eigenvalue of the ROM pencil, once computed
  int64_t steps_done = 0;      // on-line steps since the last reset
  int32_t prec = SFROM_F32;
  std::vector<int32_t> cell_m;
  double shift = 0.0;
  double build_ms = 0.0;
  int64_t n_hidden_dofs = 0;   // sum of (m-1) b
  int64_t n_hidden_rows = 0;   // sum of (m-1) ld (padded state rows)
  int64_t block_elems = 0;
  std::vector<sfrom_impl::OnlineCell> ocells;
  std::vector<sfrom_impl::OnlinePiece> opieces;
  std::vector<int64_t> rom64_off;                  // per cell into d_rom64

  // device: on-line structures
  void* d_blocks = nullptr;
  int32_t* d_prec_ptr = nullptr;   // per-piece receiver lists (receivers fused into the piece phase)
  int32_t* d_prec_list = nullptr;
  bool rec_fused = false;
  void* d_minv = nullptr;
  double* d_rom64 = nullptr;
  int64_t* d_rom64_off = nullptr;
  sfrom_impl::OnlineCell* d_ocells = nullptr;
  sfrom_impl::OnlinePiece* d_opieces = nullptr;
  int32_t* d_gather = nullptr;
  int64_t* d_inc = nullptr;
  int32_t* d_inc_cell = nullptr;
  int32_t* d_inc_col = nullptr;
  bool masses_dirty = true;

  // sources / receivers
  sfrom_impl::Columns src, rec;
  bool src_dirty = true, rec_dirty = true;
  // ROM-side device I/O
  void* d_src = nullptr;          // dense reduced sources (rows of source pieces)
  int64_t* d_rptr = nullptr;      // receivers over piece dofs
  int64_t* d_rrow = nullptr;
  double* d_rval = nullptr;
  int32_t state_ns = -1;          // n_s the state buffers are sized for
  void* d_y[2] = {nullptr, nullptr};
  void* d_h[2] = {nullptr, nullptr};
  void* d_phi = nullptr;
  int32_t* d_flag = nullptr;  // non-finite state flag
  int cur = 0;                    // which buffer holds level n
  double* d_w = nullptr;
  int64_t d_w_cap = 0;

  // fine comparator
  int32_t fine_prec = -1;
  int32_t fine_ns = -1;
  int64_t* d_frowptr = nullptr;
  int32_t* d_fcol = nullptr;
  void* d_fa = nullptr;
  void* d_fbinv = nullptr;
  void* d_u[2] = {nullptr, nullptr};
  int fcur = 0;
  int64_t* d_fsrc_row = nullptr;
  int32_t* d_fsrc_col = nullptr;
  double* d_fsrc_val = nullptr;
  int64_t fsrc_n = 0;
  int32_t* d_fsrc_idx = nullptr;   // Cartesian form: source row per node (-1: none)
  void* d_fsrc_dense = nullptr;    // and the rows, n_s values each (fine precision)
  int32_t fsrc_dense_prec = -1;
  int64_t* d_frec_ptr = nullptr;
  int64_t* d_frec_row = nullptr;
  double* d_frec_val = nullptr;
  bool fine_io_dirty = true;
  // Cartesian structure of the pencil (set by the voxel set-up)
  int32_t grid_u[3] = {0, 0, 0};
  std::vector<double> stencil;      // 8 per node, see FineArgs
  void* d_stencil = nullptr;

  // optional per-kernel timing with HIP events (kernel ids: 0 cell phase,
  // 1 piece phase, 2 receivers, 3 fine step)
  bool profiling = false;
  int32_t prof_every = 1;          // while profiling, steps timed: one in prof_every
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending[4];
  double prof_ms[4] = {0, 0, 0, 0};
  // autotuned cell-phase variant per (precision, max_b, max_m, n_s)
  std::map<std::tuple<int, int, int, int>, int> tuned;
  // cells grouped by the row-strip count of the matrix-core kernel they
  // need; one cell-phase launch (and autotuned variant) per group
  struct CellBucket {
    int32_t max_b = 0, max_m = 0, count = 0, variant = -1;
    int32_t* d_list = nullptr;
  };
  std::vector<CellBucket> buckets;
  int tuned_variant = -1;
  float tuned_ms = 0.f;

  // hipGraph form of sfrom_run: the whole run is captured once and replayed
  // while its arguments (and the state buffers and their parity) are unchanged
  bool use_graph = false;
  hipStream_t capture_stream = nullptr;   // private stream used for capture
  int pinned_variant = -1;                 // >= 0: cell-phase variant fixed by the caller
  int wide_mode = 0;                       // band kernels of the build: 0 automatic, 1 blocked, 2 per-cell
  hipGraphExec_t graph_exec = nullptr;
  std::vector<int64_t> graph_key;
  int64_t graph_launches = 0;
  int64_t prof_n[4] = {0, 0, 0, 0};
};
