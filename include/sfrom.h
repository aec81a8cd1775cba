/*
 * sfrom.h - C ABI of libsfrom, a gfx950 (MI355X) implementation of the
 * multi-scale S-fraction reduced-order model (ROM) for wavefield simulation
 * of Druskin, Mamonov and Zaslavsky.
 *
 * Problem statement (Sec. 1, eq. wave_fll): a fine-grid pencil with sparse
 * symmetric A <= 0 and diagonal B > 0, time-domain model B u'' = A u + w(t) g
 * with u = 0 for t <= 0, source columns g and receiver columns q supported on
 * the partition skeleton (Sec. 2, eq. gsupport), and a coarse-cell partition
 * with a splitting A = sum_i P_i A_i P_i^T, B = sum_i P_i B_i P_i^T
 * (eq. splitN_c). The library builds each cell's matrix S-fraction off-line
 * (Alg. alg1red stage 1) and time steps the coupled ROM on-line (stage 2).
 * A fine-grid leapfrog of the same pencil is provided as the comparator.
 *
 * Conventions
 *  - Every function returns an sfrom_status (0 = OK, < 0 = error) and never
 *    throws across the ABI; sfrom_last_error() holds a message for the last
 *    failing call on the handle.
 *  - Input arrays are caller-owned, read during the call and never retained.
 *    Output arrays are caller-owned. "host" pointers are ordinary CPU memory;
 *    "device" pointers are HIP device memory of the handle's device (for
 *    example a torch tensor's data_ptr()).
 *  - Work is enqueued on the stream given at creation. Calls that return
 *    host data synchronise that stream before returning. A handle is used by
 *    one thread at a time.
 *  - Dense matrices are column-major unless stated otherwise.
 *  - Sign convention: the source enters as +w(t) g (the paper writes the
 *    impulse on the other side of the equation; the sign is common to the
 *    fine model and the ROM and does not change any comparison).
 */
#ifndef SFROM_H
#define SFROM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfrom sfrom_t;

typedef enum {
  SFROM_OK = 0,
  SFROM_EINVAL = -1,      /* bad argument (size, index, null pointer)            */
  SFROM_ENOTSYM = -2,     /* A or A_i not symmetric                              */
  SFROM_ENOTNSD = -3,     /* A_i not <= 0 (diagonal dominance / Cholesky fails)  */
  SFROM_EBPOS = -4,       /* B or B_i not > 0                                    */
  SFROM_ESUPPORT = -5,    /* source/receiver nonzero off the skeleton (gsupport) */
  SFROM_EBREAKDOWN = -6,  /* Krylov/Lanczos block lost rank (Assumption 1)       */
  SFROM_ENOTSPD = -7,     /* S-fraction pivot not SPD (Assumption 2)             */
  SFROM_ECFL = -8,        /* dt above the leapfrog stability limit               */
  SFROM_ENONFINITE = -9,  /* NaN/Inf in an input or in the state                 */
  SFROM_EDEVICE = -10,    /* HIP runtime error                                   */
  SFROM_ESTATE = -11,     /* call out of order (e.g. run before build)           */
  SFROM_ENOMEM = -12,     /* device or host allocation failed                    */
  SFROM_ESPLIT = -13      /* sum of cell operators does not reproduce (A, B)     */
} sfrom_status;

/* Arithmetic of the on-line stage. F64: blocks and state in double.
 * F32: blocks and state in float. BF16: blocks in bfloat16, state and
 * accumulation in float. The off-line build is always double. */
typedef enum { SFROM_F64 = 0, SFROM_F32 = 1, SFROM_BF16 = 2 } sfrom_prec;

/* Create a handle on HIP device `device`; `hip_stream` is a hipStream_t (or
 * NULL for the null stream) on which all work is enqueued. device == -1
 * creates a host-only handle: problem set-up, validation and the export
 * calls work, every call that needs the GPU returns SFROM_EDEVICE. On
 * failure *out is NULL and sfrom_last_error(NULL) names the HIP call that
 * failed and its error (per calling thread). */
int sfrom_create(sfrom_t** out, int device, void* hip_stream);
void sfrom_destroy(sfrom_t* h);
/* Message for the last failing call on h, valid until the next call on h;
 * with h == NULL, why the calling thread's last sfrom_create failed. */
const char* sfrom_last_error(const sfrom_t* h);

/* ---------------------------------------------------------------------------
 * Problem definition (host data)
 * ------------------------------------------------------------------------ */

/* Fine pencil (Sec. 1, eq. wave_fll): A as CSR with both triangles, n rows,
 * rowptr[n+1] (int64), col[nnz] (int32, sorted within a row), a[nnz];
 * b[n] = diag(B). Replaces any previous pencil and partition.
 * Errors: EINVAL (shape), ENOTSYM, EBPOS, ENONFINITE. */
int sfrom_set_pencil(sfrom_t* h, int64_t n, const int64_t* rowptr, const int32_t* col,
                     const double* a, const double* b);

/* Coarse cell `cell` (0-based, added in any order, each once) with n_i local
 * nodes: global_node[n_i] maps local -> global node; (rowptr_i[n_i+1],
 * col_i, a_i) is A_i as local CSR with both triangles, b_i[n_i] = diag(B_i)
 * (eq. splitN_c). A node shared by two or more cells is a skeleton node.
 * The split is checked against the pencil at build time (ESPLIT).
 * Errors: EINVAL, ENOTSYM, EBPOS, ENONFINITE, ESTATE (no pencil). */
int sfrom_add_cell(sfrom_t* h, int32_t cell, int32_t n_i, const int64_t* global_node,
                   const int32_t* rowptr_i, const int32_t* col_i, const double* a_i,
                   const double* b_i);

/* Skeleton piece `piece` (0-based): a set of k_p skeleton nodes shared by
 * the same cells (a face interior, an edge line or a corner point of a
 * Cartesian partition), global_node[k_p], with an orthonormal boundary
 * basis S_p (k_p x b_p, column-major, S_p^T S_p = I) (Sec. 4.1). Each cell's
 * boundary basis S_i is block diagonal over its pieces in ascending piece
 * id. Every skeleton node must lie in exactly one piece.
 * Errors: EINVAL, ESTATE. */
int sfrom_add_piece(sfrom_t* h, int32_t piece, int32_t k_p, const int64_t* global_node,
                    int32_t b_p, const double* S_p);

/* Convenience set-up for the 3D acoustic example of Sec. 1: unit voxels
 * nvox[0] x nvox[1] x nvox[2], per-voxel sigma and rho (x fastest), nodes at
 * voxel corners with Dirichlet walls, each voxel adding sigma/4 to its 12
 * edges and rho/8 to its 8 corners. Cells are the boxes between the
 * interior cut planes cuts[] (ncut[0] x-planes, then y, then z, ascending
 * node coordinates); A_i, B_i are the voxel sums of cell i (eq. splitN_c).
 * Pieces are face interiors, edge lines and corner points with the lowest
 * modes_face / modes_edge orthonormal DCT-II modes (corners: 1 mode).
 * Cells are numbered x-fastest over the cell grid; pieces by first node in
 * x-fastest node order; unknowns x-fastest over interior nodes. Equivalent
 * to sfrom_set_pencil + sfrom_add_cell + sfrom_add_piece. */
int sfrom_setup_voxel_acoustic(sfrom_t* h, const int32_t nvox[3], const double* sigma,
                               const double* rho, const int32_t ncut[3], const int32_t* cuts,
                               int32_t modes_face, int32_t modes_edge);

/* sfrom_setup_voxel_acoustic with the face-mode count chosen per face from
 * its area in voxels, (n1 + 1)(n2 + 1) for a face interior of n1 x n2 nodes:
 * rule k (the first with area <= face_area_max[k]) gives face_modes[k]
 * modes; a face larger than every bound takes the last rule's count. For
 * partitions with cells of uneven size (face modes growing with the face).
 * Errors: as sfrom_setup_voxel_acoustic, EINVAL for rules without positive
 * counts or increasing bounds. */
int sfrom_setup_voxel_acoustic_rules(sfrom_t* h, const int32_t nvox[3], const double* sigma,
                                     const double* rho, const int32_t ncut[3], const int32_t* cuts,
                                     int32_t n_rules, const int32_t* face_area_max,
                                     const int32_t* face_modes, int32_t modes_edge);

/* Convenience set-up for an elastic medium (the anisotropic elastic example
 * of Sec. 9, in the form B u'' = A u + w(t) g of Sec. 1): displacements at
 * the corners of unit voxels nvox[0] x nvox[1] x nvox[2], three components
 * per node, clamped outer walls; unknown 3 k + c for interior node k
 * (x-fastest) and component c. c21 holds per voxel (x fastest) the 21
 * upper-triangle entries, row by row, of its symmetric 6 x 6 Voigt stiffness
 * (strains xx, yy, zz, yz, xz, xy, engineering shears); each voxel adds the
 * stiffness of the trilinear element on the unit cube (2 x 2 x 2 Gauss
 * rule) to A with a minus sign and rho / 8 per corner and component to B.
 * Cells and pieces as in sfrom_setup_voxel_acoustic; a piece's basis takes
 * each of its scalar DCT-II modes once per component (columns mode by mode,
 * components x, y, z; the piece's unknowns node by node). Errors: EINVAL,
 * and those of sfrom_set_pencil, sfrom_add_cell and sfrom_add_piece. */
int sfrom_setup_voxel_elastic(sfrom_t* h, const int32_t nvox[3], const double* c21, const double* rho,
                              const int32_t ncut[3], const int32_t* cuts, int32_t modes_face,
                              int32_t modes_edge);

/* Partition of a general pencil (the one given to sfrom_set_pencil) into
 * n_cells cells by the divide-and-conquer algorithm of App. A (Alg. 2):
 * each step splits the largest splittable cell with the sets O_1, O_2,
 * Gamma of Prop. 1 and the operator and mass splitting of Alg. 1 and eq.
 * alg1B with constant alpha_kl = alpha in [0, 1] and beta_k = beta in (0, 1).
 * O is a union of breadth-first levels of the cell's graph (adjacency:
 * a_kl != 0) from a pseudo-peripheral root, up to the level before the one
 * that reaches half of the cell's nodes, so Gamma is one level. For a
 * diagonally dominant A every A_i is diagonally dominant and <= 0 (Prop. 2).
 * Cells are numbered as Alg. 2 leaves them (the split cell's O_1 side keeps
 * the last position, its O_2 side is appended); each cell's local nodes are
 * in reverse Cuthill-McKee order. Pieces are the nodes held by two or more
 * cells grouped by their exact set of cells, numbered by smallest node,
 * nodes ascending, each with the normalised constant vector as its basis
 * (call sfrom_gramian_bases for richer ones). Replaces any cells, pieces,
 * sources and receivers. Requires a connected graph with a nonzero
 * diagonal. Errors: ESTATE (no pencil), EINVAL (arguments, graph, or fewer
 * than n_cells splittable cells), ENOMEM. */
int sfrom_partition_graph(sfrom_t* h, int32_t n_cells, double alpha, double beta);

/* Replace every piece's basis with the leading eigenvectors of its
 * frequency-limited Gramian (Sec. 4.1, eq. trgr): the eigenpairs (lambda,
 * z) of a local pencil with lambda <= omega_max^2 (z B-orthonormal; at least
 * the lowest pair), restricted to the piece, give G = sum z z^T; the basis
 * holds G's eigenvectors with eigenvalue above eps times the largest, at
 * most max_modes of them (single-node pieces: [1]). The local pencil is the
 * sum of the split operators of the cells holding the piece on their union,
 * cut to the nodes within graph distance depth + 1 of the piece by one
 * Prop. 1 / Alg. 1 split (alpha = beta = 1/2) with O the nodes within
 * distance depth (depth < 0: the whole union); it must have at most 4096
 * nodes (dense eigensolver on the host, one piece per thread). Works on any
 * partition; sources and receivers must be set again afterwards.
 * Errors: ESTATE (no partition), EINVAL (arguments, local pencil too
 * large), ENONFINITE, ENOMEM. */
int sfrom_gramian_bases(sfrom_t* h, double omega_max, double eps, int32_t max_modes, int32_t depth);

/* As sfrom_gramian_bases, with G taken from the spectral projector of eq.
 * trgrstep instead of the eigenpairs: Z = B^{-1/2} (I + sign(X)) / 2 B^{-1/2}
 * with X = (omega_max^2 I - C) / s, C = B^{-1/2} (-A) B^{-1/2} of the local
 * pencil and s = max(omega_max^2, h - omega_max^2) (h a Gershgorin bound of
 * C), sign(X) by Zolotarev's best rational approximation of the sign
 * function on [-1, -delta] U [delta, 1] with n_poles partial fractions and
 * delta = gamma omega_max^2 / s (eigenvalues within gamma omega_max^2 of
 * omega_max^2 get weights between 0 and 1), G = R Z R^T on the piece rows.
 * Each partial fraction is one complex symmetric band solve per piece node
 * (LDL^T without pivoting in reverse Cuthill-McKee order, valid because
 * i (X - i beta I) has a positive definite Hermitian part), so the local
 * pencil has no dense size limit (its band factor and solution columns must
 * fit in 2 GiB per piece); eps must exceed the approximant's error (about
 * 4 exp(-pi^2 n_poles / log(4 / delta))) or spurious modes are kept. The
 * Jacobi elliptic functions come from the arithmetic-geometric mean.
 * Errors: as sfrom_gramian_bases, and EINVAL for n_poles outside [1, 64],
 * gamma outside (0, 1) or a piece above the memory limit. */
int sfrom_gramian_bases_zolotarev(sfrom_t* h, double omega_max, double eps, int32_t max_modes, int32_t depth,
                                  int32_t n_poles, double gamma);

/* Remove the corner set of the current partition with hanging nodes (App. B,
 * eq. nocorners; the 2D example of Sec. 3): every node held by three or more
 * cells is replaced by one hanging node per pair of its cells that share a
 * node outside the corner set (every pair of its cells if that leaves one
 * of them out), held by those two cells only. Each cell's entries at the
 * removed node are shared equally among its copies (link weights to kept
 * nodes, the row sum on the diagonal, the mass; links between two removed
 * nodes join copies of the same pair), so that E^T A' E = A and
 * E^T B' E = B for E the map that copies an old value to its copies, and
 * A_i' <= 0 where A_i is a graph Laplacian with a non-positive remainder.
 * (App. B as printed copies each cell's row whole into every copy; that
 * leaves A' indefinite.) New numbering: old nodes ascending, a kept node
 * one id, a removed node one per pair, pairs in lexicographic order.
 * Replaces the pencil (n becomes *n_new), the cells (same ids, local order
 * kept, copies in place of the removed node) and the pieces (the pair
 * interfaces, each held by two cells, numbered by smallest node, constant
 * one-column bases: call sfrom_gramian_bases for richer ones); sources and
 * receivers are cleared and use the new numbering. Outputs (each may be
 * NULL): the new node count, the number of removed nodes and of hanging
 * nodes. A partition without a corner set is left as it is (*n_corner = 0).
 * Works on any partition (sfrom_partition_graph, sfrom_add_cell /
 * sfrom_add_piece, the voxel set-ups). Errors: ESTATE (no partition, or the
 * corner set was already removed), EINVAL (too large), ENOMEM. */
int sfrom_remove_corner_set(sfrom_t* h, int64_t* n_new, int32_t* n_corner, int64_t* n_hanging);

/* The maps of the last sfrom_remove_corner_set, into caller arrays (each may
 * be NULL): new_of_old (old node count: the new id of a kept node, -1 for a
 * removed one), corner (n_corner removed old nodes, ascending), hang_ptr
 * (n_corner + 1), hang_node (n_hanging new ids: the copies of corner[k] are
 * hang_node[hang_ptr[k] .. hang_ptr[k+1]), in pair order) and hang_weight
 * (n_hanging: b'_l / b_k, summing to one per removed node; the value at the
 * removed node is the weighted sum of its copies, and a point load there is
 * shared among the copies with the same weights). Errors: ESTATE (no corner
 * set removed). */
int sfrom_corner_map(sfrom_t* h, int64_t* new_of_old, int64_t* corner, int64_t* hang_ptr, int64_t* hang_node,
                     double* hang_weight);

/* ---------------------------------------------------------------------------
 * Off-line stage (Alg. alg1red stage 1)
 * ------------------------------------------------------------------------ */

typedef struct {
  int32_t m;                 /* S-fraction layers (Krylov blocks) per cell, >= 1      */
  const int32_t* m_per_cell; /* optional per-cell override (n_cells entries) or NULL */
  double shift;              /* Krylov shift s < 0 (Sec. 4.2, eq. npks)              */
  int32_t online_prec;       /* sfrom_prec of the on-line stage                       */
  int32_t cells_per_batch;   /* off-line batch size (0 = automatic)                   */
} sfrom_build_opts;

/* Validate the split and the partition, then build every cell's S-fraction on
 * the GPU: banded Cholesky of -(A_i + s B_i), rational block Krylov basis of
 * span{X, KX, ..., K^{m-1}X} with K = (A_i+sB_i)^{-1} B_i, X = B_i^{-1} P S_i
 * (eq. npks), projection (eq. tfprj), block Lanczos (App. C, eq. NtDtri),
 * the S-fraction change of variables (eq. GammaTrans), piece masses
 * M_p = sum_{i owns p} [(Ghat_i^1)^{-1}]_pp (eq. bdrytstep) and packing in
 * the on-line precision. On failure no ROM is kept and the message names the
 * first failing cell. The first build after the partition is defined copies
 * the build's inputs (cell operators, skeleton rows of each W_i, piece bases)
 * to device memory that the handle keeps for later builds until the pencil,
 * a cell or a piece changes or the handle is destroyed (about 300 MB for
 * 4096 cells of 8^3 voxels). Errors: ESTATE, ESPLIT, ENOTNSD, EBREAKDOWN,
 * ENOTSPD, ENOMEM, EDEVICE. */
int sfrom_build(sfrom_t* h, const sfrom_build_opts* opts);

/* What sfrom_build does when a cell breaks Assumption 1 (its rational Krylov
 * or Lanczos block k loses rank, Sec. 4.2): reduce_m = 0 (default) fails the
 * build with EBREAKDOWN naming the cell and the block; reduce_m = 1 rebuilds
 * such a cell with m_i = k - 1 (k >= 2; a rank-deficient first block still
 * fails), the per-cell layer count sfrom_export_rom reports. Partitions of
 * general graphs can have cells that touch junction nodes only through other
 * skeleton nodes with complete piece bases, which makes block 2 or 3 lose rank
 * exactly. Errors: EINVAL. */
int sfrom_set_breakdown_policy(sfrom_t* h, int32_t reduce_m);

/* Correction at the removed corner nodes after every on-line step (App. D,
 * Remark solcorr), for a partition after sfrom_remove_corner_set: with the
 * new piece state y^{n+1}, the value at each copy l of a removed node k is
 * u_l = S_p(l, :) y_p, the node's value is ubar_k = sum_l w_l u_l
 * (w_l = b'_l / b_k), delta_l = ubar_k - u_l for all copies first, then
 * y_p += S_p(l, :)^T delta_l for every copy l in piece p. Traces are read
 * after the correction (by the receivers kernel). enable: 0 (default) or 1.
 * Takes effect from the next sfrom_run; sfrom_run_noalloc refuses to run
 * while it is on. Errors: EINVAL, ESTATE (no corner set removed). */
int sfrom_set_corner_correction(sfrom_t* h, int32_t enable);

/* Persistent on-line stage (Alg. alg1red stage 2 as one kernel): with
 * enable = 1, sfrom_run executes all its steps in one cooperative launch of
 * as many workgroups as the device holds at once; each step runs the cell
 * phase over all (cell, 64-source tile) items, a grid barrier, the piece
 * phase (eq. bdrytstep) over all (piece, source) items and a grid barrier,
 * with receivers that read several pieces computed beside the next step's
 * cell phase. Same arithmetic as the default path (one cell-kernel geometry
 * for every cell instead of per-bucket autotuned variants). Requires FP32 or
 * FP64 on-line blocks, b_i <= 144 and b_p <= 16, and no corner correction
 * (EINVAL / ESTATE at sfrom_run otherwise); not captured in a graph, not
 * used by sfrom_run_noalloc, no per-kernel profile. Default 0. Errors:
 * EINVAL. */
int sfrom_set_persistent(sfrom_t* h, int32_t enable);

/* Replace cell `cell`'s S-fraction by m blocks Ghat^k and G^k (each b x b
 * symmetric, column-major, stored consecutively: Ghat[k*b*b ...]); b must
 * equal the cell's boundary dimension. Requires a built ROM; piece masses
 * are recomputed from Ghat^1 at the next run. The on-line blocks are formed
 * on the host with Cholesky factors of Ghat^2..Ghat^m (the change of
 * variables described at sfrom_run). Errors: EINVAL, ESTATE, ENOTSPD
 * (non-symmetric blocks, or Ghat^k k >= 2 not positive definite). */
int sfrom_import_rom(sfrom_t* h, int32_t cell, int32_t m, int32_t b, const double* Ghat,
                     const double* G);
/* Copy cell `cell`'s S-fraction to host: *m, *b, and (if non-NULL) Ghat, G
 * with room for m*b*b doubles each, in double precision as built. */
int sfrom_export_rom(sfrom_t* h, int32_t cell, int32_t* m, int32_t* b, double* Ghat,
                     double* G);

/* ---------------------------------------------------------------------------
 * Inputs and outputs (host data, CSC sparse columns over global nodes)
 * ------------------------------------------------------------------------ */

/* n_s source columns g_j as CSC (colptr[n_s+1], row[nnz] global node, val).
 * project != 0 replaces each column by its orthogonal projection onto the
 * piece bases (g <- S_p S_p^T g on every piece), for the fine model too;
 * project == 0 keeps g for the fine model and uses S_p^T g for the ROM.
 * Any nonzero off the skeleton gives ESUPPORT (eq. gsupport). */
int sfrom_set_sources(sfrom_t* h, int32_t n_s, const int64_t* colptr, const int64_t* row,
                      const double* val, int32_t project);
/* Receiver columns q_r, same format and meaning of `project`; traces are
 * q_r^T u (fine) and sum_p (S_p^T q_r)^T y_p (ROM, eq. solatrec). */
int sfrom_set_receivers(sfrom_t* h, int32_t n_r, const int64_t* colptr, const int64_t* row,
                        const double* val, int32_t project);
/* Projected point columns at the given global skeleton nodes: column j is
 * S_p S_p^T e_node. colptr_out[count+1] is filled; row_out/val_out need room
 * for the sum of the pieces' sizes (at most count * max k_p). */
int sfrom_point_columns(sfrom_t* h, int32_t count, const int64_t* node, int64_t* colptr_out,
                        int64_t* row_out, double* val_out);

/* ---------------------------------------------------------------------------
 * On-line stage (Alg. alg1red stage 2) and the fine-grid comparator
 * ------------------------------------------------------------------------ */

/* Zero the ROM state (eq. initial: U = 0 for t <= 0) in place and the step
 * counter. Errors: ESTATE (no ROM). */
int sfrom_reset(sfrom_t* h);
/* Advance the ROM n_steps leapfrog steps of size dt from its current state:
 * Y^{n+1} = 2Y^n - Y^{n-1} + dt^2 D^{-1} (L Y^n + w^n F), piece dofs by
 * eq. bdrytstep. The hidden layers of eq. intrtstep_td are stepped in the
 * unit-mass variables V^k = G_k^{-1} U^k (Ghat^k = G_k G_k^T, eq. GammaTrans),
 * where each cell's operator is block tridiagonal with the cell's Lanczos
 * blocks: an exactly equivalent form whose blocks stay well scaled when
 * Ghat^k and G^k of deep layers are near singular, so that rounding them
 * to F32/BF16 moves the spectrum by about a unit roundoff of its largest
 * eigenvalue. The traces are unaffected by the change of variables. w[n_steps] (double) are the
 * wavelet samples for these steps, host memory unless w_on_device.
 * traces receives n_steps x n_r x n_s values (source fastest) of the
 * receiver output at levels n+1, as double for F64 and float otherwise,
 * host memory unless traces_on_device. dt must satisfy the leapfrog
 * stability limit dt^2 lambda_max < 4 of the ROM pencil (Remark MFEM),
 * else ECFL and nothing is stepped: the limit is tested first against a
 * bound valid for built blocks (the largest Gershgorin bound of the cells'
 * pencils B_i^{-1}(-A_i), which bounds every cell's Galerkin-projected
 * pencil and hence the assembled ROM), and only when that test fails, or
 * some blocks were imported, against the ROM's own lambda_max (computed
 * once per ROM on the host, as sfrom_rom_lambda_max). After the steps the state is checked: a
 * NaN or infinity (the scheme diverged) returns ENONFINITE; the traces are
 * written either way. Errors: ESTATE, EINVAL, ECFL, EDEVICE,
 * ENONFINITE. */
int sfrom_run(sfrom_t* h, int64_t n_steps, double dt, const double* w, int32_t w_on_device,
              void* traces, int32_t traces_on_device);

/* sfrom_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same steps, kernels and results as sfrom_run, with no hipMalloc,
 * hipFree or other allocating call. w[n_steps] (double) and traces
 * (n_steps x n_r x n_s, as in sfrom_run) must be device pointers. The
 * handle must already be prepared by a sfrom_run (any n_steps, also 0)
 * since the last build, load, import, or change of sources or receivers,
 * and, for a dt beyond the cells' Gershgorin bound, the ROM's largest
 * eigenvalue must be known (sfrom_rom_lambda_max): ESTATE otherwise. The
 * Phi^1 exchange buffer (sum of the cells' b_i times n_s values of the
 * on-line precision) and the non-finite flag live in a static device array
 * of 256 MiB per GPU, held until the process ends; a run that needs more
 * returns EINVAL and steps nothing. Calls on one GPU share that array, so
 * runs that overlap on one GPU (other streams, other handles, other
 * threads) race: order them. The run is enqueued eagerly, is not timed by
 * sfrom_profile, and synchronises the stream at its end for the non-finite
 * check as sfrom_run does. Errors: as sfrom_run, plus ESTATE and EINVAL
 * as above. */
int sfrom_run_noalloc(sfrom_t* h, int64_t n_steps, double dt, const double* w, void* traces);

/* Checkpoint of the on-line stage (the ROM is built "just once" for all
 * sources and time windows, Sec. 4.2 and Alg. alg1red stage 1): writes to
 * the file `path` a versioned binary record of the partition's cell and
 * piece sizes, the piece nodes and bases, the FP64 S-fraction of every
 * cell, the on-line blocks and inverse piece masses in the on-line
 * precision, and, when a run has allocated it, both levels of the ROM
 * state with the step counter. Errors: ESTATE (no ROM), EINVAL (file). */
int sfrom_save(sfrom_t* h, const char* path);
/* Restores a checkpoint into a handle whose problem (pencil, cells, pieces)
 * is the one saved: cell and piece sizes, piece nodes and bases must match
 * exactly (EINVAL otherwise, and the current ROM is kept). Replaces any ROM
 * of the handle without building; the saved state continues at the next
 * sfrom_run when the handle has as many sources as were saved, so that n
 * steps, save, load and n more steps equal 2n steps bitwise. Sources and
 * receivers are not part of the checkpoint. A partition whose corner set was
 * removed is set up again by repeating sfrom_remove_corner_set (the removal
 * is deterministic; it also restores the corner map) before the load. A
 * failure after the file has been validated leaves no ROM. Errors: EINVAL,
 * EDEVICE, ENOMEM. */
int sfrom_load(sfrom_t* h, const char* path);

/* Zero the fine-grid state. */
int sfrom_fine_reset(sfrom_t* h);
/* Fine-grid leapfrog u^{n+1} = 2u^n - u^{n-1} + dt^2 B^{-1}(A u^n + w^n g)
 * for all sources in precision `prec` (F64 or F32); traces as in sfrom_run
 * (q^T u^{n+1}). */
int sfrom_fine_run(sfrom_t* h, int64_t n_steps, double dt, const double* w,
                   int32_t w_on_device, void* traces, int32_t traces_on_device,
                   int32_t prec);
/* Largest eigenvalue of B^{-1}(-A) (Lanczos on the GPU; relative accuracy
 * about 1e-10). The leapfrog is stable for dt < 2/sqrt(lambda). */
int sfrom_fine_lambda_max(sfrom_t* h, double* lambda);
/* Largest eigenvalue of the global ROM pencil (-L, D); needs a built ROM. */
int sfrom_rom_lambda_max(sfrom_t* h, double* lambda);

/* hipGraph form of sfrom_run (default off): the launches of a whole run are
 * captured into one graph, which is replayed by later runs with the same
 * n_steps, dt, wavelet and trace pointers, state buffers and state parity
 * (the typical case of repeated jobs with device-resident inputs and
 * outputs). Runs with host pointers are captured afresh each time. */
int sfrom_set_graph(sfrom_t* h, int32_t enable);

/* Band kernels of the off-line build (Sec. 4.2: one Cholesky factorisation
 * of -(A_i + s B_i) per cell serves every shifted solve): mode 0 (default)
 * uses the blocked kernels, spread over many workgroups per cell, for half
 * bandwidths above 128 and the one-workgroup-per-cell kernels otherwise;
 * 1 always the blocked kernels; 2 never. The results agree to rounding.
 * Meant for tests and tuning studies. Errors: EINVAL. */
int sfrom_set_build_path(sfrom_t* h, int32_t mode);

/* Kernel variant of the on-line cell phase: -1 (default) lets the
 * autotuner time the variants on the first run and keep the fastest; 0..3
 * and 5 pin a matrix-core tiling (FP32, BF16 or FP64 matrix instructions by
 * the on-line precision; 5 has 16-source tiles, for partitions with few
 * cells), 4 the scalar kernel. Meant for tests and tuning studies. */
int sfrom_set_cell_variant(sfrom_t* h, int32_t variant);

/* Per-kernel timing with HIP events recorded on the handle's stream around
 * the launches of timed steps. enable: 0 off; 1 every step; N > 1 one step
 * in N (steps 0, N, 2N, ... of each run; an event pair costs a few
 * microseconds of stream time, so sampling keeps the measurement out of the
 * run's own time); negative values return SFROM_EINVAL. Kernel ids: 0 on-line
 * cell phase, 1 on-line piece phase, 2 receivers (no launches when every
 * receiver reads a single piece: the piece phase then writes the traces),
 * 3 fine-grid step.
 * sfrom_profile_read synchronises the stream, returns the summed kernel time
 * and the number of timed launches since the last read, and clears them. */
int sfrom_profile(sfrom_t* h, int32_t enable);
int sfrom_profile_read(sfrom_t* h, int32_t kernel, double* total_ms, int64_t* launches);

/* ---------------------------------------------------------------------------
 * Introspection
 * ------------------------------------------------------------------------ */

typedef struct {
  int64_t n;               /* fine unknowns                       */
  int64_t nnz;             /* nonzeros of A                       */
  int32_t n_cells;
  int32_t n_pieces;
  int64_t n_piece_dofs;    /* sum_p b_p                            */
  int64_t n_hidden_dofs;   /* sum_i (m_i - 1) b_i (0 before build) */
  int32_t max_b;           /* max_i b_i                            */
  int32_t max_m;
  int32_t n_sources;
  int32_t n_receivers;
  int32_t built;
  int32_t online_prec;
  int64_t block_bytes;     /* on-line S-fraction storage           */
  double build_ms;         /* last sfrom_build wall time          */
  int32_t cell_variant;    /* autotuned on-line cell-phase kernel variant of the last
                              run (0-3 matrix-core tilings, 4 scalar; -1 before)    */
  int64_t steps_done;      /* on-line steps since the last reset (or as loaded)     */
} sfrom_info;

int sfrom_get_info(const sfrom_t* h, sfrom_info* info);

/* Copy the fine pencil to host (sizes from sfrom_get_info). */
int sfrom_export_pencil(sfrom_t* h, int64_t* rowptr, int32_t* col, double* a, double* b);
/* Cell sizes and (if non-NULL) its local operator: *n_i, *nnz_i, global_node,
 * rowptr_i, col_i, a_i, b_i, and its boundary dimension *b_i_out. */
int sfrom_export_cell(sfrom_t* h, int32_t cell, int32_t* n_i, int32_t* nnz_i,
                      int32_t* b_dim, int64_t* global_node, int32_t* rowptr_i,
                      int32_t* col_i, double* a_i, double* b_i);
/* Piece sizes and (if non-NULL) nodes and basis. */
int sfrom_export_piece(sfrom_t* h, int32_t piece, int32_t* k_p, int32_t* b_p,
                       int64_t* global_node, double* S_p);

/* ------------------------------------------------------------------------
 * Learned off-line stage (no counterpart in the paper, which builds every
 * cell by block Lanczos, Sec. 5 and App. C). A small 3D CNN maps a cell's
 * medium to the Cholesky factors of its S-fraction blocks Ghat^k, G^k for
 * k = 2..m; layer 1 is computed in closed form from B, W and A (Ghat^1 =
 * W^T B^{-1} W, G^1 = -(Ghat^1)^{-1} X^T A X (Ghat^1)^{-1}, X = B^{-1} W),
 * so every predicted pivot is SPD and the ROM stays Stieltjes (Prop.
 * prop1stil). A predicted cell is kept only if its ROM transfer function
 * matches the exact cell transfer function W^T (A + zB)^{-1} W to a
 * tolerance at 16 points z = -sigma_j^2, sigma_j = (j + 1/2) omega_max / 16;
 * other cells are built by block Lanczos.
 *
 * Network: input x[n][2][8][8][8] (log sigma, log rho of the cell's voxels,
 * [channel][z][y][x], float, device memory); conv3d(2 -> conv_ch, 3^3, zero
 * padding) + ReLU; 2^3 average pooling; dense(64 conv_ch -> hidden) + ReLU;
 * dense(hidden -> n_out). Parameters are one float vector [W1 (conv_ch, 2,
 * 3, 3, 3), b1, W2 (hidden, 64 conv_ch), b2, W3 (n_out, hidden), b3],
 * row-major. Outputs are normalised: factor = y * sd + mu per output.
 * Factor vectors are, for k = 2..m, the rows of the lower triangle of
 * chol(Ghat^k) and then of chol(G^k + eps I), eps = 1e-10 tr(G^k) / b:
 * n_out = (m - 1) b (b + 1).
 * ---------------------------------------------------------------------- */
typedef struct sfrom_surrogate sfrom_surrogate_t;

/* Network on `device`, launching on `hip_stream` (NULL = null stream).
 * Errors: EINVAL, EDEVICE, ENOMEM. */
int sfrom_surrogate_create(sfrom_surrogate_t** out, int32_t device, void* hip_stream, int32_t conv_ch,
                           int32_t hidden, int32_t n_out);
void sfrom_surrogate_destroy(sfrom_surrogate_t* s);
const char* sfrom_surrogate_last_error(const sfrom_surrogate_t* s);
int sfrom_surrogate_param_count(const sfrom_surrogate_t* s, int64_t* n);
/* Host parameter vector in; resets the Adam moments. Errors: ENONFINITE. */
int sfrom_surrogate_set_params(sfrom_surrogate_t* s, const float* theta);
int sfrom_surrogate_get_params(sfrom_surrogate_t* s, float* theta);
/* Output normalisation (host, n_out floats each, sd > 0). */
int sfrom_surrogate_set_scale(sfrom_surrogate_t* s, const float* mu, const float* sd);
/* Mean squared error of the batch (x: n inputs, t: n x n_out normalised
 * targets, device) and its gradient (host, param_count floats; either
 * output may be NULL). */
int sfrom_surrogate_gradients(sfrom_surrogate_t* s, const float* x, const float* t, int32_t n, float* loss,
                              float* grad);
/* One Adam step (beta 0.9, 0.999, eps 1e-8) on the batch; *loss (host, may
 * be NULL) is the loss before the step. */
int sfrom_surrogate_train_step(sfrom_surrogate_t* s, const float* x, const float* t, int32_t n, float lr,
                               float* loss);
/* Normalised outputs y (device, n x n_out) for inputs x (device); bf16 != 0
 * rounds weights and activations to bfloat16 at every layer input (float
 * accumulation). */
int sfrom_surrogate_forward(sfrom_surrogate_t* s, const float* x, int32_t n, int32_t bf16, float* y);

/* Factor vectors (device, n x n_out floats) of the listed cells of a built
 * ROM (the training targets). All listed cells must have the same b and m
 * with n_out = (m - 1) b (b + 1). Errors: ESTATE, EINVAL, ENOTSPD. */
int sfrom_surrogate_targets(sfrom_t* h, int32_t n, const int32_t* cells, float* t);

/* sfrom_build with the learned stage for the n candidate cells `cells`
 * (host ids; inputs x on the device, one per candidate, all candidates with
 * the same b and m and n_out = (m - 1) b (b + 1)): prediction with bfloat16
 * operands, closed-form layer 1, the transfer-function test with
 * `omega_max` and `tol`, and block Lanczos for every rejected or
 * non-candidate cell. accepted[i] (host, n) is 1 when candidate i kept its
 * predicted blocks; mismatch[i] (host, n, may be NULL) is its largest
 * relative transfer-function mismatch. Errors: as sfrom_build, plus
 * EINVAL for a candidate list that does not match the network. */
int sfrom_build_learned(sfrom_t* h, const sfrom_build_opts* opts, sfrom_surrogate_t* s, int32_t n,
                        const int32_t* cells, const float* x, double omega_max, double tol,
                        int32_t* accepted, double* mismatch);

#ifdef __cplusplus
}
#endif
#endif /* SFROM_H */
