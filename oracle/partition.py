"""Cartesian coarse cells, skeleton pieces, operator splitting and boundary
bases (Sec. 2 and Sec. 4.1 of the paper).

Readings (the paper leaves these open or states them for 2D only):

* Cells are boxes of voxels between interior cut planes. A cell's nodes are
  the closed node box of its voxels minus Dirichlet wall nodes, so two
  neighbouring cells share the nodes on their common plane (eq. part: the
  interfaces are one node thick).
* Splitting (eq. splitN_c): A_i and B_i are the same voxel sums as A and B
  restricted to the voxels of cell i. Then sum_i P_i A_i P_i^T = A and
  sum_i P_i B_i P_i^T = B, A_i <= 0 (each voxel's edge energy is PSD) and
  B_i > 0; for homogeneous media this reproduces the alpha/gamma/beta
  weights of the multi-domain example in Sec. 2.
* Corner set (Sec. 3, eq. nocorners): instead of removing it with hanging
  nodes, the skeleton is split into "pieces": face interiors (2 cells),
  edge lines (4 cells) and corner points (8 cells), each with its own
  reduced basis. This is the general interior-elimination form (eq. BIE)
  without the pairwise simplification (eq. BEINC).
* Boundary bases (Sec. 4.1): the frequency-limited Gramian construction
  needs a reference that is not part of the paper, so each piece gets the
  lowest separable orthonormal DCT-II modes (the constant mode included):
  face modes ordered by (max(p, q), p, q), edge modes 0, 1, ..., corners [1].
  Uneven partitions may give each face a count by its area (a rule
  (n1, n2) -> count).
  S_i is block diagonal over the cell's pieces as in Sec. 4.1.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import fine


def dct_1d(n: int, k: int) -> np.ndarray:
    """Orthonormal DCT-II vector k on n points: c_k cos(pi k (j + 1/2) / n)."""
    j = np.arange(n)
    v = np.cos(np.pi * k * (j + 0.5) / n)
    return v / np.linalg.norm(v)


def face_mode_order(n1: int, n2: int, count: int):
    """First ``count`` mode pairs (p, q), p < n1, q < n2, sorted by (max, p, q)."""
    pairs = [(p, q) for p in range(n1) for q in range(n2)]
    pairs.sort(key=lambda t: (max(t), t[0], t[1]))
    return pairs[:count]


def piece_basis(dims, kind: int, modes_face: int, modes_edge: int) -> np.ndarray:
    """Orthonormal basis S_p (k_p x b_p) of a piece whose nodes form a box with
    the given off-plane extents (x-fastest node order)."""
    if kind == 3:
        return np.ones((1, 1))
    if kind == 2:
        (n,) = dims
        cols = [dct_1d(n, k) for k in range(min(modes_edge, n))]
        return np.stack(cols, axis=1)
    n1, n2 = dims
    cols = []
    for p, q in face_mode_order(n1, n2, modes_face):
        cols.append(np.outer(dct_1d(n2, q), dct_1d(n1, p)).ravel())  # first axis fastest
    return np.stack(cols, axis=1)


@dataclass
class Piece:
    key: tuple
    kind: int                     # number of cut planes the piece lies on: 1 face, 2 edge, 3 corner
    nodes: np.ndarray             # global unknown indices, x-fastest
    dims: tuple                   # extents along the off-plane axes
    cells: List[int]              # incident cells (ascending)
    S: np.ndarray = None          # k_p x b_p


@dataclass
class Cell:
    index: tuple                  # (cx, cy, cz)
    vox_lo: np.ndarray
    vox_hi: np.ndarray            # exclusive
    nodes: np.ndarray             # global unknown indices, local x-fastest order
    shape: tuple                  # local node box extents (after wall removal)
    pieces: List[int] = field(default_factory=list)


class CartesianPartition:
    """Coarse-cell partition of a voxel grid with interior cut planes."""

    def __init__(self, nvox, cuts, modes_face, modes_edge: int):
        """``modes_face`` is a count, or a function (n1, n2) -> count of the
        face interior's node extents (face modes by face area)."""
        self.nvox = tuple(int(v) for v in nvox)
        self.cuts = [np.asarray(c, dtype=np.int64) for c in cuts]
        self.modes_face = modes_face
        self.modes_edge = modes_edge
        self.idx = fine.node_index(self.nvox)
        self.n = int(self.idx.max()) + 1
        self.edges = [np.concatenate([[0], c, [nv]]) for c, nv in zip(self.cuts, self.nvox)]
        self.ncell = tuple(len(e) - 1 for e in self.edges)
        self._build_cells()
        self._build_pieces()

    # -- cells ------------------------------------------------------------
    def cell_id(self, cx, cy, cz):
        return cx + self.ncell[0] * (cy + self.ncell[1] * cz)

    def _build_cells(self):
        self.cells: List[Cell] = []
        for cz in range(self.ncell[2]):
            for cy in range(self.ncell[1]):
                for cx in range(self.ncell[0]):
                    c = (cx, cy, cz)
                    lo = np.array([self.edges[a][c[a]] for a in range(3)])
                    hi = np.array([self.edges[a][c[a] + 1] for a in range(3)])
                    nlo = np.maximum(lo, 1)
                    nhi = np.minimum(hi, np.array(self.nvox) - 1)
                    sub = self.idx[nlo[0]:nhi[0] + 1, nlo[1]:nhi[1] + 1, nlo[2]:nhi[2] + 1]
                    nodes = sub.transpose(2, 1, 0).ravel().copy()
                    self.cells.append(Cell(c, lo, hi, nodes, tuple(int(v) for v in (nhi - nlo + 1))))

    def cell_operator(self, i, sigma, rho):
        """Split operators (A_i dense, b_i) of cell i: the voxel sums of the
        fine assembly restricted to the voxels of the cell (eq. splitN_c)."""
        Ai, b = self.cell_operator_sparse(i, sigma, rho)
        return Ai.toarray(), b

    def cell_operator_sparse(self, i, sigma, rho):
        """The same (A_i, b_i) with A_i as a scipy sparse matrix (large cells)."""
        c = self.cells[i]
        lo, hi = c.vox_lo, c.vox_hi
        sg = sigma[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        rh = rho[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        # local node numbering on the closed box; global wall nodes are removed
        shp = tuple(int(h - l + 1) for l, h in zip(lo, hi))
        lidx = -np.ones(shp, dtype=np.int64)
        gx = np.arange(lo[0], hi[0] + 1); gy = np.arange(lo[1], hi[1] + 1); gz = np.arange(lo[2], hi[2] + 1)
        okx = (gx >= 1) & (gx <= self.nvox[0] - 1)
        oky = (gy >= 1) & (gy <= self.nvox[1] - 1)
        okz = (gz >= 1) & (gz <= self.nvox[2] - 1)
        X, Y, Z = np.meshgrid(np.where(okx)[0], np.where(oky)[0], np.where(okz)[0], indexing="ij")
        ux, uy = okx.sum(), oky.sum()
        lidx[X, Y, Z] = (X - X.min()) + ux * ((Y - Y.min()) + uy * (Z - Z.min()))
        cx, cy, cz = fine.edge_conductances(sg)
        Ai = fine._laplacian_from_edges(cx, cy, cz, lidx)
        mass = fine.node_masses(rh)
        bi = mass[X, Y, Z].ravel()
        order = lidx[X, Y, Z].ravel()
        b = np.empty(len(order)); b[order] = bi
        return Ai, b

    # -- pieces -----------------------------------------------------------
    def _axis_key(self, a, coord):
        """Per-axis key: 2*j+1 if coord is cut plane j, else 2*segment."""
        cuts = self.cuts[a]
        on = np.isin(coord, cuts)
        seg = np.searchsorted(cuts, coord, side="left")   # number of cuts < coord
        return np.where(on, 2 * seg + 1, 2 * seg), on

    def _build_pieces(self):
        nx, ny, nz = self.nvox
        Z, Y, X = np.meshgrid(np.arange(1, nz), np.arange(1, ny), np.arange(1, nx), indexing="ij")
        X = X.ravel(); Y = Y.ravel(); Z = Z.ravel()   # x-fastest scan == unknown order
        kx, ox = self._axis_key(0, X)
        ky, oy = self._axis_key(1, Y)
        kz, oz = self._axis_key(2, Z)
        nplanes = ox.astype(int) + oy.astype(int) + oz.astype(int)
        skel = np.where(nplanes > 0)[0]
        keys = np.stack([kx[skel], ky[skel], kz[skel]], axis=1)
        _, first, inv = np.unique(keys, axis=0, return_index=True, return_inverse=True)
        inv = inv.ravel()
        order = np.argsort(first)                      # piece ids by first appearance
        rank = np.empty_like(order); rank[order] = np.arange(len(order))
        pid_of_skel = rank[inv]
        self.piece_of_node = -np.ones(self.n, dtype=np.int64)
        self.piece_of_node[skel] = pid_of_skel
        self.pieces: List[Piece] = []
        srt = np.argsort(pid_of_skel, kind="stable")
        bounds = np.searchsorted(pid_of_skel[srt], np.arange(len(order) + 1))
        coords = np.stack([X, Y, Z], axis=1)
        for p in range(len(order)):
            members = skel[srt[bounds[p]:bounds[p + 1]]]       # ascending => x-fastest
            key = tuple(int(v) for v in keys[first[order[p]]])
            kind = sum(k % 2 for k in key)
            cc = coords[members]
            dims = tuple(int(cc[:, a].max() - cc[:, a].min() + 1) for a in range(3) if key[a] % 2 == 0)
            per_axis = []
            for a in range(3):
                if key[a] % 2 == 1:
                    j = key[a] // 2
                    per_axis.append([j, j + 1])
                else:
                    per_axis.append([key[a] // 2])
            cells = sorted(self.cell_id(a, b, c) for c in per_axis[2] for b in per_axis[1] for a in per_axis[0])
            mf = self.modes_face(*dims) if (kind == 1 and callable(self.modes_face)) else self.modes_face
            S = piece_basis(dims, kind, mf, self.modes_edge)
            self.pieces.append(Piece(key, kind, members, dims, cells, S))
            for c in cells:
                self.cells[c].pieces.append(p)
        for c in self.cells:
            c.pieces.sort()

    # -- per-cell boundary basis -------------------------------------------
    def cell_W(self, i):
        """W_i = P^Gamma_i S_i (N_i x b_i): columns grouped by the cell's pieces
        in ascending piece id, each column supported on one piece."""
        c = self.cells[i]
        pos = {int(g): k for k, g in enumerate(c.nodes)}
        b = sum(self.pieces[p].S.shape[1] for p in c.pieces)
        W = np.zeros((len(c.nodes), b))
        col = 0
        for p in c.pieces:
            pc = self.pieces[p]
            rows = [pos[int(g)] for g in pc.nodes]
            W[rows, col:col + pc.S.shape[1]] = pc.S
            col += pc.S.shape[1]
        return W

    def piece_offsets(self):
        """Offsets of each piece's reduced dofs in the concatenated piece vector."""
        sizes = np.array([p.S.shape[1] for p in self.pieces])
        return np.concatenate([[0], np.cumsum(sizes)])

    # -- point inputs/outputs on the skeleton (eq. gsupport) ----------------
    def point_columns(self, coords):
        """Projected point columns: for node k on piece p, the fine vector
        S_p S_p^T e_k (Sec. 2, eq. gsupport; Sec. 6 reduced sources
        g_ij = S_ij^T g) and its reduced coefficients (piece, S_p^T e_k).
        Returns (G dense n x c, list of (piece, coeff vector))."""
        G = np.zeros((self.n, len(coords)))
        red = []
        for j, (x, y, z) in enumerate(coords):
            k = int(self.idx[x, y, z])
            if k < 0:
                raise ValueError("point on a wall")
            p = int(self.piece_of_node[k])
            if p < 0:
                raise ValueError("point not on the skeleton (eq. gsupport)")
            pc = self.pieces[p]
            r = int(np.searchsorted(pc.nodes, k))
            coeff = pc.S[r, :].copy()
            G[pc.nodes, j] = pc.S @ coeff
            red.append((p, coeff))
        return G, red
