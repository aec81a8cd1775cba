"""Elastic fine model on unit voxels for the layered elastic example (Sec. 9
names an anisotropic elastic medium; Sec. 1's model B u'' = A u + g w(t)
with A <= 0 covers it).

Test infrastructure only: plain numpy/scipy, FP64, no blocking.

Readings (the paper gives no discretisation for its elastic example):

* Displacements u = (u_x, u_y, u_z) at voxel corners, clamped (zero) on the
  outer walls; unknown dof 3 k + c for interior node k (x-fastest) and
  component c.
* Each voxel v contributes the trilinear (Q1) finite-element stiffness of
  the unit cube with its 6 x 6 Voigt stiffness C_v, integrated by the 2 x 2 x
  2 Gauss rule, K_v = sum_g B_g^T C_v B_g / 8; A = -sum_v K_v restricted to
  the unknowns (so A <= 0, symmetric), and a lumped mass rho_v / 8 per
  corner and component (B diagonal > 0). A cell's (A_i, B_i) are the same
  sums over its voxels (eq. splitN_c), exactly as for the acoustic model.
* Vertically transversely isotropic voxels from Thomsen's parameters
  (vertical axis z): C33 = lambda + 2 mu, C44 = C55 = mu, C11 = C22 =
  C33 (1 + 2 eps), C66 = C44, C12 = C11 - 2 C66,
  C13 = C23 = sqrt((C33 - C44)(C33 (1 + 2 delta) - C44)) - C44.
* Skeleton pieces are the scalar partition's node sets; a piece's vector
  basis takes every scalar basis vector once per component (columns mode
  by mode, components x, y, z), which stays orthonormal.

Voigt order of strains: xx, yy, zz, yz, xz, xy (engineering shears).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fine
from .partition import CartesianPartition


def vti_stiffness(lam, mu, eps, delta):
    """6 x 6 Voigt stiffness of a VTI voxel from lambda, mu (vertical P and S
    moduli C33 = lambda + 2 mu, C44 = mu) and Thomsen's epsilon, delta."""
    C33 = lam + 2.0 * mu
    C44 = mu
    C11 = C33 * (1.0 + 2.0 * eps)
    C66 = C44
    C12 = C11 - 2.0 * C66
    C13 = np.sqrt((C33 - C44) * (C33 * (1.0 + 2.0 * delta) - C44)) - C44
    C = np.zeros((6, 6))
    C[0, 0] = C[1, 1] = C11
    C[2, 2] = C33
    C[0, 1] = C[1, 0] = C12
    C[0, 2] = C[2, 0] = C[1, 2] = C[2, 1] = C13
    C[3, 3] = C[4, 4] = C44
    C[5, 5] = C66
    return C


def _corners():
    """Corners (a, b, c) of the unit cube, x fastest."""
    return [(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)]


def strain_matrix(p):
    """B (6 x 24) of the trilinear element on [0, 1]^3 at point p: strain =
    B u for the corner displacements u[3 corner + component]."""
    B = np.zeros((6, 24))
    x, y, z = p
    for k, (a, b, c) in enumerate(_corners()):
        fx = x if a else 1.0 - x
        fy = y if b else 1.0 - y
        fz = z if c else 1.0 - z
        sx = 1.0 if a else -1.0
        sy = 1.0 if b else -1.0
        sz = 1.0 if c else -1.0
        dx, dy, dz = sx * fy * fz, fx * sy * fz, fx * fy * sz     # gradient of the shape function
        B[0, 3 * k + 0] = dx
        B[1, 3 * k + 1] = dy
        B[2, 3 * k + 2] = dz
        B[3, 3 * k + 1] = dz; B[3, 3 * k + 2] = dy
        B[4, 3 * k + 0] = dz; B[4, 3 * k + 2] = dx
        B[5, 3 * k + 0] = dy; B[5, 3 * k + 1] = dx
    return B


def voxel_stiffness(C):
    """K_v = integral of B^T C B over the unit cube by the 2 x 2 x 2 Gauss rule."""
    g = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))
    K = np.zeros((24, 24))
    for z in g:
        for y in g:
            for x in g:
                B = strain_matrix((x, y, z))
                K += B.T @ C @ B / 8.0
    return K


def _assemble(Cv, rho, lo, hi, idx):
    """-sum of K_v and sum of rho_v / 8 over the voxels in the box [lo, hi)
    onto the unknown nodes numbered by ``idx`` (node index array, -1 where
    the node is not an unknown), 3 dofs per node."""
    n = 3 * (int(idx.max()) + 1)
    rows, cols, vals = [], [], []
    mass = np.zeros(n)
    cache = {}
    for vz in range(lo[2], hi[2]):
        for vy in range(lo[1], hi[1]):
            for vx in range(lo[0], hi[0]):
                C = Cv[vx, vy, vz]
                key = C.tobytes()
                if key not in cache:
                    cache[key] = voxel_stiffness(C)
                K = cache[key]
                dof = []
                for (a, b, c) in _corners():
                    k = idx[vx + a, vy + b, vz + c]
                    dof.extend([3 * k, 3 * k + 1, 3 * k + 2] if k >= 0 else [-1, -1, -1])
                dof = np.array(dof)
                ok = dof >= 0
                r, q = np.meshgrid(dof[ok], dof[ok], indexing="ij")
                rows.append(r.ravel()); cols.append(q.ravel())
                vals.append(-K[np.ix_(ok, ok)].ravel())
                np.add.at(mass, dof[ok], rho[vx, vy, vz] / 8.0)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    A.sum_duplicates()
    return A, mass


def assemble_elastic(Cv, rho):
    """Fine pencil (A, b) on all unknowns: Cv[x, y, z] is the 6 x 6 stiffness
    of voxel (x, y, z), rho[x, y, z] its density."""
    nvox = rho.shape
    idx = fine.node_index(nvox)
    return _assemble(Cv, rho, (0, 0, 0), nvox, idx)


class ElasticPartition:
    """The scalar Cartesian partition with 3 dofs per node: cells, cell
    operators, and pieces whose bases are the scalar bases per component."""

    def __init__(self, nvox, cuts, modes_face, modes_edge):
        self.scalar = CartesianPartition(nvox, cuts, modes_face, modes_edge)
        self.nvox = self.scalar.nvox
        self.n = 3 * self.scalar.n
        self.cells = self.scalar.cells
        self.pieces = []
        for pc in self.scalar.pieces:
            dofs = (3 * pc.nodes[:, None] + np.arange(3)[None, :]).ravel()     # node-major, components x, y, z
            k, bs = pc.S.shape
            S = np.zeros((3 * k, 3 * bs))
            for l in range(bs):
                for c in range(3):
                    S[c::3, 3 * l + c] = pc.S[:, l]
            self.pieces.append((dofs, S, pc.cells))

    def piece_offsets(self):
        """Offsets of each piece's reduced dofs in the concatenated piece vector."""
        sizes = np.array([S.shape[1] for _, S, _ in self.pieces])
        return np.concatenate([[0], np.cumsum(sizes)])

    def cell_dofs(self, i):
        nodes = self.cells[i].nodes
        return (3 * nodes[:, None] + np.arange(3)[None, :]).ravel()

    def cell_operator(self, i, Cv, rho):
        """(A_i dense, b_i) on the cell's dofs (node-major, x-fastest nodes)."""
        c = self.cells[i]
        lo, hi = c.vox_lo, c.vox_hi
        # local node numbering of the cell's closed box without wall nodes
        sidx = -np.ones(tuple(int(h - l + 1) for l, h in zip(lo, hi)), dtype=np.int64)
        gidx = self.scalar.idx[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1]
        pos = {int(g): k for k, g in enumerate(c.nodes)}
        for (a, b, cc), g in np.ndenumerate(gidx):
            if g >= 0:
                sidx[a, b, cc] = pos[int(g)]
        sub_C = Cv[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        sub_r = rho[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        A, m = _assemble(sub_C, sub_r, (0, 0, 0), sub_r.shape, sidx)
        return A.toarray(), m

    def cell_W(self, i):
        """W_i = P^Gamma_i S_i over the cell's dofs, columns by ascending piece."""
        dofs = self.cell_dofs(i)
        pos = {int(g): k for k, g in enumerate(dofs)}
        cols = []
        for p in self.cells[i].pieces:
            pd, S, _ = self.pieces[p]
            block = np.zeros((len(dofs), S.shape[1]))
            block[[pos[int(g)] for g in pd], :] = S
            cols.append(block)
        return np.concatenate(cols, axis=1)

    def point_columns(self, coords, comp=2):
        """Projected point forces along component ``comp`` at skeleton nodes:
        fine columns S_p S_p^T e_dof and reduced coefficients (piece, S_p^T e_dof)."""
        G = np.zeros((self.n, len(coords)))
        red = []
        for j, (x, y, z) in enumerate(coords):
            k = int(self.scalar.idx[x, y, z])
            p = int(self.scalar.piece_of_node[k])
            if k < 0 or p < 0:
                raise ValueError("point not on the skeleton (eq. gsupport)")
            pd, S, _ = self.pieces[p]
            e = np.zeros(len(pd))
            e[int(np.where(pd == 3 * k + comp)[0][0])] = 1.0
            coef = S.T @ e
            G[pd, j] = S @ coef
            red.append((p, coef))
        return G, red
