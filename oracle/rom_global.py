"""Global multi-scale ROM: boundary conjugation and time stepping (Sec. 6,
eqs. BEINCr, firsttstep_conj_td, intrtstep_td, contred, initial; Remark
Sinsubspace, eq. bdrytstep; Alg. alg1red stage 2).

The on-line step is an exactly defined linear recurrence once the
S-fraction blocks are known, so the oracle uses its plain definition: it
assembles the global stiffness L_glob = sum_i E_i^T L_i E_i and mass
D_glob = sum_i E_i^T D_i E_i explicitly as sparse matrices and runs the
textbook leapfrog D (Y^{n+1} - 2Y^n + Y^{n-1}) = dt^2 (L Y^n + w^n F).
It does not use the cell-blocked form the GPU kernels use.

Unknowns: reduced piece dofs y_p (the conjugated boundary values
u_ij = u_ji of eq. contred) first, then the hidden layers U_i^k, k = 2..m_i,
of every cell. E_i maps them to the cell's [U^1; ...; U^m], where U^1 is the
concatenation of the cell's piece dofs in the column order of W_i.
Force convention: D Y'' = L Y + w(t) F, F the reduced sources S_p^T g|_p
(the paper's source sign is common to the fine model and the ROM).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .rom_cell import layered_operator


class GlobalROM:
    def __init__(self, part, blocks):
        """``part``: CartesianPartition; ``blocks``: dict cell -> (Ghat, G)."""
        self.part = part
        self.poff = part.piece_offsets()
        npd = int(self.poff[-1])
        self.n_piece_dofs = npd
        off = npd
        self.hoff = {}
        for i in sorted(blocks):
            Ghat, G = blocks[i]
            b = G[0].shape[0]
            self.hoff[i] = off
            off += (len(G) - 1) * b
        self.ndof = off
        rows, cols, lv, dv = [], [], [], []
        for i in sorted(blocks):
            Ghat, G = blocks[i]
            L, D = layered_operator(Ghat, G)
            gl = self.cell_map(i, len(G), G[0].shape[0])
            r, c = np.meshgrid(gl, gl, indexing="ij")
            rows.append(r.ravel()); cols.append(c.ravel())
            lv.append(L.ravel()); dv.append(D.ravel())
        rows = np.concatenate(rows); cols = np.concatenate(cols)
        self.L = sp.csr_matrix((np.concatenate(lv), (rows, cols)), shape=(self.ndof, self.ndof))
        self.D = sp.csr_matrix((np.concatenate(dv), (rows, cols)), shape=(self.ndof, self.ndof))
        self.L.eliminate_zeros(); self.D.eliminate_zeros()

    def cell_map(self, i, m, b):
        """Global indices of cell i's [U^1; U^2; ...; U^m] (the map E_i)."""
        p = self.part
        u1 = np.concatenate([np.arange(self.poff[q], self.poff[q + 1]) for q in p.cells[i].pieces])
        assert len(u1) == b
        hid = self.hoff[i] + np.arange((m - 1) * b)
        return np.concatenate([u1, hid])

    def reduced_columns(self, red):
        """Reduced source/receiver columns from point_columns' (piece, coeff)."""
        F = np.zeros((self.ndof, len(red)))
        for j, (p, coeff) in enumerate(red):
            F[self.poff[p]:self.poff[p + 1], j] = coeff
        return F

    def leapfrog(self, F, Qr, w, dt, return_state=False):
        """Leapfrog of D Y'' = L Y + w(t) F from zero state; traces[n] =
        Qr^T Y^{n+1}. Shapes: F ndof x n_s, Qr ndof x n_r."""
        lu = spla.splu(self.D.tocsc())
        ns = F.shape[1]
        Y = np.zeros((self.ndof, ns)); Yp = np.zeros_like(Y)
        out = np.empty((len(w), Qr.shape[1], ns))
        dt2 = dt * dt
        for k in range(len(w)):
            acc = lu.solve(self.L @ Y + w[k] * F)
            Yn = 2.0 * Y - Yp + dt2 * acc
            Yp, Y = Y, Yn
            out[k] = Qr.T @ Y
        if return_state:
            return out, Y, Yp
        return out

    def energy(self, Yn, Y, dt):
        """Discrete leapfrog energy 1/2 v^T D v + 1/2 Yn^T (-L) Y."""
        v = (Yn - Y) / dt
        return 0.5 * np.sum(v * (self.D @ v), axis=0) + 0.5 * np.sum(Yn * (-(self.L @ Y)), axis=0)

    def lambda_max(self):
        """Largest eigenvalue of the pencil (-L, D)."""
        if self.ndof <= 3000:
            import scipy.linalg as sla
            return float(sla.eigh(-self.L.toarray(), self.D.toarray(), eigvals_only=True)[-1])
        lu = spla.splu(self.D.tocsc())
        op = spla.LinearOperator(self.L.shape, matvec=lambda x: lu.solve(-(self.L @ x)))
        return float(np.real(spla.eigs(op, k=1, which="LM", tol=1e-10, return_eigenvectors=False)[0]))
