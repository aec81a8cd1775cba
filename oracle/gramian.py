"""Frequency-limited Gramian bases of skeleton pieces (Sec. 4.1, eqs.
specdec, trgr, trgrstep).

Test infrastructure only: dense numpy eigensolvers on FP64.

For a piece Gamma_p the Gramian is G_p = sum over the eigenpairs (lambda_l,
z_l) of the pencil (-A, B) with lambda_l <= omega_max^2 of v_l v_l^T, v_l
the restriction of z_l to the piece's nodes (eq. trgr). S_p holds the
eigenvectors of G_p whose eigenvalues exceed the truncation threshold.

Readings (the approximate Gramian of Sec. 4.1 is only outlined there, its
full description being in a reference that is not available):

* Eigenvectors are B-orthonormal, z_l^T B z_l = 1 (the pencil's natural
  normalisation; the paper does not state one).
* The threshold is relative: eigenvalues of G_p above eps times the largest
  are kept, at most ``max_modes`` of them (largest first). If no pencil
  eigenvalue lies below omega_max^2, the lowest eigenpair is used.
* The exact Gramian (:func:`exact_gramian`) uses the whole pencil (A, B).
  The approximate one (:func:`local_gramian`) replaces it by a smaller pencil
  with the same rows on the piece: the operators of the cells holding the
  piece summed on their union U (eq. splitN_c restricted to those cells),
  then cut to the nodes within graph distance ``depth`` + 1 of the piece by
  one Prop. 1 / Alg. 1 split of U with O the nodes within distance
  ``depth`` (alpha = beta = 1/2), so that the cut face gets the split's
  natural boundary. depth < 0 keeps the whole union.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import divconq


def pencil_eigs_below(A, b, omega_max):
    """Eigenpairs of -A z = lambda B z (B = diag(b)) with lambda <=
    omega_max^2, B-orthonormal (eq. specdec); at least the lowest one."""
    A = A.toarray() if sp.issparse(A) else np.asarray(A)
    r = 1.0 / np.sqrt(b)
    C = -(A * r[:, None]) * r[None, :]
    lam, Y = np.linalg.eigh(0.5 * (C + C.T))
    keep = lam <= omega_max ** 2
    if not keep.any():
        keep[0] = True
    return lam[keep], Y[:, keep] * r[:, None]


def gramian(V):
    """Eq. trgr: G = sum_l v_l v_l^T from the restricted eigenvectors (columns of V)."""
    return V @ V.T


def basis_from_gramian(G, eps, max_modes):
    """Eigenvectors of G with eigenvalue > eps * (largest), largest first, at
    most ``max_modes``."""
    ev, U = np.linalg.eigh(G)
    order = np.argsort(ev)[::-1]
    ev, U = ev[order], U[:, order]
    k = int(np.sum(ev > eps * ev[0])) if ev[0] > 0 else 1
    k = max(1, min(k, max_modes))
    return U[:, :k], ev


def exact_gramian(A, b, nodes, omega_max):
    """G_p of eq. trgr with the eigenpairs of the whole pencil."""
    _, Z = pencil_eigs_below(A, b, omega_max)
    return gramian(Z[nodes, :])


def union_pencil(cells, piece_cells):
    """(nodes, A_U, b_U) of the union of the given cells: sum_c P_c A_c P_c^T
    on the union's nodes (ascending global order). ``cells`` maps a cell id
    to (global nodes, A_c sparse or dense, b_c)."""
    nodes = np.unique(np.concatenate([cells[c][0] for c in piece_cells]))
    pos = {int(g): k for k, g in enumerate(nodes)}
    n = len(nodes)
    A = sp.csr_matrix((n, n)); b = np.zeros(n)
    for c in piece_cells:
        g, Ac, bc = cells[c]
        loc = np.array([pos[int(x)] for x in g])
        Pm = sp.csr_matrix((np.ones(len(loc)), (loc, np.arange(len(loc)))), shape=(n, len(loc)))
        A = A + Pm @ sp.csr_matrix(Ac) @ Pm.T
        b = b + Pm @ bc
    return nodes, sp.csr_matrix(A), b


def local_pencil(cells, piece_cells, piece_nodes, depth):
    """The approximate pencil of the reading above: (nodes, A_s, b_s)."""
    nodes, A, b = union_pencil(cells, piece_cells)
    if depth < 0:
        return nodes, A, b
    inset = np.isin(nodes, piece_nodes)
    for _ in range(depth):
        inset = divconq.neighbourhood(A, inset)
    if divconq.neighbourhood(A, inset).all():
        return nodes, A, b
    O1, O2, G = divconq.prop1_split(A, inset)
    (n1, A1, b1), _ = divconq.alg1_split(A, b, O1, O2, G, 0.5, 0.5)
    return nodes[n1], A1, b1


def local_gramian(cells, piece_cells, piece_nodes, omega_max, depth):
    snodes, As, bs = local_pencil(cells, piece_cells, piece_nodes, depth)
    _, Z = pencil_eigs_below(As, bs, omega_max)
    rows = np.searchsorted(snodes, piece_nodes)
    return gramian(Z[rows, :])


def gramian_bases(part, cell_ops, omega_max, eps, max_modes, depth):
    """S_p for every piece of ``part`` (anything with .pieces[p].nodes /
    .cells); ``cell_ops[c]`` = (global nodes, A_c, b_c). Single-node pieces
    get [1]."""
    out = []
    for pc in part.pieces:
        if len(pc.nodes) == 1:
            out.append(np.ones((1, 1)))
            continue
        G = local_gramian(cell_ops, pc.cells, pc.nodes, omega_max, depth)
        S, _ = basis_from_gramian(G, eps, max_modes)
        out.append(S)
    return out
