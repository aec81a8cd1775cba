"""Divide-and-conquer partition and splitting of a general sparse pencil
(A, B) (App. A: Lemma 1, Prop. 1, Alg. 1 with eq. alg1B, Prop. 2 and the
multidomain algorithm Alg. 2; Sec. 2 for the notation: adjacency, the
neighbourhood of a node set, eq. part, eq. splitN_c).

Test infrastructure only: plain numpy/scipy on FP64, python loops over the
nonzeros, no blocking. Nothing here is imported by the product.

Readings (the paper leaves these choices open):

* Adjacency is the nonzero pattern of the subdomain's own operator: k and l
  are adjacent iff a_kl != 0 (Sec. 2); a node is adjacent to itself.
* Choice of the set O of Prop. 1 in Alg. 2: a breadth-first level
  structure of the subdomain's graph rooted at a pseudo-peripheral node. The
  root search starts at the subdomain's smallest node and moves to the
  node of smallest degree (then smallest index) in the last level while the
  depth grows. O is the union of levels 0..j, where level j + 1 is the
  first level at which the running count of nodes reaches half of the
  subdomain (the separator level holds the median node); j is kept in
  [0, e - 2] (e the depth) so that the neighbourhood of O is not the whole
  subdomain.
  Nodes the root cannot reach count as beyond the last level. Then
  O_2 = Omega \\ A(O) is levels j + 2 and beyond, O_1 = Omega \\ A(O_2) is
  levels 0..j and Gamma is level j + 1. A subdomain of depth < 2 is not
  split.
* Alg. 2 splits the subdomain with the most nodes (ties: the lowest
  position) among those that can be split, after swapping it with the last
  position p, and puts the O_1 side at p and the O_2 side at p + 1.
* alpha_kl = alpha and beta_k = beta are constants (1/2 by default, the
  balancing choice of the one- and two-domain examples of Sec. 2).
* Pieces of the skeleton: nodes that belong to two or more subdomains,
  grouped by the exact set of subdomains holding them (the general
  interior-elimination form instead of hanging nodes); pieces are ordered by
  their smallest node, and a piece's nodes ascend.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import scipy.sparse as sp


# ---------------------------------------------------------------------------
# Sec. 2: adjacency and neighbourhoods
# ---------------------------------------------------------------------------

def neighbourhood(A: sp.csr_matrix, inset: np.ndarray) -> np.ndarray:
    """The neighbourhood A(O) of the node set O (boolean mask over A's rows):
    every node l with a_kl != 0 for some k in O, O itself included (Lemma 1:
    the diagonal is nonzero)."""
    A = sp.csr_matrix(A)
    out = inset.copy()
    for k in np.where(inset)[0]:
        for t in range(A.indptr[k], A.indptr[k + 1]):
            if A.data[t] != 0.0:
                out[A.indices[t]] = True
    return out


# ---------------------------------------------------------------------------
# Prop. 1: the constructive two-way partition
# ---------------------------------------------------------------------------

def prop1_split(A, O: np.ndarray):
    """O_1, O_2, Gamma (boolean masks) from a set O with A(O) a proper subset
    of Omega: O_2 = Omega \\ A(O), O_1 = Omega \\ A(O_2), Gamma the rest."""
    AO = neighbourhood(A, O)
    if AO.all():
        raise ValueError("A(O) is the whole domain: Prop. 1 does not apply")
    O2 = ~AO
    O1 = ~neighbourhood(A, O2)
    Gamma = ~(O1 | O2)
    return O1, O2, Gamma


# ---------------------------------------------------------------------------
# Alg. 1 and eq. alg1B: splitting of the operator and the mass
# ---------------------------------------------------------------------------

def alg1_split(A, b, O1, O2, Gamma, alpha=0.5, beta=0.5):
    """Split (A, diag(b)) of a subdomain into (A^1, b^1) on Omega_1 = O_1 u
    Gamma and (A^2, b^2) on Omega_2 = O_2 u Gamma.

    Returns [(nodes_1, A^1, b^1), (nodes_2, A^2, b^2)]: local node indices
    (ascending) and the split operators in that order. ``alpha`` may be a
    callable alpha(k, l) (symmetric), ``beta`` a per-node array."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    O = [O1, O2]
    ent = [[dict() for _ in range(n)], [dict() for _ in range(n)]]     # row k: {l: a^i_kl}
    for k in range(n):
        for t in range(A.indptr[k], A.indptr[k + 1]):
            l = int(A.indices[t]); a = float(A.data[t])
            if (O1[k] and O2[l]) or (O2[k] and O1[l]):
                if a != 0.0:
                    raise ValueError("coupling between O_1 and O_2 (Prop. 1 violated)")
                continue
            placed = False
            for i in range(2):                 # entries at a node of O_i
                if O[i][k] or O[i][l]:
                    ent[i][k][l] = a
                    placed = True
            if placed:
                continue
            if k != l:                         # links inside Gamma, split by alpha
                al = alpha(k, l) if callable(alpha) else alpha
                ent[0][k][l] = al * a
                ent[1][k][l] = (1.0 - al) * a
    # Gamma diagonals in proportion to the off-diagonal sums
    for k in np.where(Gamma)[0]:
        s = [sum(abs(v) for l, v in ent[i][k].items() if l != k) for i in range(2)]
        akk = float(A[k, k])
        for i in range(2):
            ent[i][k][int(k)] = akk * s[i] / (s[0] + s[1])
    out = []
    for i in range(2):
        nodes = np.where(O[i] | Gamma)[0]
        pos = -np.ones(n, dtype=np.int64); pos[nodes] = np.arange(len(nodes))
        rows, cols, vals = [], [], []
        for k in nodes:
            for l, v in ent[i][k].items():
                rows.append(pos[k]); cols.append(pos[l]); vals.append(v)
        Ai = sp.csr_matrix((vals, (rows, cols)), shape=(len(nodes), len(nodes)))
        bt = beta if np.isscalar(beta) else None
        bi = np.empty(len(nodes))
        for r, k in enumerate(nodes):
            if O[i][k]:
                bi[r] = b[k]
            else:                              # eq. alg1B on Gamma
                bk = bt if bt is not None else beta[k]
                bi[r] = (bk if i == 0 else 1.0 - bk) * b[k]
        out.append((nodes, Ai, bi))
    return out


# ---------------------------------------------------------------------------
# The set O of Prop. 1 for a subdomain: breadth-first level structure
# ---------------------------------------------------------------------------

def _levels(A, root):
    """Breadth-first levels from ``root`` (unreached nodes get -1)."""
    n = A.shape[0]
    lev = -np.ones(n, dtype=np.int64)
    lev[root] = 0
    q = deque([root])
    while q:
        k = q.popleft()
        for t in range(A.indptr[k], A.indptr[k + 1]):
            l = A.indices[t]
            if A.data[t] != 0.0 and lev[l] < 0:
                lev[l] = lev[k] + 1
                q.append(l)
    return lev


def pseudo_peripheral_root(A) -> int:
    A = sp.csr_matrix(A)
    deg = np.array([np.count_nonzero(A.data[A.indptr[k]:A.indptr[k + 1]]) for k in range(A.shape[0])])
    root = 0
    lev = _levels(A, root)
    depth = int(lev.max())
    while True:
        last = np.where(lev == depth)[0]
        cand = int(last[np.lexsort((last, deg[last]))[0]])     # smallest degree, then index
        lv = _levels(A, cand)
        if int(lv.max()) > depth:
            root, lev, depth = cand, lv, int(lv.max())
        else:
            return root


def level_set_O(A) -> Optional[np.ndarray]:
    """The set O of the reading above, or None if the subdomain cannot be
    split (depth < 2)."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    lev = _levels(A, pseudo_peripheral_root(A))
    e = int(lev.max())
    if e < 2:
        return None
    counts = np.bincount(lev[lev >= 0], minlength=e + 1)
    cum = np.cumsum(counts)
    m = int(np.searchsorted(cum, 0.5 * n))              # first level with cum >= n/2
    j = min(max(m - 1, 0), e - 2)
    return (lev >= 0) & (lev <= j)


# ---------------------------------------------------------------------------
# Alg. 2: divide and conquer
# ---------------------------------------------------------------------------

@dataclass
class Subdomain:
    nodes: np.ndarray             # global node indices, ascending
    A: sp.csr_matrix              # split operator on these nodes
    b: np.ndarray


def alg2_partition(A, b, n_cells: int, alpha=0.5, beta=0.5,
                   choose_O: Callable = None) -> List[Subdomain]:
    """Alg. 2: repeatedly split one subdomain with Prop. 1 + Alg. 1 until
    there are ``n_cells``. ``choose_O(sub)`` returns the set O (mask over
    sub.nodes) or None; the default is :func:`level_set_O` on sub.A."""
    A = sp.csr_matrix(A)
    subs = [Subdomain(np.arange(A.shape[0]), A, np.asarray(b, dtype=float).copy())]
    pick = choose_O or (lambda s: level_set_O(s.A))
    while len(subs) < n_cells:
        order = sorted(range(len(subs)), key=lambda i: (-len(subs[i].nodes), i))
        found = None
        for i in order:                        # the largest splittable subdomain
            O = pick(subs[i])
            if O is not None:
                found = (i, O)
                break
        if found is None:
            raise ValueError(f"no subdomain can be split further ({len(subs)} of {n_cells})")
        i, O = found
        p = len(subs) - 1
        subs[i], subs[p] = subs[p], subs[i]    # moved to the last position
        s = subs[p]
        O1, O2, G = prop1_split(s.A, O)        # Prop. 1 sets
        (n1, A1, b1), (n2, A2, b2) = alg1_split(s.A, s.b, O1, O2, G, alpha, beta)   # Alg. 1 split
        subs[p] = Subdomain(s.nodes[n1], A1, b1)                                    # O_1 side in place
        subs.append(Subdomain(s.nodes[n2], A2, b2))
    return subs


# ---------------------------------------------------------------------------
# Cells and skeleton pieces of a general partition
# ---------------------------------------------------------------------------

@dataclass
class GPiece:
    nodes: np.ndarray             # global nodes, ascending
    cells: List[int]              # subdomains holding them, ascending
    S: np.ndarray = None          # k_p x b_p orthonormal basis


@dataclass
class GCell:
    nodes: np.ndarray
    pieces: List[int] = field(default_factory=list)


class GeneralPartition:
    """Cells from Alg. 2 and pieces grouped by owner sets, with the
    interface the global ROM uses (cells, pieces, piece_offsets, cell_W,
    point_columns) plus the split operators."""

    def __init__(self, A, b, n_cells: int, alpha=0.5, beta=0.5, choose_O=None):
        self.A = sp.csr_matrix(A)
        self.b = np.asarray(b, dtype=float)
        self.n = self.A.shape[0]
        self._index(alg2_partition(self.A, self.b, n_cells, alpha, beta, choose_O))

    def _index(self, subs):
        """Cells, and pieces grouped by owner sets, of the subdomains ``subs``."""
        self.subs = subs
        self.cells = [GCell(s.nodes) for s in self.subs]
        owners = [[] for _ in range(self.n)]
        for c, s in enumerate(self.subs):
            for g in s.nodes:
                owners[int(g)].append(c)
        groups = {}
        for g in range(self.n):
            if len(owners[g]) >= 2:
                groups.setdefault(tuple(owners[g]), []).append(g)
        keys = sorted(groups, key=lambda k: groups[k][0])
        self.pieces = [GPiece(np.array(groups[k], dtype=np.int64), list(k)) for k in keys]
        self.piece_of_node = -np.ones(self.n, dtype=np.int64)
        for p, pc in enumerate(self.pieces):
            self.piece_of_node[pc.nodes] = p
            for c in pc.cells:
                self.cells[c].pieces.append(p)

    def cell_operator(self, i):
        """(A_i dense, b_i) on the cell's nodes in ascending global order."""
        s = self.subs[i]
        return s.A.toarray(), s.b.copy()

    def set_bases(self, bases):
        for pc, S in zip(self.pieces, bases):
            pc.S = np.asarray(S, dtype=float)

    def cell_W(self, i):
        c = self.cells[i]
        pos = {int(g): k for k, g in enumerate(c.nodes)}
        b = sum(self.pieces[p].S.shape[1] for p in c.pieces)
        W = np.zeros((len(c.nodes), b))
        col = 0
        for p in c.pieces:
            pc = self.pieces[p]
            W[[pos[int(g)] for g in pc.nodes], col:col + pc.S.shape[1]] = pc.S
            col += pc.S.shape[1]
        return W

    def piece_offsets(self):
        sizes = np.array([p.S.shape[1] for p in self.pieces])
        return np.concatenate([[0], np.cumsum(sizes)])

    def point_columns(self, nodes):
        """Projected point columns S_p S_p^T e_k at skeleton nodes (eq.
        gsupport) and their reduced coefficients (piece, S_p^T e_k)."""
        G = np.zeros((self.n, len(nodes)))
        red = []
        for j, k in enumerate(nodes):
            p = int(self.piece_of_node[int(k)])
            if p < 0:
                raise ValueError("point not on the skeleton (eq. gsupport)")
            pc = self.pieces[p]
            r = int(np.searchsorted(pc.nodes, k))
            coeff = pc.S[r, :].copy()
            G[pc.nodes, j] = pc.S @ coeff
            red.append((p, coeff))
        return G, red
