"""Corner-set removal with hanging nodes (App. B, with the 2D example of
Sec. 3) and the per-step solution correction at the corner-set nodes
(App. D, Remark solcorr).

Test infrastructure only: plain numpy/scipy on FP64, python loops over the
nonzeros. Nothing here is imported by the product.

A partition with three or more cells at a node has a non-empty corner set
(eq. nocorners fails). App. B replaces every corner node k by hanging nodes,
one per pair interface Gamma_ij through k, each held by the two cells i and
j only, and removes k; afterwards every skeleton node lies in exactly two
cells and the skeleton pieces are the pair interfaces. App. D then nudges,
after each time step, the ROM values at the copies of k toward their
mass-weighted mean.

Readings (the paper leaves these open or states them inconsistently):

* Corner set: the nodes held by three or more cells.
* Pairs of a corner node k: the pairs {i, j} of cells holding k that also
  share a node outside the corner set (a face in the Cartesian case; the
  four copies up/low/left/right of the 2D example). If some cell holding k
  lies in none of those pairs, every pair of cells holding k is used.
* Entries of the hanging nodes. App. B copies each cell's whole row of k
  into every copy of k. That puts the same link several times into the rows
  of k's neighbours while their diagonals stay as they were, so A' is
  indefinite, and it multiplies the corner mass (by 2 in the 2D example),
  which App. D's weighted mean divided by b_kk cannot match. Here cell c's
  entries at k are shared equally among c's n_c(k) copies of k:
  - a link (k, l) of weight w to a node l outside the corner set gives
    w / n_c(k) from each copy of k to l;
  - a link between two corner nodes k and l goes from the copy of k to the
    copy of l of the same pair, w / |Q| for each of the Q pairs both copies
    have in c; if they have none, w / (n_c(k) n_c(l)) between every copy
    of k and every copy of l;
  - the row sum d_k of c's row k (diagonal plus links) is shared as
    d_k / n_c(k) on each copy's diagonal, and each copy's diagonal also
    loses the weights of its links;
  - the mass b_c(k) is shared as b_c(k) / n_c(k).
  With E the map that copies the value at k to all its copies, E^T A'_c E
  = A_c and E^T B'_c E = B_c, hence E^T A' E = A and E^T B' E = B; a cell
  operator that is a weighted graph Laplacian with a non-positive diagonal
  remainder stays one (Prop. 2's sign).
* App. D weights: omega_l = b'_l / b_k for the copies l of k; under the
  sharing above they sum to one, so the value at k is the mass-weighted mean
  of its copies.
* Numbering: old nodes in ascending order; a node outside the corner set
  keeps one new id, a corner node gets one id per pair, pairs in
  lexicographic order. Each cell's row sums and diagonal updates run over
  its row in ascending old column order.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np
import scipy.sparse as sp

from .divconq import GeneralPartition, Subdomain


def owner_sets(subs, n):
    owners = [[] for _ in range(n)]
    for c, s in enumerate(subs):
        for g in s.nodes:
            owners[int(g)].append(c)
    return owners


def hanging_pairs(owners) -> Dict[int, List[Tuple[int, int]]]:
    """Corner nodes (held by >= 3 cells) and their pairs, per the reading above."""
    iface = set()
    for own in owners:
        if len(own) == 2:
            iface.add((own[0], own[1]))
    out = {}
    for k, own in enumerate(owners):
        if len(own) < 3:
            continue
        allp = [(own[a], own[b]) for a in range(len(own)) for b in range(a + 1, len(own))]
        pairs = [p for p in allp if p in iface]
        covered = {c for p in pairs for c in p}
        out[k] = pairs if covered == set(own) else allp
    return out


class HangingPartition(GeneralPartition):
    """The partition of ``part`` (a GeneralPartition) after corner-set
    removal: same cells, new node numbering, pairwise pieces, and the maps
    the correction and the old-node sources and receivers need."""

    def __init__(self, part: GeneralPartition):
        self.orig = part
        n0 = part.n
        owners = owner_sets(part.subs, n0)
        pairs = hanging_pairs(owners)
        self.corner_nodes = np.array(sorted(pairs), dtype=np.int64)
        new_of_old = -np.ones(n0, dtype=np.int64)
        copy_id = {}
        nid = 0
        for g in range(n0):
            if g in pairs:
                for pr in pairs[g]:
                    copy_id[(g, pr)] = nid
                    nid += 1
            else:
                new_of_old[g] = nid
                nid += 1
        self.new_of_old = new_of_old
        self.copy_id = copy_id
        self.pairs = pairs
        n1 = nid

        def copies(c, g):
            """[(pair or None, new id)] of old node g in cell c."""
            if g in pairs:
                return [(pr, copy_id[(g, pr)]) for pr in pairs[g] if c in pr]
            return [(None, int(new_of_old[g]))]

        subs = []
        for c, s in enumerate(part.subs):
            A = sp.csr_matrix(s.A)
            A.sort_indices()
            ent = {}
            bnew = {}
            for r in range(len(s.nodes)):
                g = int(s.nodes[r])
                cg = copies(c, g)
                ng = len(cg)
                lo, hi = A.indptr[r], A.indptr[r + 1]
                d = 0.0
                for t in range(lo, hi):
                    d += A.data[t]
                for pr_a, a_id in cg:
                    diag = d / ng
                    for t in range(lo, hi):
                        l = int(A.indices[t])
                        if l == r:
                            continue
                        w = A.data[t]
                        gl = int(s.nodes[l])
                        cl = copies(c, gl)
                        nl = len(cl)
                        if g in pairs and gl in pairs:
                            Q = [p for p, _ in cg if any(p == q for q, _ in cl)]
                            if Q:
                                tg = [(i, w / len(Q)) for p, i in cl if p == pr_a] if pr_a in Q else []
                            else:
                                tg = [(i, w / (ng * nl)) for _, i in cl]
                        elif g in pairs:
                            tg = [(cl[0][1], w / ng)]
                        elif gl in pairs:
                            tg = [(i, w / nl) for _, i in cl]
                        else:
                            tg = [(cl[0][1], w)]
                        for i, wt in tg:
                            ent[(a_id, i)] = wt
                            diag -= wt
                    ent[(a_id, a_id)] = diag
                    bnew[a_id] = s.b[r] / ng
            nodes = np.array(sorted(bnew), dtype=np.int64)
            pos = {int(x): k for k, x in enumerate(nodes)}
            rr = [pos[i] for i, _ in ent]
            cc = [pos[j] for _, j in ent]
            An = sp.csr_matrix((list(ent.values()), (rr, cc)), shape=(len(nodes), len(nodes)))
            An.sort_indices()
            subs.append(Subdomain(nodes, An, np.array([bnew[int(x)] for x in nodes])))

        self.n = n1
        A1 = sp.csr_matrix((n1, n1))
        b1 = np.zeros(n1)
        for s in subs:
            P = sp.csr_matrix((np.ones(len(s.nodes)), (s.nodes, np.arange(len(s.nodes)))), shape=(n1, len(s.nodes)))
            A1 = A1 + P @ s.A @ P.T
            b1[s.nodes] += s.b
        self.A = sp.csr_matrix(A1)
        self.A.sort_indices()
        self.b = b1
        self._index(subs)

        # App. D: copies of each corner node and their weights b'_l / b_k
        ptr, hn, hw = [0], [], []
        for k in self.corner_nodes:
            for pr in pairs[int(k)]:
                l = copy_id[(int(k), pr)]
                hn.append(l)
                hw.append(self.b[l] / part.b[int(k)])
            ptr.append(len(hn))
        self.hang_ptr = np.array(ptr, dtype=np.int64)
        self.hang_node = np.array(hn, dtype=np.int64)
        self.hang_weight = np.array(hw)
        # E: old -> new, copying a corner node's value to all its copies
        rows, cols = [], []
        for g in range(n0):
            if new_of_old[g] >= 0:
                rows.append(int(new_of_old[g])); cols.append(g)
        for (g, _), i in copy_id.items():
            rows.append(i); cols.append(g)
        self.E = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n1, n0))

    def old_node_weights(self, g):
        """[(new node, weight)] whose weighted sum is the value at old node g
        (the node itself, or the mass-weighted mean of its copies)."""
        g = int(g)
        if self.new_of_old[g] >= 0:
            return [(int(self.new_of_old[g]), 1.0)]
        k = int(np.searchsorted(self.corner_nodes, g))
        lo, hi = self.hang_ptr[k], self.hang_ptr[k + 1]
        return [(int(self.hang_node[t]), float(self.hang_weight[t])) for t in range(lo, hi)]

    def old_reduced_columns(self, rom, nodes):
        """Reduced columns (rom.ndof x len(nodes)) of point sources or
        receivers at old nodes: sum over the node's copies l of omega_l
        S_p^T e_l (for a receiver, the mass-weighted mean of the copies; for
        a source, the load shared in proportion to the copies' masses)."""
        F = np.zeros((rom.ndof, len(nodes)))
        for j, g in enumerate(nodes):
            for l, wt in self.old_node_weights(g):
                p = int(self.piece_of_node[l])
                if p < 0:
                    raise ValueError("point not on the skeleton (eq. gsupport)")
                pc = self.pieces[p]
                r = int(np.searchsorted(pc.nodes, l))
                F[rom.poff[p]:rom.poff[p + 1], j] += wt * pc.S[r, :]
        return F


def correct(HP: HangingPartition, rom, Y):
    """App. D on the piece dofs of Y (rom.ndof x n_s), in place: for every
    corner node k, u_l = e_l^T S_p y_p at its copies l, the mean
    ubar_k = sum_l omega_l u_l, delta_l = ubar_k - u_l, then
    y_p += S_p^T (delta on p's copies). All deltas are taken before any
    update."""
    upd = []
    for k in range(len(HP.corner_nodes)):
        lo, hi = HP.hang_ptr[k], HP.hang_ptr[k + 1]
        uh = []
        for t in range(lo, hi):
            l = int(HP.hang_node[t])
            p = int(HP.piece_of_node[l])
            pc = HP.pieces[p]
            r = int(np.searchsorted(pc.nodes, l))
            row = pc.S[r, :]
            uh.append((p, row, row @ Y[rom.poff[p]:rom.poff[p + 1], :]))
        ubar = sum(HP.hang_weight[lo + i] * u for i, (_, _, u) in enumerate(uh))
        for p, row, u in uh:
            upd.append((p, row, ubar - u))
    for p, row, d in upd:
        Y[rom.poff[p]:rom.poff[p + 1], :] += np.outer(row, d)
    return Y


def leapfrog_corrected(HP: HangingPartition, rom, F, Qr, w, dt):
    """GlobalROM.leapfrog with App. D applied to every new level Y^{n+1}
    before it is recorded and used."""
    import scipy.sparse.linalg as spla
    lu = spla.splu(rom.D.tocsc())
    ns = F.shape[1]
    Y = np.zeros((rom.ndof, ns)); Yp = np.zeros_like(Y)
    out = np.empty((len(w), Qr.shape[1], ns))
    dt2 = dt * dt
    for k in range(len(w)):
        acc = lu.solve(rom.L @ Y + w[k] * F)
        Yn = 2.0 * Y - Yp + dt2 * acc
        correct(HP, rom, Yn)
        Yp, Y = Y, Yn
        out[k] = Qr.T @ Y
    return out
