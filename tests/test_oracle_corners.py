"""Pins of the corner-set removal (App. B) and the App. D correction in the
oracle (oracle/corners.py), against facts that do not come from the code
under test:

* conservation: E^T A' E = A and E^T B' E = B, with E the map copying an old
  node's value to its hanging copies (the reading's defining property), and
  App. D's weights b'_l / b_k summing to one;
* after the removal every skeleton node lies in exactly two cells
  (eq. nocorners) and every piece is a pair interface;
* the 2D example of Sec. 3: a 2 x 2 partition of a square grid has one
  corner node with four hanging copies, one per face-adjacent pair
  (up / low / left / right); on a 2 x 2 x 2 partition of a cube the edge
  nodes get four copies and the centre twelve;
* the cell operators stay <= 0 (Prop. 2's sign), while App. B's rule as
  printed (each cell row copied whole into every copy) gives an indefinite
  A' on the same 2D example: the reason for the reading;
* the correction at the fine level: with complete piece bases (S_p = I) the
  correction sets the copies to the value the original grid would have, so
  the hanging-node leapfrog with the correction after every step equals the
  original leapfrog (E u) to rounding; with equal-weight means instead of
  the mass-weighted ones it does not.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import corners as cn
from oracle import divconq as dc
from oracle import fine


def voxel_partition(nvox_cell, ncell, sigma=1.0, rho=1.0):
    """Uniform voxel grid in len(ncell) dimensions (Neumann), cells of
    nvox_cell voxels per axis: each voxel gives every one of its edges the
    weight sigma / 2^(d-1) and every corner the mass rho / 2^d; a cell's
    operator is the sum over its voxels. Returns a GeneralPartition built
    from these cells."""
    d = len(ncell)
    nn = [nvox_cell * c + 1 for c in ncell]
    idx = np.arange(int(np.prod(nn))).reshape(nn)
    subs = []
    for cpos in np.ndindex(*ncell):
        lo = [c * nvox_cell for c in cpos]
        nodes = idx[tuple(slice(l, l + nvox_cell + 1) for l in lo)].ravel()
        nodes = np.sort(nodes)
        pos = {int(g): k for k, g in enumerate(nodes)}
        n = len(nodes)
        A = np.zeros((n, n)); b = np.zeros(n)
        for v in np.ndindex(*([nvox_cell] * d)):
            corner = [lo[a] + v[a] for a in range(d)]
            verts = [idx[tuple(corner[a] + o[a] for a in range(d))] for o in np.ndindex(*([2] * d))]
            for g in verts:
                b[pos[int(g)]] += rho / 2 ** d
            offs = list(np.ndindex(*([2] * d)))
            for i, oi in enumerate(offs):
                for j, oj in enumerate(offs):
                    if j <= i or sum(abs(x - y) for x, y in zip(oi, oj)) != 1:
                        continue
                    p, q = pos[int(verts[i])], pos[int(verts[j])]
                    w = sigma / 2 ** (d - 1)
                    A[p, q] += w; A[q, p] += w; A[p, p] -= w; A[q, q] -= w
        subs.append(dc.Subdomain(nodes, sp.csr_matrix(A), b))
    P = dc.GeneralPartition.__new__(dc.GeneralPartition)
    N = int(np.prod(nn))
    At = sp.csr_matrix((N, N)); bt = np.zeros(N)
    for s in subs:
        E = sp.csr_matrix((np.ones(len(s.nodes)), (s.nodes, np.arange(len(s.nodes)))), shape=(N, len(s.nodes)))
        At = At + E @ s.A @ E.T
        bt[s.nodes] += s.b
    P.A, P.b, P.n = sp.csr_matrix(At), bt, N
    P._index(subs)
    return P, idx


def _acoustic_partition(nvox=(16, 16, 16), cells=8, seed=21):
    sig, rho = synth.acoustic_medium(nvox, seed, ell_sigma=5.0, ell_rho=2.0)
    A, b = fine.assemble_acoustic(sig, rho)
    A = sp.csr_matrix(A); A.sort_indices()
    return dc.GeneralPartition(A, b, cells)


def _check_conservation(P, H):
    E = H.E
    D = (E.T @ H.A @ E - P.A).tocoo()
    assert np.abs(D.data).max(initial=0.0) <= 1e-13 * np.abs(P.A.data).max()
    assert np.abs(E.T @ H.b - P.b).max() <= 1e-15 * P.b.max()
    sums = np.add.reduceat(H.hang_weight, H.hang_ptr[:-1])
    assert np.abs(sums - 1.0).max() <= 1e-14
    own = cn.owner_sets(H.subs, H.n)
    assert max(len(o) for o in own) == 2
    assert all(len(pc.cells) == 2 for pc in H.pieces)
    # every old node is either kept or has copies, never both
    kept = H.new_of_old >= 0
    assert not kept[H.corner_nodes].any() and kept.sum() + len(H.corner_nodes) == P.n


def _fallback_nodes(P):
    """Corner nodes one of whose cells shares no node outside the corner set
    with another of its cells (every pair of its cells gets a copy)."""
    owners = cn.owner_sets(P.subs, P.n)
    iface = {tuple(o) for o in owners if len(o) == 2}
    out = []
    for k, own in enumerate(owners):
        if len(own) < 3:
            continue
        pairs = [(own[a], own[c]) for a in range(len(own)) for c in range(a + 1, len(own)) if (own[a], own[c]) in iface]
        if {x for pr in pairs for x in pr} != set(own):
            out.append(k)
    return out


@pytest.mark.parametrize("case", ["acoustic", "graph", "graph_fallback"])
def test_conservation_and_pairwise_pieces(case):
    if case == "acoustic":
        P = _acoustic_partition()
    elif case == "graph":
        A, b, _ = synth.geometric_graph(1500, 6, 5)
        P = dc.GeneralPartition(A, b, 5)
    else:
        A, b, _ = synth.geometric_graph(3000, 6, 7)
        P = dc.GeneralPartition(A, b, 6)
        fb = _fallback_nodes(P)
        assert len(fb) >= 1
        own = cn.owner_sets(P.subs, P.n)
        pairs_all = len(own[fb[0]]) * (len(own[fb[0]]) - 1) // 2
    H = cn.HangingPartition(P)
    assert len(H.corner_nodes) > 0
    if case == "graph_fallback":
        assert len(H.pairs[fb[0]]) == pairs_all
    _check_conservation(P, H)
    for s in H.subs:
        assert np.linalg.eigvalsh(s.A.toarray()).max() <= 1e-12 * np.abs(s.A.data).max()


def test_2d_example_four_copies():
    P, idx = voxel_partition(3, (2, 2))
    H = cn.HangingPartition(P)
    centre = int(idx[3, 3])
    assert list(H.corner_nodes) == [centre]
    # cells in lexicographic order: 0 = (0,0), 1 = (0,1), 2 = (1,0), 3 = (1,1);
    # face-adjacent pairs only (the diagonal pairs share nothing but the centre)
    assert H.pairs[centre] == [(0, 1), (0, 2), (1, 3), (2, 3)]
    lo, hi = H.hang_ptr[0], H.hang_ptr[1]
    assert hi - lo == 4
    assert np.allclose(H.b[H.hang_node[lo:hi]], P.b[centre] / 4)
    _check_conservation(P, H)
    for s in H.subs:
        assert np.linalg.eigvalsh(s.A.toarray()).max() <= 1e-12


def test_3d_counts():
    P, idx = voxel_partition(2, (2, 2, 2))
    H = cn.HangingPartition(P)
    counts = {int(k): int(H.hang_ptr[i + 1] - H.hang_ptr[i]) for i, k in enumerate(H.corner_nodes)}
    assert counts[int(idx[2, 2, 2])] == 12
    edge = [int(idx[2, 2, 0]), int(idx[2, 0, 2]), int(idx[0, 2, 2]), int(idx[2, 2, 4])]
    assert all(counts[e] == 4 for e in edge)
    assert len(counts) == 6 * 2 + 1     # six half-edges of two nodes around the centre, and the centre
    _check_conservation(P, H)
    for s in H.subs:
        assert np.linalg.eigvalsh(s.A.toarray()).max() <= 1e-12


def _literal_app_b(P, H):
    """A' by App. B as printed: copy k_ij gets (P_i A_i P_i^T + P_j A_j P_j^T)
    at row k whole, links to kept nodes included; kept rows unchanged."""
    n = H.n
    A = np.zeros((n, n))
    Aold = P.A.toarray()
    cellA = []
    for s in P.subs:
        E = sp.csr_matrix((np.ones(len(s.nodes)), (s.nodes, np.arange(len(s.nodes)))), shape=(P.n, len(s.nodes)))
        cellA.append((E @ s.A @ E.T).toarray())
    kept = np.where(H.new_of_old >= 0)[0]
    for g in kept:
        for l in kept:
            A[H.new_of_old[g], H.new_of_old[l]] = Aold[g, l]
    for (k, (i, j)), cid in H.copy_id.items():
        rowk = cellA[i][k] + cellA[j][k]
        A[cid, cid] = rowk[k]
        for l in kept:
            if rowk[l] != 0.0:
                A[cid, H.new_of_old[l]] = A[H.new_of_old[l], cid] = rowk[l]
    return A


def test_app_b_as_printed_is_indefinite():
    P, _ = voxel_partition(3, (2, 2))
    H = cn.HangingPartition(P)
    lit = _literal_app_b(P, H)
    assert np.allclose(lit, lit.T)
    assert np.linalg.eigvalsh(lit).max() > 1e-3          # positive direction: indefinite
    assert np.linalg.eigvalsh(H.A.toarray()).max() <= 1e-12


class _IdentityRom:
    """What correct() reads of a ROM, for complete bases: the piece dofs are
    the piece nodes' values."""

    def __init__(self, H):
        sizes = [len(pc.nodes) for pc in H.pieces]
        self.poff = np.concatenate([[0], np.cumsum(sizes)])
        self.ndof = int(self.poff[-1])


def _fine_with_correction(H, G, Q, w, dt, weights=None):
    """Leapfrog of B' u'' = A' u + w G on the hanging grid, with correct()
    (complete bases) applied to every new level; traces Q^T u^{n+1}."""
    for pc in H.pieces:
        pc.S = np.eye(len(pc.nodes))
    rom = _IdentityRom(H)
    saved = H.hang_weight
    if weights is not None:
        H.hang_weight = weights
    skel = np.concatenate([pc.nodes for pc in H.pieces])
    n, ns = G.shape
    u = np.zeros((n, ns)); up = np.zeros_like(u)
    binv = (1.0 / H.b)[:, None]
    out = np.empty((len(w), Q.shape[1], ns))
    try:
        for k in range(len(w)):
            un = 2.0 * u - up + dt * dt * binv * (H.A @ u + w[k] * G)
            Y = un[skel].copy()
            cn.correct(H, rom, Y)
            un[skel] = Y
            up, u = u, un
            out[k] = Q.T @ u
    finally:
        H.hang_weight = saved
    return out


def test_correction_with_complete_bases_recovers_the_original_grid():
    P = _acoustic_partition()
    H = cn.HangingPartition(P)
    rng = np.random.default_rng(3)
    src = rng.choice(P.n, 3, replace=False)
    src[0] = H.corner_nodes[0]                  # one load on a removed node
    rec = np.concatenate([rng.choice(P.n, 10, replace=False), H.corner_nodes[:5]])
    G = np.zeros((P.n, len(src))); G[src, np.arange(len(src))] = 1.0
    Q = np.zeros((P.n, len(rec))); Q[rec, np.arange(len(rec))] = 1.0
    # a load at a removed node is shared among its copies by the weights;
    # a value there is the weighted sum of the copies
    Gh = np.zeros((H.n, len(src))); Qh = np.zeros((H.n, len(rec)))
    for j, g in enumerate(src):
        for l, wt in H.old_node_weights(g):
            Gh[l, j] += wt
    for j, g in enumerate(rec):
        for l, wt in H.old_node_weights(g):
            Qh[l, j] += wt
    dt = fine.cfl_dt(P.A, P.b, 0.5)
    w = synth.ricker(300, dt, 0.9 / (2 * np.pi * 2.5))
    ref = fine.leapfrog(P.A, P.b, G, Q, w, dt)
    got = _fine_with_correction(H, Gh, Qh, w, dt)
    e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert e <= 1e-12, e
    # without the correction, or with plain means, the hanging grid differs
    raw = fine.leapfrog(H.A, H.b, Gh, Qh, w, dt)
    assert np.linalg.norm(raw - ref) / np.linalg.norm(ref) > 1e-3
    flat = np.concatenate([np.full(H.hang_ptr[k + 1] - H.hang_ptr[k], 1.0 / (H.hang_ptr[k + 1] - H.hang_ptr[k]))
                           for k in range(len(H.corner_nodes))])
    if not np.allclose(flat, H.hang_weight):
        bad = _fine_with_correction(H, Gh, Qh, w, dt, weights=flat)
        assert np.linalg.norm(bad - ref) / np.linalg.norm(ref) > 1e-8


def test_correction_is_a_no_op_on_equal_copies():
    P = _acoustic_partition((12, 12, 12), 6, 4)
    H = cn.HangingPartition(P)
    for pc in H.pieces:
        pc.S = np.eye(len(pc.nodes))
    rom = _IdentityRom(H)
    skel = np.concatenate([pc.nodes for pc in H.pieces])
    rng = np.random.default_rng(1)
    u = H.E @ rng.standard_normal((P.n, 2))     # copies equal by construction
    Y = u[skel].copy()
    cn.correct(H, rom, Y)
    assert np.abs(Y - u[skel]).max() <= 1e-15 * np.abs(u).max() * 10
