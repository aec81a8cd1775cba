"""Pins of the oracle's partition, operator splitting (Sec. 2, eq. splitN_c;
App. A, Prop. 2) and piece bases (Sec. 4.1)."""
import numpy as np
import scipy.sparse as sp

from oracle import fine
from oracle.partition import CartesianPartition, face_mode_order, piece_basis


def _medium(nvox, seed=3):
    rng = np.random.default_rng(seed)
    return rng.uniform(1, 4, nvox), rng.uniform(1, 2, nvox)


def test_split_sums_and_signs():
    """sum_i P_i A_i P_i^T = A and sum_i P_i B_i P_i^T = B (eq. splitN_c);
    every A_i <= 0 and diagonally dominant (Prop. 2); B_i > 0."""
    nvox = (12, 10, 9)
    sigma, rho = _medium(nvox)
    A, b = fine.assemble_acoustic(sigma, rho)
    part = CartesianPartition(nvox, ([4, 8], [5], [3, 6]), 4, 2)
    n = A.shape[0]
    Asum = sp.lil_matrix((n, n))
    bsum = np.zeros(n)
    for i, c in enumerate(part.cells):
        Ai, bi = part.cell_operator(i, sigma, rho)
        ix = np.ix_(c.nodes, c.nodes)
        Asum[ix] = Asum[ix].toarray() + Ai
        bsum[c.nodes] += bi
        assert np.allclose(Ai, Ai.T, rtol=0, atol=0)
        off = np.abs(Ai).sum(axis=1) - np.abs(np.diag(Ai))
        assert np.all(np.abs(np.diag(Ai)) >= off * (1 - 1e-14))
        assert np.all(np.diag(Ai) < 0)
        assert np.linalg.eigvalsh(Ai).max() <= 1e-12 * np.abs(Ai).max()
        assert np.all(bi > 0)
    assert np.abs(Asum.tocsr() - A).max() <= 1e-14 * abs(A).max()
    assert np.abs(bsum - b).max() <= 1e-14 * b.max()


def test_split_reproduces_paper_example_weights():
    """Homogeneous medium: on a face node the cell keeps the full inward
    normal link, half of each in-plane link and half the mass (2D examples
    of Sec. 2, beta = 1/2, gamma = 1/2); on an edge node a quarter of the
    link along the edge, half of the normal links and a quarter of the
    mass; interior rows equal rows of A."""
    nvox = (8, 8, 8)
    part = CartesianPartition(nvox, ([4], [4], []), 4, 2)
    one = np.ones(nvox)
    A, b = fine.assemble_acoustic(one, one)
    i = part.cell_id(0, 0, 0)
    Ai, bi = part.cell_operator(i, one, one)
    c = part.cells[i]
    pos = {int(g): k for k, g in enumerate(c.nodes)}
    idx = part.idx

    def row(x, y, z):
        return Ai[pos[int(idx[x, y, z])]]

    def ent(r, x, y, z):
        return r[pos[int(idx[x, y, z])]]

    # face node on x = 4 (y = 2, z = 3)
    r = row(4, 2, 3)
    assert ent(r, 3, 2, 3) == 1.0                      # inward normal link
    for nb in [(4, 1, 3), (4, 3, 3), (4, 2, 2), (4, 2, 4)]:
        assert ent(r, *nb) == 0.5                      # in-plane links halved
    assert bi[pos[int(idx[4, 2, 3])]] == 0.5
    # edge node on x = 4, y = 4 (z = 3)
    r = row(4, 4, 3)
    assert ent(r, 4, 4, 2) == 0.25 and ent(r, 4, 4, 4) == 0.25
    assert ent(r, 3, 4, 3) == 0.5 and ent(r, 4, 3, 3) == 0.5
    assert bi[pos[int(idx[4, 4, 3])]] == 0.25
    # interior node equals A
    k = int(idx[2, 2, 3])
    r = row(2, 2, 3)
    Ar = A[k].toarray().ravel()
    for g, kk in pos.items():
        assert r[kk] == Ar[g]


def test_piece_inventory_small_grid():
    """4^3 cells of 8^3 voxels: 144 faces of 7x7 nodes shared by 2 cells,
    108 edges of 7 nodes shared by 4, 27 corners shared by 8."""
    cuts = [np.array([8, 16, 24])] * 3
    part = CartesianPartition((32, 32, 32), cuts, 9, 3)
    kinds = np.array([p.kind for p in part.pieces])
    assert (kinds == 1).sum() == 144 and (kinds == 2).sum() == 108 and (kinds == 3).sum() == 27
    for p in part.pieces:
        assert len(p.cells) == 2 ** p.kind
        assert len(p.nodes) == {1: 49, 2: 7, 3: 1}[p.kind]
    # an interior cell has 6 faces, 12 edges, 8 corners
    c = part.cells[part.cell_id(1, 1, 1)]
    ks = sorted(part.pieces[p].kind for p in c.pieces)
    assert ks.count(1) == 6 and ks.count(2) == 12 and ks.count(3) == 8
    assert part.cell_W(part.cell_id(1, 1, 1)).shape == (729, 6 * 9 + 12 * 3 + 8)
    # every skeleton node is in exactly one piece and on >= 1 cut plane
    assert sum(len(p.nodes) for p in part.pieces) == int((part.piece_of_node >= 0).sum())


def test_piece_bases_orthonormal_and_ordered():
    assert face_mode_order(7, 7, 4) == [(0, 0), (0, 1), (1, 0), (1, 1)]
    assert face_mode_order(7, 7, 9)[4:] == [(0, 2), (1, 2), (2, 0), (2, 1), (2, 2)]
    for dims, kind in [((7, 7), 1), ((5, 3), 1), ((7,), 2), ((), 3)]:
        S = piece_basis(dims, kind, 9, 3)
        assert np.allclose(S.T @ S, np.eye(S.shape[1]), atol=1e-14)
        # the constant vector is the first mode (low-frequency trace)
        c = np.ones(S.shape[0]) / np.sqrt(S.shape[0])
        assert np.allclose(S[:, 0], c, atol=1e-14)
    # face mode (p, q) varies along the first in-plane axis with p
    S = piece_basis((5, 3), 1, 4, 3)
    m01 = S[:, 1].reshape(3, 5)     # (q=1 along 2nd axis): rows constant along axis 1
    assert np.allclose(m01 - m01[:, :1], 0, atol=1e-14)


def test_point_columns_are_projections():
    cuts = [np.array([8])] * 3
    part = CartesianPartition((16, 16, 16), cuts, 4, 2)
    G, red = part.point_columns(np.array([[5, 3, 8], [8, 8, 3]]))
    for j, (p, coeff) in enumerate(red):
        S = part.pieces[p].S
        g = G[part.pieces[p].nodes, j]
        assert np.allclose(S @ (S.T @ g), g, atol=1e-15)
        assert np.allclose(S.T @ g, coeff, atol=1e-15)
        assert np.count_nonzero(G[:, j]) <= len(part.pieces[p].nodes)
