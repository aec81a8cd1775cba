"""Pins of the divide-and-conquer partition and the Gramian bases
(oracle/divconq.py, oracle/gramian.py) against what the paper and the
mathematics fix:

* the one- and two-domain examples of Sec. 2 (split operators and masses
  written out from the examples' formulas) and the multi-domain example
  (its gamma/alpha/beta weights) reproduced by Alg. 1 / Alg. 2;
* Prop. 1's set identities by brute force on random sparse graphs;
* eq. splitN_c after Alg. 2, and Prop. 2 (diagonal dominance and A_i <= 0);
* Alg. 2 with planar cuts equal to the voxel split of an independently
  written module (oracle/partition.py) on a homogeneous medium;
* the level-set choice of O on a path graph;
* the exact frequency-limited Gramian (eq. trgr) of a homogeneous box
  against its closed form (products of discrete sines), and the local
  Gramian equal to the exact one when the union of the cells is the whole
  domain."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import divconq as dc
from oracle import gramian as gr
from oracle import fine
from oracle.partition import CartesianPartition


def lap1d(n, h):
    """Sec. 2, first example: (A u)_k = (u_{k+1} - 2 u_k + u_{k-1}) / h^2 on
    k = -n+1..n-1 (index k + n - 1), u_{+-n} = 0."""
    N = 2 * n - 1
    A = sp.diags([np.ones(N - 1), -2 * np.ones(N), np.ones(N - 1)], [-1, 0, 1]) / h ** 2
    return sp.csr_matrix(A)


def test_example_1d_two_domains():
    n, h = 5, 0.2
    A = lap1d(n, h)
    k = np.arange(-n + 1, n)
    O = k < 0
    O1, O2, G = dc.prop1_split(A, O)
    assert np.array_equal(G, k == 0) and np.array_equal(O1, k < 0) and np.array_equal(O2, k > 0)
    beta = 0.3
    (n1, A1, b1), (n2, A2, b2) = dc.alg1_split(A, np.ones(len(k)), O1, O2, G, 0.5, beta)
    # the example's split: (A_1 u)_0 = -(u_0 - u_{-1}) / h^2, (A_2 u)_0 = (u_1 - u_0) / h^2
    E1 = A.toarray()[np.ix_(n1, n1)].copy()
    E1[-1, -1] = -1 / h ** 2
    E2 = A.toarray()[np.ix_(n2, n2)].copy()
    E2[0, 0] = -1 / h ** 2
    assert np.allclose(A1.toarray(), E1, rtol=0, atol=1e-12) and np.allclose(A2.toarray(), E2, rtol=0, atol=1e-12)
    assert b1[-1] == beta and b2[0] == 1 - beta and np.all(b1[:-1] == 1) and np.all(b2[1:] == 1)
    # variable conductances c_{k+1/2}: a_00 = -(c_- + c_+) is the negative sum
    # of its off-diagonals, so the only split with A_1, A_2 <= 0 (the remark
    # of the first example) gives node 0 the conductance of its own side
    rng = np.random.default_rng(1)
    c = 0.5 + rng.random(2 * n)                   # c[j] couples nodes j - 1 and j (index space)
    N = 2 * n - 1
    Av = np.zeros((N, N))
    for j in range(N + 1):                        # edge between index j - 1 and j (walls outside 0..N-1)
        for u in (j - 1, j):
            if 0 <= u < N:
                Av[u, u] -= c[j]
        if 1 <= j < N:
            Av[j - 1, j] += c[j]; Av[j, j - 1] += c[j]
    (m1, V1, _), (m2, V2, _) = dc.alg1_split(sp.csr_matrix(Av), np.ones(N), O1, O2, G)
    z = n - 1                                     # index of node 0
    assert abs(V1.toarray()[-1, -1] + c[z]) < 1e-14 and abs(V2.toarray()[0, 0] + c[z + 1]) < 1e-14


def lap2d(nx, ny, h):
    """5-point Laplacian on an nx x ny interior node grid (x fastest) with
    Dirichlet walls."""
    Ix, Iy = sp.eye(nx), sp.eye(ny)
    Tx = sp.diags([np.ones(nx - 1), -2 * np.ones(nx), np.ones(nx - 1)], [-1, 0, 1])
    Ty = sp.diags([np.ones(ny - 1), -2 * np.ones(ny), np.ones(ny - 1)], [-1, 0, 1])
    return sp.csr_matrix((sp.kron(Iy, Tx) + sp.kron(Ty, Ix)) / h ** 2)


def example3_operator(px, qy, lo, hi, h):
    """Split operator of one cell from the multi-domain example of Sec. 2:
    weights alpha+-, gamma, beta per node from its position in the cell
    [lo, hi] (inclusive node ranges per axis; a bound that is a wall is not
    a cell boundary). Reading: alpha+- = 1 for nodes strictly inside the
    cell along that axis."""
    xs = np.arange(lo[0], hi[0] + 1); ys = np.arange(lo[1], hi[1] + 1)
    xs = xs[(xs >= 1) & (xs <= px)]; ys = ys[(ys >= 1) & (ys <= qy)]
    nodes = [(x, y) for y in ys for x in xs]
    pos = {v: i for i, v in enumerate(nodes)}
    A = np.zeros((len(nodes), len(nodes))); B = np.zeros(len(nodes))

    def weights(c, a):
        lo_b = c == lo[a] and lo[a] >= 1          # on the cell's low boundary line
        hi_b = c == hi[a] and hi[a] <= (px, qy)[a]
        if lo_b:
            return 1.0, 0.0, 0.5
        if hi_b:
            return 0.0, 1.0, 0.5
        return 1.0, 1.0, 1.0                      # (alpha+, alpha-, beta / gamma of the other axis)

    for (x, y), i in pos.items():
        ap_x, am_x, bx = weights(x, 0)
        ap_y, am_y, by = weights(y, 1)
        gx, gy = by, bx                           # gamma_x = 0.5 on a y-boundary line, etc.
        for (dx, dy), w in (((1, 0), gx * ap_x), ((-1, 0), gx * am_x), ((0, 1), gy * ap_y), ((0, -1), gy * am_y)):
            A[i, i] -= w / h ** 2
            j = pos.get((x + dx, y + dy))
            if j is not None:
                A[i, j] += w / h ** 2
        B[i] = bx * by
    return nodes, A, B


def test_multidomain_example_by_alg2():
    """Four cells of the multi-domain example (2 x 2 coarse grid): Alg. 2
    with the cut lines as the sets O reproduces each cell's weights."""
    px, qy, h = 9, 7, 0.1                         # interior nodes x = 1..9, y = 1..7
    cx, cy = 5, 4                                 # cut lines x = 5, y = 4
    A = lap2d(px, qy, h)
    X, Y = np.meshgrid(np.arange(1, px + 1), np.arange(1, qy + 1), indexing="xy")
    X = X.ravel(); Y = Y.ravel()

    def choose(s):
        x, y = X[s.nodes], Y[s.nodes]
        if x.min() < cx < x.max():
            return x < cx
        if y.min() < cy < y.max():
            return y < cy
        return None

    subs = dc.alg2_partition(A, np.ones(px * qy), 4, 0.5, 0.5, choose)
    assert len(subs) == 4
    boxes = [((0, 0), (cx, cy)), ((cx, 0), (px + 1, cy)), ((0, cy), (cx, qy + 1)), ((cx, cy), (px + 1, qy + 1))]
    seen = set()
    for s in subs:
        x, y = X[s.nodes], Y[s.nodes]
        lo = (0 if x.min() == 1 else x.min(), 0 if y.min() == 1 else y.min())
        hi = (px + 1 if x.max() == px else x.max(), qy + 1 if y.max() == qy else y.max())
        assert (lo, hi) in boxes
        seen.add((lo, hi))
        nodes, E, EB = example3_operator(px, qy, lo, hi, h)
        order = [nodes.index((int(a), int(c))) for a, c in zip(x, y)]
        assert np.allclose(s.A.toarray(), E[np.ix_(order, order)], rtol=0, atol=1e-10)
        assert np.allclose(s.b, EB[order], rtol=0, atol=1e-15)
    assert len(seen) == 4


def test_two_domain_example_2d():
    """Second example of Sec. 2: Gamma = the line x = 0; the Gamma rows of
    A_1 are -(u_0 - u_-1)/h^2 + (1/2)(u_{q+1} - 2 u_q + u_{q-1})/h^2 and B
    is halved there."""
    px, qy, h = 7, 5, 0.25
    A = lap2d(px, qy, h)
    X = np.tile(np.arange(1, px + 1), qy)
    O1, O2, G = dc.prop1_split(A, X < 4)
    assert np.array_equal(G, X == 4)
    (n1, A1, b1), (n2, A2, b2) = dc.alg1_split(A, np.ones(px * qy), O1, O2, G)
    A1 = A1.toarray(); loc = {g: i for i, g in enumerate(n1)}
    for g in np.where(G)[0]:
        r = loc[g]
        assert abs(A1[r, r] - (-1 - 1) / h ** 2) < 1e-10          # -1 (x) - 0.5 * 2 (y)
        assert abs(A1[r, loc[g - 1]] - 1 / h ** 2) < 1e-10
        for dg in (-px, px):
            if g + dg in loc:
                assert abs(A1[r, loc[g + dg]] - 0.5 / h ** 2) < 1e-10
        assert b1[r] == 0.5
    assert np.allclose(A1.sum(axis=1)[[loc[g] for g in np.where(G)[0]]],
                       [-(1.0 if Y in (0, qy - 1) else 0.0) * 0.5 / h ** 2 for Y in range(qy)])


def random_graph(n, p, seed, dominant=True):
    rng = np.random.default_rng(seed)
    M = np.triu(rng.random((n, n)) < p, 1)
    W = np.where(M, rng.random((n, n)) + 0.1, 0.0)
    W = W + W.T
    A = W.copy()
    slack = rng.random(n) * 0.5 if dominant else -rng.random(n) * 0.5
    np.fill_diagonal(A, -(W.sum(axis=1) + slack))
    return sp.csr_matrix(A)


def test_prop1_set_identities_brute_force():
    for seed in range(20):
        A = random_graph(30, 0.08, seed)
        Ad = A.toarray() != 0
        rng = np.random.default_rng(100 + seed)
        O = np.zeros(30, bool); O[rng.choice(30, 3, replace=False)] = True
        nb = lambda S: S | Ad[S].any(axis=0)
        if nb(O).all():
            continue
        O1, O2, G = dc.prop1_split(A, O)
        assert not (O1 & O2).any() and not (O1 & G).any() and not (O2 & G).any()
        assert (O1 | O2 | G).all() and O1.any() and O2.any()
        assert np.array_equal(G, nb(O1) & ~O1) and np.array_equal(G, nb(O2) & ~O2)
        assert not (O & ~O1).any()                                  # O is inside O_1
        assert not Ad[np.ix_(O1, O2)].any()                         # no O_1 - O_2 coupling


def _check_split(A, b, subs, tol=1e-13):
    n = A.shape[0]
    S = np.zeros((n, n)); Bs = np.zeros(n)
    for s in subs:
        S[np.ix_(s.nodes, s.nodes)] += s.A.toarray()
        Bs[s.nodes] += s.b
    assert np.abs(S - A.toarray()).max() <= tol * abs(A).max()
    assert np.abs(Bs - b).max() <= tol * b.max()


def test_alg2_split_identity_and_prop2():
    done = 0
    for seed in range(8):
        A = random_graph(80, 0.05, seed)
        b = 0.5 + np.random.default_rng(seed).random(80)
        try:
            subs = dc.alg2_partition(A, b, 5)
        except ValueError:
            continue
        _check_split(A, b, subs)
        for s in subs:
            Ai = s.A.toarray()
            off = np.abs(Ai).sum(axis=1) - np.abs(np.diag(Ai))
            assert np.all(np.abs(np.diag(Ai)) >= off - 1e-12 * np.abs(Ai).max())   # Prop. 2
            assert np.linalg.eigvalsh(Ai).max() <= 1e-12 * np.abs(Ai).max()
            assert np.all(s.b > 0)
        done += 1
    assert done >= 4


def test_alg2_with_planes_equals_voxel_split():
    """Homogeneous medium, 2 x 2 x 2 cells cut at the planes 4 (voxels):
    Alg. 2 with the planes as the sets O gives the voxel split's cell
    operators."""
    nvox = (8, 8, 8)
    sigma = np.full(nvox, 1.7); rho = np.full(nvox, 0.9)
    A, b = fine.assemble_acoustic(sigma, rho)
    idx = fine.node_index(nvox)
    coords = np.argwhere(idx >= 0)
    coords = coords[np.argsort(idx[idx >= 0])]                     # row k = coordinates of unknown k

    def choose(s):
        c = coords[s.nodes]
        for a in range(3):
            if c[:, a].min() < 4 < c[:, a].max():
                return c[:, a] < 4
        return None

    subs = dc.alg2_partition(A, b, 8, 0.5, 0.5, choose)
    part = CartesianPartition(nvox, (np.array([4]),) * 3, 1, 1)
    ref = {}
    for i, c in enumerate(part.cells):
        Ai, bi = part.cell_operator(i, sigma, rho)
        o = np.argsort(c.nodes)
        ref[tuple(np.sort(c.nodes))] = (Ai[np.ix_(o, o)], bi[o])
    for s in subs:
        Ai, bi = ref[tuple(s.nodes)]
        assert np.abs(s.A.toarray() - Ai).max() <= 1e-14 * np.abs(Ai).max()
        assert np.abs(s.b - bi).max() <= 1e-15 * bi.max()


def test_level_set_choice_on_a_path():
    n = 11
    A = lap1d((n + 1) // 2, 1.0)
    assert dc.pseudo_peripheral_root(A) in (0, n - 1)
    O = dc.level_set_O(A)
    O1, O2, G = dc.prop1_split(A, O)
    assert G.sum() == 1 and abs(O1.sum() - O2.sum()) <= 1
    # depth < 2 cannot be split
    assert dc.level_set_O(lap1d(1, 1.0)) is None and dc.level_set_O(sp.csr_matrix(np.ones((2, 2)))) is None


def test_general_partition_pieces_are_owner_sets():
    nvox = (10, 9, 8)
    rng = np.random.default_rng(4)
    A, b = fine.assemble_acoustic(0.5 + rng.random(nvox), 0.5 + rng.random(nvox))
    P = dc.GeneralPartition(A, b, 6)
    _check_split(A, b, P.subs, 1e-13)
    owners = {}
    for c, s in enumerate(P.subs):
        for g in s.nodes:
            owners.setdefault(int(g), []).append(c)
    skel = sorted(g for g, o in owners.items() if len(o) >= 2)
    assert sorted(int(g) for pc in P.pieces for g in pc.nodes) == skel
    for p, pc in enumerate(P.pieces):
        assert all(owners[int(g)] == pc.cells for g in pc.nodes)
        assert all(p in P.cells[c].pieces for c in pc.cells)
    firsts = [int(pc.nodes[0]) for pc in P.pieces]
    assert firsts == sorted(firsts)
    # interior nodes of a cell couple only inside the cell (eq. part)
    for c, s in enumerate(P.subs):
        inner = [g for g in s.nodes if len(owners[int(g)]) == 1]
        cols = A[inner].indices
        assert np.all(np.isin(cols, s.nodes))


# ---------------------------------------------------------------------------
# Gramian bases
# ---------------------------------------------------------------------------

def box_modes(nvox, sigma, rho, omega_max):
    """Closed-form eigenpairs of the homogeneous Dirichlet box: lambda =
    (sigma / rho) sum_a 4 sin^2(pi k_a / (2 n_a)), z = prod_a sqrt(2 / n_a)
    sin(pi k_a x_a / n_a) / sqrt(rho) on the interior nodes (x fastest)."""
    grids = np.meshgrid(*[np.arange(1, n) for n in nvox], indexing="ij")
    lam, Z = [], []
    for ks in itertools.product(*[range(1, n) for n in nvox]):
        l = sigma / rho * sum(4 * np.sin(np.pi * k / (2 * n)) ** 2 for k, n in zip(ks, nvox))
        if l <= omega_max ** 2:
            z = np.ones_like(grids[0], dtype=float)
            for g, k, n in zip(grids, ks, nvox):
                z = z * np.sqrt(2.0 / n) * np.sin(np.pi * k * g / n)
            lam.append(l)
            Z.append(z.transpose(2, 1, 0).ravel() / np.sqrt(rho))
    return np.array(lam), np.array(Z).T


def test_exact_gramian_closed_form():
    nvox = (8, 7, 6)
    sig, rho = 1.3, 0.8
    A, b = fine.assemble_acoustic(np.full(nvox, sig), np.full(nvox, rho))
    om = 1.1
    lam_ref, Z_ref = box_modes(nvox, sig, rho, om)
    lam, Z = gr.pencil_eigs_below(A, b, om)
    assert len(lam) == len(lam_ref) and np.allclose(np.sort(lam), np.sort(lam_ref), atol=1e-12)
    idx = fine.node_index(nvox)
    plane = np.sort(idx[1:8, 1:7, 3].ravel())                     # the plane z = 3
    G = gr.exact_gramian(A, b, plane, om)
    G_ref = Z_ref[plane] @ Z_ref[plane].T
    assert np.abs(G - G_ref).max() <= 1e-12 * np.abs(G_ref).max()
    S, ev = gr.basis_from_gramian(G, 1e-8, 100)
    assert np.allclose(S.T @ S, np.eye(S.shape[1]), atol=1e-12)
    # the basis spans the plane restrictions of the modes with lambda <= omega_max^2
    V = Z_ref[plane]
    assert np.linalg.norm(V - S @ (S.T @ V)) <= 1e-10 * np.linalg.norm(V)
    assert S.shape[1] == np.linalg.matrix_rank(V, tol=1e-8 * np.linalg.norm(V, 2))


def test_local_gramian_equals_exact_on_two_cells():
    nvox = (10, 6, 6)
    rng = np.random.default_rng(9)
    sigma = 0.5 + rng.random(nvox); rho = 0.5 + rng.random(nvox)
    A, b = fine.assemble_acoustic(sigma, rho)
    P = dc.GeneralPartition(A, b, 2)
    ops = {c: (s.nodes, s.A, s.b) for c, s in enumerate(P.subs)}
    om = 1.0
    for pc in P.pieces:
        if len(pc.nodes) < 2:
            continue
        G = gr.local_gramian(ops, pc.cells, pc.nodes, om, -1)
        Gx = gr.exact_gramian(A, b, pc.nodes, om)
        assert np.abs(G - Gx).max() <= 1e-11 * np.abs(Gx).max()
        # a slab deep enough to hold the whole union changes nothing
        G9 = gr.local_gramian(ops, pc.cells, pc.nodes, om, 50)
        assert np.abs(G9 - Gx).max() <= 1e-11 * np.abs(Gx).max()


def test_local_pencil_slab_is_a_prop2_split():
    nvox = (12, 8, 8)
    rng = np.random.default_rng(2)
    A, b = fine.assemble_acoustic(0.5 + rng.random(nvox), 0.5 + rng.random(nvox))
    P = dc.GeneralPartition(A, b, 4)
    ops = {c: (s.nodes, s.A, s.b) for c, s in enumerate(P.subs)}
    pc = max(P.pieces, key=lambda q: len(q.nodes))
    nodes, As, bs = gr.local_pencil(ops, pc.cells, pc.nodes, 1)
    U, AU, bU = gr.union_pencil(ops, pc.cells)
    assert len(nodes) < len(U) and np.all(np.isin(pc.nodes, nodes))
    Ad = As.toarray()
    assert np.linalg.eigvalsh(Ad).max() <= 1e-12 * np.abs(Ad).max() and np.all(bs > 0)
    # rows of the piece's nodes are those of the union operator (the piece is inside O_1)
    loc = np.searchsorted(nodes, pc.nodes); locU = np.searchsorted(U, pc.nodes)
    AUd = AU.toarray()
    keep = np.searchsorted(U, nodes)
    assert np.abs(Ad[loc] - AUd[np.ix_(locU, keep)]).max() <= 1e-14 * np.abs(AUd).max()


def test_alg1_needs_diagonal_dominance():
    """Prop. 2's hypothesis matters: the Q1 elastic operator is not
    diagonally dominant, and Alg. 2 / Alg. 1 applied to it gives split
    operators with positive eigenvalues (so the general partition is not
    used for it; its cells are split voxel by voxel instead), while the
    diagonally dominant acoustic operator of the same grid stays A_i <= 0."""
    from oracle import elastic
    rng = np.random.default_rng(3)
    nvox = (6, 6, 6)
    Cv = np.empty(nvox + (6, 6))
    Cv[...] = elastic.vti_stiffness(2.0, 1.0, 0.1, 0.05)
    rho = 1.0 + rng.random(nvox)
    A, b = elastic.assemble_elastic(Cv, rho)
    subs = dc.alg2_partition(A, b, 4)
    _check_split(A, b, subs)
    worst = max(np.linalg.eigvalsh(s.A.toarray()).max() / abs(s.A).max() for s in subs)
    assert worst > 1e-3
    Aa, ba = fine.assemble_acoustic(1.0 + rng.random(nvox), rho)
    for s in dc.alg2_partition(Aa, ba, 4):
        assert np.linalg.eigvalsh(s.A.toarray()).max() <= 1e-12 * abs(s.A).max()
