"""Host-side parity of the corner-set removal (sfrom_remove_corner_set,
sfrom_corner_map; App. B) with the oracle (oracle/corners.py) on host-only
handles: the new pencil, every cell's operator and masses (by global node)
and the corner map bit for bit (the library takes the same quotients and
sums in the same order), the pair pieces' node sets, and Gramian bases on
the new pieces (projectors within 1e-9); the removal on a Cartesian voxel
set-up checked from the library's own outputs (E^T A' E = A); plus the
error paths and a partition without a corner set."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import corners as cn
from oracle import divconq as dc
from oracle import fine
from oracle import gramian as gr


def _lib():
    from paper_1604_06750_amd import sfrom
    return sfrom


def _handle(A, b):
    S = _lib()
    h = S.sfrom_create(-1, 0)
    A = sp.csr_matrix(A); A.sort_indices()
    S.sfrom_set_pencil(h, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data, b)
    return h


def _check(h, P, H):
    S = _lib()
    n1, nk, nh = S.sfrom_remove_corner_set(h)
    assert (n1, nk, nh) == (H.n, len(H.corner_nodes), len(H.hang_node))
    rp, cl, a, b = S.sfrom_export_pencil(h)
    A1 = sp.csr_matrix((a, cl, rp), shape=(n1, n1)).toarray()
    assert np.array_equal(A1, H.A.toarray()) and np.array_equal(b, H.b)
    info = S.sfrom_get_info(h)
    assert info["n_cells"] == len(H.subs) and info["n_pieces"] == len(H.pieces)
    for i, s in enumerate(H.subs):
        c = S.sfrom_export_cell(h, i)
        g = c["global_node"]
        o = np.argsort(g)
        assert np.array_equal(g[o], s.nodes)
        n = len(g)
        Al = sp.csr_matrix((c["a"], c["col"], c["rowptr"]), shape=(n, n)).toarray()[np.ix_(o, o)]
        assert np.array_equal(Al, s.A.toarray()), f"cell {i}: operator differs"
        assert np.array_equal(c["b"][o], s.b)
    for p, pc in enumerate(H.pieces):
        g, _ = S.sfrom_export_piece(h, p)
        assert np.array_equal(g, pc.nodes)
    new_of_old, corner, ptr, node, wt = S.sfrom_corner_map(h, P.n, nk, nh)
    assert np.array_equal(new_of_old, H.new_of_old) and np.array_equal(corner, H.corner_nodes)
    assert np.array_equal(ptr, H.hang_ptr) and np.array_equal(node, H.hang_node)
    assert np.array_equal(wt, H.hang_weight)


def test_remove_corner_set_acoustic():
    sig, rho = synth.acoustic_medium((12, 12, 12), 3, ell_sigma=4.0, ell_rho=2.0)
    A, b = fine.assemble_acoustic(sig, rho)
    P = dc.GeneralPartition(A, b, 8)
    H = cn.HangingPartition(P)
    S = _lib()
    h = _handle(A, b)
    try:
        S.sfrom_partition_graph(h, 8)
        _check(h, P, H)
        # Gramian bases on the pair pieces
        ops = {c: (s.nodes, s.A, s.b) for c, s in enumerate(H.subs)}
        ref = gr.gramian_bases(H, ops, 0.8, 1e-6, 6, 2)
        S.sfrom_gramian_bases(h, 0.8, 1e-6, 6, 2)
        for p in range(len(H.pieces)):
            _, Sb = S.sfrom_export_piece(h, p)
            assert Sb.shape[1] == ref[p].shape[1]
            assert np.abs(Sb @ Sb.T - ref[p] @ ref[p].T).max() <= 1e-9
        # once only
        with pytest.raises(S.SfromError) as e:
            S.sfrom_remove_corner_set(h)
        assert e.value.name == "ESTATE"
    finally:
        S.sfrom_destroy(h)


@pytest.mark.parametrize("n,cells,seed", [(1500, 5, 5), (3000, 6, 7)])
def test_remove_corner_set_unstructured_graph(n, cells, seed):
    """Two seeded graphs; the second has a corner node whose copies take
    every pair of its cells (one of them shares no plain interface node with
    the others)."""
    A, b, _ = synth.geometric_graph(n, 6, seed)
    P = dc.GeneralPartition(A, b, cells)
    H = cn.HangingPartition(P)
    S = _lib()
    h = _handle(A, b)
    try:
        S.sfrom_partition_graph(h, cells)
        _check(h, P, H)
    finally:
        S.sfrom_destroy(h)


def test_no_corner_set_and_errors():
    S = _lib()
    sig, rho = synth.acoustic_medium((8, 8, 8), 2, ell_sigma=4.0, ell_rho=2.0)
    A, b = fine.assemble_acoustic(sig, rho)
    h = _handle(A, b)
    try:
        with pytest.raises(S.SfromError) as e:
            S.sfrom_remove_corner_set(h)               # no partition
        assert e.value.name == "ESTATE"
        with pytest.raises(S.SfromError) as e:
            S.sfrom_corner_map(h, len(b), 0, 0)        # nothing removed
        assert e.value.name == "ESTATE"
        with pytest.raises(S.SfromError) as e:
            S.sfrom_set_corner_correction(h, 1)
        assert e.value.name == "ESTATE"
        with pytest.raises(S.SfromError) as e:
            S.sfrom_set_corner_correction(h, 2)
        assert e.value.name == "EINVAL"
        S.sfrom_partition_graph(h, 2)                  # two cells: no corner set
        before = S.sfrom_export_pencil(h)
        assert S.sfrom_remove_corner_set(h) == (len(b), 0, 0)
        after = S.sfrom_export_pencil(h)
        assert all(np.array_equal(x, y) for x, y in zip(before, after))
        S.sfrom_set_corner_correction(h, 0)
    finally:
        S.sfrom_destroy(h)


def test_remove_corner_set_on_voxel_partition():
    """The removal on the Cartesian set-up (2 x 2 x 2 cells of 8^3 voxels):
    from the library's own outputs, E^T A' E and E^T B' E equal the pencil
    before the removal (E built from the corner map), every piece is held by
    two cells, and edge nodes get 4 copies, the centre node 12."""
    S = _lib()
    sig, rho = synth.acoustic_medium((16, 16, 16), 9, ell_sigma=4.0, ell_rho=2.0)
    h = S.sfrom_create(-1, 0)
    try:
        S.sfrom_setup_voxel_acoustic(h, sig, rho, ([8], [8], [8]), 4, 2)
        rp0, cl0, a0, b0 = S.sfrom_export_pencil(h)
        n0 = len(b0)
        A0 = sp.csr_matrix((a0, cl0, rp0), shape=(n0, n0))
        n1, nk, nh = S.sfrom_remove_corner_set(h)
        new_of_old, corner, ptr, node, wt = S.sfrom_corner_map(h, n0, nk, nh)
        rp1, cl1, a1, b1 = S.sfrom_export_pencil(h)
        A1 = sp.csr_matrix((a1, cl1, rp1), shape=(n1, n1))
        rows = list(new_of_old[new_of_old >= 0]) + list(node)
        cols = list(np.where(new_of_old >= 0)[0]) + list(np.repeat(corner, np.diff(ptr)))
        E = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n1, n0))
        D = (E.T @ A1 @ E - A0).tocoo()
        assert np.abs(D.data).max(initial=0.0) <= 1e-13 * np.abs(a0).max()
        assert np.abs(E.T @ b1 - b0).max() <= 1e-15 * b0.max()
        assert np.abs(np.add.reduceat(wt, ptr[:-1]) - 1.0).max() <= 1e-14
        counts = sorted(set(np.diff(ptr).tolist()))
        assert counts == [4, 12], counts
        info = S.sfrom_get_info(h)
        own = {}
        for i in range(info["n_cells"]):
            for g in S.sfrom_export_cell(h, i)["global_node"]:
                own[int(g)] = own.get(int(g), 0) + 1
        assert max(own.values()) == 2
        for p in range(info["n_pieces"]):
            g, _ = S.sfrom_export_piece(h, p)
            assert all(own[int(x)] == 2 for x in g)
    finally:
        S.sfrom_destroy(h)
