"""GPU parity of the general sparse path: the pencil through
sfrom_set_pencil, the divide-and-conquer partition (sfrom_partition_graph,
App. A), Gramian piece bases (sfrom_gramian_bases, Sec. 4.1), the off-line
build and the on-line stage, against the oracle's own partition, bases,
cell ROMs and global leapfrog on the same inputs. Cases: a variable acoustic
medium on a 16^3-voxel grid (8 cells, slab depth 2) and a seeded
unstructured graph pencil (3000 nodes, 6 cells, whole-union Gramian).
Checks: FP64 traces (1e-9 relative, and per receiver), FP32 traces (1e-4),
and each cell's transfer function at the Krylov shift mapped to its
skeleton nodes, W F(s) W^T, which does not depend on the orientation of a
piece basis (1e-8)."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import divconq as dc
from oracle import fine
from oracle import gramian as gr
from oracle.rom_cell import Breakdown, build_cell, tf_sfraction
from oracle.rom_global import GlobalROM

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lib():
    from paper_1604_06750_amd import sfrom
    return sfrom


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


class Case:
    pass


def _build_largest_m(Ai, bi, W, shift, m):
    """The cell's ROM with the largest m_i <= m for which the rational Krylov
    and Lanczos blocks keep full rank (Assumption 1): on a general partition a
    cell can touch a few junction nodes only through other skeleton nodes
    with complete bases, and then block k loses rank exactly; such a cell
    keeps m_i = k - 1 (the per-cell m of the build)."""
    while True:
        try:
            return build_cell(Ai, bi, W, shift, m), m
        except Breakdown as e:
            k = int(str(e).split("block ")[1].split()[0])
            assert 2 <= k <= m
            m = k - 1


def _oracle(A, b, n_cells, omega_max, eps, max_modes, depth, m, n_src, n_rec, n_steps, seed):
    c = Case()
    c.A = sp.csr_matrix(A); c.A.sort_indices(); c.b = b
    c.n_cells, c.omega_max, c.eps, c.max_modes, c.depth, c.m = n_cells, omega_max, eps, max_modes, depth, m
    P = dc.GeneralPartition(c.A, b, n_cells)
    ops = {i: (s.nodes, s.A, s.b) for i, s in enumerate(P.subs)}
    P.set_bases(gr.gramian_bases(P, ops, omega_max, eps, max_modes, depth))
    skel = np.sort(np.concatenate([pc.nodes for pc in P.pieces]))
    rng = np.random.Generator(np.random.PCG64(seed))
    c.src = np.sort(rng.choice(skel, n_src, replace=False))
    c.rec = np.sort(rng.choice(skel, n_rec, replace=False))
    _, red_s = P.point_columns(c.src)
    _, red_r = P.point_columns(c.rec)
    c.shift = -omega_max ** 2 / 10.0
    c.dt = fine.cfl_dt(c.A, b, 0.5)
    c.w = synth.ricker(n_steps, c.dt, omega_max / (2.0 * np.pi * 2.5))
    c.blocks, c.m_cell = {}, []
    for i in range(len(P.subs)):
        Ai, bi = P.cell_operator(i)
        c.blocks[i], mi = _build_largest_m(Ai, bi, P.cell_W(i), c.shift, m)
        c.m_cell.append(mi)
    rom = GlobalROM(P, c.blocks)
    c.ref = rom.leapfrog(rom.reduced_columns(red_s), rom.reduced_columns(red_r), c.w, c.dt)
    c.P = P
    c.kmax = max(len(pc.nodes) for pc in P.pieces)
    return c


def _node_tf(nodes_by_piece, bases, cell_pieces, Ghat, G, s):
    """W F(s) W^T of a cell on its skeleton nodes, rows/cols by ascending node."""
    W_rows = np.concatenate([nodes_by_piece[p] for p in cell_pieces])
    nb = sum(bases[p].shape[1] for p in cell_pieces)
    W = np.zeros((len(W_rows), nb))
    r = c0 = 0
    for p in cell_pieces:
        k, bp = bases[p].shape
        W[r:r + k, c0:c0 + bp] = bases[p]
        r += k; c0 += bp
    o = np.argsort(W_rows)
    F = tf_sfraction(Ghat, G, s)
    return (W @ F @ W.T)[np.ix_(o, o)]


def _gpu(c, prec, with_blocks=False, adapt=False):
    S = _lib()
    h = S.sfrom_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        S.sfrom_set_pencil(h, c.A.indptr.astype(np.int64), c.A.indices.astype(np.int32), c.A.data, c.b)
        S.sfrom_partition_graph(h, c.n_cells)
        S.sfrom_gramian_bases(h, c.omega_max, c.eps, c.max_modes, c.depth)
        cp, rw, vl = S.sfrom_point_columns(h, c.src, c.kmax)
        S.sfrom_set_sources(h, cp, rw, vl, project=False)
        cp, rw, vl = S.sfrom_point_columns(h, c.rec, c.kmax)
        S.sfrom_set_receivers(h, cp, rw, vl, project=False)
        if adapt:
            S.sfrom_set_breakdown_policy(h, 1)
            S.sfrom_build(h, c.m, c.shift, prec)
        else:
            S.sfrom_build(h, c.m, c.shift, prec, m_per_cell=np.array(c.m_cell, np.int32))
        tr = np.zeros((len(c.w), len(c.rec), len(c.src)), np.float64 if prec == S.SFROM_F64 else np.float32)
        S.sfrom_run(h, len(c.w), c.dt, c.w, tr)
        if not with_blocks:
            return tr, None
        info = S.sfrom_get_info(h)
        pieces = [S.sfrom_export_piece(h, p) for p in range(info["n_pieces"])]
        assert [Sb.shape[1] for _, Sb in pieces] == [pc.S.shape[1] for pc in c.P.pieces]
        tfs = {}
        for i in range(info["n_cells"]):
            Ghat, G = S.sfrom_export_rom(h, i)
            cell_pieces = [p for p, pc in enumerate(c.P.pieces) if i in pc.cells]
            tfs[i] = _node_tf([g for g, _ in pieces], [Sb for _, Sb in pieces], cell_pieces, Ghat, G, c.shift)
        return tr, tfs
    finally:
        S.sfrom_destroy(h)


def _check(c, label):
    S = _lib()
    tr, tfs = _gpu(c, S.SFROM_F64, with_blocks=True)
    e = float(np.linalg.norm(tr - c.ref) / np.linalg.norm(c.ref))
    per = float((np.abs(tr - c.ref).max(axis=(0, 2)) / np.abs(c.ref).max(axis=(0, 2))).max())
    worst = 0.0
    nodes = [pc.nodes for pc in c.P.pieces]
    bases = [pc.S for pc in c.P.pieces]
    for i in range(len(c.P.subs)):
        cp = [p for p, pc in enumerate(c.P.pieces) if i in pc.cells]
        ref = _node_tf(nodes, bases, cp, *c.blocks[i], c.shift)
        worst = max(worst, np.linalg.norm(tfs[i] - ref) / np.linalg.norm(ref))
    tr32, _ = _gpu(c, S.SFROM_F32)
    e32 = float(np.linalg.norm(tr32 - c.ref) / np.linalg.norm(c.ref))
    b = [pc.S.shape[1] for pc in c.P.pieces]
    print(f"{label}: {len(c.P.subs)} cells (m_i {c.m_cell}), {len(b)} pieces, b_p {min(b)}..{max(b)}; FP64 traces {e:.2e} "
          f"(worst receiver {per:.2e}), cell TF at the shift {worst:.2e}, FP32 traces {e32:.2e}")
    assert np.abs(c.ref).max() > 0
    assert e <= 1e-9 and per <= 1e-8 and worst <= 1e-8 and e32 <= 1e-4


def test_general_acoustic_grid(dev):
    sig, rho = synth.acoustic_medium((16, 16, 16), 21, ell_sigma=5.0, ell_rho=2.0)
    A, b = fine.assemble_acoustic(sig, rho)
    c = _oracle(A, b, 8, omega_max=0.9, eps=1e-6, max_modes=6, depth=2, m=3, n_src=4, n_rec=12, n_steps=300,
                seed=5)
    _check(c, "acoustic 16^3")


def test_general_unstructured_graph(dev):
    A, b, _ = synth.geometric_graph(3000, 6, 7)
    c = _oracle(A, b, 6, omega_max=0.45, eps=1e-6, max_modes=5, depth=-1, m=3, n_src=3, n_rec=10, n_steps=300,
                seed=6)
    _check(c, "unstructured graph")


def test_general_graph_breakdown_policy(dev):
    """The same unstructured graph built with m = 3 everywhere: without the
    policy the build fails with EBREAKDOWN naming a cell and its block; with
    sfrom_set_breakdown_policy(h, 1) the library lowers m_i itself to the
    values the oracle finds (block k lost rank -> m_i = k - 1), and the
    traces equal the oracle's (1e-9)."""
    S = _lib()
    A, b, _ = synth.geometric_graph(3000, 6, 7)
    c = _oracle(A, b, 6, omega_max=0.45, eps=1e-6, max_modes=5, depth=-1, m=3, n_src=3, n_rec=10, n_steps=300,
                seed=6)
    assert min(c.m_cell) < 3
    h = S.sfrom_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        S.sfrom_set_pencil(h, c.A.indptr.astype(np.int64), c.A.indices.astype(np.int32), c.A.data, c.b)
        S.sfrom_partition_graph(h, c.n_cells)
        S.sfrom_gramian_bases(h, c.omega_max, c.eps, c.max_modes, c.depth)
        with pytest.raises(S.SfromError) as e:
            S.sfrom_build(h, c.m, c.shift, S.SFROM_F64)
        assert e.value.name == "EBREAKDOWN" and "block" in S.sfrom_last_error(h)
        S.sfrom_set_breakdown_policy(h, 1)
        S.sfrom_build(h, c.m, c.shift, S.SFROM_F64)
        got = [len(S.sfrom_export_rom(h, i)[0]) for i in range(c.n_cells)]
    finally:
        S.sfrom_destroy(h)
    assert got == c.m_cell, (got, c.m_cell)
    tr, _ = _gpu(c, S.SFROM_F64, adapt=True)
    e = float(np.linalg.norm(tr - c.ref) / np.linalg.norm(c.ref))
    print(f"breakdown policy: m_i {got}, FP64 traces {e:.2e}")
    assert e <= 1e-9
