"""Pins of the oracle's global ROM and its leapfrog (Sec. 6, Sec. 8)."""
import numpy as np
import pytest

import synth
from oracle import fine, pipeline
from oracle.partition import CartesianPartition
from oracle.rom_cell import build_cell
from oracle.rom_global import GlobalROM


def _build(nvox, cuts, mf, me, m, seed=1, m_per_cell=None):
    rng = np.random.default_rng(seed)
    sigma = 4.0 ** rng.uniform(0, 1, nvox)
    rho = rng.uniform(1, 2, nvox)
    A, b = fine.assemble_acoustic(sigma, rho)
    part = CartesianPartition(nvox, cuts, mf, me)
    blocks = {}
    for i in range(len(part.cells)):
        Ai, bi = part.cell_operator(i, sigma, rho)
        mi = m if m_per_cell is None else m_per_cell(i)
        blocks[i] = build_cell(Ai, bi, part.cell_W(i), -0.02, mi)
    return A, b, part, blocks


def _traces_both(A, b, part, blocks, src, rec, n_steps=300, f_p=0.05, dt=None):
    G, rs = part.point_columns(src)
    Q, rr = part.point_columns(rec)
    rom = GlobalROM(part, blocks)
    dt = fine.cfl_dt(A, b) if dt is None else dt
    w = synth.ricker(n_steps, dt, f_p)
    tf = fine.leapfrog(A, b, G, Q, w, dt)
    tr = rom.leapfrog(rom.reduced_columns(rs), rom.reduced_columns(rr), w, dt)
    return tf, tr, rom


@pytest.mark.parametrize("case", ["slab2", "row3", "box2"])
def test_full_order_rom_equals_fine_grid(case):
    """With full piece bases and a Krylov space that fills each cell
    (m_i b_i = N_i, every graph layer below the skeleton holding b_i
    nodes), the S-fraction ROM is an exact re-realisation of the fine model
    (Remark sfint; the 1D spectrally matched grid example of Sec. 6), so
    the leapfrog traces agree to rounding and the pencils share lambda_max."""
    mpc = None
    if case == "slab2":
        nvox, cuts, m = (8, 8, 2), ([4], [], []), 4          # cells 4 x 7 nodes, b = 7
        src = np.array([[4, 2, 1], [4, 5, 1]])
        rec = np.array([[4, 1, 1], [4, 3, 1], [4, 7, 1]])
    elif case == "row3":
        nvox, cuts, m = (9, 4, 2), ([3, 6], [], []), None     # m = 3, 2, 3 per cell
        mpc = lambda i: 2 if i == 1 else 3
        src = np.array([[3, 2, 1], [6, 1, 1]])
        rec = np.array([[3, 1, 1], [6, 3, 1], [6, 2, 1]])
    else:
        nvox, cuts, m = (6, 4, 4), ([3], [], []), 3          # cells 3 x 3 x 3 nodes, b = 9
        src = np.array([[3, 2, 1], [3, 3, 3]])
        rec = np.array([[3, 1, 2], [3, 2, 2], [3, 3, 1]])
    A, b, part, blocks = _build(nvox, cuts, 100, 100, m, m_per_cell=mpc)
    for i, c in enumerate(part.cells):
        assert len(blocks[i][1]) * blocks[i][1][0].shape[0] == len(c.nodes)
    tf, tr, rom = _traces_both(A, b, part, blocks, src, rec)
    assert np.abs(tr - tf).max() <= 1e-11 * np.abs(tf).max()
    lf = fine.lambda_max(A, b)
    assert abs(rom.lambda_max() - lf) <= 1e-10 * lf


def test_rom_energy_conserved_and_cfl_not_tighter():
    """Stieltjes ROM is conservative (Remark MFEM): its leapfrog energy is
    constant once the wavelet is zero; lambda_max(ROM) <= lambda_max(fine)."""
    nvox = (16, 16, 16)
    A, b, part, blocks = _build(nvox, ([8],) * 3, 4, 2, 3)
    rom = GlobalROM(part, blocks)
    lf = fine.lambda_max(A, b)
    lr = rom.lambda_max()
    assert lr <= lf * (1 + 1e-12)
    dt = fine.cfl_dt(A, b)
    f_p = 0.06
    w = synth.ricker(420, dt, f_p)
    _, rs = part.point_columns(np.array([[5, 3, 8]]))
    F = rom.reduced_columns(rs)
    import scipy.sparse.linalg as spla
    lu = spla.splu(rom.D.tocsc())
    Y = np.zeros((rom.ndof, 1)); Yp = np.zeros_like(Y)
    es = []
    for k in range(len(w)):
        Yn = 2 * Y - Yp + dt * dt * lu.solve(rom.L @ Y + w[k] * F)
        if k * dt > 3.0 / f_p + dt:
            es.append(rom.energy(Yn, Y, dt)[0])
        Yp, Y = Y, Yn
    es = np.array(es)
    assert len(es) > 50 and es[0] > 0
    assert np.abs(es - es[0]).max() <= 1e-11 * es[0]


def test_rom_reciprocity():
    """The global ROM is symmetric (Prop. prop1stil: its transfer function is
    Stieltjes), so the trace from point a to point b equals that from b to a."""
    nvox = (16, 16, 16)
    A, b, part, blocks = _build(nvox, ([8],) * 3, 4, 2, 3, seed=4)
    pts = np.array([[5, 3, 8], [8, 11, 4], [8, 8, 13]])
    _, tr, _ = _traces_both(A, b, part, blocks, pts, pts, n_steps=200)
    assert np.abs(tr - tr.transpose(0, 2, 1)).max() <= 1e-12 * np.abs(tr).max()


def test_per_cell_layer_counts():
    """Cells with different m_i (uneven ROM sizes) still give a conservative,
    symmetric global ROM."""
    nvox = (16, 16, 16)
    A, b, part, blocks = _build(nvox, ([8],) * 3, 4, 2, 3, m_per_cell=lambda i: 2 + i % 3)
    rom = GlobalROM(part, blocks)
    assert abs(rom.L - rom.L.T).max() <= 1e-12 * abs(rom.L).max()
    assert rom.lambda_max() <= fine.lambda_max(A, b) * (1 + 1e-12)


def test_rom_error_decreases_with_boundary_modes():
    """Qualitative convergence in the boundary basis size (Sec. 9, the
    convergence study in K; parity unpinned: the paper's curves are not
    available)."""
    errs = []
    for mf, me in [(1, 1), (4, 2), (9, 3)]:
        wl = synth.workload("tiny", modes_face=mf, modes_edge=me, m=3, n_steps=300)
        run = pipeline.setup(wl)
        pipeline.build_all(run)
        errs.append(pipeline.rel_l2(pipeline.rom_traces(run), pipeline.fine_traces(run)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 5e-3
