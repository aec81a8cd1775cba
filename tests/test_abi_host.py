"""CPU tests of libsfrom's host side through the C ABI (no GPU calls):
the library loads and exports every declared symbol; the host C++ voxel
set-up (fine pencil, voxel-wise split, pieces, bases, projected point
columns) equals the oracle's; validation rejects bad inputs with the
documented status codes."""
import os
import re
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import fine
from oracle.partition import CartesianPartition

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1604_06750_amd import sfrom
    return sfrom


def test_library_exports_every_declared_symbol():
    S = _lib()
    hdr = open(os.path.join(ROOT, "include", "sfrom.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(sfrom_\w+)\s*\(", hdr, re.M))
    assert len(declared) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", S.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert declared <= exported, declared - exported
    assert declared == set(S.EXPORTED)


@pytest.fixture()
def host():
    S = _lib()
    h = S.sfrom_create(-1)
    yield S, h
    S.sfrom_destroy(h)


@pytest.mark.parametrize("name,mf,me", [("tiny", 4, 2), ("uneven", 9, 3)])
def test_voxel_setup_matches_oracle(host, name, mf, me):
    S, h = host
    if name == "tiny":
        wl = synth.workload("tiny", modes_face=mf, modes_edge=me)
        sigma, rho, cuts, nvox = wl.sigma, wl.rho, wl.cuts, wl.nvox
    else:
        rng = np.random.default_rng(3)
        nvox = (13, 10, 11)
        sigma = rng.uniform(1, 4, nvox); rho = rng.uniform(1, 2, nvox)
        cuts = (np.array([4, 9]), np.array([6]), np.array([3, 7]))
    S.sfrom_setup_voxel_acoustic(h, sigma, rho, cuts, mf, me)
    A, b = fine.assemble_acoustic(sigma, rho)
    rp, cl, av, bv = S.sfrom_export_pencil(h)
    Ah = sp.csr_matrix((av, cl, rp), shape=A.shape)
    assert (Ah != 0).nnz == (A != 0).nnz
    assert abs(Ah - A).max() <= 1e-15 * abs(A).max()
    assert np.abs(bv - b).max() <= 1e-15 * b.max()
    part = CartesianPartition(nvox, cuts, mf, me)
    info = S.sfrom_get_info(h)
    assert info["n_cells"] == len(part.cells) and info["n_pieces"] == len(part.pieces)
    for i, c in enumerate(part.cells):
        e = S.sfrom_export_cell(h, i)
        assert np.array_equal(e["global_node"], c.nodes)
        Ai, bi = part.cell_operator(i, sigma, rho)
        Ae = sp.csr_matrix((e["a"], e["col"], e["rowptr"]), shape=Ai.shape).toarray()
        assert np.abs(Ae - Ai).max() <= 1e-15 * np.abs(Ai).max()
        assert np.abs(e["b"] - bi).max() <= 1e-15 * bi.max()
        assert e["b_dim"] == part.cell_W(i).shape[1]
    for p, pc in enumerate(part.pieces):
        g, Sp = S.sfrom_export_piece(h, p)
        assert np.array_equal(g, pc.nodes)
        assert Sp.shape == pc.S.shape
        assert np.abs(Sp - pc.S).max() <= 1e-14


def test_elastic_setup_matches_oracle(host):
    """The library's elastic set-up (its own Q1 element code) equals the
    oracle's assembly, cell split and vector piece bases; the medium's Voigt
    entries equal the oracle's VTI tensor."""
    from oracle import elastic
    S, h = host
    nvox = (9, 8, 10)
    cuts = (np.array([4]), np.array([3, 5]), np.array([5]))
    c21, rho = synth.elastic_layered_medium(nvox, 77, [3, 7])
    rho = rho * np.random.default_rng(4).uniform(1.0, 2.0, nvox)
    Cv = np.zeros(tuple(nvox) + (6, 6))
    iu = np.triu_indices(6)
    Cv[..., iu[0], iu[1]] = c21
    Cv[..., iu[1], iu[0]] = c21
    C0 = elastic.vti_stiffness(2.0, 1.0, 0.1, 0.05)
    assert np.allclose(synth.vti_voigt21(2.0, 1.0, 0.1, 0.05), C0[iu], atol=1e-15)
    S.sfrom_setup_voxel_elastic(h, c21, rho, cuts, 4, 2)
    A, b = elastic.assemble_elastic(Cv, rho)
    rp, cl, av, bv = S.sfrom_export_pencil(h)
    Ah = sp.csr_matrix((av, cl, rp), shape=A.shape)
    assert abs(Ah - A).max() <= 1e-14 * abs(A).max()
    assert np.abs(bv - b).max() <= 1e-15 * b.max()
    part = elastic.ElasticPartition(nvox, cuts, 4, 2)
    info = S.sfrom_get_info(h)
    assert info["n_cells"] == len(part.cells) and info["n_pieces"] == len(part.pieces)
    for i in range(len(part.cells)):
        e = S.sfrom_export_cell(h, i)
        assert np.array_equal(e["global_node"], part.cell_dofs(i))
        Ai, bi = part.cell_operator(i, Cv, rho)
        Ae = sp.csr_matrix((e["a"], e["col"], e["rowptr"]), shape=Ai.shape).toarray()
        assert np.abs(Ae - Ai).max() <= 1e-14 * np.abs(Ai).max()
        assert np.abs(e["b"] - bi).max() <= 1e-15 * bi.max()
        assert e["b_dim"] == part.cell_W(i).shape[1]
    for p, (dofs, Sp_o, _) in enumerate(part.pieces):
        g, Sp = S.sfrom_export_piece(h, p)
        assert np.array_equal(g, dofs)
        assert Sp.shape == Sp_o.shape and np.abs(Sp - Sp_o).max() <= 1e-14


def test_point_columns_match_oracle(host):
    S, h = host
    from paper_1604_06750_amd.problem import node_ids, max_piece_nodes
    wl = synth.workload("tiny", modes_face=4, modes_edge=2)
    S.sfrom_setup_voxel_acoustic(h, wl.sigma, wl.rho, wl.cuts, 4, 2)
    part = CartesianPartition(wl.nvox, wl.cuts, 4, 2)
    pts = np.vstack([wl.sources, wl.receivers])
    G, _ = part.point_columns(pts)
    cp, rw, vl = S.sfrom_point_columns(h, node_ids(wl.nvox, pts), max_piece_nodes(wl))
    Gh = sp.csc_matrix((vl, rw, cp), shape=G.shape).toarray()
    assert np.abs(Gh - G).max() <= 1e-15


def _small_split(S, h):
    wl = synth.workload("tiny", modes_face=4, modes_edge=2)
    S.sfrom_setup_voxel_acoustic(h, wl.sigma, wl.rho, wl.cuts, 4, 2)
    return wl


def test_source_off_skeleton_is_rejected(host):
    S, h = host
    wl = _small_split(S, h)
    from paper_1604_06750_amd.problem import node_ids
    k = node_ids(wl.nvox, [[3, 3, 3]])      # a cell-interior node
    with pytest.raises(S.SfromError) as e:
        S.sfrom_set_sources(h, np.array([0, 1]), k, np.array([1.0]))
    assert e.value.name == "ESUPPORT"
    with pytest.raises(S.SfromError) as e:
        S.sfrom_point_columns(h, k, 64)
    assert e.value.name == "ESUPPORT"


def test_split_mismatch_is_rejected(host):
    """A cell operator that does not add up to A (eq. splitN_c) is refused."""
    S, h = host
    wl = synth.workload("tiny", modes_face=4, modes_edge=2)
    A, b = fine.assemble_acoustic(wl.sigma, wl.rho)
    S.sfrom_set_pencil(h, A.indptr, A.indices, A.data, b)
    part = CartesianPartition(wl.nvox, wl.cuts, 4, 2)
    for i, c in enumerate(part.cells):
        Ai, bi = part.cell_operator(i, wl.sigma, wl.rho)
        if i == 3:
            bi = bi.copy(); bi[0] *= 1.01
        M = sp.csr_matrix(Ai)
        S.sfrom_add_cell(h, i, c.nodes, M.indptr, M.indices, M.data, bi)
    for p, pc in enumerate(part.pieces):
        S.sfrom_add_piece(h, p, pc.nodes, pc.S)
    cp, rw, vl = np.array([0, 1]), np.array([part.pieces[0].nodes[0]]), np.array([1.0])
    with pytest.raises(S.SfromError) as e:
        S.sfrom_set_sources(h, cp, rw, vl)
    assert e.value.name == "ESPLIT"


def test_pencil_validation(host):
    S, h = host
    A = sp.csr_matrix(np.array([[-2.0, 1.0], [0.5, -2.0]]))
    with pytest.raises(S.SfromError) as e:
        S.sfrom_set_pencil(h, A.indptr, A.indices, A.data, np.ones(2))
    assert e.value.name == "ENOTSYM"
    A = sp.csr_matrix(np.array([[-2.0, 1.0], [1.0, -2.0]]))
    with pytest.raises(S.SfromError) as e:
        S.sfrom_set_pencil(h, A.indptr, A.indices, A.data, np.array([1.0, -1.0]))
    assert e.value.name == "EBPOS"
    with pytest.raises(S.SfromError) as e:
        S.sfrom_set_pencil(h, A.indptr, A.indices, A.data, np.array([1.0, np.nan]))
    assert e.value.name == "ENONFINITE"


def test_piece_basis_must_be_orthonormal(host):
    S, h = host
    wl = synth.workload("tiny", modes_face=4, modes_edge=2)
    A, b = fine.assemble_acoustic(wl.sigma, wl.rho)
    S.sfrom_set_pencil(h, A.indptr, A.indices, A.data, b)
    with pytest.raises(S.SfromError) as e:
        S.sfrom_add_piece(h, 0, np.array([5, 6]), np.array([[1.0], [1.0]]))
    assert e.value.name == "EINVAL"


def test_device_calls_refused_on_host_handle(host):
    S, h = host
    _small_split(S, h)
    with pytest.raises(S.SfromError) as e:
        S.sfrom_build(h, 3, -0.02)
    assert e.value.name == "EDEVICE"


def test_binding_refuses_undersized_or_mistyped_buffers(monkeypatch):
    """The library cannot see device buffer sizes, so the binding checks the
    trace buffer's element size and count and the wavelet length before a
    run writes to them."""
    S = _lib()
    monkeypatch.setattr(S, "sfrom_get_info", lambda h: {"n_receivers": 3, "n_sources": 2, "online_prec": S.SFROM_F64})
    with pytest.raises(ValueError):
        S._check_buffers(None, 10, np.zeros(10), np.zeros((10, 3, 2), np.float32), S.SFROM_F64)
    with pytest.raises(ValueError):
        S._check_buffers(None, 10, np.zeros(10), np.zeros((9, 3, 2), np.float64), S.SFROM_F64)
    with pytest.raises(ValueError):
        S._check_buffers(None, 10, np.zeros(5), np.zeros((10, 3, 2), np.float32), S.SFROM_F32)
    S._check_buffers(None, 10, np.zeros(10), np.zeros((10, 3, 2), np.float64), S.SFROM_F64)
    S._check_buffers(None, 0, np.zeros(0), np.zeros((0, 3, 2), np.float32), S.SFROM_F64)


def test_binding_refuses_host_tensors_and_bad_numpy_layouts():
    """Device pointers come only from GPU tensors (a CPU tensor's address
    would be dereferenced by the kernels); host trace buffers must be
    C-contiguous and writeable, since the library copies into them as one
    flat block."""
    S = _lib()
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):
        S._wave_arg(torch.zeros(10, dtype=torch.float64))
    with pytest.raises(ValueError):
        S._trace_arg(torch.zeros((4, 3, 2), dtype=torch.float32))
    t = np.zeros((4, 3, 2), np.float32)
    with pytest.raises(ValueError):
        S._trace_arg(t[::-1])
    with pytest.raises(ValueError):
        S._trace_arg(np.asfortranarray(np.zeros((4, 3, 2), np.float32)))
    ro = np.zeros((4, 3, 2), np.float32)
    ro.flags.writeable = False
    with pytest.raises(ValueError):
        S._trace_arg(ro)
    with pytest.raises(ValueError):
        S._trace_arg([[0.0]])
    p, dev = S._trace_arg(t)
    assert dev == 0 and p.value == t.ctypes.data


def test_checkpoint_calls_need_a_device(host, tmp_path):
    S, h = host
    _small_split(S, h)
    for f in (S.sfrom_save, S.sfrom_load):
        with pytest.raises(S.SfromError) as e:
            f(h, str(tmp_path / "x.ckp"))
        assert e.value.name == "EDEVICE"


def test_face_modes_by_area_match_oracle(host):
    """Uneven cells with face-mode counts by face area (voxel areas <= 20 ->
    1 mode, <= 40 -> 3, else 5): every piece's basis equals the oracle's
    DCT modes for the count its face's area selects."""
    S, h = host
    rng = np.random.default_rng(8)
    nvox = (13, 12, 9)
    sigma = rng.uniform(1, 4, nvox); rho = rng.uniform(1, 2, nvox)
    cuts = (np.array([4, 10]), np.array([5]), np.array([4]))
    area_max, modes = [20, 40, 10 ** 6], [1, 3, 5]

    def rule(n1, n2):
        area = (n1 + 1) * (n2 + 1)
        return next(mo for am, mo in zip(area_max, modes) if area <= am)

    S.sfrom_setup_voxel_acoustic_rules(h, sigma, rho, cuts, area_max, modes, 2)
    part = CartesianPartition(nvox, cuts, rule, 2)
    info = S.sfrom_get_info(h)
    assert info["n_pieces"] == len(part.pieces)
    counts = set()
    for p, pc in enumerate(part.pieces):
        g, Sp = S.sfrom_export_piece(h, p)
        assert np.array_equal(g, pc.nodes)
        assert Sp.shape == pc.S.shape and np.abs(Sp - pc.S).max() <= 1e-14
        if pc.kind == 1:
            counts.add(pc.S.shape[1])
    assert counts == {1, 3, 5}
    with pytest.raises(S.SfromError):
        S.sfrom_setup_voxel_acoustic_rules(h, sigma, rho, cuts, [40, 20], [1, 3], 2)
