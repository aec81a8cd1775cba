"""GPU tests of the ABI's contracts around the on-line stage: checkpoint and
restart, the leapfrog stability check, non-finite inputs and states, state
reset under graph replay, and skeleton pieces wider than the piece phase's
unrolled bodies."""
import numpy as np
import pytest

import synth
from oracle import pipeline

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lib():
    from paper_1604_06750_amd import sfrom, problem
    return sfrom, problem


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _handle(S):
    return S.sfrom_create(0, torch.cuda.current_stream().cuda_stream)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _traces(S, h, n):
    info = S.sfrom_get_info(h)
    return np.zeros((n, info["n_receivers"], info["n_sources"]),
                    np.float64 if info["online_prec"] == S.SFROM_F64 else np.float32)


@pytest.mark.parametrize("prec", [0, 1])
def test_save_load_continues_bitwise(dev, tmp_path, prec):
    """n steps straight equal n/2 steps, sfrom_save, sfrom_load into a new
    handle with the same problem (no build there), n/2 more steps: bitwise,
    with the step counter carried over."""
    S, P = _lib()
    wl = synth.workload("tiny", modes_face=4, modes_edge=2, m=3, n_steps=200)
    run = pipeline.setup(wl)
    w = np.random.default_rng(3).standard_normal(200)
    path = str(tmp_path / "rom.ckp")
    h = _handle(S)
    try:
        P.setup(h, wl)
        S.sfrom_build(h, wl.m, wl.shift, prec)
        full = _traces(S, h, 200)
        S.sfrom_run(h, 200, run.dt, w, full)
        S.sfrom_reset(h)
        assert S.sfrom_get_info(h)["steps_done"] == 0
        first = _traces(S, h, 100)
        S.sfrom_run(h, 100, run.dt, w[:100], first)
        S.sfrom_save(h, path)
    finally:
        S.sfrom_destroy(h)
    h = _handle(S)
    try:
        P.setup(h, wl)
        S.sfrom_load(h, path)
        info = S.sfrom_get_info(h)
        assert info["built"] == 1 and info["steps_done"] == 100 and info["online_prec"] == prec
        second = _traces(S, h, 100)
        S.sfrom_run(h, 100, run.dt, w[100:], second)
        assert S.sfrom_get_info(h)["steps_done"] == 200
    finally:
        S.sfrom_destroy(h)
    assert np.abs(full).max() > 0
    assert np.array_equal(np.concatenate([first, second]), full)


def test_load_refuses_a_different_partition(dev, tmp_path):
    """A checkpoint of one boundary basis does not load into a problem with
    another (EINVAL); the handle's own ROM stays usable."""
    S, P = _lib()
    path = str(tmp_path / "rom.ckp")
    wl = synth.workload("tiny", modes_face=4, modes_edge=2, m=3, n_steps=20)
    run = pipeline.setup(wl)
    h = _handle(S)
    try:
        P.setup(h, wl)
        S.sfrom_build(h, 3, wl.shift, S.SFROM_F64)
        S.sfrom_save(h, path)
    finally:
        S.sfrom_destroy(h)
    other = synth.workload("tiny", modes_face=9, modes_edge=2, m=3, n_steps=20)
    h = _handle(S)
    try:
        P.setup(h, other)
        S.sfrom_build(h, 3, other.shift, S.SFROM_F64)
        with pytest.raises(S.SfromError) as e:
            S.sfrom_load(h, path)
        assert e.value.name == "EINVAL"
        with pytest.raises(S.SfromError) as e:
            S.sfrom_load(h, str(tmp_path / "missing.ckp"))
        assert e.value.name == "EINVAL"
        tr = _traces(S, h, 20)
        S.sfrom_run(h, 20, run.dt, run.w[:20], tr)
        assert np.isfinite(tr).all()
    finally:
        S.sfrom_destroy(h)


def test_cfl_limit_is_enforced(dev):
    """dt^2 lambda_max < 4 (Remark MFEM): a dt just above the ROM's own
    limit is refused with ECFL before any step; a dt just below it runs (the
    cells' Gershgorin bound is above the ROM's lambda_max there, so the run
    needs the exact eigenvalue); imported blocks with a 100x stiffer layer
    make a dt that was fine unstable, and it is refused too."""
    S, P = _lib()
    wl = synth.workload("tiny", modes_face=4, modes_edge=2, m=3, n_steps=50)
    run = pipeline.setup(wl)
    h = _handle(S)
    try:
        P.setup(h, wl)
        S.sfrom_build(h, wl.m, wl.shift, S.SFROM_F64)
        lam = S.sfrom_rom_lambda_max(h)
        dt_lim = 2.0 / np.sqrt(lam)
        tr = _traces(S, h, 50)
        S.sfrom_run(h, 50, run.dt, run.w, tr)                 # half the fine limit
        assert run.dt < dt_lim
        with pytest.raises(S.SfromError) as e:
            S.sfrom_run(h, 50, 1.01 * dt_lim, run.w, tr)
        assert e.value.name == "ECFL"
        assert S.sfrom_get_info(h)["steps_done"] == 50         # nothing was stepped
        S.sfrom_reset(h)
        S.sfrom_run(h, 50, 0.99 * dt_lim, run.w, tr)
        assert np.isfinite(tr).all()
        Gh, G = S.sfrom_export_rom(h, 0)
        S.sfrom_import_rom(h, 0, Gh, 100.0 * G)
        lam2 = S.sfrom_rom_lambda_max(h)
        assert lam2 > 10 * lam
        S.sfrom_reset(h)
        with pytest.raises(S.SfromError) as e:
            S.sfrom_run(h, 50, 0.99 * dt_lim, run.w, tr)
        assert e.value.name == "ECFL"
        S.sfrom_run(h, 50, 0.9 * 2.0 / np.sqrt(lam2), run.w, tr)
    finally:
        S.sfrom_destroy(h)


def test_nonfinite_wavelet_and_state(dev):
    """A NaN among host wavelet samples is refused before any step
    (ENONFINITE); a NaN among device wavelet samples reaches the state and the
    run ends with ENONFINITE; after sfrom_reset the handle steps exactly as a
    fresh one."""
    S, P = _lib()
    wl = synth.workload("tiny", modes_face=4, modes_edge=2, m=3, n_steps=60)
    run = pipeline.setup(wl)
    bad = run.w.copy()
    bad[7] = np.nan
    h = _handle(S)
    try:
        P.setup(h, wl)
        S.sfrom_build(h, wl.m, wl.shift, S.SFROM_F32)
        tr = _traces(S, h, 60)
        with pytest.raises(S.SfromError) as e:
            S.sfrom_run(h, 60, run.dt, bad, tr)
        assert e.value.name == "ENONFINITE"
        assert S.sfrom_get_info(h)["steps_done"] == 0
        with pytest.raises(S.SfromError) as e:
            S.sfrom_run(h, 60, run.dt, torch.tensor(bad, dtype=torch.float64, device="cuda"), tr)
        assert e.value.name == "ENONFINITE"
        assert np.isnan(tr[-1]).any()
        S.sfrom_reset(h)
        again = _traces(S, h, 60)
        S.sfrom_run(h, 60, run.dt, run.w, again)
    finally:
        S.sfrom_destroy(h)
    h = _handle(S)
    try:
        P.setup(h, wl)
        S.sfrom_build(h, wl.m, wl.shift, S.SFROM_F32)
        fresh = _traces(S, h, 60)
        S.sfrom_run(h, 60, run.dt, run.w, fresh)
    finally:
        S.sfrom_destroy(h)
    assert np.array_equal(again, fresh)


def test_graph_replay_across_reset_and_new_source_count(dev):
    """Graph replay on: run, reset, run (replayed), then a different number
    of sources (state buffers reallocated: the captured run must not be
    replayed against freed memory), each run equal to the eager handle's
    bitwise."""
    S, P = _lib()
    wl = synth.workload("tiny", modes_face=4, modes_edge=2, m=3, n_steps=80)
    run = pipeline.setup(wl)
    w = torch.tensor(run.w, dtype=torch.float64, device="cuda")
    fi = synth.face_interior_nodes(wl.nvox, wl.cuts)
    more = fi[np.sort(np.random.default_rng(8).choice(len(fi), 7, replace=False))]
    out = {}
    for mode in ("eager", "graph"):
        h = _handle(S)
        try:
            P.setup(h, wl)
            S.sfrom_build(h, wl.m, wl.shift, S.SFROM_F32)
            S.sfrom_set_graph(h, mode == "graph")
            res = []
            for k, srcs in enumerate([wl.sources, wl.sources, more, more]):
                if k == 2:
                    cp, rw, vl = S.sfrom_point_columns(h, P.node_ids(wl.nvox, srcs), P.max_piece_nodes(wl))
                    S.sfrom_set_sources(h, cp, rw, vl, project=False)
                info = S.sfrom_get_info(h)
                tr = torch.zeros((80, info["n_receivers"], info["n_sources"]), dtype=torch.float32, device="cuda")
                S.sfrom_reset(h)
                S.sfrom_run(h, 80, run.dt, w, tr)
                torch.cuda.synchronize()
                res.append(tr.cpu().numpy().copy())
                _ = torch.ones(4096, device="cuda").sum().item()
            out[mode] = res
        finally:
            S.sfrom_destroy(h)
    for a, b in zip(out["eager"], out["graph"]):
        assert np.array_equal(a, b)
    assert np.array_equal(out["eager"][0], out["eager"][1])
    assert np.abs(out["eager"][3]).max() > 0


def test_wide_edge_pieces_match_oracle(dev):
    """Cells of 16 x 6 x 6 voxels: the edge lines along x have 15 nodes and
    carry 10 DCT modes each, wider than the piece phase's unrolled body for
    4-cell pieces; sources and receivers sit on those edges and on faces.
    FP64 (1e-10) and FP32 (1e-4) against the oracle."""
    S, P = _lib()
    rng = np.random.default_rng(12)
    nvox = (32, 12, 12)
    sigma, rho = synth.acoustic_medium(nvox, 7001)
    cuts = (np.array([16]), np.array([6]), np.array([6]))
    edge = np.array([[x, 6, 6] for x in range(1, 32) if x != 16], np.int64)
    fi = synth.face_interior_nodes(nvox, cuts)
    src = np.vstack([edge[[2, 9]], fi[rng.choice(len(fi), 6, replace=False)]])
    rec = np.vstack([edge[[0, 5, 12, 14]], fi[rng.choice(len(fi), 12, replace=False)]])
    f_p, omega_max = 0.7071 / 25.0, 2 * np.pi * 0.7071 / 10.0
    wl = synth.Workload("edges", nvox, sigma, rho, cuts, 3, 4, 10, src, rec, 300, f_p, omega_max,
                        -omega_max ** 2 / 10.0)
    run = pipeline.setup(wl)
    run.w = rng.standard_normal(300)
    assert max(pc.S.shape[1] for pc in run.part.pieces) == 10
    pipeline.build_all(run)
    ref = pipeline.rom_traces(run)
    h = _handle(S)
    try:
        P.setup(h, wl)
        for prec, tol in ((S.SFROM_F64, 1e-10), (S.SFROM_F32, 1e-4)):
            S.sfrom_build(h, 3, wl.shift, prec)
            tr = _traces(S, h, 300)
            S.sfrom_run(h, 300, run.dt, run.w, tr)
            e = rel(tr, ref)
            d = np.abs(tr - ref).max(axis=(0, 2)) / np.abs(ref).max(axis=(0, 2))
            print(f"10-mode edges, prec {prec}: rel L2 {e:.2e}, worst receiver {d.max():.2e}")
            assert e <= tol and d.max() <= 10 * tol
    finally:
        S.sfrom_destroy(h)
