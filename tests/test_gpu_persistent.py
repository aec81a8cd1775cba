"""GPU parity of the persistent on-line stage (sfrom_set_persistent: all steps
of a run in one cooperative launch with grid barriers between the cell and
piece phases) against the FP64 oracle and against the default path, on the
same seeded inputs: b = 98 with 16 sources (the source count not a multiple
of 64) in FP64 (1e-10) and FP32 (1e-4), b = 56 with 64 sources and a
receiver column spanning two pieces (the receivers computed beside the next
step's cell phase; FP64 within 1e-12 of the default path), a run split in
two continuing the state of the first, per-cell layer counts 1..4, and the
refusals (BF16 blocks)."""
import numpy as np
import pytest

import synth
from oracle import pipeline
from oracle.rom_cell import build_cell

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lib():
    from paper_1604_06750_amd import problem, sfrom
    return sfrom, problem


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - b) / np.linalg.norm(b))


def _run(wl, prec, dt, w, persistent, split=None, receivers=None, m_per_cell=None):
    S, P = _lib()
    h = S.sfrom_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        P.setup(h, wl)
        if receivers is not None:
            S.sfrom_set_receivers(h, *receivers, project=False)
        S.sfrom_build(h, wl.m, wl.shift, prec, m_per_cell=m_per_cell)
        S.sfrom_set_persistent(h, int(persistent))
        info = S.sfrom_get_info(h)
        dtype = np.float64 if prec == S.SFROM_F64 else np.float32
        parts = [len(w)] if split is None else [split, len(w) - split]
        out, k = [], 0
        for n in parts:
            tr = np.zeros((n, info["n_receivers"], info["n_sources"]), dtype)
            S.sfrom_run(h, n, dt, w[k:k + n], tr)
            out.append(tr)
            k += n
        return np.concatenate(out, axis=0)
    finally:
        S.sfrom_destroy(h)


def test_persistent_matches_oracle_b98(dev):
    S, P = _lib()
    print("[persistent] b = 98, 16 sources, 300 steps", flush=True)
    wl = synth.workload("small", modes_face=9, modes_edge=3, m=3, n_steps=300)
    fi = synth.face_interior_nodes(wl.nvox, wl.cuts)
    rng = np.random.default_rng(21)
    wl.sources = fi[np.sort(rng.choice(len(fi), 16, replace=False))]
    run = pipeline.setup(wl)
    ref = pipeline.rom_traces(pipeline.build_all(run))
    t64 = _run(wl, S.SFROM_F64, run.dt, run.w, True)
    t32 = _run(wl, S.SFROM_F32, run.dt, run.w, True)
    d32 = _run(wl, S.SFROM_F32, run.dt, run.w, False)
    split = _run(wl, S.SFROM_F64, run.dt, run.w, True, split=137)
    print(f"persistent FP64 {rel(t64, ref):.2e}, FP32 {rel(t32, ref):.2e}, FP32 vs default {rel(t32, d32):.2e}, "
          f"split run vs whole {rel(split, t64):.2e}")
    assert rel(t64, ref) <= 1e-10 and rel(t32, ref) <= 1e-4 and rel(t32, d32) <= 1e-5
    assert rel(split, t64) <= 1e-13


def test_persistent_receivers_across_pieces_b56(dev):
    S, P = _lib()
    print("[persistent] b = 56, 64 sources, receiver over two pieces", flush=True)
    wl = synth.workload("tiny", modes_face=4, modes_edge=2, m=3, n_steps=120)
    fi = synth.face_interior_nodes(wl.nvox, wl.cuts)
    rng = np.random.default_rng(5)
    wl.sources = fi[np.sort(rng.choice(len(fi), 64, replace=len(fi) < 64))]
    run = pipeline.setup(wl)
    h = S.sfrom_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        P.setup(h, wl)
        cp, rw, vl = S.sfrom_point_columns(h, P.node_ids(wl.nvox, wl.receivers), P.max_piece_nodes(wl))
    finally:
        S.sfrom_destroy(h)
    last = len(cp) - 2
    rows = np.concatenate([rw[cp[0]:cp[1]], rw[cp[last]:cp[last + 1]], rw[cp[1]:cp[2]]])
    vals = np.concatenate([vl[cp[0]:cp[1]], vl[cp[last]:cp[last + 1]], vl[cp[1]:cp[2]]])
    n0 = cp[1] - cp[0] + cp[last + 1] - cp[last]
    recv = (np.array([0, n0, len(rows)], np.int64), rows, vals)
    a = _run(wl, S.SFROM_F64, run.dt, run.w, True, receivers=recv)
    b = _run(wl, S.SFROM_F64, run.dt, run.w, False, receivers=recv)
    print(f"persistent vs default (receivers kernel): {rel(a, b):.2e}")
    assert np.abs(b).max() > 0 and rel(a, b) <= 1e-12


def test_persistent_uneven_layers(dev):
    """Per-cell layer counts 1..4 (every branch of the strip sequence) in the
    persistent kernel: FP64 within 1e-10 of the oracle and equal to the
    default path."""
    S, P = _lib()
    print("[persistent] per-cell m 1..4", flush=True)
    wl = synth.workload("tiny", modes_face=4, modes_edge=2, m=3, n_steps=200)
    run = pipeline.setup(wl)
    mpc = np.array([1, 2, 3, 4, 4, 3, 2, 1], np.int32)
    for i in range(len(run.part.cells)):
        Ai, bi = run.part.cell_operator(i, wl.sigma, wl.rho)
        run.blocks[i] = build_cell(Ai, bi, run.part.cell_W(i), wl.shift, int(mpc[i]))
    ref = pipeline.rom_traces(run)
    a = _run(wl, S.SFROM_F64, run.dt, run.w, True, m_per_cell=mpc)
    b = _run(wl, S.SFROM_F64, run.dt, run.w, False, m_per_cell=mpc)
    print(f"persistent uneven m: vs oracle {rel(a, ref):.2e}, vs default {rel(a, b):.2e}")
    assert rel(a, ref) <= 1e-10 and rel(a, b) <= 1e-13


def test_persistent_refusals(dev):
    S, P = _lib()
    wl = synth.workload("tiny", modes_face=4, modes_edge=2, m=3, n_steps=20)
    run = pipeline.setup(wl)
    h = S.sfrom_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        P.setup(h, wl)
        S.sfrom_build(h, wl.m, wl.shift, S.SFROM_BF16)
        S.sfrom_set_persistent(h, 1)
        info = S.sfrom_get_info(h)
        tr = np.zeros((20, info["n_receivers"], info["n_sources"]), np.float32)
        with pytest.raises(S.SfromError) as e:
            S.sfrom_run(h, 20, run.dt, run.w, tr)
        assert e.value.name == "EINVAL"
        with pytest.raises(S.SfromError) as e:
            S.sfrom_set_persistent(h, 2)
        assert e.value.name == "EINVAL"
        S.sfrom_set_persistent(h, 0)
        S.sfrom_run(h, 20, run.dt, run.w, tr)
    finally:
        S.sfrom_destroy(h)
