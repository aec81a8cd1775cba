"""GPU tests of sfrom_run_noalloc, the on-line run that allocates no device
memory (its Phi^1 exchange buffer and non-finite flag live in a static
device array): results equal to sfrom_run's, over two calls in a row with
the second on a smaller problem, and its refusals."""
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


def _pair(S, P, dev, wl, prec, n_steps):
    """Traces of the same run through sfrom_run and sfrom_run_noalloc
    (device buffers, state reset in between)."""
    run = pipeline.setup(wl, n_steps=n_steps)
    h = _handle(S)
    try:
        P.setup(h, wl)
        S.sfrom_build(h, wl.m, wl.shift, prec)
        info = S.sfrom_get_info(h)
        dt_t = torch.float64 if prec == S.SFROM_F64 else torch.float32
        shape = (n_steps, info["n_receivers"], info["n_sources"])
        w = torch.tensor(run.w[:n_steps], dtype=torch.float64, device=dev)
        ref = torch.full(shape, float("nan"), dtype=dt_t, device=dev)
        S.sfrom_run(h, n_steps, run.dt, w, ref)
        S.sfrom_reset(h)
        got = torch.full(shape, float("nan"), dtype=dt_t, device=dev)
        S.sfrom_run_noalloc(h, n_steps, run.dt, w, got)
        assert S.sfrom_get_info(h)["steps_done"] == n_steps
        torch.cuda.synchronize()
        return ref.cpu().numpy(), got.cpu().numpy()
    finally:
        S.sfrom_destroy(h)


@pytest.mark.parametrize("prec", [1, 0])
def test_noalloc_equals_run_on_two_calls(dev, prec):
    """First call: 27 cells of 8^3 with 64 sources; second call, in the same
    process and so on the same static scratch array (which keeps the first
    call's contents): 8 cells with one source and fewer steps. Each is
    bitwise equal to sfrom_run on the same inputs (same kernels, same
    order), finite and not all zero."""
    S, P = _lib()
    big = synth.workload("cube3", modes_face=4, modes_edge=2, m=4, n_steps=240)
    small = synth.workload("tiny", modes_face=4, modes_edge=2, m=3, n_steps=120)
    for wl, n in ((big, 240), (small, 120)):
        ref, got = _pair(S, P, dev, wl, prec, n)
        assert np.all(np.isfinite(ref)) and np.abs(ref).max() > 0
        assert np.array_equal(ref, got), (wl.name, float(np.abs(ref - got).max()))


def test_noalloc_refusals(dev):
    """ESTATE before the handle is prepared by a sfrom_run, a binding error
    for host buffers, and EINVAL (nothing stepped) when the Phi^1 buffer
    would exceed the static array."""
    S, P = _lib()
    wl = synth.workload("tiny", modes_face=4, modes_edge=2, m=3, n_steps=50)
    run = pipeline.setup(wl, n_steps=50)
    h = _handle(S)
    try:
        P.setup(h, wl)
        S.sfrom_build(h, wl.m, wl.shift, S.SFROM_F32)
        info = S.sfrom_get_info(h)
        w = torch.tensor(run.w[:50], dtype=torch.float64, device=dev)
        tr = torch.zeros((50, info["n_receivers"], info["n_sources"]), dtype=torch.float32, device=dev)
        with pytest.raises(S.SfromError) as e:
            S.sfrom_run_noalloc(h, 50, run.dt, w, tr)
        assert e.value.name == "ESTATE"
        S.sfrom_run(h, 0, run.dt, w, tr)          # prepares the on-line stage
        with pytest.raises(ValueError):
            S.sfrom_run_noalloc(h, 50, run.dt, run.w[:50], tr)
        S.sfrom_run_noalloc(h, 50, run.dt, w, tr)
        assert S.sfrom_get_info(h)["steps_done"] == 50
    finally:
        S.sfrom_destroy(h)

    # enough sources that sum_i b_i * n_s doubles exceed 256 MiB
    wl = synth.workload("medium", modes_face=4, modes_edge=2, m=2, n_steps=4)
    h = _handle(S)
    try:
        P.setup(h, wl, sources=False)
        sum_b = sum(P_b for P_b in _cell_dims(S, h))
        ns = (256 << 20) // (8 * sum_b) + 1
        fi = synth.face_interior_nodes(wl.nvox, wl.cuts)
        nodes = fi[np.arange(ns) % len(fi)]
        cp, rw, vl = S.sfrom_point_columns(h, P.node_ids(wl.nvox, nodes), P.max_piece_nodes(wl))
        S.sfrom_set_sources(h, cp, rw, vl, project=False)
        S.sfrom_build(h, wl.m, wl.shift, S.SFROM_F64)
        S.sfrom_set_cell_variant(h, 0)
        nr = S.sfrom_get_info(h)["n_receivers"]
        w = torch.zeros(4, dtype=torch.float64, device=dev)
        tr = torch.zeros((4, nr, ns), dtype=torch.float64, device=dev)
        S.sfrom_run(h, 0, 0.1, w, tr)
        with pytest.raises(S.SfromError) as e:
            S.sfrom_run_noalloc(h, 4, 0.1, w, tr)
        assert e.value.name == "EINVAL" and "scratch" in str(e.value)
        assert S.sfrom_get_info(h)["steps_done"] == 0
    finally:
        S.sfrom_destroy(h)


def _cell_dims(S, h):
    import ctypes as C
    out = []
    for i in range(S.sfrom_get_info(h)["n_cells"]):
        n, nnz, bd = C.c_int32(), C.c_int32(), C.c_int32()
        rc = S._lib.sfrom_export_cell(h, i, C.byref(n), C.byref(nnz), C.byref(bd), None, None, None, None, None)
        assert rc == 0
        out.append(bd.value)
    return out
