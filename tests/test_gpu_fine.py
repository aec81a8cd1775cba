"""GPU parity of the fine-grid comparator's Cartesian kernel for n_s a
multiple of 64 (2.5D-blocked planes, point sources in the flux, traces of
the level each launch reads): against the oracle's leapfrog (eq. wave_fll)
element by element on grids whose unknown counts leave ragged tiles in x,
y and z, with one and two groups of 64 sources, and over a run split in
two calls."""
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


def _case(ns, seed):
    """24^3 voxels (23^3 unknowns: tiles of 16 x 8 and 8 x 8 columns are
    ragged), ns seeded face-interior sources, 48 receivers."""
    return synth.workload("cube3", modes_face=4, modes_edge=2, n_sources=ns, n_receivers=48, n_steps=240,
                          realisation=seed)


def _check(tr, ref, tol):
    tr = np.asarray(tr, np.float64)
    scale = np.abs(ref).max()
    assert scale > 0
    # element by element, relative to the largest trace value
    err = np.abs(tr - ref).max() / scale
    # and per receiver, relative to that receiver's own peak
    per = np.abs(tr - ref).max(axis=(0, 2)) / np.maximum(np.abs(ref).max(axis=(0, 2)), 1e-300)
    print("max elementwise", err, "worst receiver", per.max())
    assert err <= tol and per.max() <= 50 * tol


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)])
@pytest.mark.parametrize("ns", [64, 128])
def test_fine_cartesian_many_sources_match_oracle(dev, prec, tol, ns):
    S, P = _lib()
    wl = _case(ns, 1)
    run = pipeline.setup(wl)
    ref = pipeline.fine_traces(run)
    h = _handle(S)
    try:
        P.setup(h, wl)
        tr = np.zeros(ref.shape, np.float64 if prec == 0 else np.float32)
        S.sfrom_fine_run(h, len(run.w), run.dt, run.w, tr, prec)
    finally:
        S.sfrom_destroy(h)
    _check(tr, ref, tol)


def test_fine_cartesian_split_run_equals_whole(dev):
    """240 steps in one call equal 100 + 140 steps in two calls bitwise
    (state and trace bookkeeping of the fused receivers across calls), and
    the device-buffer form equals the host form."""
    S, P = _lib()
    wl = _case(64, 2)
    run = pipeline.setup(wl)
    h = _handle(S)
    try:
        P.setup(h, wl)
        info = S.sfrom_get_info(h)
        shape = (240, info["n_receivers"], info["n_sources"])
        whole = np.zeros(shape, np.float32)
        S.sfrom_fine_run(h, 240, run.dt, run.w, whole, S.SFROM_F32)
        S.sfrom_fine_reset(h)
        a = np.zeros((100,) + shape[1:], np.float32)
        b = np.zeros((140,) + shape[1:], np.float32)
        S.sfrom_fine_run(h, 100, run.dt, run.w[:100], a, S.SFROM_F32)
        S.sfrom_fine_run(h, 140, run.dt, run.w[100:], b, S.SFROM_F32)
        S.sfrom_fine_reset(h)
        d = torch.zeros(shape, dtype=torch.float32, device=dev)
        wd = torch.tensor(run.w, dtype=torch.float64, device=dev)
        S.sfrom_fine_run(h, 240, run.dt, wd, d, S.SFROM_F32)
        torch.cuda.synchronize()
    finally:
        S.sfrom_destroy(h)
    assert np.abs(whole).max() > 0
    assert np.array_equal(np.concatenate([a, b]), whole)
    assert np.array_equal(d.cpu().numpy(), whole)
