"""End-to-end oracle run of a synthetic workload (Alg. alg1red, both stages,
plus the fine-grid reference of Sec. 1)."""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

import synth
from . import fine
from .partition import CartesianPartition
from .rom_cell import build_cell
from .rom_global import GlobalROM


@dataclass
class OracleRun:
    wl: object
    part: CartesianPartition
    A: object
    b: np.ndarray
    dt: float
    w: np.ndarray
    G_src: np.ndarray
    Q_rec: np.ndarray
    red_src: list
    red_rec: list
    blocks: dict = field(default_factory=dict)
    rom: GlobalROM = None
    timings: dict = field(default_factory=dict)


def setup(wl, dt=None, n_steps=None):
    """Fine pencil, partition, projected point sources/receivers, dt, wavelet."""
    A, b = fine.assemble_acoustic(wl.sigma, wl.rho)
    rules = getattr(wl, "extra", {}).get("face_rules")
    if rules is None:
        mf = wl.modes_face
    else:
        def mf(n1, n2):
            area = (n1 + 1) * (n2 + 1)
            return next((mo for am, mo in zip(*rules) if area <= am), rules[1][-1])
    part = CartesianPartition(wl.nvox, wl.cuts, mf, wl.modes_edge)
    if dt is None:
        dt = fine.cfl_dt(A, b, wl.cfl_fraction)
    w = synth.ricker(n_steps or wl.n_steps, dt, wl.f_p)
    G, red_s = part.point_columns(wl.sources)
    Q, red_r = part.point_columns(wl.receivers)
    return OracleRun(wl, part, A, b, dt, w, G, Q, red_s, red_r)


def build_all(run: OracleRun, cells=None):
    """Off-line stage for every cell (or the given subset)."""
    t0 = time.perf_counter()
    part, wl = run.part, run.wl
    for i in (range(len(part.cells)) if cells is None else cells):
        Ai, bi = part.cell_operator(i, wl.sigma, wl.rho)
        W = part.cell_W(i)
        run.blocks[i] = build_cell(Ai, bi, W, wl.shift, wl.m)
    run.timings["build_s"] = time.perf_counter() - t0
    return run


def rom_traces(run: OracleRun):
    run.rom = GlobalROM(run.part, run.blocks)
    F = run.rom.reduced_columns(run.red_src)
    Qr = run.rom.reduced_columns(run.red_rec)
    t0 = time.perf_counter()
    out = run.rom.leapfrog(F, Qr, run.w, run.dt)
    run.timings["rom_step_s"] = time.perf_counter() - t0
    return out


def fine_traces(run: OracleRun):
    t0 = time.perf_counter()
    out = fine.leapfrog(run.A, run.b, run.G_src, run.Q_rec, run.w, run.dt)
    run.timings["fine_step_s"] = time.perf_counter() - t0
    return out


def rel_l2(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
