"""Training driver of the learned off-line stage (argument marshalling and
the loop over batches; the network's forward, backward and Adam steps, the
targets and the learned build run in libsfrom's kernels)."""
from __future__ import annotations

import numpy as np

from . import problem
from . import sfrom as S


def n_outputs(b: int, m: int) -> int:
    """Factor-vector length (m - 1) b (b + 1) of a cell with (b, m)."""
    return (m - 1) * b * (b + 1)


def init_params(conv_ch: int, hidden: int, n_out: int, seed: int) -> np.ndarray:
    """He-scaled normal weights and zero biases, in the network's flat order
    [W1, b1, W2, b2, W3, b3]; the last layer starts at zero so that the
    first prediction is the target mean."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w1 = rng.normal(0.0, np.sqrt(2.0 / 54), conv_ch * 54)
    w2 = rng.normal(0.0, np.sqrt(2.0 / (64 * conv_ch)), hidden * 64 * conv_ch)
    w3 = np.zeros(n_out * hidden)
    return np.concatenate([w1, np.zeros(conv_ch), w2, np.zeros(hidden), w3, np.zeros(n_out)]).astype(np.float32)


def training_set(workloads, m: int, prec=S.SFROM_F32, stream: int = 0):
    """Inputs (n, 2, 8, 8, 8) and factor targets (n, P) of the interior cells
    of each workload, labelled by the library's block-Lanczos build."""
    import torch
    xs, ts = [], []
    for wl in workloads:
        h = S.sfrom_create(0, stream)
        try:
            problem.setup(h, wl, sources=False, receivers=False)
            S.sfrom_build(h, m, wl.shift, prec)
            cells = problem.interior_cells(wl)
            b = S.sfrom_get_info(h)["max_b"]
            t = torch.empty((len(cells), n_outputs(b, m)), dtype=torch.float32, device="cuda")
            S.sfrom_surrogate_targets(h, cells, t)
            torch.cuda.synchronize()
            ts.append(t.cpu().numpy())
            xs.append(problem.cell_features(wl, cells))
        finally:
            S.sfrom_destroy(h)
    return np.concatenate(xs), np.concatenate(ts)


def train(s, x, t, epochs: int, lr: float, batch: int, seed: int):
    """Adam over shuffled mini-batches of normalised targets; returns the
    mean loss of every epoch. x, t are float32 CUDA tensors."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    n = x.shape[0]
    hist = []
    for _ in range(epochs):
        perm = torch.as_tensor(rng.permutation(n), device=x.device)
        tot, cnt = 0.0, 0
        for i in range(0, n, batch):
            idx = perm[i:i + batch]
            xb = x[idx].contiguous()
            tb = t[idx].contiguous()
            tot += S.sfrom_surrogate_train_step(s, xb, tb, lr) * len(idx)
            cnt += len(idx)
        hist.append(tot / cnt)
    return hist


def experiment(n_train_media: int = 8, n_eval_media: int = 10, epochs: int = 40, m: int = 4, tol: float = 1e-3,
               conv_ch: int = 8, hidden: int = 128, workload: str = "large", log=print):
    """The learned off-line stage at scale: train on the interior cells of
    ``n_train_media`` realisations of the 128^3 medium generator (2744
    interior cells each), then, on each of ``n_eval_media`` held-out
    realisations, build the ROM with the learned stage and without it and
    compare acceptance, build times and receiver traces. Returns a dict of
    the figures (the network's forward/backward/Adam, targets, prediction and
    transfer-function tests run in libsfrom)."""
    import time
    import torch
    import synth
    stream = torch.cuda.current_stream().cuda_stream
    train_wl = [synth.workload(workload, modes_face=4, modes_edge=2, m=m, realisation=100 + r)
                for r in range(n_train_media)]
    t0 = time.perf_counter()
    x, t = training_set(train_wl, m, stream=stream)
    label_s = time.perf_counter() - t0
    P = t.shape[1]
    mu = t.mean(axis=0)
    sd = t.std(axis=0) + 1e-3 * np.abs(t).mean() + 1e-12
    s = S.sfrom_surrogate_create(0, stream, conv_ch, hidden, P)
    out = {"train_cells": int(len(x)), "label_s": label_s}
    try:
        S.sfrom_surrogate_set_params(s, init_params(conv_ch, hidden, P, seed=7))
        S.sfrom_surrogate_set_scale(s, mu.astype(np.float32), sd.astype(np.float32))
        xd = torch.tensor(x.reshape(len(x), -1), device="cuda")
        td = torch.tensor(((t - mu) / sd).astype(np.float32), device="cuda")
        del t
        t0 = time.perf_counter()
        hist = train(s, xd, td, epochs=epochs, lr=1e-3, batch=256, seed=3)
        torch.cuda.synchronize()
        out.update({"epochs": epochs, "train_s": time.perf_counter() - t0, "loss_first": hist[0], "loss_last": hist[-1]})
        log(f"[learned] {len(x)} cells, loss {hist[0]:.3e} -> {hist[-1]:.3e} in {out['train_s']:.1f} s")
        del xd, td
        evals = []
        for r in range(n_eval_media):
            wl = synth.workload(workload, modes_face=4, modes_edge=2, m=m, realisation=r)
            h = S.sfrom_create(0, stream)
            try:
                problem.setup(h, wl)
                cells = problem.interior_cells(wl)
                xe = torch.tensor(problem.cell_features(wl, cells).reshape(len(cells), -1), device="cuda")
                S.sfrom_build(h, m, wl.shift, S.SFROM_F32)          # warm (staged inputs)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                S.sfrom_build(h, m, wl.shift, S.SFROM_F32)
                torch.cuda.synchronize()
                plain = time.perf_counter() - t0
                t0 = time.perf_counter()
                acc, mis = S.sfrom_build_learned(h, m, wl.shift, S.SFROM_F32, s, cells, xe, wl.omega_max, tol)
                torch.cuda.synchronize()
                learned = time.perf_counter() - t0
                evals.append({"cells": int(len(cells)), "accepted": int(acc.sum()),
                              "median_mismatch": float(np.median(mis)), "min_mismatch": float(np.min(mis)),
                              "plain_build_s": plain, "learned_build_s": learned})
                log(f"[learned] medium {r}: {int(acc.sum())}/{len(cells)} accepted, median mismatch "
                    f"{np.median(mis):.2e} (min {np.min(mis):.2e}), build {learned:.2f} s learned vs {plain:.2f} s plain")
            finally:
                S.sfrom_destroy(h)
        out["eval"] = evals
        out["accepted"] = int(sum(e["accepted"] for e in evals))
        out["evaluated"] = int(sum(e["cells"] for e in evals))
    finally:
        S.sfrom_surrogate_destroy(s)
    return out
