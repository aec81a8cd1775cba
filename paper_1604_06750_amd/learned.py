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
