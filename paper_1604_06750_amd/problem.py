"""Marshal a synthetic voxel workload into libsfrom ABI calls.

Argument marshalling only: node coordinates become global node indices
(x-fastest over interior nodes), point receivers/sources become projected
skeleton columns through sfrom_point_columns, and every computation runs in
the library.
"""
from __future__ import annotations

import numpy as np

from . import sfrom as S


def node_ids(nvox, coords) -> np.ndarray:
    """Global unknown index of each node (x, y, z), x fastest over 1..n-1."""
    nx, ny, nz = nvox
    c = np.asarray(coords, dtype=np.int64).reshape(-1, 3)
    if np.any(c <= 0) or np.any(c[:, 0] >= nx) or np.any(c[:, 1] >= ny) or np.any(c[:, 2] >= nz):
        raise ValueError("node on or outside the Dirichlet walls")
    return (c[:, 0] - 1) + (nx - 1) * ((c[:, 1] - 1) + (ny - 1) * (c[:, 2] - 1))


def max_piece_nodes(wl) -> int:
    """Upper bound on the nodes of one skeleton piece (largest face)."""
    ext = [np.diff(np.concatenate([[0], np.asarray(c), [n]])).max() for c, n in zip(wl.cuts, wl.nvox)]
    ext = sorted(ext)
    return int(ext[-1] * ext[-2])


def setup(h, wl, sources=True, receivers=True, gramian=None):
    """Voxel set-up plus projected point sources/receivers of a Workload.
    ``gramian`` = (omega, eps, max_modes, depth) replaces the DCT piece bases
    by frequency-limited Gramian bases (sfrom_gramian_bases) before the
    columns are set."""
    rules = getattr(wl, "extra", {}).get("face_rules")
    if rules is not None:
        S.sfrom_setup_voxel_acoustic_rules(h, wl.sigma, wl.rho, wl.cuts, rules[0], rules[1], wl.modes_edge)
    else:
        S.sfrom_setup_voxel_acoustic(h, wl.sigma, wl.rho, wl.cuts, wl.modes_face, wl.modes_edge)
    if gramian is not None:
        S.sfrom_gramian_bases(h, *gramian)
    mp = max_piece_nodes(wl)
    if sources:
        cp, rw, vl = S.sfrom_point_columns(h, node_ids(wl.nvox, wl.sources), mp)
        S.sfrom_set_sources(h, cp, rw, vl, project=False)
    if receivers:
        cp, rw, vl = S.sfrom_point_columns(h, node_ids(wl.nvox, wl.receivers), mp)
        S.sfrom_set_receivers(h, cp, rw, vl, project=False)


def setup_elastic(h, wl, sources=True, receivers=True):
    """Elastic voxel set-up plus projected point forces (component
    wl.extra['source_component'], default z) and receivers of all three
    components at the receiver nodes (receiver r, component c is column
    3 r + c)."""
    S.sfrom_setup_voxel_elastic(h, wl.extra["c21"], wl.rho, wl.cuts, wl.modes_face, wl.modes_edge)
    mp = 3 * max_piece_nodes(wl)
    comp = int(wl.extra.get("source_component", 2))
    if sources:
        d = 3 * node_ids(wl.nvox, wl.sources) + comp
        cp, rw, vl = S.sfrom_point_columns(h, d, mp)
        S.sfrom_set_sources(h, cp, rw, vl, project=False)
    if receivers:
        d = (3 * node_ids(wl.nvox, wl.receivers)[:, None] + np.arange(3)[None, :]).ravel()
        cp, rw, vl = S.sfrom_point_columns(h, d, mp)
        S.sfrom_set_receivers(h, cp, rw, vl, project=False)


def interior_cells(wl):
    """Ids (x-fastest over the cut grid) of the 8^3-voxel cells that touch no
    wall: the cells the learned off-line stage predicts."""
    lo = [np.concatenate([[0], np.asarray(c)]) for c in wl.cuts]
    hi = [np.concatenate([np.asarray(c), [n]]) for c, n in zip(wl.cuts, wl.nvox)]
    ncx, ncy, ncz = (len(a) for a in lo)
    out = []
    for k in range(ncz):
        for j in range(ncy):
            for i in range(ncx):
                box = [(lo[0][i], hi[0][i]), (lo[1][j], hi[1][j]), (lo[2][k], hi[2][k])]
                inner = 0 < i < ncx - 1 and 0 < j < ncy - 1 and 0 < k < ncz - 1
                if inner and all(b - a == 8 for a, b in box):
                    out.append(i + ncx * (j + ncy * k))
    return np.asarray(out, dtype=np.int32)


def cell_features(wl, cells):
    """Network inputs of the given cells: log sigma and log rho of each cell's
    8^3 voxels, float32 [cell][channel][z][y][x]."""
    lo = [np.concatenate([[0], np.asarray(c)]) for c in wl.cuts]
    ncx, ncy = len(lo[0]), len(lo[1])
    ls, lr = np.log(wl.sigma), np.log(wl.rho)
    out = np.empty((len(cells), 2, 8, 8, 8), np.float32)
    for t, c in enumerate(cells):
        i, j, k = c % ncx, (c // ncx) % ncy, c // (ncx * ncy)
        x0, y0, z0 = lo[0][i], lo[1][j], lo[2][k]
        out[t, 0] = ls[x0:x0 + 8, y0:y0 + 8, z0:z0 + 8].transpose(2, 1, 0)
        out[t, 1] = lr[x0:x0 + 8, y0:y0 + 8, z0:z0 + 8].transpose(2, 1, 0)
    return out
