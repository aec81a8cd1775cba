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


def setup(h, wl, sources=True, receivers=True):
    """Voxel set-up plus projected point sources/receivers of a Workload."""
    S.sfrom_setup_voxel_acoustic(h, wl.sigma, wl.rho, wl.cuts, wl.modes_face, wl.modes_edge)
    mp = max_piece_nodes(wl)
    if sources:
        cp, rw, vl = S.sfrom_point_columns(h, node_ids(wl.nvox, wl.sources), mp)
        S.sfrom_set_sources(h, cp, rw, vl, project=False)
    if receivers:
        cp, rw, vl = S.sfrom_point_columns(h, node_ids(wl.nvox, wl.receivers), mp)
        S.sfrom_set_receivers(h, cp, rw, vl, project=False)
