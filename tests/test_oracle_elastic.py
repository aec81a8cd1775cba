"""Pins of the elastic oracle (oracle/elastic.py): the Q1 voxel stiffness
against what mechanics fixes (symmetry, the six rigid-body motions as its
null space, the exact energy of a constant strain, the isotropic limit of
the VTI tensor), the assembled pencil and its cell split (eq. splitN_c), the
rigid motions of a floating cell, the exact modal solution of the fine
leapfrog, and the Pade property of a built elastic cell (Sec. 4.2)."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import elastic, fine
from oracle.rom_cell import build_cell, tf_full, tf_sfraction


def _corner_coords():
    return np.array([(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)], dtype=float)


def _rigid_modes():
    """Three translations and three infinitesimal rotations of the unit
    cube's corners (24-vectors, corner-major, components x, y, z)."""
    X = _corner_coords()
    modes = []
    for t in np.eye(3):
        modes.append(np.tile(t, 8))
    for axis in np.eye(3):
        modes.append(np.cross(axis, X - 0.5).ravel())
    return np.array(modes).T


def _C(seed=0):
    rng = np.random.default_rng(seed)
    return elastic.vti_stiffness(1.0 + rng.random(), 0.5 + rng.random(), 0.2 * rng.random(), 0.2 * rng.random())


def test_isotropic_limit():
    lam, mu = 1.7, 0.9
    C = elastic.vti_stiffness(lam, mu, 0.0, 0.0)
    iso = np.zeros((6, 6))
    iso[:3, :3] = lam
    iso[np.arange(3), np.arange(3)] = lam + 2 * mu
    iso[np.arange(3, 6), np.arange(3, 6)] = mu
    assert np.allclose(C, iso, atol=1e-14)
    assert np.all(np.linalg.eigvalsh(_C()) > 0)


def test_voxel_stiffness_symmetric_with_rigid_null_space():
    K = elastic.voxel_stiffness(_C(1))
    assert np.allclose(K, K.T, atol=1e-13)
    R = _rigid_modes()
    assert np.abs(K @ R).max() <= 1e-12 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    # exactly six zero modes; the 2x2x2 Gauss rule integrates the trilinear
    # element exactly, so the other 18 are positive
    assert np.sum(ev < 1e-10 * ev[-1]) == 6 and ev[0] > -1e-12 * ev[-1]


def test_constant_strain_energy_is_exact():
    """u = E x (any 3x3 E) gives strain sym(E) everywhere; the element energy
    u^T K u equals eps^T C eps times the unit volume."""
    rng = np.random.default_rng(3)
    C = _C(2)
    K = elastic.voxel_stiffness(C)
    for _ in range(3):
        E = rng.standard_normal((3, 3))
        u = (_corner_coords() @ E.T).ravel()
        eps = np.array([E[0, 0], E[1, 1], E[2, 2], E[1, 2] + E[2, 1], E[0, 2] + E[2, 0], E[0, 1] + E[1, 0]])
        assert abs(u @ K @ u - eps @ C @ eps) <= 1e-12 * abs(eps @ C @ eps)


def _medium(nvox, seed=5):
    rng = np.random.default_rng(seed)
    Cv = np.empty(tuple(nvox) + (6, 6))
    layers = [elastic.vti_stiffness(1.0 + j, 0.5 * (1 + j), 0.1 * j, 0.05 * j) for j in range(3)]
    for z in range(nvox[2]):
        Cv[:, :, z] = layers[min(2, 3 * z // nvox[2])]
    rho = 1.0 + rng.random(nvox)
    return Cv, rho


def test_assembly_split_and_floating_cell():
    nvox = (8, 8, 8)
    Cv, rho = _medium(nvox)
    A, b = elastic.assemble_elastic(Cv, rho)
    n = A.shape[0]
    assert n == 3 * 7 ** 3
    assert abs(A - A.T).max() <= 1e-13 * abs(A).max()
    assert np.linalg.eigvalsh(A.toarray())[-1] <= 1e-12 * abs(A).max()     # A <= 0 (clamped walls: < 0)
    assert np.all(b > 0)
    part = elastic.ElasticPartition(nvox, (np.array([4]), np.array([4]), np.array([4])), 4, 2)
    S = np.zeros((n, n)); Bs = np.zeros(n)
    for i in range(len(part.cells)):
        Ai, bi = part.cell_operator(i, Cv, rho)
        d = part.cell_dofs(i)
        S[np.ix_(d, d)] += Ai
        Bs[d] += bi
    assert np.abs(S - A.toarray()).max() <= 1e-13 * abs(A).max()
    assert np.abs(Bs - b).max() <= 1e-14 * b.max()
    # an interior cell of a 3^3 partition touches no wall: its operator has
    # exactly the six rigid motions in its null space
    nv3 = (12, 12, 12)
    Cv3, rho3 = _medium(nv3)
    p3 = elastic.ElasticPartition(nv3, tuple(np.array([4, 8]) for _ in range(3)), 4, 2)
    Ai, _ = p3.cell_operator(p3.scalar.cell_id(1, 1, 1), Cv3, rho3)
    ev = np.linalg.eigvalsh(Ai)
    assert np.sum(np.abs(ev) <= 1e-11 * np.abs(ev).max()) == 6 and ev[-1] <= 1e-11 * np.abs(ev).max()


def test_fine_leapfrog_matches_modal_solution():
    nvox = (6, 6, 6)
    Cv, rho = _medium(nvox, 8)
    A, b = elastic.assemble_elastic(Cv, rho)
    part = elastic.ElasticPartition(nvox, (np.array([3]),) * 3, 4, 2)
    G, _ = part.point_columns(np.array([[2, 2, 3]]), comp=2)
    Q, _ = part.point_columns(np.array([[3, 4, 3], [4, 3, 2]]), comp=0)
    dt = fine.cfl_dt(A, b, 0.5)
    w = synth.ricker(300, dt, 0.05)
    tr = fine.leapfrog(A, b, G, Q, w, dt)
    ref = fine.modal_traces(A, b, G, Q, w, dt)
    assert np.abs(tr).max() > 0
    assert np.linalg.norm(tr - ref) <= 1e-11 * np.linalg.norm(ref)


def test_elastic_cell_pade_at_the_shift():
    """Rational Krylov ROM of an interior elastic cell (vector piece bases):
    the S-fraction's transfer function equals the cell's at the shift."""
    nv3 = (24, 24, 24)
    Cv, rho = _medium(nv3, 11)
    part = elastic.ElasticPartition(nv3, tuple(np.array([8, 16]) for _ in range(3)), 4, 2)
    i = part.scalar.cell_id(1, 1, 1)
    Ai, bi = part.cell_operator(i, Cv, rho)
    W = part.cell_W(i)
    assert W.shape[1] == 3 * (6 * 4 + 12 * 2 + 8)
    assert np.allclose(W.T @ W, np.eye(W.shape[1]), atol=1e-13)
    s = -0.05
    Ghat, G = build_cell(Ai, bi, W, s, 3)
    F = tf_full(Ai, bi, W, s)
    U = tf_sfraction(Ghat, G, s)
    assert np.linalg.norm(U - F) <= 1e-10 * np.linalg.norm(F)
