"""Pins of the oracle's fine-grid model (Sec. 1, eq. wave_fll) against
closed forms, brute force and the exact modal solution."""
import itertools

import numpy as np
import scipy.sparse as sp

import synth
from oracle import fine


def test_homogeneous_is_kronecker_laplacian():
    """sigma = rho = 1: A must be the standard 7-point Dirichlet Laplacian
    (Kronecker sum of 1D second differences) and B = I."""
    nvox = (5, 4, 3)
    A, b = fine.assemble_acoustic(np.ones(nvox), np.ones(nvox))

    def d2(n):
        return sp.diags([np.ones(n - 1), -2 * np.ones(n), np.ones(n - 1)], [-1, 0, 1])

    nx, ny, nz = (v - 1 for v in nvox)
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    ref = sp.kron(Iz, sp.kron(Iy, d2(nx))) + sp.kron(Iz, sp.kron(d2(ny), Ix)) + sp.kron(d2(nz), sp.kron(Iy, Ix))
    assert abs(A - ref).max() == 0.0
    assert np.all(b == 1.0)


def test_assembly_matches_voxel_energy_brute_force():
    """-u^T A u and u^T B u equal per-voxel sums over the 12 edges and 8
    corners of every voxel (pure-Python loops, wall nodes held at zero)."""
    rng = np.random.default_rng(7)
    nvox = (3, 4, 3)
    sigma = rng.uniform(1, 4, nvox)
    rho = rng.uniform(1, 2, nvox)
    A, b = fine.assemble_acoustic(sigma, rho)
    idx = fine.node_index(nvox)
    for _ in range(3):
        u = rng.standard_normal(A.shape[0])

        def val(x, y, z):
            k = idx[x, y, z]
            return 0.0 if k < 0 else u[k]

        e_pot = 0.0
        e_kin = 0.0
        for i, j, k in itertools.product(*(range(n) for n in nvox)):
            corners = [(i + a, j + c, k + d) for a in (0, 1) for c in (0, 1) for d in (0, 1)]
            for p, q in itertools.combinations(corners, 2):
                if sum(abs(p[t] - q[t]) for t in range(3)) == 1:
                    e_pot += sigma[i, j, k] / 4.0 * (val(*p) - val(*q)) ** 2
            for p in corners:
                e_kin += rho[i, j, k] / 8.0 * val(*p) ** 2
        assert np.isclose(-u @ (A @ u), e_pot, rtol=1e-13)
        assert np.isclose(u @ (b * u), e_kin, rtol=1e-13)


def test_leapfrog_equals_modal_solution():
    """Leapfrog traces equal the eigen-expansion solution of the same
    recurrence (closed form) on a tiny heterogeneous grid."""
    rng = np.random.default_rng(11)
    nvox = (4, 3, 3)
    sigma = rng.uniform(1, 4, nvox)
    rho = rng.uniform(1, 2, nvox)
    A, b = fine.assemble_acoustic(sigma, rho)
    n = A.shape[0]
    G = rng.standard_normal((n, 2))
    Q = rng.standard_normal((n, 3))
    dt = fine.cfl_dt(A, b, 0.9)
    w = synth.ricker(300, dt, 0.08)
    lf = fine.leapfrog(A, b, G, Q, w, dt)
    md = fine.modal_traces(A, b, G, Q, w, dt)
    assert np.abs(lf - md).max() <= 1e-11 * np.abs(md).max()


def test_leapfrog_energy_conserved_after_source():
    rng = np.random.default_rng(5)
    nvox = (6, 5, 4)
    sigma = rng.uniform(1, 4, nvox)
    rho = rng.uniform(1, 2, nvox)
    A, b = fine.assemble_acoustic(sigma, rho)
    n = A.shape[0]
    dt = fine.cfl_dt(A, b)
    f_p = 0.1
    w = synth.ricker(400, dt, f_p)
    assert w[-1] == 0.0
    G = rng.standard_normal((n, 1))
    u_prev = np.zeros((n, 1)); u = np.zeros((n, 1))
    energies = []
    for k in range(len(w)):
        u_next = 2 * u - u_prev + dt * dt * (A @ u + w[k] * G) / b[:, None]
        if k * dt > 2 * 1.5 / f_p + dt:
            energies.append(fine.leapfrog_energy(A, b, u_next, u, dt)[0])
        u_prev, u = u, u_next
    e = np.array(energies)
    assert e[0] > 0
    assert np.abs(e - e[0]).max() <= 1e-12 * e[0]


def test_ricker_shape():
    dt = 0.1
    f_p = 0.05
    w = synth.ricker(2000, dt, f_p)
    t0 = 1.5 / f_p
    k0 = int(round(t0 / dt))
    assert abs(w[k0] - 1.0) < 1e-12
    assert np.all(w[np.arange(2000) * dt > 2 * t0] == 0.0)
