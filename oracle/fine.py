"""Fine-grid reference model (Sec. 1, eq. wave_fll) and its leapfrog.

The acoustic example of Sec. 1 (div sigma grad u - rho u_tt = g delta(t))
is discretised conservatively on unit voxels: nodes sit at voxel corners,
nodes on the outer faces are Dirichlet (removed), every voxel v adds
sigma_v/4 to the conductance of each of its 12 edges and rho_v/8 to the
mass of each of its 8 corners. A = -sum_edges c (e_a - e_b)(e_a - e_b)^T is
then a symmetric non-positive graph Laplacian with nontrivial diagonal and B
is diagonal positive, as Sec. 1 requires.

Force convention used throughout the oracle (see rom_global): the time-domain
model is B u'' = A u + w(t) g with u = 0 for t <= 0; the paper's sign of the
source term is a global sign common to the fine model and the ROM.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import scipy.linalg as sla


def node_index(nvox):
    """Map from node coordinates to unknown index (x fastest), -1 on walls."""
    nx, ny, nz = nvox
    idx = -np.ones((nx + 1, ny + 1, nz + 1), dtype=np.int64)
    ux, uy, uz = nx - 1, ny - 1, nz - 1
    xs, ys, zs = np.meshgrid(np.arange(1, nx), np.arange(1, ny), np.arange(1, nz), indexing="ij")
    idx[1:nx, 1:ny, 1:nz] = (xs - 1) + ux * ((ys - 1) + uy * (zs - 1))
    return idx


def edge_conductances(sigma):
    """Conductances of all grid edges from per-voxel sigma.

    Returns (cx, cy, cz): cx[i, j, k] is the conductance of the edge from node
    (i, j, k) to (i+1, j, k), the sum of sigma_v / 4 over the (up to) four
    voxels sharing that edge; likewise cy, cz.
    """
    nx, ny, nz = sigma.shape
    q = sigma / 4.0
    cx = np.zeros((nx, ny + 1, nz + 1))
    cy = np.zeros((nx + 1, ny, nz + 1))
    cz = np.zeros((nx + 1, ny + 1, nz))
    for a in (0, 1):
        for b in (0, 1):
            cx[:, a:a + ny, b:b + nz] += q
            cy[a:a + nx, :, b:b + nz] += q
            cz[a:a + nx, b:b + ny, :] += q
    return cx, cy, cz


def node_masses(rho):
    """Mass of every grid node: sum of rho_v / 8 over its voxels."""
    nx, ny, nz = rho.shape
    m = np.zeros((nx + 1, ny + 1, nz + 1))
    q = rho / 8.0
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                m[a:a + nx, b:b + ny, c:c + nz] += q
    return m


def _laplacian_from_edges(cx, cy, cz, idx):
    """A = -sum_e c_e (e_a - e_b)(e_a - e_b)^T over edges, restricted to the
    unknowns in ``idx`` (edges to wall nodes keep only their diagonal part)."""
    n = int(idx.max()) + 1
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    for c, (dx, dy, dz) in ((cx, (1, 0, 0)), (cy, (0, 1, 0)), (cz, (0, 0, 1))):
        sx, sy, sz = c.shape
        a = idx[0:sx, 0:sy, 0:sz]
        b = idx[dx:dx + sx, dy:dy + sy, dz:dz + sz]
        c = c.ravel(); a = a.ravel(); b = b.ravel()
        keep = c != 0.0
        c, a, b = c[keep], a[keep], b[keep]
        ma, mb = a >= 0, b >= 0
        np.add.at(diag, a[ma], -c[ma])
        np.add.at(diag, b[mb], -c[mb])
        both = ma & mb
        rows += [a[both], b[both]]
        cols += [b[both], a[both]]
        vals += [c[both], c[both]]
    rows.append(np.arange(n)); cols.append(np.arange(n)); vals.append(diag)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    A.sum_duplicates()
    A.sort_indices()
    return A


def assemble_acoustic(sigma, rho):
    """Fine pencil (A, b) of Sec. 1 for per-voxel sigma, rho (arrays [x,y,z]).

    Returns A (CSR, n x n, symmetric, <= 0) and b = diag(B) (length n), with
    unknowns numbered x-fastest over nodes 1..n_axis-1 on each axis.
    """
    nvox = sigma.shape
    idx = node_index(nvox)
    cx, cy, cz = edge_conductances(sigma)
    A = _laplacian_from_edges(cx, cy, cz, idx)
    mass = node_masses(rho)
    b = mass[1:nvox[0], 1:nvox[1], 1:nvox[2]].transpose(2, 1, 0).ravel().copy()
    return A, b


def lambda_max(A, b, tol=1e-10):
    """Largest eigenvalue of the pencil (-A, B), i.e. of B^{-1}(-A)."""
    d = 1.0 / np.sqrt(b)
    M = sp.diags(d) @ (-A) @ sp.diags(d)
    n = A.shape[0]
    if n <= 400:
        return float(np.linalg.eigvalsh(M.toarray())[-1])
    return float(spla.eigsh(M, k=1, which="LA", tol=tol, return_eigenvectors=False)[0])


def cfl_dt(A, b, fraction=0.5):
    """Leapfrog time step at ``fraction`` of the stability limit 2/sqrt(lambda_max)."""
    return fraction * 2.0 / np.sqrt(lambda_max(A, b))


def leapfrog(A, b, G, Q, w, dt):
    """Explicit leapfrog for B u'' = A u + w(t) G, u^0 = u^{-1} = 0.

    u^{n+1} = 2 u^n - u^{n-1} + dt^2 B^{-1} (A u^n + w^n G), n = 0..N-1, and
    traces[n] = Q^T u^{n+1}. G is n x n_s, Q is n x n_r (dense or sparse).
    Returns traces with shape (N, n_r, n_s).
    """
    G = G.toarray() if sp.issparse(G) else np.asarray(G)
    Qt = (Q.T.tocsr() if sp.issparse(Q) else np.asarray(Q).T)
    n, ns = G.shape
    binv = (1.0 / b)[:, None]
    u_prev = np.zeros((n, ns))
    u = np.zeros((n, ns))
    out = np.empty((len(w), Qt.shape[0], ns))
    dt2 = dt * dt
    for k in range(len(w)):
        acc = A @ u + w[k] * G
        u_next = 2.0 * u - u_prev + dt2 * binv * acc
        u_prev, u = u, u_next
        out[k] = Qt @ u
    return out


def leapfrog_energy(A, b, u_next, u, dt):
    """Conserved discrete energy of the source-free leapfrog between levels
    n and n+1: 1/2 v^T B v + 1/2 u_next^T (-A) u, v = (u_next - u)/dt."""
    v = (u_next - u) / dt
    return 0.5 * np.sum(b[:, None] * v * v, axis=0) + 0.5 * np.sum(u_next * (-(A @ u)), axis=0)


def modal_traces(A, b, G, Q, w, dt):
    """Exact solution of the leapfrog recurrence by eigen-expansion.

    With B^{-1}(-A) z_l = mu_l z_l, z_l^T B z_l = 1 and cos(theta_l) =
    1 - mu_l dt^2 / 2, each modal amplitude obeys a scalar three-term
    recurrence whose Green's function is sin((n+1-j) theta)/sin(theta), so
    traces[n] = sum_l (Q^T z_l)(z_l^T G) dt^2 sum_{j<=n} w^j
    sin((n+1-j) theta_l)/sin(theta_l). Dense; for tiny grids only.
    """
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    G = G.toarray() if sp.issparse(G) else np.asarray(G)
    Q = Q.toarray() if sp.issparse(Q) else np.asarray(Q)
    mu, Z = sla.eigh(-Ad, np.diag(b))          # Z^T B Z = I
    theta = np.arccos(1.0 - mu * dt * dt / 2.0)
    qz = Q.T @ Z                                 # n_r x L
    zg = Z.T @ G                                 # L x n_s
    N = len(w)
    n = np.arange(N)
    out = np.zeros((N, Q.shape[1], G.shape[1]))
    for l in range(len(mu)):
        # h[n] = sum_{j<=n} w_j sin((n+1-j) th)/sin th  (direct convolution)
        kern = np.sin((n + 1) * theta[l]) / np.sin(theta[l])
        h = np.convolve(w, kern)[:N] * dt * dt
        out += h[:, None, None] * np.outer(qz[:, l], zg[l, :])[None, :, :]
    return out
