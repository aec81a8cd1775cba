"""Spectral projector of eq. trgrstep by Zolotarev's rational approximation of
the sign function (Sec. 4.1), and the Gramian of a piece built from it.

Test infrastructure only: FP64 numpy/scipy, sparse complex LU for the
shifted solves. Nothing here is imported by the product.

The Gramian of eq. trgr is G = R Z_w R^T with Z_w = sum over the
B-orthonormal eigenvectors z_l of the pencil (-A, B) with lambda_l <= w^2
of z_l z_l^T, and R the restriction to the piece. With
C = B^{-1/2} (-A) B^{-1/2}, Z_w = B^{-1/2} eta(w^2 I - C) B^{-1/2}, and
eta(x) = (1 + sign(x)) / 2 (eq. trgrstep).

Zolotarev's best uniform rational approximation of sign(x) on
[-1, -delta] U [delta, 1] (type (2n-1, 2n)), in partial fractions:

    Z(x) = M x sum_{j=1..n} a_j / (x^2 + c_{2j-1}),
    c_i = delta^2 sn^2(i K'/(2n); k') / cn^2(i K'/(2n); k'),  k' = sqrt(1 - delta^2),
    a_j = prod_{i=1..n-1} (c_{2i} - c_{2j-1}) / prod_{i != j} (c_{2i-1} - c_{2j-1}),

with K' the complete elliptic integral of modulus k' and M set so that the
error equioscillates about zero on [delta, 1] (M = 2 / (max + min of the
unscaled function there); the function is monotone between its extrema, so
they are taken on a dense grid). The Jacobi functions come from the
arithmetic-geometric mean (descending Landen) algorithm.

Readings (the paper only names the approach):
* The spectrum is mapped to [-1, 1] by X = (w^2 I - C) / s with
  s = max(w^2, lam_hi - w^2), lam_hi a Gershgorin bound of C; the
  transition band is |lambda - w^2| < gamma w^2, so delta = gamma w^2 / s.
  Eigenvalues inside the band get a weight between 0 and 1.
* Each term is one complex shifted solve: for real symmetric X and beta > 0,
  (X^2 + beta^2 I)^{-1} = Im[(X - i beta I)^{-1}] / beta.
* The B^{-1/2} scaling of Z_w is kept (the printed expression omits it; it
  is what makes the result equal the eigen-sum of eq. trgr).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def agm_ellipk(k):
    """K(k) = pi / (2 AGM(1, sqrt(1 - k^2)))."""
    a, b = 1.0, np.sqrt(1.0 - k * k)
    for _ in range(64):
        if abs(a - b) <= 1e-16 * a:
            break
        a, b = 0.5 * (a + b), np.sqrt(a * b)
    return np.pi / (2.0 * a)


def jacobi_sn_cn_dn(u, k):
    """Jacobi elliptic functions of argument u and modulus k by the
    arithmetic-geometric mean: a_0 = 1, b_0 = k', c_0 = k; run the means to
    a_N; phi_N = 2^N a_N u; then phi_{n-1} = (phi_n + asin(c_n sin(phi_n) /
    a_n)) / 2; sn = sin phi_0, cn = cos phi_0, dn = sqrt(1 - k^2 sn^2)."""
    a, b, c = [1.0], [np.sqrt(1.0 - k * k)], [k]
    for _ in range(64):
        if abs(c[-1]) <= 1e-17:
            break
        a.append(0.5 * (a[-1] + b[-1]))
        c.append(0.5 * (a[-2] - b[-1]))
        b.append(np.sqrt(a[-2] * b[-1]))
    N = len(a) - 1
    phi = (2.0 ** N) * a[N] * u
    for n in range(N, 0, -1):
        phi = 0.5 * (phi + np.arcsin(c[n] * np.sin(phi) / a[n]))
    sn, cn = np.sin(phi), np.cos(phi)
    return sn, cn, np.sqrt(1.0 - k * k * sn * sn)


def zolotarev_sign(n, delta):
    """(M, beta2, a) of Z(x) = M x sum_j a_j / (x^2 + beta2_j)."""
    kp = np.sqrt(1.0 - delta * delta)
    Kp = agm_ellipk(kp)
    c = np.empty(2 * n)
    for i in range(1, 2 * n):
        sn, cn, _ = jacobi_sn_cn_dn(i * Kp / (2 * n), kp)
        c[i] = delta * delta * sn * sn / (cn * cn)
    odd = c[1:2 * n:2]            # c_1, c_3, ..., c_{2n-1}
    even = c[2:2 * n:2]           # c_2, ..., c_{2n-2}
    a = np.empty(n)
    for j in range(n):
        num = np.prod(even - odd[j])
        den = np.prod(np.delete(odd, j) - odd[j])
        a[j] = num / den
    x = np.geomspace(delta, 1.0, 20001)
    f = x * np.sum(a[None, :] / (x[:, None] ** 2 + odd[None, :]), axis=1)
    M = 2.0 / (f.max() + f.min())
    return M, odd, a


def eval_sign(x, M, beta2, a):
    x = np.asarray(x, dtype=float)
    return M * x * np.sum(a[None, :] / (x.ravel()[:, None] ** 2 + beta2[None, :]), axis=1).reshape(x.shape)


def gershgorin_hi(A, b):
    """Upper bound of the spectrum of C = B^{-1/2} (-A) B^{-1/2}."""
    A = sp.csr_matrix(A)
    r = 1.0 / np.sqrt(b)
    C = sp.diags(r) @ (-A) @ sp.diags(r)
    C = sp.csr_matrix(C)
    d = C.diagonal()
    off = np.asarray(abs(C).sum(axis=1)).ravel() - np.abs(d)
    return float((d + off).max())


def projector_columns(A, b, cols, omega_max, n, gamma):
    """Z_w[:, cols] of the pencil (-A, B) (n x len(cols)) by the Zolotarev
    route of the reading above."""
    A = sp.csr_matrix(A)
    N = A.shape[0]
    w2 = omega_max ** 2
    r = 1.0 / np.sqrt(b)
    C = sp.csr_matrix(sp.diags(r) @ (-A) @ sp.diags(r))
    s = max(w2, gershgorin_hi(A, b) - w2)
    delta = min(gamma * w2 / s, 0.5)
    M, beta2, a = zolotarev_sign(n, delta)
    X = sp.csr_matrix((w2 * sp.identity(N) - C) / s)
    E = np.zeros((N, len(cols)))
    E[cols, np.arange(len(cols))] = r[cols]           # B^{-1/2} e_col
    acc = np.zeros_like(E)
    for j in range(n):
        beta = np.sqrt(beta2[j])
        lu = spla.splu(sp.csc_matrix(X - 1j * beta * sp.identity(N)))
        acc += a[j] * np.imag(lu.solve(E.astype(complex))) / beta
    sgn = M * (X @ acc)
    return r[:, None] * 0.5 * (E + sgn)


def rational_gramian(A, b, rows, omega_max, n, gamma):
    """G = R Z_w R^T for the piece rows ``rows`` of the pencil (-A, B)."""
    Z = projector_columns(A, b, rows, omega_max, n, gamma)
    G = Z[rows, :]
    return 0.5 * (G + G.T)


def gramian_bases_zolotarev(part, cell_ops, omega_max, eps, max_modes, depth, n, gamma):
    """S_p for every piece as gramian.gramian_bases, with G from the
    Zolotarev projector of the same local pencil."""
    from . import gramian as gr
    out = []
    for pc in part.pieces:
        if len(pc.nodes) == 1:
            out.append(np.ones((1, 1)))
            continue
        snodes, As, bs = gr.local_pencil(cell_ops, pc.cells, pc.nodes, depth)
        rows = np.searchsorted(snodes, pc.nodes)
        G = rational_gramian(As, bs, rows, omega_max, n, gamma)
        S, _ = gr.basis_from_gramian(G, eps, max_modes)
        out.append(S)
    return out
