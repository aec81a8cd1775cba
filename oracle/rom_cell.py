"""Per-cell reduced-order model and its matrix S-fraction.

Steps, in the paper's order:

1. Rational block Krylov subspace at a negative shift s (Sec. 4.2, eq. npks),
   projection of the cell pencil onto it (eq. tfprj).
2. Block Lanczos on the projected pencil (App. C, eq. NtDtri): a block
   tridiagonal T with T_{k+1,k} = beta_{k+1}, T_{k,k+1} = beta_{k+1}^T and
   R = [beta_1; 0; ...].
3. The recursive block-diagonal change of variables (App. C, eq. GammaTrans)
   giving the S-fraction blocks Ghat^k, G^k (eq. S-fraction) of the
   three-point scheme (eqs. GammaU1st, GammaUrem).

Readings:

* Krylov operator (eq. npks). Moment matching at s (the Pade remark after
  Assumption 1) and a piece-block-diagonal Ghat^1 (Remark Sinsubspace) both
  need the B-weighted operator, so the subspace is
  span{X, K X, ..., K^{m-1} X} with K = (A + sB)^{-1} B and X = B^{-1} W,
  W = P^Gamma S (the zero-power term is included, as Remark Sinsubspace
  recommends). The basis is B-orthonormal, so B^m = I.
* beta blocks from a QR step are triangular, not symmetric as App. C
  assumes; with T_{k+1,k} = beta_{k+1} the change of variables reads
  G_1 = beta_1^T, G_{k+1} = (G_k^T G^k)^{-1} beta_{k+1}^T.
* The printed middle relation of eq. GammaTrans has G_k^T where the
  derivation from the three-term relations (eq. tridiagW) gives G_k^{-T}:
  G^k = -G_k^{-T} alpha_k G_k^{-1} - G^{k-1}.
* The last displayed formula of App. C is read as
  U^1(z) = E_1^T (L + z D)^{-1} E_1 with D = blkdiag((Ghat^k)^{-1}) and L
  the block tridiagonal operator of eqs. GammaU1st-GammaUrem.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class Breakdown(RuntimeError):
    """Krylov or Lanczos block lost rank (Assumption 1 / Assumption 2)."""


def _bchol(gram, what):
    try:
        return sla.cholesky(gram, lower=False)
    except np.linalg.LinAlgError as e:  # pragma: no cover - exercised by tests
        raise Breakdown(what) from e


def rational_krylov(A, b, W, s, m):
    """B-orthonormal basis V (N x m b) of span{X, KX, ..., K^{m-1}X},
    K = (A + sB)^{-1} B, X = B^{-1} W (Sec. 4.2, eq. npks).

    Each new block is orthogonalised against all previous blocks in the
    B inner product by classical Gram-Schmidt applied twice, then
    normalised by the Cholesky factor of its B-Gram matrix.
    """
    if s >= 0:
        raise ValueError("shift must be negative")
    C = -(A + s * np.diag(b))                 # SPD because A <= 0, B > 0, s < 0
    fac = sla.cho_factor(C, lower=True)
    X = W / b[:, None]
    blocks = []
    for j in range(m):
        if blocks:
            V = np.hstack(blocks)
            for _ in range(2):
                X = X - V @ (V.T @ (b[:, None] * X))
        gram = X.T @ (b[:, None] * X)
        R = _bchol(0.5 * (gram + gram.T), f"Krylov block {j + 1}")
        scale = np.abs(np.diag(R)).min() / max(np.abs(np.diag(R)).max(), 1e-300)
        if scale < 1e-10:
            raise Breakdown(f"Krylov block {j + 1} nearly rank deficient")
        q = sla.solve_triangular(R, X.T, trans="T", lower=False).T   # X R^{-1}
        blocks.append(q)
        if j < m - 1:
            X = -sla.cho_solve(fac, b[:, None] * q)                  # (A + sB)^{-1} B q
    return np.hstack(blocks)


def project(A, V, W):
    """Projected pencil and input (eq. tfprj): A^m = V^T A V (symmetrised),
    S^m = V^T W."""
    Am = V.T @ (A @ V)
    return 0.5 * (Am + Am.T), V.T @ W


def block_lanczos(Am, Sm, m):
    """Block Lanczos on (A^m, I) started from S^m (App. C).

    Q_1 beta_1 = S^m (QR), alpha_k = Q_k^T A^m Q_k,
    Q_{k+1} beta_{k+1} = A^m Q_k - Q_k alpha_k - Q_{k-1} beta_k^T
    (reorthogonalised twice against all previous Q). Returns (alphas, betas)
    with betas[0] = beta_1 and betas[k] = beta_{k+1}.
    """
    Q1, beta1 = np.linalg.qr(Sm)
    Qs, alphas, betas = [Q1], [], [beta1]
    for k in range(m):
        Qk = Qs[k]
        AQ = Am @ Qk
        alpha = Qk.T @ AQ
        alphas.append(0.5 * (alpha + alpha.T))
        if k == m - 1:
            break
        Z = AQ - Qk @ alphas[k]
        if k > 0:
            Z = Z - Qs[k - 1] @ betas[k].T
        Qall = np.hstack(Qs)
        for _ in range(2):
            Z = Z - Qall @ (Qall.T @ Z)
        Qn, beta = np.linalg.qr(Z)
        d = np.abs(np.diag(beta))
        if d.min() < 1e-12 * max(d.max(), 1e-300):
            raise Breakdown(f"Lanczos block {k + 2} rank deficient")
        Qs.append(Qn)
        betas.append(beta)
    return alphas, betas


def sfraction(alphas, betas):
    """S-fraction blocks from the block tridiagonal form (App. C, eq.
    GammaTrans, corrected as stated in the module docstring).

    G_1 = beta_1^T, G^0 = 0; for k = 1..m: Ghat^k = G_k G_k^T,
    G^k = -G_k^{-T} alpha_k G_k^{-1} - G^{k-1},
    G_{k+1} = (G_k^T G^k)^{-1} beta_{k+1}^T.
    Returns (Ghat list, G list), each of m symmetric b x b blocks.
    """
    m = len(alphas)
    b = alphas[0].shape[0]
    Gk = betas[0].T.copy()
    Gprev = np.zeros((b, b))
    Ghat, G = [], []
    for k in range(m):
        Ghat.append(Gk @ Gk.T)
        Ginv = np.linalg.inv(Gk)
        Gc = -Ginv.T @ alphas[k] @ Ginv - Gprev
        Gc = 0.5 * (Gc + Gc.T)
        G.append(Gc)
        if k < m - 1:
            Gk = np.linalg.solve(Gk.T @ Gc, betas[k + 1].T)
        Gprev = Gc
    return Ghat, G


def build_cell(A, b, W, s, m):
    """Off-line stage of one cell (Alg. alg1red, stage 1)."""
    V = rational_krylov(A, b, W, s, m)
    Am, Sm = project(A, V, W)
    alphas, betas = block_lanczos(Am, Sm, m)
    return sfraction(alphas, betas)


# --------------------------------------------------------------------------
# transfer functions used as pins
# --------------------------------------------------------------------------

def tf_full(A, b, W, z):
    """Projected cell transfer function W^T (A + z B)^{-1} W (eqs. tfcur, project)."""
    return W.T @ np.linalg.solve(A + z * np.diag(b), W.astype(complex) if np.iscomplexobj(z) else W)


def tf_rom(Am, Sm, z):
    """ROM transfer function (S^m)^T (A^m + z I)^{-1} S^m (eq. tfprj, B^m = I)."""
    n = Am.shape[0]
    return Sm.T @ np.linalg.solve(Am + z * np.eye(n), Sm.astype(complex) if np.iscomplexobj(z) else Sm)


def tf_tridiag(alphas, betas, z):
    """beta_1^T [(T + zI)^{-1}]_{11} beta_1 (App. C, eq. NtDtri)."""
    m = len(alphas)
    b = alphas[0].shape[0]
    T = np.zeros((m * b, m * b), dtype=complex if np.iscomplexobj(z) else float)
    for k in range(m):
        T[k * b:(k + 1) * b, k * b:(k + 1) * b] = alphas[k]
        if k + 1 < m:
            T[(k + 1) * b:(k + 2) * b, k * b:(k + 1) * b] = betas[k + 1]
            T[k * b:(k + 1) * b, (k + 1) * b:(k + 2) * b] = betas[k + 1].T
    R = np.zeros((m * b, b)); R[:b] = betas[0]
    return R.T @ np.linalg.solve(T + z * np.eye(m * b), R)


def layered_operator(Ghat, G):
    """(L, D) of the three-point scheme (eqs. GammaU1st, GammaUrem): L is block
    tridiagonal with L_kk = -(G^k + G^{k-1}), L_{k,k+1} = L_{k+1,k} = G^k,
    and D = blkdiag((Ghat^k)^{-1})."""
    m = len(G)
    b = G[0].shape[0]
    L = np.zeros((m * b, m * b))
    D = np.zeros((m * b, m * b))
    for k in range(m):
        sl = slice(k * b, (k + 1) * b)
        L[sl, sl] = -(G[k] + (G[k - 1] if k > 0 else 0.0))
        if k + 1 < m:
            nx = slice((k + 1) * b, (k + 2) * b)
            L[sl, nx] = G[k]
            L[nx, sl] = G[k]
        D[sl, sl] = np.linalg.inv(Ghat[k])
    return L, D


def tf_sfraction(Ghat, G, z):
    """U^1(z) = E_1^T (L + z D)^{-1} E_1 (eqs. GammaU1st-tfgamma)."""
    L, D = layered_operator(Ghat, G)
    b = G[0].shape[0]
    E = np.zeros((L.shape[0], b)); E[:b] = np.eye(b)
    return E.T @ np.linalg.solve(L + z * D, E)


def tf_continued_fraction(Ghat, G, z):
    """Nested matrix continued fraction of eq. S-fraction, with the overall
    sign that makes it equal to U^1 of the three-point scheme:
    Y_m = z Ghat_m^{-1} - G^m, Y_k = z Ghat_k^{-1} - (G_k^{-1} - Y_{k+1}^{-1})^{-1},
    U^1 = Y_1^{-1}."""
    inv = np.linalg.inv
    m = len(G)
    Y = z * inv(Ghat[m - 1]) - G[m - 1]
    for k in range(m - 2, -1, -1):
        Y = z * inv(Ghat[k]) - inv(inv(G[k]) - inv(Y))
    return inv(Y)
