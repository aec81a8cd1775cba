"""Pins of the oracle's per-cell ROM: rational Krylov projection (Sec. 4.2),
block Lanczos (App. C) and S-fraction (Sec. 5, App. C eq. GammaTrans)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import rom_cell as rc
from oracle.partition import CartesianPartition


@pytest.fixture(scope="module")
def cells():
    """A wall cell (Dirichlet nodes on three sides) and a floating interior
    cell (A_i has the constant null vector)."""
    rng = np.random.default_rng(21)
    nvox = (24, 24, 24)
    sigma = 4.0 ** rng.uniform(0, 1, nvox)
    rho = rng.uniform(1, 2, nvox)
    part = CartesianPartition(nvox, ([8, 16],) * 3, 4, 2)
    out = {}
    for name, idx in (("wall", part.cell_id(0, 0, 0)), ("floating", part.cell_id(1, 1, 1))):
        A, b = part.cell_operator(idx, sigma, rho)
        out[name] = (A, b, part.cell_W(idx), part, idx)
    return out


S_SHIFT = -0.02
ZS = [S_SHIFT, -0.5, 0.3 + 0.2j, 2.0 + 1.0j, -0.01 + 0.5j, 5.0]


def _rom(A, b, W, m):
    V = rc.rational_krylov(A, b, W, S_SHIFT, m)
    Am, Sm = rc.project(A, V, W)
    al, be = rc.block_lanczos(Am, Sm, m)
    Ghat, G = rc.sfraction(al, be)
    return V, Am, Sm, al, be, Ghat, G


@pytest.mark.parametrize("name", ["wall", "floating"])
def test_krylov_basis_and_pade_moments(cells, name):
    A, b, W, _, _ = cells[name]
    m = 3
    V, Am, Sm, *_ = _rom(A, b, W, m)
    assert np.abs(V.T @ (b[:, None] * V) - np.eye(V.shape[1])).max() < 1e-11
    X = W / b[:, None]
    assert np.linalg.norm(X - V @ (V.T @ (b[:, None] * X))) < 1e-10 * np.linalg.norm(X)
    # Lemma lemStil: projected pencil is non-positive
    assert np.linalg.eigvalsh(Am).max() <= 1e-12 * np.abs(Am).max()
    # Pade at s: derivatives j = 0..2m-3 of W^T (A + zB)^{-1} W match at z = s.
    # Full side: F^{(j)}(s) = (-1)^j j! W^T [(A+sB)^{-1} B]^j (A+sB)^{-1} W by dense LU.
    Cs = A + S_SHIFT * np.diag(b)
    n = Am.shape[0]
    Cm = Am + S_SHIFT * np.eye(n)
    Y = np.linalg.solve(Cs, W)
    Ym = np.linalg.solve(Cm, Sm)
    for j in range(2 * m - 2):
        full = W.T @ Y
        red = Sm.T @ Ym
        assert np.abs(full - red).max() <= 1e-8 * np.abs(full).max(), j
        Y = np.linalg.solve(Cs, b[:, None] * Y)
        Ym = np.linalg.solve(Cm, Ym)


@pytest.mark.parametrize("name", ["wall", "floating"])
def test_sfraction_transfer_function_identity(cells, name):
    """U^1(z) of the three-point scheme, the nested continued fraction
    (eq. S-fraction), the block tridiagonal form (eq. NtDtri) and the
    projected ROM (eq. tfprj) are one function of z."""
    A, b, W, _, _ = cells[name]
    V, Am, Sm, al, be, Ghat, G = _rom(A, b, W, 3)
    for z in ZS:
        ref = rc.tf_rom(Am, Sm, z)
        sc = np.abs(ref).max()
        assert np.abs(rc.tf_tridiag(al, be, z) - ref).max() <= 1e-11 * sc
        assert np.abs(rc.tf_sfraction(Ghat, G, z) - ref).max() <= 1e-10 * sc
        assert np.abs(rc.tf_continued_fraction(Ghat, G, z) - ref).max() <= 1e-10 * sc
    full = rc.tf_full(A, b, W, S_SHIFT)
    assert np.abs(rc.tf_sfraction(Ghat, G, S_SHIFT) - full).max() <= 1e-9 * np.abs(full).max()


@pytest.mark.parametrize("name", ["wall", "floating"])
def test_first_layer_closed_forms_and_definiteness(cells, name):
    A, b, W, part, idx = cells[name]
    V, Am, Sm, al, be, Ghat, G = _rom(A, b, W, 3)
    Gh1 = W.T @ (W / b[:, None])
    assert np.abs(Ghat[0] - Gh1).max() <= 1e-12 * np.abs(Gh1).max()
    Xa = W.T @ (A @ (W / b[:, None])) / 1.0
    Xa = (W / b[:, None]).T @ (A @ (W / b[:, None]))
    inv = np.linalg.inv(Gh1)
    G1 = -inv @ Xa @ inv
    assert np.abs(G[0] - G1).max() <= 1e-9 * np.abs(G1).max()
    # Ghat^1 is block diagonal over the cell's pieces (Remark Sinsubspace)
    col = 0
    mask = np.zeros_like(Gh1, dtype=bool)
    for p in part.cells[idx].pieces:
        k = part.pieces[p].S.shape[1]
        mask[col:col + k, col:col + k] = True
        col += k
    assert np.abs(Ghat[0][~mask]).max() <= 1e-14 * np.abs(Ghat[0]).max()
    # SPD pivots (eq. S-fraction); the deepest G^m of a floating cell is only
    # semidefinite to rounding, so it gets a relative tolerance
    for k in range(3):
        assert np.linalg.eigvalsh(Ghat[k]).min() > 0
        ev = np.linalg.eigvalsh(G[k])
        if k < 2:
            assert ev.min() > 0
        else:
            assert ev.min() > -1e-10 * ev.max()


def _lanczos_symmetric_normalisation(Am, Sm, m):
    """Same block Lanczos with symmetric square-root normalisation
    beta = (Z^T Z)^{1/2}, Q = Z beta^{-1}: a different basis of the same
    Krylov space."""
    def nrm(Z):
        w, U = np.linalg.eigh(Z.T @ Z)
        beta = (U * np.sqrt(w)) @ U.T
        return Z @ np.linalg.inv(beta), beta
    Q1, b1 = nrm(Sm)
    Qs, al, be = [Q1], [], [b1]
    for k in range(m):
        AQ = Am @ Qs[k]
        a = Qs[k].T @ AQ
        al.append(0.5 * (a + a.T))
        if k == m - 1:
            break
        Z = AQ - Qs[k] @ al[k] - (Qs[k - 1] @ be[k].T if k else 0)
        Qa = np.hstack(Qs)
        for _ in range(2):
            Z = Z - Qa @ (Qa.T @ Z)
        Qn, bn = nrm(Z)
        Qs.append(Qn); be.append(bn)
    return al, be


def test_sfraction_is_basis_independent(cells):
    """Uniqueness of the S-fraction (Sec. 5): QR and symmetric Lanczos
    normalisations give the same blocks."""
    A, b, W, _, _ = cells["wall"]
    V, Am, Sm, al, be, Ghat, G = _rom(A, b, W, 3)
    al2, be2 = _lanczos_symmetric_normalisation(Am, Sm, 3)
    Gh2, G2 = rc.sfraction(al2, be2)
    for k in range(3):
        assert np.abs(Gh2[k] - Ghat[k]).max() <= 1e-10 * np.abs(Ghat[k]).max()
        assert np.abs(G2[k] - G[k]).max() <= 1e-9 * np.abs(G[k]).max()


def test_scalar_single_layer_closed_form():
    """b = 1, m = 1: F = beta^2/(alpha + z) = 1/(z/Ghat - G) gives
    Ghat = beta^2, G = -alpha/beta^2."""
    alpha, beta = -0.7, 1.3
    Ghat, G = rc.sfraction([np.array([[alpha]])], [np.array([[beta]])])
    assert np.isclose(Ghat[0][0, 0], beta ** 2, rtol=1e-15)
    assert np.isclose(G[0][0, 0], -alpha / beta ** 2, rtol=1e-15)


def _printed_gammatrans(alphas, betas):
    """eq. GammaTrans exactly as printed (G_k^T in the second relation,
    beta taken symmetric): kept only to show it does not reproduce the TF."""
    m = len(alphas)
    b = alphas[0].shape[0]
    Gk = betas[0].copy(); Gprev = np.zeros((b, b)); Ghat, G = [], []
    for k in range(m):
        Ghat.append(Gk @ Gk.T)
        Gc = -Gk.T @ alphas[k] @ np.linalg.inv(Gk) - Gprev
        G.append(Gc)
        if k < m - 1:
            Gk = np.linalg.solve(Gk.T @ Gc, betas[k + 1])
        Gprev = Gc
    return Ghat, G


def test_printed_gammatrans_fails_tf_identity(cells):
    A, b, W, _, _ = cells["wall"]
    V, Am, Sm, al, be, *_ = _rom(A, b, W, 3)
    Gh, G = _printed_gammatrans(al, be)
    ref = rc.tf_rom(Am, Sm, -0.5)
    err = np.abs(rc.tf_sfraction(Gh, G, -0.5) - ref).max() / np.abs(ref).max()
    assert err > 1e-3


def test_breakdown_on_dependent_inputs(cells):
    """Assumption 1: a duplicated boundary column makes the first Krylov
    block rank deficient."""
    A, b, W, _, _ = cells["wall"]
    W2 = np.hstack([W, W[:, :1]])
    with pytest.raises(rc.Breakdown):
        rc.rational_krylov(A, b, W2, S_SHIFT, 2)
