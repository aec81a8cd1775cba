"""Learned off-line stage: a small 3D CNN from a cell's medium to its
S-fraction, with the fallback test (plain FP64 numpy; test infrastructure).

The paper builds each cell's S-fraction by block Lanczos (Sec. 5, App. C).
This module is the reference for a learned replacement of that build for
interior cells (parity unpinned against the paper, which has no learned
part; pinned here against finite differences, closed forms and the Lanczos
route):

* Layer 1 in closed form. With X = B^{-1} W the start of the Krylov space
  and B-orthonormal V spanning it, the first S-fraction blocks are
  Ghat^1 = W^T B^{-1} W and G^1 = -(Ghat^1)^{-1} (X^T A X) (Ghat^1)^{-1}
  (from G_1 = beta_1^T, Ghat^1 = G_1 G_1^T and eq. GammaTrans with
  G^0 = 0), so the network predicts layers 2..m only.
* Targets: the lower Cholesky factors of Ghat^k and of G^k + eps_k I for
  k = 2..m (eps_k = 1e-10 tr(G^k) / b, since G^m of a floating cell is only
  semidefinite), rows of the lower triangles concatenated. Reconstruction
  as L L^T + eps I gives SPD blocks by construction, hence a Stieltjes ROM
  (Prop. prop1stil).
* Network: conv3d(2 -> C, 3^3, zero padding) + ReLU, 2^3 average pooling,
  dense(C*64 -> H) + ReLU, dense(H -> P); loss = mean squared error over
  the batch and the P normalised outputs; Adam.
* Fallback test: relative Frobenius mismatch of the ROM transfer function
  U^1(z) against the exact cell transfer function W^T (A + z B)^{-1} W at
  16 points z = -sigma_j^2 of the Laplace axis, sigma_j = (j + 1/2)
  omega_max / 16 (no poles there); a cell is accepted when the largest
  mismatch is at most the tolerance.
"""
from __future__ import annotations

import numpy as np

from .rom_cell import tf_full, tf_sfraction

VOX = 8


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------

def param_shapes(conv_ch: int, hidden: int, n_out: int):
    """Shapes of (W1, b1, W2, b2, W3, b3) in the flat parameter order."""
    return [(conv_ch, 2, 3, 3, 3), (conv_ch,), (hidden, conv_ch * 64), (hidden,),
            (n_out, hidden), (n_out,)]


def unflatten(theta, conv_ch, hidden, n_out):
    out, o = [], 0
    for s in param_shapes(conv_ch, hidden, n_out):
        k = int(np.prod(s))
        out.append(np.asarray(theta[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def flatten(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------

def _pad(x):
    return np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))


def forward(theta, x, conv_ch, hidden, n_out):
    """x: (N, 2, 8, 8, 8) -> (y (N, P), cache)."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta, conv_ch, hidden, n_out)
    n = x.shape[0]
    xp = _pad(x)
    z1 = np.zeros((n, conv_ch, VOX, VOX, VOX))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                win = xp[:, :, dz:dz + VOX, dy:dy + VOX, dx:dx + VOX]        # (N, 2, 8, 8, 8)
                z1 += np.einsum("oc,nczyx->nozyx", W1[:, :, dz, dy, dx], win)
    z1 += b1[None, :, None, None, None]
    h1 = np.maximum(z1, 0.0)
    p = h1.reshape(n, conv_ch, 4, 2, 4, 2, 4, 2).mean(axis=(3, 5, 7)).reshape(n, conv_ch * 64)
    z2 = p @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3.T + b3
    return y, (xp, z1, h1, p, z2, h2)


def loss_and_grad(theta, x, t, conv_ch, hidden, n_out):
    """Mean squared error and its gradient with respect to theta."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta, conv_ch, hidden, n_out)
    y, (xp, z1, h1, p, z2, h2) = forward(theta, x, conv_ch, hidden, n_out)
    n = x.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / r.size
    gW3 = dy.T @ h2
    gb3 = dy.sum(axis=0)
    dh2 = dy @ W3
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ p
    gb2 = dz2.sum(axis=0)
    dp = (dz2 @ W2).reshape(n, conv_ch, 4, 1, 4, 1, 4, 1) / 8.0
    dh1 = np.broadcast_to(dp, (n, conv_ch, 4, 2, 4, 2, 4, 2)).reshape(n, conv_ch, VOX, VOX, VOX)
    dz1 = dh1 * (z1 > 0)
    gW1 = np.zeros_like(W1)
    for dz in range(3):
        for dy_ in range(3):
            for dx in range(3):
                win = xp[:, :, dz:dz + VOX, dy_:dy_ + VOX, dx:dx + VOX]
                gW1[:, :, dz, dy_, dx] = np.einsum("nozyx,nczyx->oc", dz1, win)
    gb1 = dz1.sum(axis=(0, 2, 3, 4))
    return loss, flatten([gW1, gb1, gW2, gb2, gW3, gb3])


def adam_step(theta, g, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; state = (m, v, t) is updated in place and returned."""
    m, v, t = state
    t += 1
    m[:] = beta1 * m + (1.0 - beta1) * g
    v[:] = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    theta = theta - lr * mh / (np.sqrt(vh) + eps)
    return theta, (m, v, t)


# ---------------------------------------------------------------------------
# S-fraction <-> network outputs
# ---------------------------------------------------------------------------

def cell_features(sigma, rho, lo):
    """(2, 8, 8, 8) input of the cell whose voxel box starts at lo = (x, y, z):
    log sigma and log rho of its voxels, [channel][z][y][x]."""
    x0, y0, z0 = lo
    s = sigma[x0:x0 + VOX, y0:y0 + VOX, z0:z0 + VOX]
    r = rho[x0:x0 + VOX, y0:y0 + VOX, z0:z0 + VOX]
    return np.stack([np.log(s).transpose(2, 1, 0), np.log(r).transpose(2, 1, 0)])


def _eps(M):
    return 1e-10 * np.trace(M) / M.shape[0]


def targets(Ghat, G):
    """Lower Cholesky factors of Ghat^k and G^k + eps I, k = 2..m, as one
    vector (row-major lower triangles, Ghat before G per layer)."""
    b = G[0].shape[0]
    il = np.tril_indices(b)
    out = []
    for k in range(1, len(G)):
        out.append(np.linalg.cholesky(Ghat[k])[il])
        out.append(np.linalg.cholesky(G[k] + _eps(G[k]) * np.eye(b))[il])
    return np.concatenate(out)


def reconstruct(y, b, m):
    """Ghat^k, G^k for k = 2..m from the factor vector: L L^T + eps I."""
    il = np.tril_indices(b)
    nt = len(il[0])
    Gh, G = [], []
    for k in range(m - 1):
        for j, dst in enumerate((Gh, G)):
            L = np.zeros((b, b))
            L[il] = y[(2 * k + j) * nt:(2 * k + j + 1) * nt]
            M = L @ L.T
            dst.append(M + _eps(M) * np.eye(b))
    return Gh, G


def layer1_closed_form(A, bdiag, W):
    """Ghat^1 = W^T B^{-1} W, G^1 = -(Ghat^1)^{-1} X^T A X (Ghat^1)^{-1},
    X = B^{-1} W."""
    X = W / bdiag[:, None]
    Gh1 = W.T @ X
    Gi = np.linalg.inv(Gh1)
    G1 = -Gi @ (X.T @ (A @ X)) @ Gi
    return 0.5 * (Gh1 + Gh1.T), 0.5 * (G1 + G1.T)


def laplace_points(omega_max, count=16):
    """z_j = -sigma_j^2, sigma_j = (j + 1/2) omega_max / count."""
    s = (np.arange(count) + 0.5) * omega_max / count
    return -s * s


def tf_mismatch(A, bdiag, W, Ghat, G, omega_max, count=16):
    """Largest relative Frobenius mismatch of the ROM transfer function
    against the exact cell transfer function on the Laplace axis."""
    worst = 0.0
    for z in laplace_points(omega_max, count):
        ex = tf_full(A, bdiag, W, z)
        ro = tf_sfraction(Ghat, G, z)
        worst = max(worst, np.linalg.norm(ro - ex) / np.linalg.norm(ex))
    return worst
