"""Pins of the learned off-line stage's reference (oracle/surrogate.py):
finite differences, brute-force convolution, the Lanczos route for the
closed-form first layer, exact factor round trips, and the sensitivity of
the transfer-function test."""
import numpy as np
import pytest

from oracle import surrogate as sg
from oracle import rom_cell as rc
from oracle.partition import CartesianPartition

C, H, P = 2, 5, 7


def _theta(rng, p=P):
    return np.concatenate([rng.normal(0, 0.3, int(np.prod(s))) for s in sg.param_shapes(C, H, p)])


def test_conv_pool_matches_brute_force():
    """The vectorised 3^3 convolution with zero padding and the 2^3 average
    pooling against explicit loops over every output voxel and tap."""
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 2, 8, 8, 8))
    th = _theta(rng)
    W1, b1, W2, b2, W3, b3 = sg.unflatten(th, C, H, P)
    _, (xp, z1, h1, p, z2, h2) = sg.forward(th, x, C, H, P)
    ref = np.zeros_like(z1)
    for n in range(2):
        for o in range(C):
            for z in range(8):
                for y in range(8):
                    for xx in range(8):
                        acc = b1[o]
                        for c in range(2):
                            for dz in (-1, 0, 1):
                                for dy in (-1, 0, 1):
                                    for dx in (-1, 0, 1):
                                        zz, yy, x3 = z + dz, y + dy, xx + dx
                                        if 0 <= zz < 8 and 0 <= yy < 8 and 0 <= x3 < 8:
                                            acc += W1[o, c, dz + 1, dy + 1, dx + 1] * x[n, c, zz, yy, x3]
                        ref[n, o, z, y, xx] = acc
    assert np.abs(z1 - ref).max() < 1e-12
    h = np.maximum(ref, 0)
    pool = np.zeros((2, C, 4, 4, 4))
    for a in range(2):
        for b in range(2):
            for c in range(2):
                pool += h[:, :, a::2, b::2, c::2] / 8
    assert np.abs(p - pool.reshape(2, -1)).max() < 1e-12


def test_gradient_matches_finite_differences():
    """Backward pass against central differences (FP64, step 1e-6)."""
    rng = np.random.default_rng(2)
    x = rng.normal(size=(3, 2, 8, 8, 8))
    t = rng.normal(size=(3, P))
    th = _theta(rng)
    loss, g = sg.loss_and_grad(th, x, t, C, H, P)
    idx = rng.choice(len(th), 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th); e[i] = h
        fd = (sg.loss_and_grad(th + e, x, t, C, H, P)[0] - sg.loss_and_grad(th - e, x, t, C, H, P)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_first_adam_step_is_signed_learning_rate():
    """With zero moments, the bias-corrected first Adam step moves every
    parameter by -lr * g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    th = rng.normal(size=11)
    g = rng.normal(size=11)
    st = (np.zeros(11), np.zeros(11), 0)
    th1, st = sg.adam_step(th, g, st, 1e-2)
    assert np.allclose(th1, th - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert st[2] == 1


@pytest.fixture(scope="module")
def floating_cell():
    rng = np.random.default_rng(4)
    nvox = (24, 24, 24)
    sigma = 4.0 ** rng.uniform(0, 1, nvox)
    rho = rng.uniform(1, 2, nvox)
    part = CartesianPartition(nvox, ([8, 16],) * 3, 4, 2)
    i = part.cell_id(1, 1, 1)
    A, b = part.cell_operator(i, sigma, rho)
    W = part.cell_W(i)
    Gh, G = rc.build_cell(A, b, W, -0.02, 4)
    return A, b, W, Gh, G


def test_layer1_closed_form_equals_lanczos(floating_cell):
    """Ghat^1 and G^1 from B, W and A alone equal the Lanczos route's first
    S-fraction blocks."""
    A, b, W, Gh, G = floating_cell
    gh1, g1 = sg.layer1_closed_form(A, b, W)
    assert np.linalg.norm(gh1 - Gh[0]) / np.linalg.norm(Gh[0]) < 1e-12
    assert np.linalg.norm(g1 - G[0]) / np.linalg.norm(G[0]) < 1e-10


def test_factor_round_trip(floating_cell):
    """reconstruct(targets(blocks)) returns the deep blocks (G^m of the
    floating cell is only semidefinite: the eps shift is 1e-10 relative)."""
    A, b, W, Gh, G = floating_cell
    y = sg.targets(Gh, G)
    assert len(y) == 2 * 3 * (56 * 57 // 2)
    rGh, rG = sg.reconstruct(y, 56, 4)
    for k in range(3):
        assert np.linalg.norm(rGh[k] - Gh[k + 1]) / np.linalg.norm(Gh[k + 1]) < 1e-9
        assert np.linalg.norm(rG[k] - G[k + 1]) / np.linalg.norm(G[k + 1]) < 1e-9


def test_tf_mismatch_accepts_lanczos_and_rejects_perturbed(floating_cell):
    """The plain ROM matches the exact cell transfer function on the Laplace
    axis far below 1e-3; a 1% error in a deep block is caught."""
    A, b, W, Gh, G = floating_cell
    wmax = 0.444
    assert sg.tf_mismatch(A, b, W, Gh, G, wmax) < 1e-7
    G2 = [g.copy() for g in G]
    G2[1] = 1.01 * G2[1]
    assert sg.tf_mismatch(A, b, W, Gh, G2, wmax) > 1e-3


def test_adam_constant_gradient_and_scale_invariance():
    """Invariants of the moment recurrences beyond the first step: for a
    constant gradient the bias-corrected moments equal g and g^2 at every
    step, so every step moves by -lr g / (|g| + eps); and scaling all
    gradients by c > 0 leaves the steps unchanged (eps negligible). A
    dropped decay term, a wrong bias-correction power or a missing square
    root fails one of these from step 2 on."""
    rng = np.random.default_rng(5)
    th = rng.normal(size=7)
    g = rng.normal(size=7)
    st = (np.zeros(7), np.zeros(7), 0)
    cur = th.copy()
    for t in range(1, 11):
        nxt, st = sg.adam_step(cur, g, st, 1e-2)
        assert np.allclose(nxt - cur, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-16), t
        cur = nxt
    gs = [rng.normal(size=7) for _ in range(6)]
    a, sa = th.copy(), (np.zeros(7), np.zeros(7), 0)
    c, sc = th.copy(), (np.zeros(7), np.zeros(7), 0)
    for gk in gs:
        a, sa = sg.adam_step(a, gk, sa, 1e-3, eps=1e-30)
        c, sc = sg.adam_step(c, 1e4 * gk, sc, 1e-3, eps=1e-30)
    assert np.allclose(a, c, rtol=0, atol=1e-13)
    # a sign flip of the gradient at step 2 partly cancels the first moment:
    # m_2 = 0.9 * 0.1 g - 0.1 g = -0.01 g, v_2 = 0.001999 g^2 (bias factors 0.19, 0.001999)
    th0 = np.array([0.0]); s2 = (np.zeros(1), np.zeros(1), 0)
    th1, s2 = sg.adam_step(th0, np.array([2.0]), s2, 1.0, eps=0.0)
    th2, s2 = sg.adam_step(th1, np.array([-2.0]), s2, 1.0, eps=0.0)
    mh = -0.01 * 2.0 / (1 - 0.9 ** 2)
    vh = (0.999 * 0.001 * 4.0 + 0.001 * 4.0) / (1 - 0.999 ** 2)
    assert abs((th2 - th1)[0] - (-mh / np.sqrt(vh))) < 1e-12


def test_reconstruct_layout_by_hand():
    """b = 2, m = 3: the factor vector is [L(Ghat^2), L(G^2), L(Ghat^3),
    L(G^3)], each the row-major lower triangle (l11, l21, l22); the blocks
    are L L^T plus the relative shift, written out by hand here."""
    y = np.array([1.0, 2.0, 3.0,   4.0, 0.5, 1.0,   2.0, -1.0, 1.0,   3.0, 0.0, 2.0])
    Gh, G = sg.reconstruct(y, 2, 3)
    hand = [np.array([[1.0, 2.0], [2.0, 13.0]]), np.array([[16.0, 2.0], [2.0, 1.25]]),
            np.array([[4.0, -2.0], [-2.0, 2.0]]), np.array([[9.0, 0.0], [0.0, 4.0]])]
    got = [Gh[0], G[0], Gh[1], G[1]]
    for M, H in zip(got, hand):
        shift = M - H
        assert np.allclose(shift, shift[0, 0] * np.eye(2), atol=1e-15)
        assert 0.0 <= shift[0, 0] <= 1e-9 * np.trace(H)
