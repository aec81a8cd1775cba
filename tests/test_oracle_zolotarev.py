"""Pins of the Zolotarev route to the spectral projector of eq. trgrstep
(oracle/zolotarev.py), against facts that do not come from the code under
test:

* the complete elliptic integral and the Jacobi elliptic functions from the
  arithmetic-geometric mean equal scipy's (library routines);
* Zolotarev's approximant is odd, its error on [delta, 1] equals the
  asymptotic optimal error 4 exp(-pi^2 n / log(4 / delta)) to within 2%,
  and it equioscillates (at least 2n interior extrema of equal size);
* the projector's Gramian differs from the eigen-sum Gramian of eq. trgr by
  at most (eps / 2) max_k 1/b_k in the 2-norm when no eigenvalue lies in the
  transition band (eps the approximant's maximal error: the projector is
  B^{-1/2} (I + sign) / 2 B^{-1/2}), and the difference shrinks as poles are
  added.
"""
import numpy as np
import pytest
import scipy.special as ss
import scipy.sparse as sp

import synth
from oracle import fine
from oracle import gramian as gr
from oracle import zolotarev as z


@pytest.mark.parametrize("k", [0.1, 0.5, 0.9, 0.999, 1 - 1e-9])
def test_elliptic_functions_match_scipy(k):
    assert abs(z.agm_ellipk(k) - ss.ellipk(k * k)) <= 1e-13 * ss.ellipk(k * k)
    for u in (0.05, 0.7, 1.5, 2.5):
        sn, cn, dn = z.jacobi_sn_cn_dn(u, k)
        ref = ss.ellipj(u, k * k)
        assert max(abs(sn - ref[0]), abs(cn - ref[1]), abs(dn - ref[2])) <= 1e-13


@pytest.mark.parametrize("n,delta", [(4, 0.1), (8, 0.01), (12, 1e-3)])
def test_zolotarev_sign_is_optimal(n, delta):
    M, beta2, a = z.zolotarev_sign(n, delta)
    x = np.geomspace(delta, 1.0, 200001)
    f = z.eval_sign(x, M, beta2, a)
    assert np.allclose(z.eval_sign(-x, M, beta2, a), -f, rtol=0, atol=1e-15)
    err = f - 1.0
    emax = np.abs(err).max()
    bound = 4.0 * np.exp(-np.pi ** 2 * n / np.log(4.0 / delta))
    assert abs(emax / bound - 1.0) <= 0.02, (emax, bound)
    # equal ripple: every interior local extremum of the error has size ~emax
    inner = np.where((np.abs(err[1:-1]) >= np.abs(err[:-2])) & (np.abs(err[1:-1]) >= np.abs(err[2:])))[0] + 1
    peaks = np.abs(err[inner])
    assert len(peaks) >= 2 * n - 1
    assert peaks.min() >= 0.99 * emax


def _pencil():
    sig, rho = synth.acoustic_medium((10, 10, 10), 3, ell_sigma=4.0, ell_rho=2.0)
    A, b = fine.assemble_acoustic(sig, rho)
    return sp.csr_matrix(A), b


def test_projector_gramian_within_the_approximation_bound():
    A, b = _pencil()
    r = 1.0 / np.sqrt(b)
    C = (r[:, None] * (-A.toarray())) * r[None, :]
    lam = np.linalg.eigvalsh(0.5 * (C + C.T))
    # omega^2 in the middle of the widest gap among the lowest 30 eigenvalues
    gaps = np.diff(lam[:30])
    i = int(np.argmax(gaps))
    w2 = 0.5 * (lam[i] + lam[i + 1])
    gap = 0.5 * gaps[i] / w2
    rows = np.arange(0, 120)
    Gex = gr.exact_gramian(A, b, rows, np.sqrt(w2))
    s = max(w2, z.gershgorin_hi(A, b) - w2)
    prev = None
    for n in (6, 10, 14):
        gamma = 0.9 * gap
        Gz = z.rational_gramian(A, b, rows, np.sqrt(w2), n, gamma)
        delta = min(gamma * w2 / s, 0.5)
        M, beta2, a = z.zolotarev_sign(n, delta)
        xg = np.geomspace(delta, 1.0, 200001)
        eps = np.abs(z.eval_sign(xg, M, beta2, a) - 1.0).max()
        d = np.linalg.norm(Gz - Gex, 2)
        assert d <= 0.5 * eps * (1.0 / b[rows]).max() * (1 + 1e-6) + 1e-12, (n, d, eps)
        if prev is not None:
            assert d < prev
        prev = d
