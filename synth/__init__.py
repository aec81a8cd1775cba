"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds only input generation: voxel media, grid geometry,
source/receiver locations, the source wavelet and random test matrices.
It contains none of the reduced-order method's arithmetic (no operator
assembly, splitting, Krylov, Lanczos or time stepping), so importing it
from both the CPU oracle and the GPU path shares no method code.

Workload shapes follow the paper's numerical section (Sec. 9): 3D acoustic
media on a Cartesian grid with Dirichlet walls, split into cubic coarse
cells, point sources and receivers on the partition skeleton (Sec. 2,
eq. gsupport), and a band-limited wavelet (Sec. 1).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "gaussian_field", "acoustic_medium", "layered_medium", "ricker",
    "Workload", "workload", "face_interior_nodes", "random_spd",
]


# --------------------------------------------------------------------------
# media
# --------------------------------------------------------------------------

def gaussian_field(shape: Tuple[int, ...], ell: float, rng: np.random.Generator,
                   uniform: bool = False) -> np.ndarray:
    """Smooth random field on a periodic voxel grid, min-max scaled to [0, 1].

    White noise (standard normal, or U[0,1] when ``uniform``) is filtered in
    Fourier space by exp(-2 pi^2 ell^2 |k|^2) (k in cycles per voxel), i.e. a
    Gaussian kernel with standard deviation ``ell`` voxels.
    """
    noise = rng.random(shape) if uniform else rng.standard_normal(shape)
    spec = np.fft.fftn(noise)
    k2 = np.zeros(shape)
    for ax, n in enumerate(shape):
        k = np.fft.fftfreq(n)
        sh = [1] * len(shape)
        sh[ax] = n
        k2 = k2 + (k.reshape(sh)) ** 2
    f = np.real(np.fft.ifftn(spec * np.exp(-2.0 * np.pi ** 2 * ell ** 2 * k2)))
    lo, hi = f.min(), f.max()
    return (f - lo) / (hi - lo) if hi > lo else np.zeros(shape)


def acoustic_medium(nvox: Tuple[int, int, int], seed: int,
                    sigma_range=(1.0, 4.0), rho_range=(1.0, 2.0),
                    ell_sigma: float = 6.0, ell_rho: float = 2.0):
    """Per-voxel stiffness sigma and density rho, arrays indexed [x, y, z].

    sigma = lo * (hi/lo)^f with f a smooth Gaussian field (log-uniform range,
    the exponential of a smooth field); rho = lo + (hi-lo) * smooth(U[0,1]).
    sigma is drawn before rho from one PCG64 stream seeded with ``seed``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    f = gaussian_field(tuple(nvox), ell_sigma, rng)
    s0, s1 = sigma_range
    sigma = s0 * (s1 / s0) ** f
    r = gaussian_field(tuple(nvox), ell_rho, rng, uniform=True)
    r0, r1 = rho_range
    rho = r0 + (r1 - r0) * r
    return np.ascontiguousarray(sigma), np.ascontiguousarray(rho)


def layered_medium(nvox: Tuple[int, int, int], seed: int,
                   z_bounds: Sequence[int], contrast: float = 3.0,
                   perturb: float = 0.10, ell: float = 6.0):
    """Horizontally layered medium with a smooth multiplicative perturbation.

    Layer j gets sigma = contrast^(j/(L-1)) in a seeded order, rho ~ U[1,2]
    per layer; both are multiplied by (1 + perturb * (2 f - 1)) with f a
    smooth field of correlation length ``ell``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nz = nvox[2]
    edges = [0] + list(z_bounds) + [nz]
    L = len(edges) - 1
    order = rng.permutation(L)
    sig_layer = contrast ** (order / max(L - 1, 1))
    rho_layer = 1.0 + rng.random(L)
    sigma = np.empty(nvox)
    rho = np.empty(nvox)
    for j in range(L):
        sigma[:, :, edges[j]:edges[j + 1]] = sig_layer[j]
        rho[:, :, edges[j]:edges[j + 1]] = rho_layer[j]
    f1 = gaussian_field(tuple(nvox), ell, rng)
    f2 = gaussian_field(tuple(nvox), ell, rng)
    sigma *= 1.0 + perturb * (2.0 * f1 - 1.0)
    rho *= 1.0 + perturb * (2.0 * f2 - 1.0)
    return np.ascontiguousarray(sigma), np.ascontiguousarray(rho)


def vti_voigt21(lam, mu, eps, delta):
    """Upper triangle (21 values, row by row) of the 6 x 6 Voigt stiffness of
    a vertically transversely isotropic medium from lambda, mu and Thomsen's
    epsilon, delta (vertical axis z): C33 = lambda + 2 mu, C44 = C55 = C66 =
    mu, C11 = C22 = C33 (1 + 2 eps), C12 = C11 - 2 C66,
    C13 = C23 = sqrt((C33 - C44)(C33 (1 + 2 delta) - C44)) - C44."""
    lam, mu, eps, delta = (np.asarray(v, np.float64) for v in (lam, mu, eps, delta))
    C33 = lam + 2.0 * mu
    C44 = mu
    C11 = C33 * (1.0 + 2.0 * eps)
    C12 = C11 - 2.0 * C44
    C13 = np.sqrt((C33 - C44) * (C33 * (1.0 + 2.0 * delta) - C44)) - C44
    z = np.zeros_like(C33)
    rows = [[C11, C12, C13, z, z, z], [C11, C13, z, z, z], [C33, z, z, z], [C44, z, z], [C44, z], [C44]]
    return np.stack([v for r in rows for v in r], axis=-1)


def elastic_layered_medium(nvox: Tuple[int, int, int], seed: int, z_bounds: Sequence[int],
                           contrast: float = 3.0, aniso: float = 0.2):
    """Layered VTI medium (piecewise-constant phases): layer j gets mu and
    lambda scaled by contrast^(j/(L-1)) in a seeded order (lambda = 2 mu),
    Thomsen epsilon, delta ~ U[0, aniso] and rho = 1. Returns the per-voxel
    21 Voigt entries (nx, ny, nz, 21) and rho (nx, ny, nz)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nz = nvox[2]
    edges = [0] + list(z_bounds) + [nz]
    L = len(edges) - 1
    order = rng.permutation(L)
    mu = contrast ** (order / max(L - 1, 1))
    eps = aniso * rng.random(L)
    dl = aniso * rng.random(L)
    c21 = np.empty(tuple(nvox) + (21,))
    for j in range(L):
        c21[:, :, edges[j]:edges[j + 1]] = vti_voigt21(2.0 * mu[j], mu[j], eps[j], dl[j])
    return np.ascontiguousarray(c21), np.ones(nvox)


# --------------------------------------------------------------------------
# wavelet
# --------------------------------------------------------------------------

def ricker(n_steps: int, dt: float, f_p: float) -> np.ndarray:
    """Ricker wavelet samples w[n] = w(n dt), n = 0..n_steps-1.

    w(t) = (1 - 2 pi^2 f_p^2 tau^2) exp(-pi^2 f_p^2 tau^2), tau = t - t0,
    t0 = 1.5 / f_p, and w = 0 exactly for t > 2 t0 (so energy tests see a
    source-free tail).
    """
    t = np.arange(n_steps, dtype=np.float64) * dt
    t0 = 1.5 / f_p
    tau = t - t0
    a = (np.pi * f_p * tau) ** 2
    w = (1.0 - 2.0 * a) * np.exp(-a)
    w[t > 2.0 * t0] = 0.0
    return w


# --------------------------------------------------------------------------
# geometry helpers (plain coordinate logic)
# --------------------------------------------------------------------------

def face_interior_nodes(nvox, cuts) -> np.ndarray:
    """All grid nodes (x, y, z) strictly inside the domain that lie on exactly
    one interior cut plane. Returns an (n, 3) int64 array in x-fastest order."""
    out = []
    cutsets = [set(int(c) for c in cuts[a]) for a in range(3)]
    nx, ny, nz = nvox
    for z in range(1, nz):
        for y in range(1, ny):
            for x in range(1, nx):
                k = (x in cutsets[0]) + (y in cutsets[1]) + (z in cutsets[2])
                if k == 1:
                    out.append((x, y, z))
    return np.array(out, dtype=np.int64).reshape(-1, 3)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    """One synthetic workload: medium, partition geometry, ROM sizes,
    sources, receivers and time stepping parameters."""
    name: str
    nvox: Tuple[int, int, int]
    sigma: np.ndarray
    rho: np.ndarray
    cuts: Tuple[np.ndarray, np.ndarray, np.ndarray]   # interior cut planes per axis
    m: int                                           # S-fraction layers (Krylov blocks)
    modes_face: int
    modes_edge: int
    sources: np.ndarray                              # (n_s, 3) node coords
    receivers: np.ndarray                            # (n_r, 3) node coords
    n_steps: int
    f_p: float                                       # Ricker peak frequency
    omega_max: float                                 # band edge 2 pi f_max
    shift: float                                     # Krylov shift s < 0
    cfl_fraction: float = 0.5
    seed: int = 0
    extra: dict = field(default_factory=dict)


def _band(c_min: float, ppw: float = 10.0):
    """Ricker peak frequency for ``ppw`` points per shortest wavelength on a
    unit grid: f_max = 2.5 f_p and c_min / f_max = ppw."""
    f_max = c_min / ppw
    f_p = f_max / 2.5
    omega_max = 2.0 * np.pi * f_max
    return f_p, omega_max


def workload(name: str, *, modes_face: Optional[int] = None, modes_edge: Optional[int] = None,
             m: Optional[int] = None, n_steps: Optional[int] = None,
             n_sources: Optional[int] = None, n_receivers: Optional[int] = None,
             realisation: int = 0, ppw: float = 10.0, cell: Optional[int] = None,
             ncell: Optional[int] = None) -> Workload:
    """Build a named workload.

    ``tiny``   : 16^3 voxels, 2^3 cells of 8^3 (fast CPU tests)
    ``cube3``  : 24^3 voxels, 3^3 cells of 8^3 (one interior cell), seeded
                 face-interior sources and receivers
    ``small``  : 32^3 voxels, 4^3 cells of 8^3, one source, 64 receivers,
                 1500 steps (the FP64 case)
    ``medium`` : 64^3 voxels, 8^3 cells, 16 sources (parity case that spans
                 many cells but stays within seconds for the oracle)
    ``large``  : 128^3 voxels, 16^3 cells of 8^3, 64 sources on an 8x8 grid,
                 1024 receivers, 4000 steps (the batched FP32 case)
    ``layered``: 256x256x128 voxels, 6 layers of contrast 3:1 with a +-10%
                 smooth perturbation, non-uniform cells of 8..16 voxels aligned
                 to the layers, per-cell layer count 3..8 from the cell size
                 (``extra['m_per_cell']``), face modes 4/6/8 by face area
                 (``extra['face_rules']``), 256 sources, 6000 steps
    ``layered_small``: the same recipe on 64x64x32 voxels (parity case)
    ``paper``  : ``ncell``^3 (default 4^3) cubic cells of ``cell`` voxels
                 (default 40) at ``ppw`` points per wavelength (default: one
                 wavelength per cell), 64 sources, 32 x 32 receivers (the
                 paper's example shape)
    """
    extra_cell = cell
    mf = 9 if modes_face is None else modes_face
    me = 2 if modes_edge is None else modes_edge
    c_min = np.sqrt(1.0 / 2.0)        # sqrt(sigma_lo / rho_hi) of the generator bounds
    f_p, omega_max = _band(c_min, ppw)
    shift = -omega_max ** 2 / 10.0
    if name == "tiny":
        nvox = (16, 16, 16)
        seed = 9001 + realisation
        sigma, rho = acoustic_medium(nvox, seed)
        cuts = tuple(np.array([8]) for _ in range(3))
        src = np.array([[5, 3, 8]], dtype=np.int64)
        rec_all = face_interior_nodes(nvox, cuts)
        rng = np.random.Generator(np.random.PCG64(seed + 100))
        nr = 16 if n_receivers is None else n_receivers
        rec = rec_all[np.sort(rng.choice(len(rec_all), size=nr, replace=False))]
        return Workload(name, nvox, sigma, rho, cuts, m or 3, mf, me, src, rec,
                        n_steps or 400, f_p, omega_max, shift, seed=seed)
    if name == "cube3":
        # 24^3 voxels, 3^3 cells of 8^3: the centre cell is interior (the
        # boundary dimension of the 128^3 workload's interior cells) while
        # the oracle stays within seconds; sources and receivers are seeded
        # picks among face-interior nodes
        nvox = (24, 24, 24)
        seed = 6001 + realisation
        sigma, rho = acoustic_medium(nvox, seed)
        cuts = tuple(np.array([8, 16]) for _ in range(3))
        fi = face_interior_nodes(nvox, cuts)
        rng = np.random.Generator(np.random.PCG64(seed + 100))
        ns = 64 if n_sources is None else n_sources
        nr = 48 if n_receivers is None else n_receivers
        src = fi[np.sort(rng.choice(len(fi), size=ns, replace=False))]
        rec = fi[np.sort(rng.choice(len(fi), size=nr, replace=False))]
        return Workload(name, nvox, sigma, rho, cuts, m or 4, mf, me, src, rec,
                        n_steps or 300, f_p, omega_max, shift, seed=seed)
    if name == "small":
        nvox = (32, 32, 32)
        seed = 1001 + realisation
        sigma, rho = acoustic_medium(nvox, seed)
        cuts = tuple(np.array([8, 16, 24]) for _ in range(3))
        src = np.array([[20, 20, 16]], dtype=np.int64)
        rec_all = face_interior_nodes(nvox, cuts)
        rng = np.random.Generator(np.random.PCG64(1101 + realisation))
        nr = 64 if n_receivers is None else n_receivers
        rec = rec_all[np.sort(rng.choice(len(rec_all), size=nr, replace=False))]
        return Workload(name, nvox, sigma, rho, cuts, m or 4, mf, me, src, rec,
                        n_steps or 1500, f_p, omega_max, shift, seed=seed)
    if name == "medium":
        nvox = (64, 64, 64)
        seed = 3001 + realisation
        sigma, rho = acoustic_medium(nvox, seed)
        cuts = tuple(np.arange(8, 64, 8) for _ in range(3))
        a = np.arange(4)
        src = np.array([[12 + 16 * i, 12 + 16 * j, 56] for j in a for i in a], dtype=np.int64)
        if n_sources is not None:
            src = src[:n_sources]
        b = np.arange(16)
        rec = np.array([[2 + 4 * i, 2 + 4 * j, 56] for j in b for i in b], dtype=np.int64)
        return Workload(name, nvox, sigma, rho, cuts, m or 4, mf, me, src, rec,
                        n_steps or 600, f_p, omega_max, shift, seed=seed)
    if name == "large":
        nvox = (128, 128, 128)
        seed = 2001 + realisation
        sigma, rho = acoustic_medium(nvox, seed)
        cuts = tuple(np.arange(8, 128, 8) for _ in range(3))
        a = np.arange(8)
        src = np.array([[12 + 16 * i, 12 + 16 * j, 120] for j in a for i in a], dtype=np.int64)
        if n_sources is not None:
            src = src[:n_sources]
        b = np.arange(32)
        rec = np.array([[2 + 4 * i, 2 + 4 * j, 120] for j in b for i in b], dtype=np.int64)
        return Workload(name, nvox, sigma, rho, cuts, m or 4, mf, me, src, rec,
                        n_steps or 4000, f_p, omega_max, shift, seed=seed)
    if name in ("layered", "layered_small"):
        # layered medium, non-uniform cells of 8..16 voxels aligned to the
        # layers, per-cell layer count from the cell size (uneven (m, b))
        if name == "layered":
            nvox = (256, 256, 128)
            nsrc_side, nrec_side, steps = 16, 32, 6000
        else:
            nvox = (64, 64, 32)
            nsrc_side, nrec_side, steps = 4, 8, 600
        seed = 4001 + realisation
        rng = np.random.Generator(np.random.PCG64(seed + 50))
        nz = nvox[2]
        nl = 6 if nz >= 96 else 3
        zb = [int(round(nz * j / nl)) for j in range(1, nl)]
        sigma, rho = layered_medium(nvox, seed, zb, contrast=3.0)

        def segments(total):
            cuts, pos = [], 0
            while total - pos > 16:
                step = int(rng.integers(8, 17))
                if total - pos - step < 8:
                    step = total - pos - 8
                pos += step
                cuts.append(pos)
            return np.array(cuts, dtype=np.int64)

        zcuts = []
        for lo, hi in zip([0] + zb, zb + [nz]):
            zcuts.append((lo + hi) // 2)
            if hi < nz:
                zcuts.append(hi)
        cuts = (segments(nvox[0]), segments(nvox[1]), np.array(sorted(zcuts), dtype=np.int64))
        plane = int(cuts[2][-1])                       # first interface below the top wall

        def off_cut(v, c):
            while v in set(int(x) for x in c) or v <= 0:
                v += 1
            return v

        xs = [off_cut(int(v), cuts[0]) for v in np.linspace(4, nvox[0] - 5, nsrc_side).astype(int)]
        ys = [off_cut(int(v), cuts[1]) for v in np.linspace(4, nvox[1] - 5, nsrc_side).astype(int)]
        src = np.array([[x, y, plane] for y in ys for x in xs], dtype=np.int64)
        if n_sources is not None:
            src = src[:n_sources]
        xr = [off_cut(int(v), cuts[0]) for v in np.linspace(2, nvox[0] - 3, nrec_side).astype(int)]
        yr = [off_cut(int(v), cuts[1]) for v in np.linspace(2, nvox[1] - 3, nrec_side).astype(int)]
        rec = np.array([[x, y, plane] for y in yr for x in xr], dtype=np.int64)
        c_min = np.sqrt(0.9 / 2.2)                      # generator bounds of sigma and rho
        f_p, omega_max = _band(c_min, ppw)
        wl = Workload(name, nvox, sigma, rho, cuts, m or 3, mf, me, src, rec,
                      n_steps or steps, f_p, omega_max, -omega_max ** 2 / 10.0, seed=seed)
        # layers per cell grow with the cell size: 3 at 8 voxels, 8 at 16
        edges = [np.diff(np.concatenate([[0], c, [n]])) for c, n in zip(cuts, nvox)]
        mpc = []
        for ez in edges[2]:
            for ey in edges[1]:
                for ex in edges[0]:
                    v13 = (ex * ey * ez) ** (1.0 / 3.0)
                    mpc.append(int(np.clip(round(3 + 5 * (v13 - 8) / 8), 3, 8)))
        wl.extra["m_per_cell"] = np.array(mpc, dtype=np.int32)
        if name == "layered":
            # face modes by face area in voxels: <= 100 -> 4, <= 169 -> 6, else 8
            wl.extra["face_rules"] = ([100, 169, 2 ** 31 - 1], [4, 6, 8])
        return wl
    if name in ("elastic", "elastic_tiny"):
        # layered VTI elastic medium (three piecewise-constant phases, shear
        # modulus contrast 3:1, lambda = 2 mu, Thomsen eps, delta <= 0.2,
        # rho = 1), cells of 8^3 voxels, vertical point forces on a grid of
        # face-interior nodes of the first interior z-interface, receivers on
        # a denser grid of the same plane; the unknown of node k's component
        # c is 3 k + c
        if name == "elastic":
            nvox, zb, nsx, nsy, nrx, nry, steps = (96, 96, 96), [32, 64], 8, 4, 32, 16, 3000
        else:
            nvox, zb, nsx, nsy, nrx, nry, steps = (16, 16, 16), [5, 11], 2, 1, 4, 3, 400
        seed = 9101 + realisation
        c21, rho = elastic_layered_medium(nvox, seed, zb)
        cuts = tuple(np.arange(8, n, 8) for n in nvox)
        plane = 8

        def grid(k, n, lo):
            v = [int(round(lo + (n - 2 * lo) * (i + 0.5) / k)) for i in range(k)]
            return [x + 1 if x % 8 == 0 else x for x in v]

        src = np.array([[x, y, plane] for y in grid(nsy, nvox[1], 2) for x in grid(nsx, nvox[0], 2)], dtype=np.int64)
        rec = np.array([[x, y, plane] for y in grid(nry, nvox[1], 1) for x in grid(nrx, nvox[0], 1)], dtype=np.int64)
        c_s = 1.0                       # slowest shear speed of the generator (mu >= 1, rho = 1)
        f_p2, om2 = _band(c_s, ppw)
        wl = Workload(name, nvox, None, rho, cuts, m or 4, mf if modes_face is not None else 4, me, src, rec,
                      n_steps or steps, f_p2, om2, -om2 ** 2 / 10.0, seed=seed)
        wl.extra["c21"] = c21
        wl.extra["source_component"] = 2
        return wl
    if name == "paper":
        # the shape of the paper's acoustic examples (Sec. 9): a fine grid far
        # finer than the wavelength (``ppw`` points per shortest wavelength,
        # 40 in the paper) split into 4^3 cubic cells of ``cell`` voxels (40 in
        # the paper), i.e. about one wavelength per cell at the band edge. The
        # medium is the acoustic generator with its correlation lengths scaled
        # with the wavelength (6 and 2 voxels at 10 points per wavelength), so
        # the medium per wavelength matches the 8^3-cell workloads. 64 sources
        # on an 8 x 8 grid on the first interior z-interface below the top
        # wall and 32 x 32 receivers on the first one above the bottom wall
        # (the paper's examples place source and receiver apart), at
        # coordinates off the cut planes.
        L = int(extra_cell or 40)
        ppw_p = float(ppw if ppw != 10.0 else L)
        nc = int(ncell or 4)
        nvox = (nc * L,) * 3
        seed = 7001 + realisation
        sc = ppw_p / 10.0
        sigma, rho = acoustic_medium(nvox, seed, ell_sigma=6.0 * sc, ell_rho=2.0 * sc)
        cuts = tuple(np.arange(L, nc * L, L) for _ in range(3))
        plane = (nc - 1) * L
        n = nc * L

        def grid(k, lo):
            step = (n - 2 * lo) / (k - 1)
            v = [int(round(lo + step * i)) for i in range(k)]
            return [x + 1 if x % L == 0 else x for x in v]

        src = np.array([[x, y, plane] for y in grid(8, L // 4) for x in grid(8, L // 4)], dtype=np.int64)
        if n_sources is not None:
            src = src[:n_sources]
        nrs = 32 if n_receivers is None else n_receivers
        rec = np.array([[x, y, L] for y in grid(nrs, 2) for x in grid(nrs, 2)], dtype=np.int64)
        f_p2, om2 = _band(np.sqrt(1.0 / 2.0), ppw_p)
        return Workload(name, nvox, sigma, rho, cuts, m or 4, mf, me, src, rec,
                        n_steps or 4000, f_p2, om2, -om2 ** 2 / 10.0, seed=seed,
                        extra={"cell": L, "ppw": ppw_p})
    raise ValueError(f"unknown workload {name!r}")


# --------------------------------------------------------------------------
# random test matrices
# --------------------------------------------------------------------------

def random_spd(n: int, rng: np.random.Generator, cond: float = 10.0, scale: float = 1.0) -> np.ndarray:
    """Random symmetric positive definite n x n matrix with eigenvalues
    log-spaced in [scale/cond, scale]."""
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = scale * np.logspace(-np.log10(cond), 0.0, n)
    m = (q * ev) @ q.T
    return 0.5 * (m + m.T)


# --------------------------------------------------------------------------
# unstructured input pencil
# --------------------------------------------------------------------------

def geometric_graph(n: int, k: int, seed: int):
    """A synthetic unstructured-mesh pencil (the input of a general
    partition, standing in for a non-Cartesian discretisation): n seeded
    points in the unit cube, each joined to its k nearest neighbours
    (symmetrised), edge weight 1 / |x_i - x_j|^2 scaled to mean 1; A = minus
    the weighted graph Laplacian minus a sink of 0.2 on nodes within 0.08 of
    the cube's faces (so A < 0, diagonally dominant); b = 0.8 + 0.4 u,
    u uniform. Returns (A as scipy CSR with sorted columns, b, points)."""
    import scipy.sparse as sp
    from scipy.spatial import cKDTree
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.random((n, 3))
    _, nb = cKDTree(x).query(x, k + 1)
    rows = np.repeat(np.arange(n), k)
    cols = nb[:, 1:].ravel()
    W = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n)).tocsr()
    W = ((W + W.T) > 0).astype(float).tocoo()
    d2 = np.sum((x[W.row] - x[W.col]) ** 2, axis=1)
    w = 1.0 / d2
    w /= w.mean()
    W = sp.csr_matrix((w, (W.row, W.col)), shape=(n, n))
    near = np.any((x < 0.08) | (x > 0.92), axis=1)
    diag = -np.asarray(W.sum(axis=1)).ravel() - 0.2 * near
    A = (W + sp.diags(diag)).tocsr()
    A.sort_indices()
    b = 0.8 + 0.4 * rng.random(n)
    return A, b, x
