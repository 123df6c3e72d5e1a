"""Seeded synthetic inputs shared by the tests, the smoke check and bench.py.

This module holds input generation only: coefficient fields and point sets
with the shapes and structure of the paper's workloads.  It contains none of
the evaluation arithmetic (no window, no oversampled grid, no trigonometric
sum) and imports neither the oracle nor the HIP library.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).

Workloads (coefficients are C-order (N0, N1, N2), index i <-> frequency
i - N/2; points are (M, 3) in the unit box [-1/2, 1/2)^3):

* ``smooth_coeffs``   -- complex Gaussian * exp(-|k|^2/200): the small FP64 case.
* ``powerlaw_coeffs`` -- |k|^-2 spectral decay with random phase: the
  turbulence-like spectrum of a quantum-vortex field (Sec. 3, Sec. 5).
* ``vortex_pair_field`` -- a field sampled on the periodic box made of two
  antiparallel straight vortex lines, psi = prod tanh(r/sqrt 2) e^{+-i theta}
  (the single-vortex profile and product initial condition of Sec. 3 with the
  tanh approximation of the core), turned into coefficients by the FFT of
  Sec. 2 (psihat = fftshift(fftn(psi)) up to normalisation and the sign rule
  that maps the box to [-1/2, 1/2)).  The paper's own field comes from a GPE
  run with the Pade core profile; neither is reproducible here, so this
  stands in for it.
* ``uniform_points``, ``clustered_points`` -- uniform and Gaussian-cluster
  point sets (the vortex-core clustering of Sec. 5 is strongly localised).
* ``subbox_grid_points`` -- a fine regular grid in a small sub-box around the
  closest approach of the two lines (the localised high-resolution
  evaluation of Sec. 5).
* ``gpe_two_vortices`` -- the initial state of the reconnection run of Sec. 5
  (two straight vortices with a tanh core) on its 80^3 grid.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def _freq_grid(N):
    ks = [np.arange(n) - n // 2 for n in N]
    return np.meshgrid(*ks, indexing="ij")


def smooth_coeffs(N, seed: int) -> np.ndarray:
    """fhat_k = (a + i b) exp(-|k|^2 / 200), a, b ~ N(0, 1)."""
    N = tuple(int(v) for v in N)
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(N)
    b = rng.standard_normal(N)
    k0, k1, k2 = _freq_grid(N)
    env = np.exp(-(k0.astype(np.float64) ** 2 + k1 ** 2 + k2 ** 2) / 200.0)
    return (a + 1j * b) * env


def powerlaw_coeffs(N, seed: int) -> np.ndarray:
    """fhat_k = max(|k|, 1)^-2 exp(i theta_k), theta ~ U[0, 2 pi)."""
    N = tuple(int(v) for v in N)
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, 2.0 * math.pi, size=N)
    k0, k1, k2 = _freq_grid(N)
    kk = np.sqrt(k0.astype(np.float64) ** 2 + k1 ** 2 + k2 ** 2)
    amp = 1.0 / np.maximum(kk, 1.0) ** 2
    out = np.empty(N, dtype=np.complex128)
    out.real = amp * np.cos(theta)
    out.imag = amp * np.sin(theta)
    return out


def wrap(x: np.ndarray) -> np.ndarray:
    """Periodic wrap into [-1/2, 1/2)."""
    return x - np.floor(x + 0.5)


def uniform_points(M: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-0.5, 0.5, size=(int(M), 3))


def clustered_points(M: int, n_clusters: int, width: float, seed_centres: int,
                     seed_offsets: int) -> np.ndarray:
    """M points in ``n_clusters`` isotropic Gaussian clusters of std ``width``
    (per axis), centres uniform in the box, wrapped periodically."""
    rc = np.random.default_rng(seed_centres)
    centres = rc.uniform(-0.5, 0.5, size=(n_clusters, 3))
    ro = np.random.default_rng(seed_offsets)
    which = ro.integers(0, n_clusters, size=int(M))
    pts = centres[which] + width * ro.standard_normal((int(M), 3))
    return wrap(pts)


def mixed_points(M: int, n_clusters: int, width: float, seeds) -> np.ndarray:
    """Half uniform, half clustered, shuffled.  ``seeds`` = (uniform, centres,
    offsets, shuffle)."""
    Mu = int(M) // 2
    Mc = int(M) - Mu
    pu = uniform_points(Mu, seeds[0])
    pc = clustered_points(Mc, n_clusters, width, seeds[1], seeds[2])
    pts = np.concatenate([pu, pc], axis=0)
    perm = np.random.default_rng(seeds[3]).permutation(pts.shape[0])
    return np.ascontiguousarray(pts[perm])


def sample_indices(M: int, count: int, seed: int) -> np.ndarray:
    """``count`` distinct indices in [0, M), sorted."""
    count = min(int(count), int(M))
    return np.sort(np.random.default_rng(seed).choice(int(M), size=count, replace=False))


# ---------------------------------------------------------------------------
# Vortex-pair field (GPE-like)
# ---------------------------------------------------------------------------

@dataclass
class VortexPair:
    N: int                       # coarse grid / coefficient count per axis
    L: float                     # physical box side
    points: np.ndarray           # two points on the lines (physical units)
    dirs: np.ndarray             # unit direction vectors
    signs: tuple = (1, -1)       # circulation signs (antiparallel pair)
    midpoint_unit: np.ndarray = field(default=None)


def _rotation(ax: float, ay: float) -> np.ndarray:
    cx, sx, cy, sy = math.cos(ax), math.sin(ax), math.cos(ay), math.sin(ay)
    rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    return ry @ rx


def vortex_pair(N: int = 128, L: float = 64.0, seed: int = 201) -> VortexPair:
    """Two antiparallel lines along axis 0 (coordinates are (x0, x1, x2) in array
    axis order) through (., +-2, 0) with offsets U(-1/2, 1/2)^3 and tilts
    U(-10, 10) degrees."""
    rng = np.random.default_rng(seed)
    base = np.array([[0.0, 2.0, 0.0], [0.0, -2.0, 0.0]])
    pts = base + rng.uniform(-0.5, 0.5, size=(2, 3))
    tilt = np.deg2rad(rng.uniform(-10.0, 10.0, size=(2, 2)))
    dirs = np.stack([_rotation(tilt[i, 0], tilt[i, 1]) @ np.array([1.0, 0.0, 0.0]) for i in range(2)])
    # closest approach of the two (skew) lines
    p, q, u, v = pts[0], pts[1], dirs[0], dirs[1]
    w0 = p - q
    a, b, c, d, e = u @ u, u @ v, v @ v, u @ w0, v @ w0
    den = a * c - b * b
    s = (b * e - c * d) / den if abs(den) > 1e-14 else 0.0
    t = (a * e - b * d) / den if abs(den) > 1e-14 else 0.0
    mid = 0.5 * ((p + s * u) + (q + t * v))
    return VortexPair(N=N, L=L, points=pts, dirs=dirs, midpoint_unit=mid / L)


def vortex_pair_field(vp: VortexPair) -> np.ndarray:
    """psi on the coarse nodes x_n = L (n/N - 1/2), n = 0..N-1 per axis."""
    N, L = vp.N, vp.L
    g = L * (np.arange(N) / N - 0.5)
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1)        # (N,N,N,3)
    psi = np.ones((N, N, N), dtype=np.complex128)
    for i in range(2):
        u = vp.dirs[i]
        # orthonormal frame (e1, e2) perpendicular to the line
        tmp = np.array([0.0, 0.0, 1.0]) if abs(u[2]) < 0.9 else np.array([0.0, 1.0, 0.0])
        e1 = np.cross(u, tmp); e1 /= np.linalg.norm(e1)
        e2 = np.cross(u, e1)
        rel = X - vp.points[i]
        # nearest periodic image of the line: wrap the perpendicular offset
        rel = rel - L * np.round(rel / L)
        a1 = rel @ e1
        a2 = rel @ e2
        r = np.sqrt(a1 * a1 + a2 * a2)
        theta = np.arctan2(a2, a1)
        psi *= np.tanh(r / math.sqrt(2.0)) * np.exp(1j * vp.signs[i] * theta)
    return psi


def coeffs_from_samples(psi: np.ndarray) -> np.ndarray:
    """Coefficients whose series, evaluated at the unit-box nodes n/N - 1/2,
    returns ``psi``: fhat = (-1)^{sum k} fftshift(ifftn(psi)).  This is the
    trapezoidal-rule step of Sec. 2 written for the NFFT sign and the unit
    box (the (-1)^k factor is the shift by 1/2 of the sign rule of Sec. 2.2.1)."""
    N = psi.shape
    c = np.fft.fftshift(np.fft.ifftn(psi))
    k0, k1, k2 = _freq_grid(N)
    sgn = 1 - 2 * ((k0 + k1 + k2) & 1)
    return c * sgn


def subbox_grid_points(vp: VortexPair, fine: int = 128, width: float = 1.0 / 16) -> tuple:
    """``fine``^3 regular points with spacing width/fine in a cube of side
    ``width`` centred on the coarse node nearest to the closest approach;
    returns (points (fine^3, 3), mask of points that coincide with coarse nodes)."""
    N = vp.N
    centre = np.round((vp.midpoint_unit + 0.5) * N) / N - 0.5      # snapped to a coarse node
    h = width / fine
    offs = (np.arange(fine) - fine // 2) * h
    P = np.stack(np.meshgrid(offs, offs, offs, indexing="ij"), axis=-1).reshape(-1, 3) + centre
    step = int(round((1.0 / N) / h))                                   # fine points per coarse cell
    ii = np.arange(fine) - fine // 2
    on = (ii % step) == 0
    mask = (on[:, None, None] & on[None, :, None] & on[None, None, :]).reshape(-1)
    return wrap(P), mask


def coarse_index_of(points_unit: np.ndarray, N: int) -> np.ndarray:
    """Integer coarse-node index (i0, i1, i2) of points lying on coarse nodes."""
    return np.mod(np.rint((points_unit + 0.5) * N).astype(np.int64), N)


def gpe_two_vortices(N: int = 80, a: float = -20.0, b: float = 60.0) -> np.ndarray:
    """Initial state of the reconnection run of Sec. 5 on the regular grid of
    [a, b)^3: the product of two straight vortices, one through (2, 0, 0)
    along (0, 1, 0), one through (-2, 0, 0) along (0, 0, 1), each with the
    tanh(r / sqrt 2) core (the paper's Pade core profile is not given), the
    distance to each line taken to its nearest periodic image."""
    L = b - a
    g = a + np.arange(N) * (L / N)
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1)
    psi = np.ones((N, N, N), dtype=np.complex128)
    for p0, u, sgn in ((np.array([2.0, 0.0, 0.0]), 1, 1), (np.array([-2.0, 0.0, 0.0]), 2, 1)):
        rel = X - p0
        rel = rel - L * np.round(rel / L)
        axes = [d for d in range(3) if d != u]
        a1, a2 = rel[..., axes[0]], rel[..., axes[1]]
        r = np.sqrt(a1 * a1 + a2 * a2)
        psi *= np.tanh(r / math.sqrt(2.0)) * np.exp(1j * sgn * np.arctan2(a2, a1))
    return psi


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def smooth_uniform_case(N: int = 32, M: int = 10_000):
    """FP64, sigma=2, m=6 case: smooth Gaussian-envelope coefficients, uniform points."""
    return smooth_coeffs((N, N, N), 101), uniform_points(M, 102)


def vortex_subbox_case(N: int = 128, fine: int = 128):
    """GPE-like vortex-pair coefficients and a fine sub-box grid of points."""
    vp = vortex_pair(N, 64.0, 201)
    psi = vortex_pair_field(vp)
    fhat = coeffs_from_samples(psi)
    pts, mask = subbox_grid_points(vp, fine)
    return fhat, pts, mask, psi


def powerlaw_mixed_case(N: int = 256, M: int = 10_000_000):
    """|k|^-2 coefficients; half uniform points, half in 16 clusters (std 0.02)."""
    fhat = powerlaw_coeffs((N, N, N), 301)
    x = mixed_points(M, 16, 0.02, (302, 303, 304, 305))
    return fhat, x


def batched_sets(T: int = 64, sizes=(64, 96, 128), seed: int = 401, mmin: int = 10_000,
                 mmax: int = 1_000_000, mmed: float = 1e5):
    """T coefficient sets with uneven cubic N and lognormal point counts.
    Returns a list of (N, fhat, x)."""
    rs = np.random.default_rng(seed)
    Ns = rs.choice(np.asarray(sizes), size=T)
    rm = np.random.default_rng(seed + 1)
    z = rm.standard_normal(T)
    Ms = np.clip(np.rint(np.exp(math.log(mmed) + 1.1513 * z)), mmin, mmax).astype(np.int64)
    out = []
    for t in range(T):
        N = int(Ns[t])
        x = mixed_points(int(Ms[t]), 4, 0.02, (seed + 2 + 4 * t, seed + 3 + 4 * t,
                                                  seed + 4 + 4 * t, seed + 5 + 4 * t))
        fhat = powerlaw_coeffs((N, N, N), 500 + t)
        out.append((N, fhat, x))
    return out


def lowdim_case(d: int, N: int, M: int, seed: int = 801):
    """One- or two-dimensional case (Appendix B's infft / infft2 sizes scaled
    up): |k|^-2 random-phase coefficients on N^d, M uniform points (M, d)."""
    rng = np.random.default_rng(seed)
    shape = (int(N),) * d
    ks = np.meshgrid(*[np.arange(N) - N // 2 for _ in range(d)], indexing="ij")
    kk = np.sqrt(sum(k.astype(np.float64) ** 2 for k in ks))
    theta = rng.uniform(0.0, 2.0 * math.pi, size=shape)
    fhat = (np.cos(theta) + 1j * np.sin(theta)) / np.maximum(kk, 1.0) ** 2
    x = np.random.default_rng(seed + 1).uniform(-0.5, 0.5, size=(int(M), d))
    return fhat, x


def clustered_grad_case(N: int = 128, M: int = 1_000_000):
    """Differentiation case: |k|^-2 coefficients, 16 clusters, random cotangent w."""
    fhat = powerlaw_coeffs((N, N, N), 701)
    x = clustered_points(M, 16, 0.02, 702, 7020)
    rw = np.random.default_rng(703)
    w = (rw.standard_normal(M) + 1j * rw.standard_normal(M)) / math.sqrt(2.0)
    return fhat, x, w
