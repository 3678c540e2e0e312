"""Seeded synthetic hyperspectral neutron-tomography inputs.

This module is the one thing shared by the FP64 oracle tests and the GPU
path: it produces *inputs* only (phantoms, attenuation spectra, analytic
projections and Poisson counts) and holds none of the method's arithmetic
(no normalisation, no factorisation, no discrete projector).

The simulation follows the paper's data section: a phantom of
non-overlapping single-material objects (volume fraction 1 inside), a
dictionary of mu-spectra over 1.5-4.5 Angstrom, projections p = L (D^m)^T
(eq. 3 without noise, with L the exact chord length of each ray through
each material region), counts y = y^o exp(-p) (eq. 10) and independent
Poisson noise on both y and the open beam y^o.  The paper's Bragg-edge
library is not available, so each material's spectrum is a smooth
a + b/lambda baseline plus 2-4 step drops at seeded wavelengths.

Geometry conventions (shared with every consumer):
  * parallel beam, detector row r is an independent N_c x N_c slice;
  * view angle theta_v = v*pi/N_v, v = 0..N_v-1;
  * pixel pitch = detector pitch = 1, centres at index - (N-1)/2;
  * the image x coordinate follows the column index i, y the row index j;
  * a ray of view v at detector column c is {(x, y): x cos + y sin = s_c}.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

LAMBDA_LO = 1.5   # Angstrom, wavelength range of the paper's data
LAMBDA_HI = 4.5


def wavelengths(n_bins: int) -> np.ndarray:
    """Bin centres uniform on [1.5, 4.5] Angstrom."""
    k = np.arange(n_bins, dtype=np.float64)
    return LAMBDA_LO + (k + 0.5) * (LAMBDA_HI - LAMBDA_LO) / n_bins


def view_angles(n_views: int) -> np.ndarray:
    """theta_v = v*pi/N_v (180 degrees, endpoint excluded)."""
    return np.arange(n_views, dtype=np.float64) * (math.pi / n_views)


def material_spectra(n_mat: int, n_bins: int, seed: int) -> np.ndarray:
    """Unscaled attenuation spectra mu_m(lambda), shape [n_bins][n_mat].

    mu_m = a_m + b_m / lambda + sum_e h_e * [lambda < lambda_e]: a smooth
    1/lambda-like baseline with 2-4 Bragg-edge-style drops at seeded edge
    wavelengths lambda_e ~ U[1.8, 4.2]; steps are hard at bin resolution.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = wavelengths(n_bins)
    mu = np.zeros((n_bins, n_mat))
    for m in range(n_mat):
        a = rng.uniform(0.2, 1.0)
        b = rng.uniform(0.5, 2.0)
        col = a + b / lam
        n_edge = int(rng.integers(2, 5))
        for _ in range(n_edge):
            lam_e = rng.uniform(1.8, 4.2)
            h = rng.uniform(0.15, 0.6)
            col = col + h * (lam < lam_e)
        mu[:, m] = col
    return mu


@dataclasses.dataclass
class Ellipsoid:
    cx: float
    cy: float
    cz: float
    a: float      # semi-axis along the rotated x' direction (pixels)
    b: float      # semi-axis along y'
    c: float      # semi-axis along z (slices); inf for a 2D disc/ellipse
    phi: float    # in-plane rotation
    material: int


def phantom(n: int, n_slices: int, n_obj: int, n_mat: int, rng: np.random.Generator,
            max_tries: int = 10000) -> List[Ellipsoid]:
    """Non-overlapping ellipses (1 slice) or z-aligned ellipsoids.

    Centres lie within 0.6*N/2 of the rotation axis, in-plane semi-axes are
    U[0.08, 0.22]*N.  Objects are rejected until their bounding circles in
    the x-y plane are disjoint, so no voxel holds two materials.  Object o
    is made of material o mod n_mat, so every material is present.
    """
    objs: List[Ellipsoid] = []
    tries = 0
    while len(objs) < n_obj:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("phantom: could not place non-overlapping objects")
        a = rng.uniform(0.08, 0.22) * n
        b = rng.uniform(0.08, 0.22) * n
        rad = 0.6 * n / 2
        ang = rng.uniform(0, 2 * math.pi)
        dist = rad * math.sqrt(rng.uniform(0, 1))
        cx, cy = dist * math.cos(ang), dist * math.sin(ang)
        phi = rng.uniform(0, math.pi)
        if n_slices > 1:
            c = rng.uniform(0.5, 1.0) * n_slices
            cz = rng.uniform(-0.25, 0.25) * n_slices
        else:
            c, cz = math.inf, 0.0
        r_new = max(a, b)
        # keep inside the field of view
        if math.hypot(cx, cy) + r_new > 0.5 * (n - 2):
            continue
        if any(math.hypot(cx - o.cx, cy - o.cy) <= r_new + max(o.a, o.b) + 1.0 for o in objs):
            continue
        objs.append(Ellipsoid(cx, cy, cz, a, b, c, phi, len(objs) % n_mat))
    return objs


def _slice_scale(o: Ellipsoid, z: float) -> float:
    if math.isinf(o.c):
        return 1.0
    t = (z - o.cz) / o.c
    return math.sqrt(1.0 - t * t) if abs(t) < 1.0 else 0.0


def chord_lengths(objs: Sequence[Ellipsoid], n_views: int, n_rows: int, n_cols: int,
                  n_mat: int, angles: Optional[np.ndarray] = None) -> np.ndarray:
    """Exact chord length of every ray through every material region.

    Returns L[v][r][c][m] (float64, pixel units).  For an ellipse with
    semi-axes (a, b) rotated by phi and centred at (x0, y0), the ray
    x cos t + y sin t = s has chord 2ab sqrt(q^2 - u^2) / q^2 with
    u = s - (x0 cos t + y0 sin t) and q^2 = a^2 cos^2(t-phi) + b^2 sin^2(t-phi).
    """
    th = view_angles(n_views) if angles is None else np.asarray(angles, np.float64)
    s = np.arange(n_cols, dtype=np.float64) - (n_cols - 1) / 2.0
    L = np.zeros((len(th), n_rows, n_cols, n_mat))
    for r in range(n_rows):
        z = r - (n_rows - 1) / 2.0
        for o in objs:
            sc = _slice_scale(o, z)
            if sc <= 0.0:
                continue
            a, b = o.a * sc, o.b * sc
            ct, st = np.cos(th), np.sin(th)
            u = s[None, :] - (o.cx * ct + o.cy * st)[:, None]
            al = th - o.phi
            q2 = (a * np.cos(al)) ** 2 + (b * np.sin(al)) ** 2
            inside = q2[:, None] - u * u
            chord = np.where(inside > 0, 2 * a * b * np.sqrt(np.maximum(inside, 0)) / q2[:, None], 0.0)
            L[:, r, :, o.material] += chord
    return L


def volume_fractions(objs: Sequence[Ellipsoid], n: int, n_rows: int, n_mat: int,
                     supersample: int = 4) -> np.ndarray:
    """Ground-truth x^m[r][j][i][m]: fraction of each pixel inside each object."""
    q = supersample
    off = (np.arange(q) + 0.5) / q - 0.5
    g = np.arange(n, dtype=np.float64) - (n - 1) / 2.0
    X = (g[None, :, None, None] + off[None, None, None, :])  # [1][i][1][q]
    Y = (g[:, None, None, None] + off[None, None, :, None])  # [j][1][q][1]
    xm = np.zeros((n_rows, n, n, n_mat))
    for r in range(n_rows):
        z = r - (n_rows - 1) / 2.0
        for o in objs:
            sc = _slice_scale(o, z)
            if sc <= 0.0:
                continue
            a, b = o.a * sc, o.b * sc
            cp, sp = math.cos(o.phi), math.sin(o.phi)
            dx, dy = X - o.cx, Y - o.cy
            xr = dx * cp + dy * sp
            yr = -dx * sp + dy * cp
            ins = ((xr / a) ** 2 + (yr / b) ** 2 < 1.0)
            xm[r, :, :, o.material] += ins.mean(axis=(2, 3))
    return np.minimum(xm, 1.0)


@dataclasses.dataclass
class Scan:
    """One synthetic hyperspectral scan (all arrays host numpy)."""
    n_views: int
    n_rows: int
    n_cols: int
    n_bins: int
    n_mat: int
    flux: float
    objs: List[Ellipsoid]
    L: np.ndarray          # [N_v][N_r][N_c][N_m] chord lengths
    mu: np.ndarray         # [N_k][N_m] scaled spectra (D^m)
    y: Optional[np.ndarray] = None    # [N_v][N_r][N_c][N_k] uint16 counts
    yo: Optional[np.ndarray] = None   # [N_r][N_c][N_k] uint16 open beam

    @property
    def n_p(self) -> int:
        return self.n_views * self.n_rows * self.n_cols

    def p_clean(self) -> np.ndarray:
        """Noiseless projections [N_p][N_k] (eq. 3 with w = 0)."""
        return self.L.reshape(-1, self.n_mat) @ self.mu.T


def make_scan(n_views: int, n_rows: int, n_cols: int, n_bins: int, n_mat: int,
              flux: float, seed: int, n_obj: Optional[int] = None,
              library_seed: Optional[int] = None, p_max: float = 2.0,
              counts: bool = True) -> Scan:
    """Build a seeded scan.  Spectra come from `library_seed` (default: seed),
    so several scans can share one material library; geometry and noise come
    from `seed`.  mu is scaled so that the largest noiseless p equals p_max."""
    ss = np.random.SeedSequence(seed)
    g_geom, g_noise = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(2)]
    objs = phantom(n_cols, n_rows, n_obj if n_obj is not None else n_mat, n_mat, g_geom)
    L = chord_lengths(objs, n_views, n_rows, n_cols, n_mat)
    mu = material_spectra(n_mat, n_bins, seed if library_seed is None else library_seed)
    Lf = L.reshape(-1, n_mat)
    peak = max(float((Lf[r0:r0 + (1 << 16)] @ mu.T).max()) for r0 in range(0, Lf.shape[0], 1 << 16))
    mu = mu * (p_max / peak)
    scan = Scan(n_views, n_rows, n_cols, n_bins, n_mat, float(flux), objs, L, mu)
    if counts:
        scan.y, scan.yo = poisson_counts(scan, g_noise)
    return scan


def poisson_counts(scan: Scan, rng: np.random.Generator, chunk_rows: int = 1 << 15):
    """y ~ Poisson(flux e^{-p}) and y^o ~ Poisson(flux), independently (eq. 10
    plus the paper's Poisson noise on both), clipped into uint16."""
    yo = rng.poisson(scan.flux, size=(scan.n_rows, scan.n_cols, scan.n_bins))
    yo = np.minimum(yo, 65535).astype(np.uint16)
    Lf = scan.L.reshape(-1, scan.n_mat)
    y = np.empty((scan.n_p, scan.n_bins), np.uint16)
    for r0 in range(0, scan.n_p, chunk_rows):
        lam = scan.flux * np.exp(-(Lf[r0:r0 + chunk_rows] @ scan.mu.T))
        y[r0:r0 + chunk_rows] = np.minimum(rng.poisson(lam), 65535)
    y = y.reshape(scan.n_views, scan.n_rows, scan.n_cols, scan.n_bins)
    return y, yo


def device_counts(scan: Scan, seed: int, device="cuda", chunk_rows: int = 1 << 18):
    """The counts of `scan` drawn on a GPU with torch's seeded Philox
    generator (same model as poisson_counts: y^o ~ Poisson(flux),
    y ~ Poisson(flux e^{-p}), clipped into uint16), for workloads whose
    15.7 G counts would take minutes on the host.  Returns (y, y^o) as int16
    tensors holding the uint16 bits, shapes [N_v][N_r][N_c][N_k] and
    [N_r][N_c][N_k]."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    yo = torch.poisson(torch.full((scan.n_rows, scan.n_cols, scan.n_bins), float(scan.flux), device=device),
                       generator=g)
    yo = torch.clamp(yo, max=65535.0).to(torch.int32).to(torch.int16)
    Lf = torch.from_numpy(scan.L.reshape(-1, scan.n_mat)).to(device)
    muT = torch.from_numpy(scan.mu.T.copy()).to(device)
    y = torch.empty((scan.n_p, scan.n_bins), dtype=torch.int16, device=device)
    for r0 in range(0, scan.n_p, chunk_rows):
        lam = scan.flux * torch.exp(-(Lf[r0:r0 + chunk_rows] @ muT))
        cnt = torch.poisson(lam.float(), generator=g)
        y[r0:r0 + chunk_rows] = torch.clamp(cnt, max=65535.0).to(torch.int32).to(torch.int16)
        del lam, cnt
    return y.view(scan.n_views, scan.n_rows, scan.n_cols, scan.n_bins), yo


# Named workloads.  Shapes follow the paper's problem statement (N_v views,
# N_r slices, N_c columns, N_k bins, N_m materials, K = N_m).
CONFIGS = {
    "tiny":  dict(n_views=90, n_rows=1, n_cols=64, n_bins=256, n_mat=3, flux=1e4, seed=1),
    "mid":   dict(n_views=60, n_rows=16, n_cols=128, n_bins=1024, n_mat=4, flux=2e3, seed=2),
    "full":  dict(n_views=120, n_rows=256, n_cols=256, n_bins=2000, n_mat=5, flux=1e3, seed=5),
}


def config_scan(name: str, counts: bool = True, **over) -> Scan:
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    return make_scan(counts=counts, **cfg)


def batched_instances(n: int = 32, seed: int = 3):
    """Shapes of the uneven batch: columns U{64..256}, views U{30..180},
    bins U{512..2048}, K = N_m U{2..6}; one slice each, flux 1e4."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        out.append(dict(n_views=int(rng.integers(30, 181)), n_rows=1,
                        n_cols=int(rng.integers(64, 257)), n_bins=int(rng.integers(512, 2049)),
                        n_mat=int(rng.integers(2, 7)), flux=1e4, seed=seed * 1000 + i))
    return out


def batched_scans(n: int = 32, seed: int = 3, counts: bool = True):
    """The scans of batched_instances.  An instance whose objects cannot be
    placed without overlap keeps its shape and draws its geometry again from
    seed + 100000 * attempt (deterministic)."""
    out = []
    for d in batched_instances(n, seed):
        for attempt in range(20):
            try:
                out.append(make_scan(counts=counts, **dict(d, seed=d["seed"] + 100000 * attempt)))
                break
            except RuntimeError:
                continue
        else:
            raise RuntimeError("batched_scans: could not place objects")
    return out


def random_factors(n_p: int, n_k: int, k: int, seed: int, lo: float = 0.1, hi: float = 1.0):
    """Strictly positive seeded (V, D) pair, used as an explicit NMF start."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, (n_p, k)), rng.uniform(lo, hi, (n_k, k))


def random_volume(n_rows: int, n: int, k: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((n_rows, n, n, k))


def mlp_init(k: int, seed: int, n_in: int = 256, n_h: int = 128) -> np.ndarray:
    """Seeded Glorot-uniform weights with zero biases for the
    n_in -> n_h -> n_h -> k network, as one flat float64 vector in the order
    W1[n_in][n_h], b1, W2[n_h][n_h], b2, W3[n_h][k], b3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fi, fo in ((n_in, n_h), (n_h, n_h), (n_h, k)):
        a = math.sqrt(6.0 / (fi + fo))
        parts.append(rng.uniform(-a, a, fi * fo))
        parts.append(np.zeros(fo))
    return np.concatenate(parts)
