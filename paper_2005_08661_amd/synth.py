"""Seeded synthetic multi-echo, multi-coil MRI volumes.

This module only *generates inputs*: phantoms, smooth field maps, coil
sensitivities, the signal model of Sec. II eq. (model) with complex Gaussian
noise, and the support mask of Sec. IV.  It holds none of the estimator's
arithmetic (no coil combination, no cost, no solver), so both the GPU path
and the CPU oracle can consume the same inputs without sharing any of the
method's code.

Layout: every volume is a C-ordered numpy array of shape (nx, ny, nz), z
fastest.  Images are ``y[coil, echo, x, y, z]`` (complex64) and coil maps
``s[coil, x, y, z]`` (complex64).  Field maps are in Hz, echo times in
seconds; the phase of echo l is ``2*pi*f*t_l`` (Sec. II eq. (model) with
omega = 2*pi*f).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

SEED_BASE = 200508661

# Proton gyromagnetic ratio over 2*pi in MHz/T, used to turn ppm into Hz.
GAMMA_MHZ_PER_T = 42.577478

# A six-peak fat spectrum chosen for this project: offsets in ppm relative to
# water (the main methylene peak near -3.4 ppm carries most of the weight)
# and relative amplitudes summing to one (Sec. II, multipeak fat model).
FAT_PPM = np.array([-3.80, -3.40, -2.70, -2.00, -0.50, 0.60])
FAT_AMP = np.array([0.08, 0.70, 0.12, 0.02, 0.03, 0.05])


@dataclasses.dataclass
class Volume:
    """One synthetic acquisition plus its ground truth."""

    y: np.ndarray            # complex64 [ncoil, necho, nx, ny, nz]
    sens: Optional[np.ndarray]  # complex64 [ncoil, nx, ny, nz] or None (s = 1)
    te: np.ndarray           # float64 [necho], seconds
    mask: np.ndarray         # uint8 [nx, ny, nz]
    f_true: np.ndarray       # float64 [nx, ny, nz], Hz
    beta: float
    niter: int
    nmls: int = 3
    model: str = "fieldmap"  # or "waterfat"
    fat_hz: Optional[np.ndarray] = None
    fat_amp: Optional[np.ndarray] = None
    water: Optional[np.ndarray] = None
    fat: Optional[np.ndarray] = None
    name: str = ""
    reg_order: int = 1       # finite differences of the regulariser C: 1 or 2

    @property
    def shape(self):
        return self.mask.shape

    @property
    def ncoil(self):
        return self.y.shape[0]

    @property
    def necho(self):
        return self.y.shape[1]


def _grid(shape):
    return np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")


def ellipsoid(shape, inside=1.0, outside=0.05):
    """Ellipsoid centred at (dims-1)/2 with semi-axes 0.4*dims."""
    g = _grid(shape)
    r2 = np.zeros(shape)
    for ax, n in enumerate(shape):
        c = (n - 1) / 2.0
        a = max(0.4 * n, 0.5)
        r2 += ((g[ax] - c) / a) ** 2
    return np.where(r2 <= 1.0, inside, outside), r2 <= 1.0


def smooth_field(rng, shape, k, span):
    """Sum of k random anisotropic 3D Gaussians, rescaled to max |.| = span."""
    g = _grid(shape)
    out = np.zeros(shape)
    dims = np.array(shape, dtype=np.float64)
    for _ in range(k):
        c = rng.uniform(0.2, 0.8, 3) * dims
        sig = rng.uniform(0.1, 0.3, 3) * dims
        amp = rng.uniform(-1.0, 1.0)
        e = np.zeros(shape)
        for ax in range(3):
            e += ((g[ax] - c[ax]) / max(sig[ax], 1e-3)) ** 2
        out += amp * np.exp(-0.5 * e)
    m = np.abs(out).max()
    if m > 0:
        out *= span / m
    return out


def dipole_field(rng, shape, inside_ell, peak=400.0, radius=4.0):
    """Localized susceptibility-like dipole: (R^3/2)(3 dz^2 - r^2)/r^5 outside
    radius R around a seeded centre inside the ellipsoid, 0 inside R; scaled
    so its on-axis value at r = R is ``peak`` and clipped to +-peak."""
    idx = np.argwhere(inside_ell)
    c = idx[rng.integers(len(idx))].astype(np.float64)
    g = _grid(shape)
    dx, dy, dz = g[0] - c[0], g[1] - c[1], g[2] - c[2]
    r2 = dx * dx + dy * dy + dz * dz
    r = np.sqrt(r2)
    with np.errstate(divide="ignore", invalid="ignore"):
        d = (radius ** 3 / 2.0) * (3 * dz * dz - r2) / np.maximum(r, 1e-12) ** 5
    d = np.where(r >= radius, d, 0.0)
    return np.clip(peak * d, -peak, peak)


def coil_maps(rng, shape, ncoil):
    """Smooth complex coil sensitivities normalised to sum_c |s_c|^2 = 1."""
    nx, ny, nz = shape
    g = _grid(shape)
    R = max(nx, ny)
    sig = 0.5 * R
    cx, cy, cz = (nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0
    s = np.zeros((ncoil,) + tuple(shape), dtype=np.complex128)
    for c in range(ncoil):
        th = 2 * np.pi * c / ncoil
        px = cx + 0.6 * R * np.cos(th)
        py = cy + 0.6 * R * np.sin(th)
        pz = cz + (0.25 * nz if c % 2 == 0 else -0.25 * nz)
        mag = np.exp(-0.5 * (((g[0] - px) ** 2 + (g[1] - py) ** 2 + (g[2] - pz) ** 2) / sig ** 2))
        ph0 = rng.uniform(-np.pi, np.pi)
        ramp = rng.normal(size=3)
        ramp *= rng.uniform(0, np.pi) / max(np.linalg.norm(ramp), 1e-12)
        ph = ph0 + ramp[0] * g[0] / max(nx, 1) + ramp[1] * g[1] / max(ny, 1) + ramp[2] * g[2] / max(nz, 1)
        s[c] = mag * np.exp(1j * ph)
    ss = np.sqrt((np.abs(s) ** 2).sum(0))
    return s / ss


def add_noise(rng, clean, inside, snr_db):
    """Complex Gaussian noise at SNR in dB relative to the rms of the clean
    signal over the ellipsoid; real and imaginary parts each N(0, sigma^2/2)."""
    sel = np.broadcast_to(inside, clean.shape)
    rms = np.sqrt(np.mean(np.abs(clean[sel]) ** 2))
    sigma = rms * 10 ** (-snr_db / 20.0)
    noise = (rng.normal(size=clean.shape) + 1j * rng.normal(size=clean.shape)) * (sigma / np.sqrt(2))
    return clean + noise


def paper_mask(y, sens=None, frac=0.1, dilate=2):
    """Support mask following Sec. IV: threshold the first-echo magnitude at
    frac * max, take the 3D convex hull, dilate by ``dilate`` voxels.

    The magnitude used is the root-sum-of-squares over coils (a standard
    combination that is not part of the estimator)."""
    from scipy import ndimage
    from scipy.spatial import ConvexHull

    mag = np.sqrt((np.abs(y[:, 0].astype(np.complex128)) ** 2).sum(0))
    pts = np.argwhere(mag >= frac * mag.max()).astype(np.float64)
    shape = mag.shape
    m = np.zeros(shape, dtype=bool)
    try:
        hull = ConvexHull(pts)
        eq = hull.equations
        allp = np.stack([a.ravel() for a in _grid(shape)], 1)
        inside = np.ones(len(allp), dtype=bool)
        for s0 in range(0, len(allp), 1 << 18):
            blk = allp[s0:s0 + (1 << 18)]
            inside[s0:s0 + len(blk)] = np.all(blk @ eq[:, :3].T + eq[:, 3] <= 1e-9, axis=1)
        m = inside.reshape(shape)
    except Exception:  # degenerate (flat) point sets: fall back to the threshold set
        m[tuple(pts.astype(int).T)] = True
    if dilate > 0:
        m = ndimage.binary_dilation(m, structure=np.ones((3, 3, 3), bool), iterations=dilate)
    return m.astype(np.uint8)


def _signal(rng, shape, te, f, x_echo, sens, snr_db, inside):
    """y[c, l] = s_c * x_l * exp(i 2 pi f t_l) + noise (Sec. II eq. (model))."""
    necho = len(te)
    ncoil = 1 if sens is None else sens.shape[0]
    y = np.zeros((ncoil, necho) + tuple(shape), dtype=np.complex128)
    for l in range(necho):
        ph = np.exp(1j * 2 * np.pi * f * te[l])
        for c in range(ncoil):
            sc = 1.0 if sens is None else sens[c]
            y[c, l] = sc * x_echo[l] * ph
    y = add_noise(rng, y, inside, snr_db)
    return y.astype(np.complex64)


def fieldmap_volume(shape, ncoil, te, beta, niter, seed, field_k, field_span, dipole, snr_db,
                    mask="full", name=""):
    rng = np.random.default_rng(seed)
    te = np.asarray(te, dtype=np.float64)
    mag, inside = ellipsoid(shape)
    f = smooth_field(rng, shape, field_k, field_span)
    if dipole:
        f = f + dipole_field(rng, shape, inside)
    phi0 = smooth_field(rng, shape, 3, np.pi)
    m = mag * np.exp(1j * phi0)
    sens = coil_maps(rng, shape, ncoil) if ncoil > 1 else None
    y = _signal(rng, shape, te, f, [m] * len(te), sens, snr_db, inside)
    msk = np.ones(shape, np.uint8) if mask == "full" else paper_mask(y)
    return Volume(y=y, sens=None if sens is None else sens.astype(np.complex64), te=te, mask=msk,
                  f_true=f, beta=beta, niter=niter, name=name)


def waterfat_volume(shape, ncoil, te, beta, niter, seed, field_span, snr_db, b0=3.0,
                    mask="full", name=""):
    rng = np.random.default_rng(seed)
    te = np.asarray(te, dtype=np.float64)
    mag, inside = ellipsoid(shape)
    f = smooth_field(rng, shape, 8, field_span)
    ff_s = smooth_field(rng, shape, 4, 1.0)
    ff = 0.25 + 0.25 * ff_s / max(np.abs(ff_s).max(), 1e-12)
    phi0 = smooth_field(rng, shape, 3, np.pi)
    water = mag * (1 - ff) * np.exp(1j * phi0)
    fat = mag * ff * np.exp(1j * phi0)
    fat_hz = FAT_PPM * GAMMA_MHZ_PER_T * b0
    cl = np.array([np.sum(FAT_AMP * np.exp(1j * 2 * np.pi * fat_hz * t)) for t in te])
    x_echo = [water + fat * cl[l] for l in range(len(te))]
    sens = coil_maps(rng, shape, ncoil) if ncoil > 1 else None
    y = _signal(rng, shape, te, f, x_echo, sens, snr_db, inside)
    msk = np.ones(shape, np.uint8) if mask == "full" else paper_mask(y)
    return Volume(y=y, sens=None if sens is None else sens.astype(np.complex64), te=te, mask=msk,
                  f_true=f, beta=beta, niter=niter, model="waterfat", fat_hz=fat_hz,
                  fat_amp=FAT_AMP.copy(), water=water, fat=fat, name=name)


# --- The workloads -----------------------------------------------------------

def tiny_fieldmap(mask="paper", seed_offset=0):
    """32x32x16, 1 coil, TE 0/2/10 ms, SNR 20, beta 2^-3, 50 iterations."""
    return fieldmap_volume((32, 32, 16), 1, [0.0, 2.0e-3, 10.0e-3], 2.0 ** -3, 50,
                           SEED_BASE + 0 + seed_offset, 4, 100.0, False, 20.0, mask=mask,
                           name="fieldmap 32x32x16 1 coil 3 echoes")


def mid_fieldmap(mask="full", shape=(128, 128, 64), seed_offset=0):
    """128x128x64, 8 coils, TE 0/2.2/4.4 ms, SNR 30, beta 2^-4, 100 iterations;
    smooth field (8 blobs, +-250 Hz) plus a +-400 Hz dipole."""
    return fieldmap_volume(shape, 8, [0.0, 2.2e-3, 4.4e-3], 2.0 ** -4, 100,
                           SEED_BASE + 1 + seed_offset, 8, 250.0, True, 30.0, mask=mask,
                           name="fieldmap %dx%dx%d 8 coils 3 echoes" % tuple(shape))


def waterfat(mask="full", shape=(192, 192, 64)):
    """192x192x64, 8 coils, 6 echoes TE = 1.2 + k ms, field +-300 Hz, SNR 25."""
    te = [1.2e-3 + 1.0e-3 * k for k in range(6)]
    return waterfat_volume(shape, 8, te, 2.0 ** -4, 100, SEED_BASE + 2, 300.0, 25.0, mask=mask,
                           name="water-fat %dx%dx%d 8 coils 6 echoes" % tuple(shape))


def batched(nvol=16, scale=1.0):
    """16 volumes, X,Y in {64..160 step 8}, Z in {32..96 step 8}, 4 coils,
    TE 0/2/5 ms, beta_v = 2^U[-6,-2], otherwise generated as mid_fieldmap."""
    out = []
    for v in range(nvol):
        rng = np.random.default_rng(SEED_BASE * 100 + v)
        nx = int(rng.choice(np.arange(64, 161, 8)))
        ny = int(rng.choice(np.arange(64, 161, 8)))
        nz = int(rng.choice(np.arange(32, 97, 8)))
        beta = float(2.0 ** rng.uniform(-6, -2))
        shp = tuple(max(4, int(round(d * scale))) for d in (nx, ny, nz))
        vol = fieldmap_volume(shp, 4, [0.0, 2.0e-3, 5.0e-3], beta, 100,
                              SEED_BASE * 100 + v + 1000, 8, 250.0, True, 30.0, mask="full",
                              name="batched volume %d %dx%dx%d" % ((v,) + shp))
        out.append(vol)
    return out


def random_volume(shape, ncoil, necho, seed, beta=0.1, niter=10, mask_frac=1.0, te=None,
                  snr_db=20.0, field_span=60.0):
    """Small random problem for unit tests (optionally with a random mask)."""
    rng = np.random.default_rng(seed)
    if te is None:
        te = np.sort(rng.uniform(0, 6e-3, necho))
        te[0] = 0.0
    vol = fieldmap_volume(shape, ncoil, te, beta, niter, seed + 7, 2, field_span, False, snr_db)
    if mask_frac < 1.0:
        vol.mask = (rng.uniform(size=shape) < mask_frac).astype(np.uint8)
    return vol
