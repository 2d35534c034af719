"""Seeded input generation (no transforms, no operators, no solves).

Random numbers: numpy ``Generator(PCG64)``.  Every stream is a child of the
master ``SeedSequence(seed)`` addressed by an explicit spawn key, so any one
stream can be regenerated without drawing the others:

* key (r,)          right-hand-side draws of RHS r, in this order:
                    omega1 (nalm), omega2 (npix), g_signal (nalm), g_noise (npix)
* key (1000,)       point-source disc centres: z ~ U(-1, 1), then phi ~ U(0, 2 pi)
* key (2000 + r,)   white draw for a prior sample x_true of RHS r (nalm)

Layout conventions (the public data layout of the library, not arithmetic):

* maps are HEALPix RING ordered (Gorski et al. 2005): rings run north to
  south, pixels within a ring by increasing phi;
* harmonic vectors are "real packed, m-major": the m = 0 block holds x_l0 for
  l = 0..lmax, then for each m >= 1 a cosine block (l = m..lmax) followed by a
  sine block (l = m..lmax); length (lmax+1)^2.  The basis is orthonormal, so
  the prior covariance of every entry with multipole l is C_l.
"""
from __future__ import annotations

import math
import numpy as np

from .configs import WorkloadConfig


# --------------------------------------------------------------------------
# layout helpers
# --------------------------------------------------------------------------
def alm_size(lmax: int) -> int:
    return (lmax + 1) ** 2


def packed_ell(lmax: int) -> np.ndarray:
    """Multipole l of every entry of a real packed harmonic vector."""
    out = np.empty(alm_size(lmax), dtype=np.int64)
    out[: lmax + 1] = np.arange(lmax + 1)
    pos = lmax + 1
    for m in range(1, lmax + 1):
        n = lmax - m + 1
        ells = np.arange(m, lmax + 1)
        out[pos: pos + n] = ells
        out[pos + n: pos + 2 * n] = ells
        pos += 2 * n
    return out


def ring_layout(nside: int):
    """Per-ring (z, npix_in_ring, phi of first pixel) of the HEALPix RING grid.

    Rings i = 1..4 nside - 1 from north to south (Gorski et al. 2005):
    north cap i < nside has 4i pixels at z = 1 - i^2/(3 nside^2), first pixel
    at phi = pi/(4i); the equatorial belt has 4 nside pixels at
    z = 4/3 - 2i/(3 nside) with first pixel at pi/(4 nside) when i - nside is
    even and at 0 when it is odd (base pixel 4 centred on phi = 0); the south
    cap mirrors the north cap.
    """
    nrings = 4 * nside - 1
    z = np.empty(nrings)
    npr = np.empty(nrings, dtype=np.int64)
    phi0 = np.empty(nrings)
    for i in range(1, nrings + 1):
        if i < nside:
            ii = i
            npr[i - 1] = 4 * ii
            z[i - 1] = 1.0 - ii * ii / (3.0 * nside * nside)
            phi0[i - 1] = math.pi / (4.0 * ii)
        elif i <= 3 * nside:
            npr[i - 1] = 4 * nside
            z[i - 1] = (4.0 * nside - 2.0 * i) / (3.0 * nside)
            phi0[i - 1] = math.pi / (4.0 * nside) if (i - nside) % 2 == 0 else 0.0
        else:
            ii = 4 * nside - i
            npr[i - 1] = 4 * ii
            z[i - 1] = -(1.0 - ii * ii / (3.0 * nside * nside))
            phi0[i - 1] = math.pi / (4.0 * ii)
    return z, npr, phi0


def pixel_centres(nside: int):
    """(z, phi) of every pixel centre, RING order."""
    z, npr, phi0 = ring_layout(nside)
    zz = np.repeat(z, npr)
    ring_of = np.repeat(np.arange(len(npr)), npr)
    start = np.concatenate([[0], np.cumsum(npr)[:-1]])
    j = np.arange(int(npr.sum())) - start[ring_of]
    phi = phi0[ring_of] + 2.0 * math.pi * j / npr[ring_of]
    return zz, phi


# --------------------------------------------------------------------------
# model inputs
# --------------------------------------------------------------------------
def power_spectrum(cfg: WorkloadConfig) -> np.ndarray:
    """C_l = A/(l(l+1)) for l >= 2 with sum_{l>=2} (2l+1) C_l / (4 pi) =
    sky_rms^2 (uK^2); C_0 = C_1 = C_2 (the wide monopole/dipole prior of the
    paper's experiment, Sec. 4.1) when cfg.wide_low_l, else C_0 = C_1 = 0."""
    ell = np.arange(cfg.lmax + 1, dtype=np.float64)
    shape = np.zeros(cfg.lmax + 1)
    shape[2:] = 1.0 / (ell[2:] * (ell[2:] + 1.0))
    var = np.sum((2.0 * ell + 1.0) * shape) / (4.0 * math.pi)
    cl = shape * (cfg.sky_rms_uK ** 2 / var)
    cl[:2] = cl[2] if cfg.wide_low_l else 0.0
    return cl


def gaussian_beam(cfg: WorkloadConfig, lmax: int | None = None) -> np.ndarray:
    """b_l = exp(-l(l+1) sigma_b^2 / 2), sigma_b = FWHM / sqrt(8 ln 2); p_l = 1."""
    lmax = cfg.lmax if lmax is None else lmax
    ell = np.arange(lmax + 1, dtype=np.float64)
    sig = cfg.fwhm_rad / math.sqrt(8.0 * math.log(2.0))
    return np.exp(-0.5 * ell * (ell + 1.0) * sig * sig)


def _disc_centres(cfg: WorkloadConfig, seed: int):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(1000,))))
    zc = rng.uniform(-1.0, 1.0, cfg.n_discs)
    phic = rng.uniform(0.0, 2.0 * math.pi, cfg.n_discs)
    return zc, phic


def mask_map(cfg: WorkloadConfig, seed: int = 0) -> np.ndarray:
    """Boolean map, True = masked (N^-1 = 0 there)."""
    nside = cfg.nside
    z, npr, phi0 = ring_layout(nside)
    start = np.concatenate([[0], np.cumsum(npr)[:-1]])
    npix = int(npr.sum())
    masked = np.zeros(npix, dtype=bool)
    # galactic band |b| < band, i.e. |z| < sin(band) (map coordinates, no rotation)
    zb = math.sin(math.radians(cfg.band_deg))
    band_rings = np.nonzero(np.abs(z) < zb)[0]
    for k in band_rings:
        masked[start[k]: start[k] + npr[k]] = True
    # discs: masked iff angular distance to the centre < radius
    r = math.radians(cfg.disc_radius_deg)
    cosr = math.cos(r)
    theta_ring = np.arccos(np.clip(z, -1.0, 1.0))
    zc, phic = _disc_centres(cfg, seed)
    for zc_i, phic_i in zip(zc, phic):
        thc = math.acos(zc_i)
        sc = math.sqrt(max(0.0, 1.0 - zc_i * zc_i))
        sel = np.nonzero((theta_ring >= thc - r - 1e-12) & (theta_ring <= thc + r + 1e-12))[0]
        for k in sel:
            n = int(npr[k])
            phi = phi0[k] + 2.0 * math.pi * np.arange(n) / n
            sk = math.sqrt(max(0.0, 1.0 - z[k] * z[k]))
            cosd = z[k] * zc_i + sk * sc * np.cos(phi - phic_i)
            hit = cosd > cosr
            if hit.any():
                masked[start[k]: start[k] + n] |= hit
    return masked


def inverse_noise_map(cfg: WorkloadConfig, seed: int = 0):
    """(N^-1 map in uK^-2 with zeros in the mask, sigma map in uK, mask)."""
    z, npr, _ = ring_layout(cfg.nside)
    zz = np.repeat(z, npr)
    sigma = cfg.sigma0_uK * (1.0 + 2.0 * zz * zz)
    masked = mask_map(cfg, seed)
    ninv = np.where(masked, 0.0, 1.0 / (sigma * sigma))
    return ninv, sigma, masked


def active_mode_mask(cl: np.ndarray) -> np.ndarray:
    """Packed-vector mask of the unknowns: modes with C_l > 0."""
    lmax = len(cl) - 1
    return cl[packed_ell(lmax)] > 0.0


# --------------------------------------------------------------------------
# random draws
# --------------------------------------------------------------------------
def _rng(seed: int, key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(key,))))


def draw_rhs_white(cfg: WorkloadConfig, r: int, seed: int = 0):
    """White draws for RHS r: (omega1[nalm], omega2[npix], g_signal[nalm], g_noise[npix])."""
    rng = _rng(seed, r)
    w1 = rng.standard_normal(cfg.nalm)
    w2 = rng.standard_normal(cfg.npix)
    gs = rng.standard_normal(cfg.nalm)
    gn = rng.standard_normal(cfg.npix)
    return w1, w2, gs, gn


def draw_prior_white(cfg: WorkloadConfig, r: int, seed: int = 0) -> np.ndarray:
    """White draw (nalm) for a prior sample x_true = S^{1/2} g of RHS r."""
    return _rng(seed, 2000 + r).standard_normal(cfg.nalm)


def prior_sample(cfg: WorkloadConfig, r: int, seed: int = 0) -> np.ndarray:
    """x ~ N(0, S): sqrt(C_l) times the white draw (zero where C_l = 0)."""
    cl = power_spectrum(cfg)
    return np.sqrt(cl)[packed_ell(cfg.lmax)] * draw_prior_white(cfg, r, seed)


def workload_inputs(cfg: WorkloadConfig, seed: int = 0):
    """Fixed inputs of one problem: dict(cl, bl, ninv, sigma, mask)."""
    cl = power_spectrum(cfg)
    bl = gaussian_beam(cfg)
    ninv, sigma, masked = inverse_noise_map(cfg, seed)
    return dict(cl=cl, bl=bl, ninv=ninv, sigma=sigma, mask=masked)
