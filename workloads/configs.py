"""Synthetic workload specifications.

The paper's experiment (Sec. 4.1) uses the Planck 143 GHz channel: an
N_side=2048 observation grid, lmax 3000, an 80%-sky mask plus point-source
mask, and the best-fit LCDM C_l.  None of that data is available, so these
synthetic configurations stand in for it.  They keep the paper's structure:

* a power-law prior C_l = A / (l (l+1)) for l >= 2, with A chosen so the
  l >= 2 sky rms is 100 uK, and C_0 = C_1 = C_2 (the paper's wide prior for
  the monopole and dipole, which its multi-level method needs); the tiny
  dense-solve case instead conditions on a zero monopole and dipole,
  C_0 = C_1 = 0;
* a symmetric Gaussian beam (Sec. 2.2, beam matrix B diagonal in l) with the
  pixel window p_l taken as 1;
* white, inhomogeneous noise sigma_p = sigma0 (1 + 2 cos^2 theta_p);
* a mask given by zeros in N^-1 (Sec. 2.3): a |b| < 20 deg band in map
  coordinates plus seeded circular discs standing in for point sources.
"""
from dataclasses import dataclass
import math


@dataclass(frozen=True)
class WorkloadConfig:
    name: str
    nside: int
    lmax: int
    fwhm_arcmin: float        # Gaussian beam FWHM; <= 0 means "3 pixel sizes"
    sigma0_uK: float          # noise rms at the equator
    band_deg: float           # galactic-band half width (|b| < band_deg masked)
    n_discs: int              # seeded point-source discs
    disc_radius_deg: float
    nrhs: int
    sky_rms_uK: float = 100.0
    wide_low_l: bool = True   # C_0 = C_1 = C_2 (multi-level solves); False: C_0 = C_1 = 0

    @property
    def npix(self) -> int:
        return 12 * self.nside * self.nside

    @property
    def nalm(self) -> int:
        return (self.lmax + 1) ** 2

    @property
    def fwhm_rad(self) -> float:
        if self.fwhm_arcmin > 0:
            return math.radians(self.fwhm_arcmin / 60.0)
        # pixel size = sqrt(4 pi / Npix)
        return 3.0 * math.sqrt(4.0 * math.pi / self.npix)


# Five workloads: tiny FP64 solve (dense Cholesky check), FP64 GPU solve,
# precision form, batching form, full scale.
CONFIGS = {
    "c1": WorkloadConfig("c1", 16, 32, -1.0, 10.0, 20.0, 5, 5.0, 1, wide_low_l=False),
    "c2": WorkloadConfig("c2", 256, 512, 30.0, 20.0, 20.0, 50, 1.0, 1),
    "c3": WorkloadConfig("c3", 1024, 2048, 10.0, 30.0, 20.0, 200, 0.5, 1),
    "c4": WorkloadConfig("c4", 1024, 2048, 10.0, 30.0, 20.0, 200, 0.5, 32),
    "c5": WorkloadConfig("c5", 2048, 4096, 7.0, 40.0, 20.0, 1000, 0.2, 8),
    # member of the mixed batch at N_side 512
    "m512": WorkloadConfig("m512", 512, 1024, 20.0, 25.0, 20.0, 100, 0.7, 1),
}

# Mixed batch of 8 problems with different resolutions.
MIXED_BATCH = ["c2", "c2", "c2", "m512", "m512", "m512", "c3", "c3"]


def get_config(name: str) -> WorkloadConfig:
    return CONFIGS[name]
