"""Seeded synthetic inputs for the constrained-realization (CR) system.

This package is the ONLY code shared by the CPU oracle (``oracle/``) and the
GPU product path (``paper_1308_5299_amd``).  It draws random numbers and
builds the fixed inputs of the CR system of Seljebotn et al. (2013), Sec. 2.2
(data model) and Sec. 2.3 (CR system): the prior power spectrum C_l, the beam
b_l, the inverse-noise map N^-1 with its mask, and the white Gaussian draws
used for right-hand sides and manufactured solutions.  It contains none of the
method's arithmetic (no spherical-harmonic transform, no operator, no solve).
"""
from .configs import CONFIGS, MIXED_BATCH, WorkloadConfig, get_config
from .generate import (
    alm_size,
    packed_ell,
    pixel_centres,
    mask_map,
    prior_sample,
    ring_layout,
    power_spectrum,
    gaussian_beam,
    inverse_noise_map,
    active_mode_mask,
    draw_rhs_white,
    draw_prior_white,
    workload_inputs,
)

__all__ = [
    "CONFIGS", "MIXED_BATCH", "WorkloadConfig", "get_config",
    "alm_size", "packed_ell", "pixel_centres", "mask_map", "prior_sample", "ring_layout", "power_spectrum",
    "gaussian_beam", "inverse_noise_map", "active_mode_mask",
    "draw_rhs_white", "draw_prior_white", "workload_inputs",
]
