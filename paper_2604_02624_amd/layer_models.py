"""Layer models besides the dielectric thickness of Eq. 1-2.

Phase-only layers (paper Eq. 3, the spatial light modulators of the experiment): a pixel with
phase phi at a reference wavelength lambda_ref imposes exp(+j phi lambda_ref / lambda) (a fixed
optical path; the sign as read for Eq. 1).  That is the thickness model with a material whose
index exceeds the medium's by exactly 1 at every wavelength, no absorption, and thickness
h = phi lambda_ref / (2 pi), so a phase-only design runs on the same kernels: build it with
phase_only_design and pass heights_from_phase(phi).
"""
from __future__ import annotations

import math

import numpy as np


def phase_only_design(design: dict) -> dict:
    """The design with phase-only layers: unit index contrast to the medium, no absorption."""
    d = dict(design)
    d["n_mat"] = np.full(d["n_wl"], float(d["n_medium"]) + 1.0)
    d["kappa"] = None
    return d


def heights_from_phase(phi: np.ndarray, lam_ref: float) -> np.ndarray:
    """Equivalent thicknesses (metres, float32) of phases phi (radians) at lam_ref."""
    return (np.asarray(phi, np.float64) * (lam_ref / (2.0 * math.pi))).astype(np.float32)


def phase_from_heights(h: np.ndarray, lam_ref: float) -> np.ndarray:
    """Phases (radians) at lam_ref of equivalent thicknesses h."""
    return np.asarray(h, np.float64) * (2.0 * math.pi / lam_ref)
