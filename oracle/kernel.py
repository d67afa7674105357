"""Scalar Helmholtz point kernel (oracle).

The paper's matrix entries (Eq. 7) integrate the free-space Green's function
exp(-jkR)/R of Eq. 5-6 against RWG basis functions. The synthetic workloads
replace the Galerkin integrals by point collocation of the same kernel:

    G(a, b) = exp(-j k r) / (4 pi r),   r = |a - b|,   a != b
    G(a, a) = (1 - j k h / 2) / (2 pi h)

with h the mean point spacing supplied by the caller. exp(-jkr) is taken as
cos(kr) - j sin(kr). Pinned by closed-form scalar evaluation in the tests.
"""
from __future__ import annotations

import math

import numpy as np


def self_term(k: float, h: float) -> complex:
    """Diagonal entry (1 - j k h / 2) / (2 pi h)."""
    return complex(1.0, -k * h / 2.0) / (2.0 * math.pi * h)


def kernel_block(pa: np.ndarray, pb: np.ndarray, k: float, h: float,
                 same: bool = False) -> np.ndarray:
    """Dense block G(pa[i], pb[j]) for point arrays pa (m x 3), pb (n x 3).

    ``same`` marks a diagonal block (pa is pb): its diagonal gets the self
    term. Distinct coincident points (r = 0 off the diagonal) raise
    ValueError, since the kernel is singular there.
    """
    d = pa[:, None, :] - pb[None, :, :]
    r = np.sqrt(d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2])
    if same:
        np.fill_diagonal(r, 1.0)
    if np.any(r == 0.0):
        raise ValueError("coincident distinct points: kernel is singular")
    kr = k * r
    out = (np.cos(kr) - 1j * np.sin(kr)) / (4.0 * math.pi * r)
    if same:
        np.fill_diagonal(out, self_term(k, h))
    return out


def kernel_row(p_obs: np.ndarray, pb: np.ndarray, k: float) -> np.ndarray:
    """One row G(p_obs, pb[j]) for an observer that is not among pb."""
    d = pb - p_obs[None, :]
    r = np.sqrt(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2])
    kr = k * r
    return (np.cos(kr) - 1j * np.sin(kr)) / (4.0 * math.pi * r)
