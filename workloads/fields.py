"""Synthetic scalar fields that stand in for the paper's turbulence-like
datasets (vorticity magnitudes of pseudo-spectral simulations): seeded,
standardised, with a Kolmogorov-like k^(-5/3) amplitude spectrum.
"""

from __future__ import annotations

import numpy as np


def fourier_modes(n_modes: int, kmax: int, seed: int):
    """Wave vectors k in Z^3 with 1 <= |k| <= kmax drawn uniformly over the
    lattice points, amplitudes |k|^(-5/3), phases U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    r = np.arange(-kmax, kmax + 1)
    K = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    norm = np.linalg.norm(K, axis=1)
    K = K[(norm >= 1) & (norm <= kmax)]
    k = K[rng.integers(0, K.shape[0], n_modes)]
    amp = np.linalg.norm(k, axis=1) ** (-5.0 / 3.0)
    phase = rng.uniform(0.0, 2.0 * np.pi, n_modes)
    return k.astype(np.float64), amp, phase


def fourier_field_grid(res: int, n_modes: int = 512, kmax: int = 16, seed: int = 2):
    """sum_m A_m cos(pi k_m . x + phi_m) on linspace(-1, 1, res)^3 (index
    order [i, j, k] = [x, y, z]), standardised to mean 0, std 1.  Returns
    (grid float32, (mean, std) of the raw field)."""
    k, amp, phase = fourier_modes(n_modes, kmax, seed)
    x = np.linspace(-1.0, 1.0, res)
    # separable: Re sum_m c_m e^{i pi k1 x} e^{i pi k2 y} e^{i pi k3 z}
    c = amp * np.exp(1j * phase)
    X = np.exp(1j * np.pi * k[:, 0:1] * x[None, :])  # [m, res]
    Y = np.exp(1j * np.pi * k[:, 1:2] * x[None, :])
    Z = np.exp(1j * np.pi * k[:, 2:3] * x[None, :])
    out = np.empty((res, res, res), dtype=np.float64)
    for i in range(res):
        T = (c * X[:, i])[:, None] * Y  # [m, j]
        out[i] = (T.T @ Z).real  # [j, k]
    mean, std = out.mean(), out.std()
    return ((out - mean) / std).astype(np.float32), (mean, std)
