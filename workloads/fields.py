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


def blob_params(n_blobs: int = 4096, seed: int = 5):
    """Anisotropic Gaussian blobs: centres U[-1,1]^3, a random rotation (QR
    of a Gaussian matrix, signs fixed so that the factor is unique), axis
    scales log-uniform in [0.01, 0.1], amplitudes U[0.5, 1.5] with a random
    sign, all from default_rng(seed) in that order."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-1.0, 1.0, (n_blobs, 3))
    rots = np.empty((n_blobs, 3, 3))
    for b in range(n_blobs):
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        rots[b] = q * np.sign(np.diag(r))[None, :]
    scales = np.exp(rng.uniform(np.log(0.01), np.log(0.1), (n_blobs, 3)))
    amps = rng.uniform(0.5, 1.5, n_blobs) * rng.choice([-1.0, 1.0], n_blobs)
    return centres, rots, scales, amps


def blob_field_points(x, params, chunk: int = 4096):
    """sum_b a_b exp(-|diag(1/s_b) R_b^T (x - c_b)|^2 / 2) at points x [N, 3]
    (float64, numpy)."""
    centres, rots, scales, amps = params
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(x.shape[0])
    for s0 in range(0, x.shape[0], chunk):
        d = x[s0:s0 + chunk, None, :] - centres[None, :, :]          # [n, B, 3]
        u = np.einsum("nbi,bij->nbj", d, rots) / scales[None, :, :]  # local axes
        out[s0:s0 + chunk] = (amps[None, :] * np.exp(-0.5 * (u * u).sum(-1))).sum(1)
    return out


def fourier_field_points(x, n_modes: int = 512, kmax: int = 16, seed: int = 6):
    """sum_m A_m cos(pi k_m . x + phi_m) at points x [N, 3] (unstandardised)."""
    k, amp, phase = fourier_modes(n_modes, kmax, seed)
    x = np.asarray(x, dtype=np.float64)
    return np.cos(np.pi * x @ k.T + phase[None, :]) @ amp
