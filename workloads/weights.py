"""MLP weight container, He-normal initialisation and the on-disk weight file.

File layout (little endian)::

    char[4]  magic  = b"ISXW"
    uint32   version = 1
    uint32   n_linear             (number of linear layers, L)
    uint32   widths[L + 1]        (widths[0] = input dim, widths[L] = 1)
    for each layer l in 0..L-1:
        float32 W_l[widths[l+1] * widths[l]]   row-major (out x in)
        float32 b_l[widths[l+1]]

A ReLU follows every linear layer except the last.  Both the oracle and the
GPU library read the same float32 values; the oracle widens them to float64.
"""

from __future__ import annotations

import struct
from dataclasses import dataclass
from pathlib import Path
from typing import List, Sequence, Tuple

import numpy as np

MAGIC = b"ISXW"
VERSION = 1


@dataclass
class MLPWeights:
    """Coordinate MLP f: R^3 -> R with ReLU on every hidden layer."""

    Ws: List[np.ndarray]  # float32 [out, in]
    bs: List[np.ndarray]  # float32 [out]

    @property
    def widths(self) -> List[int]:
        return [self.Ws[0].shape[1]] + [w.shape[0] for w in self.Ws]

    @property
    def n_linear(self) -> int:
        return len(self.Ws)

    def layers(self) -> List[Tuple[np.ndarray, np.ndarray]]:
        return list(zip(self.Ws, self.bs))

    def n_params(self) -> int:
        return sum(w.size + b.size for w, b in zip(self.Ws, self.bs))


def he_normal_mlp(widths: Sequence[int], seed: int) -> MLPWeights:
    """He-normal weights AND biases, N(0, 2/fan_in), drawn in the order
    W1, b1, W2, b2, ... from numpy's PCG64 ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for fan_in, fan_out in zip(widths[:-1], widths[1:]):
        std = np.sqrt(2.0 / fan_in)
        Ws.append((rng.standard_normal((fan_out, fan_in)) * std).astype(np.float32))
        bs.append((rng.standard_normal(fan_out) * std).astype(np.float32))
    return MLPWeights(Ws, bs)


def siren_mlp(widths: Sequence[int], seed: int, w0: float) -> MLPWeights:
    """Sine network in the SIREN initialisation (Sitzmann et al. 2020): first
    layer U(-w0/fan_in, w0/fan_in) (the frequency w0 folded into it), later
    layers U(-sqrt(6/fan_in), sqrt(6/fan_in)), biases from the same ranges,
    drawn in the order W1, b1, W2, b2, ... from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for li, (fan_in, fan_out) in enumerate(zip(widths[:-1], widths[1:])):
        lim = w0 / fan_in if li == 0 else np.sqrt(6.0 / fan_in)
        Ws.append(rng.uniform(-lim, lim, (fan_out, fan_in)).astype(np.float32))
        bs.append(rng.uniform(-lim, lim, fan_out).astype(np.float32))
    return MLPWeights(Ws, bs)


def write_weights(path, mlp: MLPWeights) -> None:
    widths = mlp.widths
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<II", VERSION, mlp.n_linear))
        f.write(struct.pack("<%dI" % len(widths), *widths))
        for W, b in zip(mlp.Ws, mlp.bs):
            f.write(np.ascontiguousarray(W, dtype="<f4").tobytes())
            f.write(np.ascontiguousarray(b, dtype="<f4").tobytes())


def read_weights(path) -> MLPWeights:
    data = Path(path).read_bytes()
    if data[:4] != MAGIC:
        raise ValueError(f"{path}: not an ISXW weight file")
    version, n_linear = struct.unpack_from("<II", data, 4)
    if version != VERSION:
        raise ValueError(f"{path}: unsupported version {version}")
    off = 12
    widths = list(struct.unpack_from("<%dI" % (n_linear + 1), data, off))
    off += 4 * (n_linear + 1)
    Ws, bs = [], []
    for fan_in, fan_out in zip(widths[:-1], widths[1:]):
        W = np.frombuffer(data, dtype="<f4", count=fan_out * fan_in, offset=off).reshape(fan_out, fan_in)
        off += 4 * fan_out * fan_in
        b = np.frombuffer(data, dtype="<f4", count=fan_out, offset=off)
        off += 4 * fan_out
        Ws.append(W.astype(np.float32))
        bs.append(b.astype(np.float32))
    if off != len(data):
        raise ValueError(f"{path}: {len(data) - off} trailing bytes")
    return MLPWeights(Ws, bs)
