"""Fit a wide ReLU coordinate MLP to the blob + Fourier field (workload
preparation, run once on a GPU).

The field: 4096 anisotropic Gaussian blobs (``fields.blob_params``, seed 5)
plus 0.25 times a Fourier background of 512 modes with a k^(-5/3) spectrum
(``fields.fourier_modes``, seed 6, scaled to unit std), the sum standardised
to mean 0 and std 1; it is evaluated on the fly at random points of the 512^3
grid linspace(-1, 1, 512)^3 (mean and std estimated from 2^22 random grid
points).  The MLP starts from He-normal weights (seed 0) and takes Adam steps
(lr 1e-3) on the MSE of random batches of grid points.  PyTorch on the GPU
only prepares the input: the weight file is then read by both the oracle and
the library.

Usage::

    python -m workloads.fit_gpu --out workloads/data/relu_512x8_blobs.isxw
"""

from __future__ import annotations

import argparse
import time

import numpy as np
import torch

from .fields import blob_params, fourier_modes
from .weights import MLPWeights, he_normal_mlp, write_weights


class Field:
    def __init__(self, device, n_blobs=4096, blob_seed=5, fourier_seed=6, background=0.25):
        c, r, s, a = blob_params(n_blobs, blob_seed)
        t = lambda v: torch.tensor(v, dtype=torch.float32, device=device)
        self.c, self.r, self.inv_s, self.a = t(c), t(r), t(1.0 / s), t(a)
        k, amp, ph = fourier_modes(512, 16, fourier_seed)
        self.k, self.amp, self.ph = t(k), t(amp), t(ph)
        self.bg, self.fstd = background, 1.0
        self.mean, self.std = 0.0, 1.0

    def raw(self, x, chunk=512):
        out = torch.zeros(x.shape[0], device=x.device)
        for b0 in range(0, self.c.shape[0], chunk):
            d = x[:, None, :] - self.c[None, b0:b0 + chunk]
            u = torch.einsum("nbi,bij->nbj", d, self.r[b0:b0 + chunk]) * self.inv_s[None, b0:b0 + chunk]
            out += (self.a[None, b0:b0 + chunk] * torch.exp(-0.5 * (u * u).sum(-1))).sum(1)
        four = torch.cos(torch.pi * x @ self.k.T + self.ph[None, :]) @ self.amp
        return out + self.bg * four / self.fstd

    def __call__(self, x):
        return (self.raw(x) - self.mean) / self.std


def grid_points(n, res, gen, device):
    idx = torch.randint(0, res, (n, 3), generator=gen, device=device)
    return idx.float() * (2.0 / (res - 1)) - 1.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--res", type=int, default=512)
    ap.add_argument("--width", type=int, default=512)
    ap.add_argument("--hidden", type=int, default=8)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--data-seed", type=int, default=50)
    ap.add_argument("--device", default="cuda")
    ap.add_argument("--stat-points", type=int, default=1 << 22)
    a = ap.parse_args()
    dev = torch.device(a.device)
    gen = torch.Generator(device=dev).manual_seed(a.data_seed)
    field = Field(dev)
    with torch.no_grad():
        # unit-std Fourier background, then the standardisation of the sum
        pts = grid_points(a.stat_points, a.res, gen, dev)
        four = torch.cos(torch.pi * pts @ field.k.T + field.ph[None, :]) @ field.amp
        field.fstd = float(four.std())
        v = torch.cat([field.raw(pts[i:i + 65536]) for i in range(0, pts.shape[0], 65536)])
        field.mean, field.std = float(v.mean()), float(v.std())
    print(f"field mean {field.mean:.4f} std {field.std:.4f} (Fourier background std {field.fstd:.4f})", flush=True)
    widths = [3] + [a.width] * a.hidden + [1]
    init = he_normal_mlp(widths, a.init_seed)
    params = []
    for W, b in zip(init.Ws, init.bs):
        params.append(torch.tensor(W, device=dev, requires_grad=True))
        params.append(torch.tensor(b, device=dev, requires_grad=True))
    opt = torch.optim.Adam(params, lr=a.lr)
    nl = len(params) // 2
    t0 = time.time()
    for step in range(a.steps):
        x = grid_points(a.batch, a.res, gen, dev)
        with torch.no_grad():
            y = field(x)
        h = x
        for li in range(nl):
            h = h @ params[2 * li].T + params[2 * li + 1]
            if li + 1 < nl:
                h = torch.relu(h)
        loss = torch.mean((h[:, 0] - y) ** 2)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        if step % 200 == 0 or step == a.steps - 1:
            print(f"step {step:5d} mse {loss.item():.5f} ({time.time() - t0:.0f}s)", flush=True)
    Ws = [params[2 * l].detach().cpu().numpy().astype(np.float32) for l in range(nl)]
    bs = [params[2 * l + 1].detach().cpu().numpy().astype(np.float32) for l in range(nl)]
    write_weights(a.out, MLPWeights(Ws, bs))
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()
