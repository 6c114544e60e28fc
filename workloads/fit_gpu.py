"""Fit a coordinate MLP to a synthetic target (workload preparation, run
once on a GPU): the blob + Fourier field, or the signed distance function of
a small analytic scene (``--target sdf``) for ray casting.

The field: 4096 anisotropic Gaussian blobs (``fields.blob_params``, seed 5)
plus 0.25 times a Fourier background of 512 modes with a k^(-5/3) spectrum
(``fields.fourier_modes``, seed 6, scaled to unit std), the sum standardised
to mean 0 and std 1; it is evaluated on the fly at random points of the 512^3
grid linspace(-1, 1, 512)^3 (mean and std estimated from 2^22 random grid
points).  The MLP starts from He-normal weights (seed 0) and takes Adam steps
(lr 1e-3) on the MSE of random batches of grid points.  PyTorch on the GPU
only prepares the input: the weight file is then read by both the oracle and
the library.

The SDF scene (``--target sdf``): the union (minimum) of a sphere of
radius 0.35 at (-0.35, -0.1, 0), a torus of major radius 0.3 and minor
radius 0.1 centred at (0.35, 0, 0.05) in the plane x = 0.35 (axis along x),
and a box of half-sizes (0.3, 0.08, 0.2) at (0, 0.45, -0.1); exact
distances, sampled uniformly on [-1, 1]^3 and, for half of each batch, near
the surface (a uniform point moved along the gradient of the distance to
the surface, then jittered by N(0, 0.02^2) per axis).  No standardisation:
the MLP learns the distance itself.  ``--act elu`` trains an ELU net.

Usage::

    python -m workloads.fit_gpu --out workloads/data/relu_512x8_blobs.isxw
    python -m workloads.fit_gpu --target sdf --width 64 --hidden 2 --last 48 --steps 3000 \
        --out workloads/data/relu_sdf_7k.isxw
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


def scene_sdf(x):
    """Exact signed distance of the scene in the module docstring."""
    s = torch.linalg.norm(x - torch.tensor([-0.35, -0.1, 0.0], device=x.device), dim=1) - 0.35
    q = x - torch.tensor([0.35, 0.0, 0.05], device=x.device)
    ring = torch.sqrt(q[:, 1] ** 2 + q[:, 2] ** 2) - 0.3  # torus about the x axis
    t = torch.sqrt(ring ** 2 + q[:, 0] ** 2) - 0.1
    d = torch.abs(x - torch.tensor([0.0, 0.45, -0.1], device=x.device)) - torch.tensor([0.3, 0.08, 0.2],
                                                                                       device=x.device)
    b = torch.linalg.norm(torch.clamp(d, min=0.0), dim=1) + torch.clamp(d.max(dim=1).values, max=0.0)
    return torch.minimum(torch.minimum(s, t), b)


def sdf_batch(n, gen, device):
    """Half uniform points, half points pulled onto the surface and jittered."""
    x = torch.rand((n, 3), generator=gen, device=device) * 2.0 - 1.0
    h = n // 2
    p = x[:h].clone().requires_grad_(True)
    d = scene_sdf(p)
    (g,) = torch.autograd.grad(d.sum(), p)
    with torch.no_grad():
        p = p - d[:, None] * g / torch.clamp(torch.linalg.norm(g, dim=1, keepdim=True), min=1e-6)
        p = p + 0.02 * torch.randn(p.shape, generator=gen, device=device)
        x[:h] = torch.clamp(p, -1.0, 1.0)
    with torch.no_grad():
        y = scene_sdf(x)
    return x, y


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
    ap.add_argument("--target", default="blobs", choices=["blobs", "sdf"])
    ap.add_argument("--act", default="relu", choices=["relu", "elu"])
    ap.add_argument("--last", type=int, default=0, help="width of the last hidden layer (0: --width)")
    a = ap.parse_args()
    dev = torch.device(a.device)
    gen = torch.Generator(device=dev).manual_seed(a.data_seed)
    act = torch.relu if a.act == "relu" else torch.nn.functional.elu
    if a.target == "sdf":
        widths = [3] + [a.width] * a.hidden + ([a.last] if a.last else []) + [1]
        return fit(widths, a, dev, lambda: sdf_batch(a.batch, gen, dev), act)
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

    def batch():
        x = grid_points(a.batch, a.res, gen, dev)
        with torch.no_grad():
            y = field(x)
        return x, y

    return fit(widths, a, dev, batch, act)


def fit(widths, a, dev, batch, act):
    """Adam on the MSE of batches from ``batch()``; writes the weight file."""
    init = he_normal_mlp(widths, a.init_seed)
    params = []
    for W, b in zip(init.Ws, init.bs):
        params.append(torch.tensor(W, device=dev, requires_grad=True))
        params.append(torch.tensor(b, device=dev, requires_grad=True))
    opt = torch.optim.Adam(params, lr=a.lr)
    nl = len(params) // 2
    t0 = time.time()
    for step in range(a.steps):
        x, y = batch()
        h = x
        for li in range(nl):
            h = h @ params[2 * li].T + params[2 * li + 1]
            if li + 1 < nl:
                h = act(h)
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
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
