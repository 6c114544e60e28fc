"""Fit a ReLU coordinate MLP to a synthetic field (workload preparation).

This only prepares an input: a trained INR whose weight file both the
oracle and the GPU library then read.  It is plain PyTorch on the CPU
(float32, Adam, MSE on random grid points) and is not part of the
extraction path.

Usage::

    python -m workloads.fit --out workloads/data/relu_256x5_fourier.isxw
"""

from __future__ import annotations

import argparse
import time

import numpy as np
import torch

from .fields import fourier_field_grid
from .weights import MLPWeights, he_normal_mlp, write_weights


def fit_mlp(widths, grid: np.ndarray, steps: int, lr: float, batch: int, init_seed: int, data_seed: int,
            log_every: int = 100):
    """Adam on MSE between the MLP and ``grid`` values at random grid points
    (grid index -> coordinate linspace(-1, 1, res)).  Starts from the
    He-normal initialisation with ``init_seed``."""
    torch.manual_seed(data_seed)
    init = he_normal_mlp(widths, init_seed)
    params = []
    for W, b in zip(init.Ws, init.bs):
        params.append(torch.tensor(W, requires_grad=True))
        params.append(torch.tensor(b, requires_grad=True))
    opt = torch.optim.Adam(params, lr=lr)
    res = grid.shape[0]
    target = torch.from_numpy(grid.reshape(-1))
    coords = torch.linspace(-1.0, 1.0, res, dtype=torch.float32)
    gen = torch.Generator().manual_seed(data_seed)
    t0 = time.time()
    for step in range(steps):
        idx = torch.randint(0, res ** 3, (batch,), generator=gen)
        i = idx // (res * res)
        j = (idx // res) % res
        k = idx % res
        h = torch.stack([coords[i], coords[j], coords[k]], dim=1)
        for li in range(len(params) // 2):
            h = h @ params[2 * li].T + params[2 * li + 1]
            if li + 1 < len(params) // 2:
                h = torch.relu(h)
        loss = torch.mean((h[:, 0] - target[idx]) ** 2)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        if log_every and (step % log_every == 0 or step == steps - 1):
            print(f"step {step:5d} mse {loss.item():.5f} ({time.time() - t0:.0f}s)", flush=True)
    Ws = [params[2 * l].detach().numpy().astype(np.float32) for l in range(len(params) // 2)]
    bs = [params[2 * l + 1].detach().numpy().astype(np.float32) for l in range(len(params) // 2)]
    return MLPWeights(Ws, bs)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--res", type=int, default=256)
    ap.add_argument("--width", type=int, default=256)
    ap.add_argument("--hidden", type=int, default=5)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--field-seed", type=int, default=2)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--data-seed", type=int, default=20)
    ap.add_argument("--threads", type=int, default=8)
    a = ap.parse_args()
    torch.set_num_threads(a.threads)
    grid, _ = fourier_field_grid(a.res, seed=a.field_seed)
    widths = [3] + [a.width] * a.hidden + [1]
    mlp = fit_mlp(widths, grid, a.steps, a.lr, a.batch, a.init_seed, a.data_seed)
    write_weights(a.out, mlp)
    print("wrote", a.out)


if __name__ == "__main__":
    main()
