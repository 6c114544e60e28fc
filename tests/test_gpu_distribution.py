"""Distribution-quality report (Sec. V-E, Eq. 11) on the GPU against the
float64 oracle, on octree blocks of levels 1..6 of the 3->64x3->1
He-normal net and the 3->256x5->1 Fourier INR.

* UP and RA-UA Gaussians (float64 propagation): within 1e-10 of
  max(|o|, S).
* Monte Carlo statistics of the float32 evaluation (mean, std, min, max,
  and the first-n_fit-samples fit): within 2e-5 of max(|o|, S).
* Histogram: counts differ only by samples that lie within the float32
  evaluation error of a bin edge (at most two bins per such sample).
* KL: the library's value equals Eq. 11 (the oracle's formula) on the
  library's own histogram and Gaussians to 1e-9, and the oracle's KL within
  1e-3 nats.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.distribution import FIELDS, block_report, kl_histogram_gaussian
from workloads import he_normal_mlp

from _parity import output_scale

pytestmark = pytest.mark.gpu

N_SAMPLES, N_BINS, N_FIT, SEED = 20_000, 64, 100, 9


@pytest.fixture(scope="module")
def ctx():
    import paper_2402_13861_amd as isx

    assert torch.cuda.is_available()
    c = isx.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _blocks(seed=4):
    """One octree cell per level 1..6, positions from a seeded generator."""
    rng = np.random.default_rng(seed)
    cs, hs = [], []
    for L in range(1, 7):
        n = 1 << L
        idx = rng.integers(0, n, 3)
        h = 1.0 / n
        cs.append(-1.0 + (2 * idx + 1) * h)
        hs.append([h, h, h])
    return np.array(cs, np.float32), np.array(hs, np.float32)


def _nets():
    from workloads.configs import load_mlp

    return {"he64x3": he_normal_mlp([3, 64, 64, 64, 1], seed=0), "fourier256x5": load_mlp("relu256x5_fourier")}


@pytest.mark.parametrize("name", ["he64x3", "fourier256x5"])
def test_distribution_report_matches_oracle(ctx, name):
    mlp = _nets()[name]
    S = output_scale(mlp)
    c, h = _blocks()
    vals = []
    ref, ref_hist = block_report(mlp, c, h, N_SAMPLES, N_BINS, N_FIT, SEED, values_out=vals)
    mid = ctx.load_weights(mlp)
    try:
        out, hist = ctx.distribution_kl(mid, torch.from_numpy(c).cuda(), torch.from_numpy(h).cuda(),
                                        n_samples=N_SAMPLES, n_bins=N_BINS, n_fit=N_FIT, seed=SEED, with_hist=True)
        torch.cuda.synchronize()
    finally:
        ctx.unload_mlp(mid)
    g = out.cpu().numpy()
    gh = hist.cpu().numpy().astype(np.int64)
    col = {f: i for i, f in enumerate(FIELDS)}
    scale = np.maximum(np.abs(ref), S)
    for f in ("up_mu", "up_sigma", "raua_mu", "raua_sigma"):
        err = np.abs(g[:, col[f]] - ref[:, col[f]]) / scale[:, col[f]]
        assert err.max() <= 1e-10, (f, err)
    for f in ("mc_mean", "mc_std", "lo", "hi", "fit_mu", "fit_sigma"):
        err = np.abs(g[:, col[f]] - ref[:, col[f]]) / scale[:, col[f]]
        assert err.max() <= 2e-5, (f, err)
    for b in range(c.shape[0]):
        assert gh[b].sum() == N_SAMPLES
        lo, hi = ref[b, col["lo"]], ref[b, col["hi"]]
        edges = lo + (hi - lo) * np.arange(1, N_BINS) / N_BINS
        tol = 2e-5 * S + abs(g[b, col["lo"]] - lo) + abs(g[b, col["hi"]] - hi)
        d = np.abs(vals[b][:, None] - edges[None, :]).min(axis=1)
        near = int((d <= tol).sum())
        moved = int(np.abs(gh[b] - ref_hist[b]).sum())
        print(f"{name} block {b}: KL up {g[b, col['kl_up']]:.4f} (oracle {ref[b, col['kl_up']]:.4f}), raua "
              f"{g[b, col['kl_raua']]:.4f}, fit {g[b, col['kl_fit']]:.4f}; count differences {moved}, samples "
              f"near an edge {near}", flush=True)
        assert moved <= 2 * near
        for kf, mf, sf in (("kl_up", "up_mu", "up_sigma"), ("kl_raua", "raua_mu", "raua_sigma"),
                           ("kl_fit", "fit_mu", "fit_sigma")):
            own = kl_histogram_gaussian(gh[b], g[b, col["lo"]], g[b, col["hi"]], g[b, col[mf]], g[b, col[sf]])
            assert g[b, col[kf]] == pytest.approx(own, rel=1e-9, abs=1e-9)
            assert abs(g[b, col[kf]] - ref[b, col[kf]]) <= 1e-3


def test_distribution_report_edge_cases(ctx):
    import paper_2402_13861_amd as isx

    mlp = he_normal_mlp([3, 32, 32, 1], seed=2)
    mid = ctx.load_weights(mlp)
    try:
        c = torch.zeros((2, 3), device="cuda")
        h = torch.tensor([[0.5, 0.5, 0.5], [0.0, 0.0, 0.0]], device="cuda")
        out = ctx.distribution_kl(mid, c, h, n_samples=1000, n_bins=1, n_fit=1000, seed=1).cpu().numpy()
        # a zero-size block: all samples equal, KL undefined
        assert np.all(np.isnan(out[1, 10:]))
        # one bin and the fit over every sample: the fit is the sample mean and std
        assert out[0, 8] == pytest.approx(out[0, 0], rel=1e-12) and out[0, 9] == pytest.approx(out[0, 1], rel=1e-12)
        assert ctx.distribution_kl(mid, c[:0], h[:0], n_samples=10, n_fit=10).shape == (0, 13)
        for kw in (dict(n_bins=0), dict(n_bins=8193), dict(n_fit=0), dict(n_samples=10, n_fit=11)):
            args = dict(n_samples=100, n_bins=8, n_fit=10, seed=0)
            args.update(kw)
            with pytest.raises(isx.IsxError) as e:
                ctx.distribution_kl(mid, c, h, **args)
            assert e.value.status == -1
    finally:
        ctx.unload_mlp(mid)
