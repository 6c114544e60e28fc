"""The bf16 uncertainty propagation's output read-off on bf16 MFMA with
hi/lo splits (the default) against the float32 MFMA read-off on the same
hidden-layer vectors (ISX_BF16_READOFF = 1): the spread is a sum of
squares of the downward row vectors' products, each split part carrying
about 2^-16 relative error, so the two agree to 1e-4 relative on the spread
and 1e-6 of max(|o|, S) on the centre, for deep narrow and wide nets and
both bf16 forms."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import he_normal_mlp, random_boxes

from _parity import output_scale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2402_13861_amd as isx

    assert torch.cuda.is_available()
    c = isx.Context(0)
    yield c
    torch.cuda.synchronize()
    c.set_option(isx.BF16_READOFF, 0)
    c.set_option(isx.UP_FORM, 0)
    c.close()


@pytest.mark.parametrize("widths", [[3] + [32] * 7 + [1], [3] + [256] * 5 + [1], [3, 128, 128, 128, 128, 1]],
                         ids=lambda w: f"{w[1]}x{len(w) - 2}")
@pytest.mark.parametrize("form", [0, 1], ids=["covariance", "coefficient"])
def test_bf16_readoff_matches_float32_readoff(ctx, widths, form):
    import paper_2402_13861_amd as isx

    mlp = he_normal_mlp(widths, seed=31)
    S = output_scale(mlp)
    c, h, _ = random_boxes(2000, range(0, 10), seed=14)
    mid = ctx.load_weights(mlp)
    res = []
    try:
        ctx.set_option(isx.UP_FORM, form)
        ctx.set_option(isx.CANCEL_CHECK, 0)  # the same vectors for both read-offs
        for ro in (0, 1):
            ctx.set_option(isx.BF16_READOFF, ro)
            out = torch.full((c.shape[0], 2), float("nan"), device="cuda")
            ctx.propagate(mid, isx.UP, isx.BF16, torch.from_numpy(c).cuda(), torch.from_numpy(h).cuda(), out)
            torch.cuda.synchronize()
            res.append(out.cpu().numpy().astype(np.float64))
    finally:
        ctx.set_option(isx.BF16_READOFF, 0)
        ctx.set_option(isx.UP_FORM, 0)
        ctx.set_option(isx.CANCEL_CHECK, 1)
        ctx.unload_mlp(mid)
    a, b = res
    ec = np.abs(a[:, 0] - b[:, 0]) / np.maximum(np.abs(b[:, 0]), S)
    es = np.abs(a[:, 1] - b[:, 1]) / np.maximum(b[:, 1], 1e-3 * S)
    print(f"read-offs {widths[1]}x{len(widths) - 2} form {form}: centre {ec.max():.2e}, spread {es.max():.2e}",
          flush=True)
    assert ec.max() <= 1e-6
    assert es.max() <= 1e-4
