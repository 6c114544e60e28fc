"""The allocation-free classify/compact entry point against the ordinary
one, through the C ABI: two calls in a row (the second on a smaller input, so
that the fixed working memory still holds the first call's contents), a call
at the capacity limit, and the capacity error above it."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import he_normal_mlp

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    out = np.stack([rng.normal(0, 1, n), np.abs(rng.normal(0, 0.5, n))], 1).astype(np.float32)
    out[::89, 1] = 0.0
    pmask = rng.integers(0, 8, n).astype(np.uint32)
    return torch.from_numpy(out).cuda(), torch.from_numpy(pmask.view(np.int32)).cuda()


def test_noalloc_classify_compact_matches_allocating_call():
    import paper_2402_13861_amd as isx

    assert torch.cuda.is_available()
    with isx.Context(0) as ctx:
        mid = ctx.load_weights(he_normal_mlp([3, 32, 32, 1], seed=0))
        ctx.set_isovalues(mid, [-0.5, 0.0, 0.7])
        cap = isx._lib.NOALLOC_MAX_CELLS
        for n, seed, k in ((50_021, 1, 3.0), (7_013, 2, 1.0), (cap, 3, 3.0), (1, 4, 3.0)):
            print(f"noalloc classify/compact: n={n} seed={seed} k={k}", flush=True)
            out, pm = _inputs(n, seed)
            idx_a, msk_a, cnt_a = ctx.classify_compact(mid, k, out, pm)
            idx_b = torch.full((n,), -1, dtype=torch.int32, device="cuda")
            msk_b = torch.full((n,), -1, dtype=torch.int32, device="cuda")
            cnt_b = torch.full((1,), -1, dtype=torch.int64, device="cuda")
            ctx.classify_compact_noalloc(mid, k, out, pm, idx_b, msk_b, cnt_b)
            torch.cuda.synchronize()
            m = int(cnt_a.item())
            assert int(cnt_b.item()) == m
            assert torch.equal(idx_a[:m], idx_b[:m])
            assert torch.equal(msk_a[:m], msk_b[:m])
        # above the fixed capacity: a clear error, nothing launched
        big = torch.zeros((cap + 1, 2), dtype=torch.float32, device="cuda")
        small = torch.zeros(1, dtype=torch.int32, device="cuda")
        with pytest.raises(isx.IsxError) as e:
            ctx.classify_compact_noalloc(mid, 3.0, big, None, small, small, torch.zeros(1, dtype=torch.int64,
                                                                                       device="cuda"))
        assert e.value.status == isx._lib.ECAPACITY
        ctx.unload_mlp(mid)
