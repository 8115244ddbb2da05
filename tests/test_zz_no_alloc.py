"""The allocation-free entry point (lq_inner_products_noalloc) against the
entry point it is a variant of (lq_inner_products), through the C ABI: two
calls in a row on one context, the second with a smaller input, each checked
against lq_inner_products on the same vectors and against numpy."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _vecs(nb, nw, n, seed):
    rng = np.random.default_rng(seed)
    E = rng.standard_normal((nb, n)) + 1j * rng.standard_normal((nb, n))
    W = rng.standard_normal((nw, n)) + 1j * rng.standard_normal((nw, n))
    return E, W


def test_noalloc_inner_products_match_the_allocating_entry_point():
    from paper_1509_06865_amd import Context
    c = Context((4, 4, 4, 4), 1)
    # the first call is long enough that its chunk count is capped by the
    # scratch (96 rows: at most 680 chunks; the allocating call uses 977)
    for nb, nw, n, seed in ((96, 16, 1_000_003, 1), (37, 5, 40_000 + 3, 2)):
        print(f"[noalloc] nb={nb} nw={nw} n={n}", flush=True)
        E, W = _vecs(nb, nw, n, seed)
        Ed = torch.from_numpy(E).cuda()
        Wd = torch.from_numpy(W).cuda()
        got = c.inner_products_noalloc(Ed, Wd)
        ref = c.inner_products(Ed, Wd)
        scale = np.abs(ref).max()
        # FP64 sums over n terms in another chunking: rounding only
        assert np.abs(got - ref).max() <= 1e-13 * scale
        exact = E.conj() @ W.T
        assert np.abs(got - exact).max() <= 1e-12 * np.abs(exact).max()
        del Ed, Wd
        torch.cuda.synchronize()


def test_noalloc_inner_products_reject_sizes_beyond_the_limits():
    from paper_1509_06865_amd import Context
    from paper_1509_06865_amd.lqmg import LQError
    c = Context((4, 4, 4, 4), 1)
    E = torch.zeros((193, 8), dtype=torch.complex128, device="cuda")
    W = torch.zeros((2, 8), dtype=torch.complex128, device="cuda")
    with pytest.raises(LQError) as e:
        c.inner_products_noalloc(E, W)
    assert e.value.code == -1
