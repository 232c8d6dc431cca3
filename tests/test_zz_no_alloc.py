"""The non-allocating entry point fvk_multidot_noalloc (static device scratch)
against fvk_multidot, on two calls in a row, the second with a smaller input,
and its size limit."""
import numpy as np
import pytest
import torch

pytestmark = [pytest.mark.gpu]


def test_multidot_noalloc_matches_multidot(fvk):
    print("case multidot_noalloc", flush=True)
    ctx = fvk.Ctx(12, 10, 14, grid=fvk.TANH, s=1.5)
    rng = np.random.default_rng(11)
    for m, n in ((13, ctx.N), (5, ctx.N // 3 + 7)):
        Vh = rng.standard_normal((m + 1, ctx.N))
        V = torch.as_tensor(Vh).cuda()
        w = V[m].clone()
        ref = ctx.multidot(V, m, w) if n == ctx.N else None
        out = torch.full((m,), np.nan, dtype=torch.float64, device="cuda")
        ctx.multidot_noalloc(V, m, w, out, n=n)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        exact = Vh[:m, :n] @ Vh[m, :n]
        assert np.max(np.abs(got - exact)) < 1e-12 * np.abs(exact).max() * 10
        if ref is not None:
            assert np.array_equal(got, ref)   # same kernels, same summation order
    # a second context (another scratch user on the same GPU), in turn
    ctx2 = fvk.Ctx(6, 5, 7, grid=fvk.UNIFORM, s=0.0)
    V2 = torch.as_tensor(rng.standard_normal((3, ctx2.N))).cuda()
    out2 = torch.empty(2, dtype=torch.float64, device="cuda")
    ctx2.multidot_noalloc(V2, 2, V2[2].clone(), out2)
    assert np.allclose(out2.cpu().numpy(), ctx2.multidot(V2, 2, V2[2].clone()), rtol=0, atol=0)
    with pytest.raises(fvk.FvkError):
        ctx.multidot_noalloc(V, 257, w, torch.empty(257, dtype=torch.float64, device="cuda"))
