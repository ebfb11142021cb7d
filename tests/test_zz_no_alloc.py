"""The loss-and-gradient entry point that allocates nothing
(mkf_surrogate_grad_noalloc, for callers that cannot allocate) against the
allocating one (mkf_surrogate_grad), through the C ABI: the same kernels in
the same order, so the same values bit for bit; two calls in a row, the
second smaller, and a size beyond the fixed scratch refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_noalloc_gradient_equals_the_allocating_one():
    from paper_1811_04141_amd import mkf
    from synth import barrel_endcap
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    w = barrel_endcap()
    ctx = mkf.Context(w.find)
    try:
        ctx.load_geometry(w.layers)
        rng = np.random.default_rng(41)
        p = (rng.normal(size=5191) * 0.1).astype(np.float32)
        ctx.surrogate_set(p)
        lw = np.array([1.0, 0.5, 0.5, 0.25, 1.0, 1.0, 0.0], np.float32)
        grad = torch.full((5191,), np.nan, device="cuda")
        loss = torch.full((1,), np.nan, device="cuda")
        for n, seed in ((mkf.NOALLOC_MAX_SAMPLES, 7), (1024, 8)):
            print("noalloc gradient, n =", n, flush=True)
            x = torch.zeros((n, 8), device="cuda")
            t = torch.zeros((n, 7), device="cuda")
            v = torch.zeros(n, device="cuda")
            ctx.surrogate_samples(n, seed, x, t, v)
            ctx.surrogate_grad_noalloc(x, t, lw, grad, loss)
            torch.cuda.synchronize()
            g_ref, l_ref = ctx.surrogate_grad(x, t, lw)
            g = grad.cpu().numpy()
            assert np.all(np.isfinite(g))
            assert np.array_equal(g, g_ref), float(np.abs(g - g_ref).max())
            assert float(loss.cpu()[0]) == l_ref
        n = mkf.NOALLOC_MAX_SAMPLES + 64
        x = torch.zeros((n, 8), device="cuda")
        t = torch.zeros((n, 7), device="cuda")
        with pytest.raises(mkf.MkfError) as e:
            ctx.surrogate_grad_noalloc(x, t, lw, grad, loss)
        assert e.value.status == mkf.MKF_E_CAPACITY
    finally:
        ctx.close()
