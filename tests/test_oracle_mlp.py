"""Pins of the FP64 oracle of the learned propagation surrogate (forward,
backpropagated gradient, Adam), against facts fixed independently of its
code: finite differences, a linear regime that reduces to matrix products,
a saturated regime with a closed-form loss, and Adam's first step."""
import numpy as np
import pytest

from oracle import oracle as O

NI, NH, NO = O.MLP_NI, O.MLP_NH, O.MLP_NO


def split(p):
    o = 0
    out = []
    for shape in [(NH, NI), (NH,), (NH, NH), (NH,), (NO, NH), (NO,)]:
        n = int(np.prod(shape))
        out.append(p[o:o + n].reshape(shape))
        o += n
    assert o == O.MLP_NPARAM
    return out


def join(*parts):
    return np.concatenate([np.ravel(a) for a in parts])


def random_params(rng, scale=0.4):
    return rng.normal(size=O.MLP_NPARAM) * scale


def test_parameter_count():
    assert O.MLP_NPARAM == 5191


def test_gradient_matches_central_differences():
    """Every parameter block, including the biases and an output with zero
    weight in the loss, against central differences of the loss."""
    rng = np.random.default_rng(3)
    p = random_params(rng)
    x = rng.normal(size=(5, NI))
    t = rng.normal(size=(5, NO))
    w = np.array([1.0, 0.5, 0.0, 2.0, 1.0, 0.25, 1.0])
    L, g = O.mlp_grad(p, x, t, w)
    y = O.mlp_forward(p, x)
    assert L == pytest.approx(np.mean(np.sum(w * (y - t) ** 2, axis=1)), rel=1e-12)
    offs = np.cumsum([0, NH * NI, NH, NH * NH, NH, NO * NH, NO])
    picks = np.concatenate([rng.choice(np.arange(offs[i], offs[i + 1]), min(12, offs[i + 1] - offs[i]), replace=False)
                            for i in range(6)])
    h = 1e-6
    for i in picks:
        e = np.zeros_like(p)
        e[i] = h
        fd = (O.mlp_grad(p + e, x, t, w)[0] - O.mlp_grad(p - e, x, t, w)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_linear_regime_reduces_to_matrix_products():
    """With every pre-activation far above zero, silu(z) = z to within
    z exp(-z), and the network is the affine map W3 (W2 (W1 x + b1) + b2) + b3."""
    rng = np.random.default_rng(4)
    A1 = rng.normal(size=(NH, NI)) * 0.3
    A2 = rng.normal(size=(NH, NH)) * 0.05
    A3 = rng.normal(size=(NO, NH)) * 0.1
    c = 60.0  # silu(z) - z = -z / (1 + e^z) ~ 1e-24 at z = 60
    b1 = np.full(NH, c)
    b2 = c - A2 @ b1   # z2 = A2 (A1 x) + c
    b3 = rng.normal(size=NO)
    p = join(A1, b1, A2, b2, A3, b3)
    x = rng.uniform(-1, 1, size=(7, NI))
    y = O.mlp_forward(p, x)
    z1 = x @ A1.T + b1
    z2 = z1 @ A2.T + b2
    assert z1.min() > 50 and z2.min() > 50
    np.testing.assert_allclose(y, z2 @ A3.T + b3, rtol=1e-12, atol=1e-10)


def test_saturated_regime_outputs_the_bias_and_only_b3_learns():
    """With every second-layer pre-activation far below zero, h2 = 0: the
    output is b3, the loss is sum w_j (b3_j - t_j)^2 averaged over samples,
    and only b3 gets a gradient, 2 w_j mean(b3_j - t_j)."""
    rng = np.random.default_rng(5)
    W1 = rng.normal(size=(NH, NI))
    b1 = rng.normal(size=NH)
    W2 = np.zeros((NH, NH))
    b2 = np.full(NH, -80.0)
    W3 = rng.normal(size=(NO, NH))
    b3 = rng.normal(size=NO)
    p = join(W1, b1, W2, b2, W3, b3)
    x = rng.normal(size=(6, NI))
    t = rng.normal(size=(6, NO))
    w = rng.uniform(0.5, 2.0, NO)
    y = O.mlp_forward(p, x)
    np.testing.assert_allclose(y, np.broadcast_to(b3, y.shape), atol=1e-30)
    L, g = O.mlp_grad(p, x, t, w)
    assert L == pytest.approx(np.mean(np.sum(w * (b3 - t) ** 2, axis=1)), rel=1e-13)
    gW1, gb1, gW2, gb2, gW3, gb3 = split(g)
    np.testing.assert_allclose(gb3, 2 * w * np.mean(b3 - t, axis=0), rtol=1e-12)
    for a in (gW1, gb1, gW2, gb2, gW3):
        assert np.max(np.abs(a)) < 1e-25


def test_adam_first_step_moves_each_parameter_by_lr():
    """From zero moments, bias correction makes the first step
    lr * g / (|g| + eps): each parameter moves by lr against its gradient's
    sign (up to eps); a second identical gradient moves it by the same step."""
    rng = np.random.default_rng(6)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    g[0] = 0.0
    p, m, v = O.adam(p0, np.zeros(50), np.zeros(50), g, 1, 0.01)
    exp = p0 - 0.01 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(p, exp, rtol=0, atol=1e-15)
    assert p[0] == p0[0]
    p, m, v = O.adam(p, m, v, g, 2, 0.01)
    # bias-corrected moments of two equal gradients are g and g^2 again
    np.testing.assert_allclose(p, p0 - 0.02 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-14)


def test_bf16_rounding_mode_is_a_small_perturbation():
    """round_bf16 changes outputs by at most a few bf16 ulps of the
    activations, and not at all for inputs and activations that bf16 holds
    exactly (a network whose hidden layers are all zero)."""
    rng = np.random.default_rng(7)
    p = random_params(rng, 0.3)
    x = rng.uniform(-1, 1, size=(32, NI))
    y = O.mlp_forward(p, x)
    yb = O.mlp_forward(p, x, round_bf16=True)
    d = np.abs(yb - y)
    assert d.max() > 0
    assert d.max() < 3e-2 * (1 + np.abs(y).max())
    W1, b1, W2, b2, W3, b3 = split(p.copy())
    p0 = join(np.zeros_like(W1), np.zeros_like(b1), W2, np.zeros_like(b2), W3, b3)
    # zero pre-activations: h1 = silu(0) = 0 and h2 = 0 exactly in both modes
    np.testing.assert_array_equal(O.mlp_forward(p0, x), O.mlp_forward(p0, x, round_bf16=True))


def test_cosine_schedule_endpoints_midpoint_and_shape():
    """The step size starts at lr, ends at lr / 100, is their mean half way
    (cos(pi/2) = 0), falls monotonically, and its steps are symmetric about
    the middle (cos(pi - a) = -cos(a)): lr(s) + lr(S-1-s) = lr + lr/100."""
    lr, S = 3e-3, 101
    lrs = np.array([O.lr_cosine(lr, S, s) for s in range(S)])
    assert lrs[0] == pytest.approx(lr, rel=1e-15)
    assert lrs[-1] == pytest.approx(lr / 100, rel=1e-13)
    assert lrs[50] == pytest.approx((lr + lr / 100) / 2, rel=1e-13)
    assert np.all(np.diff(lrs) < 0)
    np.testing.assert_allclose(lrs + lrs[::-1], lr + lr / 100, rtol=1e-13)
    assert O.lr_cosine(lr, 1, 0) == lr
