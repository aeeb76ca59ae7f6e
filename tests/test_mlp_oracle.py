"""Pins of the numpy MLP oracle: BF16 rounding against its integer
definition on hand-picked bit patterns, backward against central finite
differences, Adam's first step against its closed form, forward special
cases."""
import numpy as np
import pytest

from oracle import mlp
from paper_1612_01501_amd import inputs as I


def _bits(x):
    return np.array([x], np.uint32).view(np.float32)


@pytest.mark.parametrize("src,dst", [
    (0x3F800000, 0x3F80),   # 1.0 exact
    (0x3F808000, 0x3F80),   # tie, kept part even: down
    (0x3F818000, 0x3F82),   # tie, kept part odd: up to even
    (0x3F808001, 0x3F81),   # just above the tie: up
    (0x3F807FFF, 0x3F80),   # just below the tie: down
    (0xBFC00000, 0xBFC0),   # -1.5 exact
    (0x7F800000, 0x7F80),   # +inf
    (0xFF800000, 0xFF80),   # -inf
    (0x7F7FFFFF, 0x7F80),   # largest finite float rounds to +inf
    (0x00000001, 0x0000),   # smallest denormal: to +0
    (0x00008000, 0x0000),   # denormal tie, even: down
    (0x00018000, 0x0002),   # denormal tie, odd: up
    (0x80000000, 0x8000),   # -0
])
def test_bf16_round_bit_patterns(src, dst):
    r = mlp.bf16_round(_bits(src)).view(np.uint32)[0]
    assert r == (dst << 16), (hex(src), hex(r))


def test_bf16_round_nan_stays_nan():
    for src in (0x7FC00000, 0x7F800001, 0xFFFFFFFF):
        assert np.isnan(mlp.bf16_round(_bits(src))[0])


def test_bf16_round_is_nearest():
    x = np.random.default_rng(1).normal(0, 100, 20000).astype(np.float32)
    r = mlp.bf16_round(x).astype(np.float64)
    ulp = np.abs(r) * 2.0 ** -7
    assert np.all(np.abs(r - x) <= 0.5 * ulp + 1e-45)


def test_backward_matches_finite_differences():
    w = I.mlp_init_params(11).astype(np.float64)
    w += np.random.default_rng(2).normal(0, 0.05, w.shape)     # non-zero biases too
    x, t = I.mlp_batch(7, 3)
    _, g = mlp.loss_and_grad(w, x, t)
    rs = np.random.default_rng(4)
    idx = np.concatenate([rs.choice(mlp.N_PARAMS, 60, replace=False),
                          np.arange(2048, 2048 + 5), np.arange(mlp.N_PARAMS - 16, mlp.N_PARAMS)])
    h = 1e-6
    for k in idx:
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        num = (mlp.loss_and_grad(wp, x, t)[0] - mlp.loss_and_grad(wm, x, t)[0]) / (2 * h)
        assert g[k] == pytest.approx(num, rel=1e-5, abs=1e-9), k


def test_padding_outputs_carry_no_gradient():
    w = I.mlp_init_params(12).astype(np.float64)
    x, t = I.mlp_batch(5, 5)
    _, g = mlp.loss_and_grad(w, x, t)
    gp = mlp.unpack(g)
    assert np.all(gp["W3"][14:] == 0) and np.all(gp["b3"][14:] == 0)


def test_adam_first_step_closed_form():
    """After one step m_hat = g and v_hat = g^2, so w moves by lr*g/(|g|+eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    w, m, v = mlp.adam_step(np.ones(4), np.zeros(4), np.zeros(4), g, 1, lr=0.01)
    np.testing.assert_allclose(w, 1.0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_forward_special_cases():
    p = {name: np.zeros(shp) for name, shp in mlp.SHAPES}
    p["b3"] = np.arange(16.0)
    x = np.random.default_rng(6).normal(0, 1, (3, 16))
    y, _ = mlp.forward(mlp.pack(p), x)
    np.testing.assert_array_equal(y, np.tile(np.arange(16.0), (3, 1)))     # silu(0) = 0
    # a chain that passes x0 through both SiLUs; for large inputs silu(z) ~ z
    p["b3"][:] = 0.0
    p["W1"][0, 0] = p["W2"][0, 0] = p["W3"][0, 0] = 1.0
    x = np.zeros((1, 16))
    x[0, 0] = 40.0
    y, _ = mlp.forward(mlp.pack(p), x)
    assert y[0, 0] == pytest.approx(40.0, rel=1e-15)
    x[0, 0] = -40.0
    y, _ = mlp.forward(mlp.pack(p), x)
    assert abs(y[0, 0]) < 1e-15


def test_bf16_mode_close_to_exact():
    w = I.mlp_init_params(13).astype(np.float64)
    x, t = I.mlp_batch(64, 7)
    y0, _ = mlp.forward(w, x)
    y1, _ = mlp.forward(w, x, bf16=True)
    assert np.abs(y1 - y0).max() <= 0.05 * np.abs(y0).max()
    l0, g0 = mlp.loss_and_grad(w, x, t)
    l1, g1 = mlp.loss_and_grad(w, x, t, bf16=True)
    assert abs(l1 - l0) <= 0.02 * l0
    assert np.linalg.norm(g1 - g0) <= 0.05 * np.linalg.norm(g0)
