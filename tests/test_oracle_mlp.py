"""Pins of the surrogate oracle (oracle/mlp.py) against facts it does not compute
itself: finite differences, closed forms of SiLU and of Adam's first steps, hand-worked
networks, bfloat16 rounding cases, and the particle-number invariant of the warm start."""
import math

import numpy as np
import pytest

from oracle import mlp


def _tiny(seed=0, width=6, depth=3):
    dims = mlp.layer_dims(width=width, depth=depth)
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.7, mlp.param_count(dims))
    X = rng.uniform(-1, 1, (5, mlp.D_IN))
    T = rng.normal(0, 1, (5, mlp.D_OUT))
    return dims, theta, X, T


def test_param_count_of_the_surrogate():
    # 4*128+128 + 2*(128*128+128) + 128*4+4
    assert mlp.param_count() == 34180


def test_gradient_matches_central_differences():
    """Every component of the reverse-mode gradient against a central difference of the
    loss (step 1e-6, FP64): agreement to 1e-7 relative to the gradient's max-norm."""
    dims, theta, X, T = _tiny()
    L, g = mlp.loss_and_grad(theta, X, T, dims)
    assert L == pytest.approx(mlp.loss(theta, X, T, dims), rel=1e-15)
    h = 1e-6
    fd = np.empty_like(theta)
    for i in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd[i] = (mlp.loss(tp, X, T, dims) - mlp.loss(tm, X, T, dims)) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-7 * np.abs(fd).max()


def test_gradient_of_full_width_network_on_sampled_components():
    dims = mlp.layer_dims()
    rng = np.random.default_rng(3)
    theta = rng.normal(0, 0.1, mlp.param_count(dims))
    X = rng.uniform(-1, 1, (9, 4))
    T = rng.normal(0, 1, (9, 4))
    _, g = mlp.loss_and_grad(theta, X, T, dims)
    h = 1e-6
    for i in rng.choice(len(theta), 60, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, X, T, dims) - mlp.loss(tm, X, T, dims)) / (2 * h)
        assert abs(g[i] - fd) <= 1e-8 + 1e-6 * abs(fd), i


def test_silu_closed_forms():
    assert mlp.silu(0.0) == 0.0
    assert mlp.dsilu(0.0) == 0.5
    assert mlp.silu(1.0) == pytest.approx(1.0 / (1.0 + math.exp(-1.0)), rel=1e-15)
    z = np.linspace(-8, 8, 33)
    # sigmoid(z) + sigmoid(-z) = 1  =>  silu(z) - silu(-z) = z
    assert np.allclose(mlp.silu(z) - mlp.silu(-z), z, rtol=0, atol=1e-14)
    assert mlp.silu(40.0) == pytest.approx(40.0, rel=1e-15)
    assert abs(mlp.silu(-40.0)) < 1e-15


def test_forward_of_hand_worked_network():
    """Width 1, depth 1: y_o = v_o silu(sum_i w_i x_i + c) + e_o."""
    dims = mlp.layer_dims(width=1, depth=1)
    w = np.array([0.5, -1.0, 0.25, 2.0])
    c = 0.1
    v = np.array([1.0, -2.0, 3.0, 0.5])
    e = np.array([0.0, 1.0, -1.0, 2.0])
    theta = np.concatenate([w, [c], v, e])
    x = np.array([[0.2, 0.4, -0.8, 0.3]])
    z = 0.5 * 0.2 - 1.0 * 0.4 + 0.25 * -0.8 + 2.0 * 0.3 + 0.1       # = 0.2
    s = z / (1 + math.exp(-z))
    want = v * s + e
    assert np.allclose(mlp.forward(theta, x, dims)[0], want, rtol=1e-15, atol=1e-15)


def test_loss_is_zero_with_zero_gradient_at_exact_fit():
    dims, theta, X, _ = _tiny(1)
    Y = mlp.forward(theta, X, dims)
    L, g = mlp.loss_and_grad(theta, X, Y, dims)
    assert L == 0.0 and not np.any(g)


def test_adam_first_steps_closed_form():
    """Bias correction makes step 1 move every parameter by lr g / (|g| + eps); after
    gradients g1 then g2: m_hat = (b1(1-b1) g1 + (1-b1) g2)/(1-b1^2), likewise v_hat."""
    rng = np.random.default_rng(7)
    th0 = rng.normal(size=11)
    g1, g2 = rng.normal(size=11), rng.normal(size=11)
    opt = mlp.Adam(11, lr=1e-3)
    th1 = opt.step(th0, g1)
    assert np.allclose(th1, th0 - 1e-3 * g1 / (np.abs(g1) + 1e-8), rtol=0, atol=1e-18)
    th2 = opt.step(th1, g2)
    mh = (0.9 * 0.1 * g1 + 0.1 * g2) / (1 - 0.81)
    vh = (0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2) / (1 - 0.999 ** 2)
    assert np.allclose(th2, th1 - 1e-3 * mh / (np.sqrt(vh) + 1e-8), rtol=0, atol=1e-17)


def test_training_reduces_the_loss():
    """Adam on a smooth target (two hundred full-batch steps, width 16) cuts the loss
    tenfold: the gradient points downhill."""
    dims = mlp.layer_dims(width=16, depth=2)
    rng = np.random.default_rng(11)
    theta = rng.normal(0, 0.4, mlp.param_count(dims))
    X = rng.uniform(-1, 1, (64, 4))
    T = np.stack([np.sin(X[:, 0]), X[:, 1] * X[:, 2], np.cos(X[:, 3]), X.sum(1) / 4], axis=1)
    opt = mlp.Adam(len(theta), lr=1e-2)
    L0 = mlp.loss(theta, X, T, dims)
    for _ in range(200):
        _, g = mlp.loss_and_grad(theta, X, T, dims)
        theta = opt.step(theta, g)
    assert mlp.loss(theta, X, T, dims) < 0.1 * L0


def test_bf16_rounding_cases():
    e = 2.0 ** -8
    assert mlp.bf16(1.0) == 1.0
    assert mlp.bf16(1 + e) == 1.0                      # tie -> even (1.0)
    assert mlp.bf16(1 + 3 * e) == 1 + 4 * e             # tie -> even (mantissa 2)
    assert mlp.bf16(1 + e + 2.0 ** -20) == 1 + 2 * e    # above the tie
    assert mlp.bf16(-2.5) == -2.5
    assert mlp.bf16(3.0e38) == pytest.approx(2.9975e38, rel=3e-3)
    x = np.random.default_rng(5).normal(size=1000)
    assert np.all(np.abs(mlp.bf16(x) - x) <= np.abs(x) * 2.0 ** -8)   # half an ulp of 7 stored bits


def test_bf16_forward_error_is_bounded():
    """bfloat16 operands perturb each product by at most 2^-8 relative."""
    dims = mlp.layer_dims()
    rng = np.random.default_rng(2)
    theta = rng.normal(0, 0.1, mlp.param_count(dims))
    X = rng.uniform(-1, 1, (32, 4))
    Y = mlp.forward(theta, X, dims)
    Yb = mlp.forward_bf16(theta, X, dims)
    assert 0 < np.abs(Yb - Y).max() <= 2e-2 * np.abs(Y).max()


def test_features_map_the_box_to_unit_cube():
    lo = mlp.features(1e-2, 0.05, 0.3, 0.0)
    hi = mlp.features(10.0, 0.5, 0.8, 1.0)
    assert np.allclose(lo, -1.0, atol=1e-15) and np.allclose(hi, 1.0, atol=1e-15)


def test_warm_profile_keeps_the_cold_particle_number():
    from oracle.couette import CouetteOracle
    o = CouetteOracle(R_in=1.0, R_out=2.5, N_R=40, ax1=(1, 4, 2), ax2=(0, 4, 2), Kn=0.3, u_in=0.3)
    rng = np.random.default_rng(4)
    Y = rng.normal(0, 0.3, (40, 4))
    cold = o.mass(o.equilibrium(1.0, 0.0, 0.0, 1.0))
    n, uR, uphi, T = mlp.warm_profile(Y, 0.3, o.dchi, float(np.sum(o.dchi)))
    assert not np.any(uR)
    assert o.mass(o.equilibrium(n, uR, uphi, T)) == pytest.approx(cold, rel=1e-14)
    # the targets invert the profile map (n before rescaling)
    t = mlp.targets(1 + Y[:, 0] / mlp.S_N, Y[:, 1] / mlp.S_U, uphi, T, 0.3)
    assert np.allclose(t[:, [0, 2, 3]], Y[:, [0, 2, 3]], rtol=0, atol=1e-13)
