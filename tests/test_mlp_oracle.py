"""Pins the surrogate's numpy oracle against independent implementations:
PyTorch's bfloat16 conversion, its tanh GELU, a float64 torch network with
autograd, torch's Adam, and central finite differences."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as mo


def test_parameter_count():
    assert mo.N_PARAMS == 33665


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    vals = np.concatenate([
        rng.normal(size=5000) * 10.0 ** rng.integers(-30, 30, size=5000),
        rng.uniform(-3, 3, size=2000),
        np.array([0.0, -0.0, 1.0, -1.0, 3.0e38, -3.0e38, 1e-40, -1e-40, np.inf, -np.inf]),
    ]).astype(np.float32)
    # exact ties: bfloat16 grid points plus half an ulp (even and odd mantissas)
    base = (np.arange(1, 400, dtype=np.uint32) << 16) | np.uint32(0x3F800000)
    ties = (base | np.uint32(0x8000)).view(np.float32)
    vals = np.concatenate([vals, ties])
    ours = mo.bf16(vals)
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(ours, ref)


def test_gelu_matches_torch_tanh_form():
    z = np.linspace(-8, 8, 2001)
    ref = torch.nn.functional.gelu(torch.from_numpy(z), approximate="tanh").numpy()
    np.testing.assert_allclose(mo.gelu(z), ref, rtol=1e-14, atol=1e-14)
    # derivative against torch autograd
    zt = torch.from_numpy(z).requires_grad_(True)
    torch.nn.functional.gelu(zt, approximate="tanh").sum().backward()
    np.testing.assert_allclose(mo.gelu_grad(z), zt.grad.numpy(), rtol=1e-12, atol=1e-12)


def _torch_net(theta):
    P = {k: torch.from_numpy(np.array(v, dtype=np.float64)) for k, v in mo.unpack(theta).items()}
    for v in P.values():
        v.requires_grad_(True)
    return P


def _torch_forward(P, x):
    g = lambda z: torch.nn.functional.gelu(z, approximate="tanh")
    h1 = g(x @ P["W1"].T + P["b1"])
    h2 = g(h1 @ P["W2"].T + P["b2"])
    h3 = g(h2 @ P["W3"].T + P["b3"])
    return h3 @ P["w4"] + P["b4"][0]


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = np.stack([rng.uniform(0.2, 1.0, n), rng.choice([0.1, 0.5, 0.9], n),
                  rng.uniform(0, 1, n)], axis=1)
    t = -2.0 * x[:, 2] * x[:, 0] + 0.3 * x[:, 1] - 0.5
    m = (rng.random(n) < 0.8).astype(np.float64)
    return x, t, m


def test_forward_and_gradient_match_torch_float64():
    theta = mo.init_params(3)
    x, t, m = _data(257, 1)
    y, _ = mo.forward(theta, x, bf=False)
    P = _torch_net(theta)
    xt = torch.from_numpy(x)
    yt = _torch_forward(P, xt)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    mt = torch.from_numpy(m)
    loss_t = (mt * (yt - torch.from_numpy(t)) ** 2).sum() / mt.sum()
    loss_t.backward()
    ref = np.concatenate([P[name].grad.numpy().reshape(-1) for name, _ in mo.SIZES])
    loss, grad = mo.loss_and_grad(theta, x, t, m, bf=False)
    assert abs(loss - float(loss_t.detach())) < 1e-12
    np.testing.assert_allclose(grad, ref, rtol=1e-10, atol=1e-13)


def test_gradient_matches_finite_differences():
    theta = mo.init_params(4)
    x, t, m = _data(64, 2)
    _, grad = mo.loss_and_grad(theta, x, t, m, bf=False)
    rng = np.random.default_rng(9)
    idx = np.concatenate([rng.choice(mo.N_PARAMS, 40, replace=False), [0, 383, 384, 33664]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mo.loss_and_grad(tp, x, t, m, bf=False)[0] - mo.loss_and_grad(tm, x, t, m, bf=False)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-7 + 1e-5 * abs(grad[i]), (i, fd, grad[i])


def test_bf16_rounding_perturbs_only_slightly():
    theta = mo.init_params(5)
    x, t, m = _data(512, 3)
    y32, _ = mo.forward(theta, x, bf=False)
    y16, _ = mo.forward(theta, x, bf=True)
    assert np.abs(y16 - y32).max() < 0.02
    _, g32 = mo.loss_and_grad(theta, x, t, m, bf=False)
    _, g16 = mo.loss_and_grad(theta, x, t, m, bf=True)
    cos = g16 @ g32 / np.linalg.norm(g16) / np.linalg.norm(g32)
    assert cos > 0.999


def test_masked_rows_do_not_contribute():
    theta = mo.init_params(6)
    x, t, m = _data(100, 4)
    l1, g1 = mo.loss_and_grad(theta, x, t, m)
    t2 = t.copy()
    t2[m == 0] += 100.0
    l2, g2 = mo.loss_and_grad(theta, x, t2, m)
    assert l1 == l2
    np.testing.assert_array_equal(g1, g2)


def test_adam_matches_torch():
    theta = mo.init_params(7)
    x, t, m = _data(128, 5)
    opt = mo.Adam(mo.N_PARAMS, lr=1e-3)
    tp = torch.from_numpy(theta.copy()).requires_grad_(True)
    topt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    th = theta.copy()
    for _ in range(5):
        _, g = mo.loss_and_grad(th, x, t, m, bf=False)
        th = opt.step(th, g)
        topt.zero_grad()
        tp.grad = torch.from_numpy(mo.loss_and_grad(tp.detach().numpy().copy(), x, t, m, bf=False)[1])
        topt.step()
    np.testing.assert_allclose(th, tp.detach().numpy(), rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("seed", [1, 2])
def test_training_reduces_the_loss(seed):
    theta = mo.init_params(seed)
    x, t, m = _data(256, seed)
    opt = mo.Adam(mo.N_PARAMS, lr=3e-3)
    l0 = mo.loss_and_grad(theta, x, t, m)[0]
    for _ in range(60):
        _, g = mo.loss_and_grad(theta, x, t, m)
        theta = opt.step(theta, g)
    assert mo.loss_and_grad(theta, x, t, m)[0] < 0.2 * l0
