"""GPU parity of the density surrogate's kernels (forward, gradient, Adam)
against the numpy oracle, through the C ABI.

Tolerances. Both sides round the operands of every product to bfloat16, so
they differ only by float32 versus float64 accumulation (relative ~1e-6) and
by the rare bfloat16 rounding decision that flips between the two (one
bfloat16 ulp, 2^-8 relative, on one activation). For outputs of size O(1)
that bounds |dy| well below 5e-3; for gradients the relative L2 error stays
below 1e-2 and the direction (cosine) above 0.9999."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as mo

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pcpd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1301_6082_amd import pcpd as mod
    return mod


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = mo.features(rng.uniform(0.05, 0.25, n), rng.choice([0.1, 0.5, 0.9], n),
                    10.0 ** rng.uniform(0, 6, n))
    t = -1.5 * x[:, 2] * x[:, 0] + 0.4 * x[:, 1] - 0.2 + 0.05 * rng.normal(size=n)
    m = (rng.random(n) < 0.85).astype(np.float64)
    return x, t, m


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _theta(seed):
    # float32-representable parameters so that both sides start identical
    return mo.init_params(seed).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 4097])
def test_forward_matches_oracle(pcpd, n):
    theta = _theta(1)
    x, _, _ = _data(n, n)
    x = x.astype(np.float32).astype(np.float64)
    net = pcpd.Surrogate(seed=0)
    net.set_params(theta)
    np.testing.assert_array_equal(net.params(), theta.astype(np.float32))
    y = net.predict(_cuda(x)).cpu().numpy().astype(np.float64)
    ref, _ = mo.forward(theta, x)
    err = np.abs(y - ref)
    print(f"[mlp fwd] n={n} max|dy|={err.max():.2e}", flush=True)
    assert err.max() < 5e-3
    assert np.median(err) < 1e-4


@pytest.mark.parametrize("n", [200, 777, 4096])
def test_gradient_matches_oracle(pcpd, n):
    theta = _theta(2)
    x, t, m = _data(n, 10 + n)
    x = x.astype(np.float32).astype(np.float64)
    t = t.astype(np.float32).astype(np.float64)
    net = pcpd.Surrogate(seed=0)
    net.set_params(theta)
    loss, g = net.grads(_cuda(x), _cuda(t), _cuda(m))
    rl, rg = mo.loss_and_grad(theta, x, t, m)
    g = g.astype(np.float64)
    assert abs(loss - rl) <= 1e-4 * max(1.0, rl)
    o = 0
    for name, shape in mo.SIZES:
        k = int(np.prod(shape))
        a, b = g[o:o + k], rg[o:o + k]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        print(f"[mlp grad] n={n} {name}: rel L2 {rel:.2e}", flush=True)
        assert rel < 1e-2, name
        o += k
    cos = g @ rg / np.linalg.norm(g) / np.linalg.norm(rg)
    assert cos > 0.9999


def test_mask_all_zero_gives_zero_gradient(pcpd):
    theta = _theta(3)
    x, t, _ = _data(130, 3)
    net = pcpd.Surrogate(seed=0)
    net.set_params(theta)
    loss, g = net.grads(_cuda(x), _cuda(t), _cuda(np.zeros(130)))
    assert loss == 0.0 and not np.any(g)


def test_adam_steps_match_oracle(pcpd):
    """Three Adam steps on both sides from the same start. Early Adam steps
    move each parameter by about lr * sign(gradient), so the parameters must
    agree to a small fraction of lr except where a gradient component is so
    close to zero that its sign is decided by rounding."""
    theta = _theta(4)
    x, t, m = _data(512, 4)
    x = x.astype(np.float32).astype(np.float64)
    t = t.astype(np.float32).astype(np.float64)
    lr = 1e-3
    net = pcpd.Surrogate(seed=0)
    net.set_params(theta)
    opt = mo.Adam(mo.N_PARAMS, lr=lr)
    th = theta.copy()
    xs, ts, ms = _cuda(x), _cuda(t), _cuda(m)
    for step in range(3):
        loss = net.train_step(xs, ts, ms, lr=lr, want_loss=True)
        rl, rg = mo.loss_and_grad(th, x, t, m)
        assert abs(loss - rl) <= 1e-3 * max(1.0, rl), step
        th = opt.step(th, rg)
        gpu = net.params().astype(np.float64)
        close = np.abs(gpu - th) <= 0.05 * lr
        print(f"[mlp adam] step {step}: {close.mean():.4f} of parameters within 0.05 lr", flush=True)
        assert close.mean() > 0.99, step
        assert np.abs(gpu - th).max() <= 2.5 * lr * (step + 1)


def test_training_on_gpu_reduces_the_loss(pcpd):
    x, t, m = _data(8192, 5)
    net = pcpd.Surrogate(seed=7)
    xs, ts, ms = _cuda(x), _cuda(t), _cuda(m)
    l0 = net.grads(xs, ts, ms)[0]
    for _ in range(300):
        net.train_step(xs, ts, ms, lr=2e-3)
    l1 = net.grads(xs, ts, ms)[0]
    print(f"[mlp train] loss {l0:.4f} -> {l1:.4f}", flush=True)
    assert l1 < 0.1 * l0
