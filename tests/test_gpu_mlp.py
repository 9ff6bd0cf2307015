"""GPU parity of the density surrogate's kernels (forward, gradient, Adam)
against the numpy oracle, through the C ABI.

Tolerances, element by element. Both sides round the operands of every
product to bfloat16 at the same points, so they differ only by float32 versus
float64 accumulation (a few 1e-7 of an element's scale, the sum of the
magnitudes of its terms) and by the rare bfloat16 rounding decision that falls
the other way on one side (one bfloat16 ulp, 2^-8 relative, on one operand).
Every output, gradient element and parameter is compared on its own."""
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
    share, worst = _elementwise(y, ref, mo.forward_scale(theta, x), f"fwd n={n}")
    assert share <= max(FLIP_SHARE, 1.0 / n)
    assert worst <= FLIP


# Element-wise bounds, relative to the per-element scale of the oracle (the sum
# of the magnitudes of the terms the element adds up; mlp_oracle.grad_scale,
# forward_scale): float32 accumulation of at most a few hundred partial sums
# moves an element by well under EXACT of its scale; an element where one side
# rounds an operand to the other neighbouring bfloat16 value (a tie decided by
# the last float32 bit) moves by at most FLIP, and only a small share of the
# elements may do so.
EXACT = 2e-5
FLIP = 2.0 ** -6
FLIP_SHARE = 0.01


def _elementwise(a, b, scale, tag):
    """(share of elements beyond EXACT, largest relative error) of a vs b."""
    rel = np.abs(a - b) / (scale + 1e-30)
    share = float((rel > EXACT).mean())
    print(f"[mlp elem] {tag}: max rel {rel.max():.2e}, 99.9% {np.quantile(rel, 0.999):.2e}, "
          f"share beyond {EXACT:g}: {share:.2e}", flush=True)
    return share, float(rel.max())


@pytest.mark.parametrize("n", [200, 777, 4096])
def test_gradient_matches_oracle_elementwise(pcpd, n):
    theta = _theta(2)
    x, t, m = _data(n, 10 + n)
    x = x.astype(np.float32).astype(np.float64)
    t = t.astype(np.float32).astype(np.float64)
    net = pcpd.Surrogate(seed=0)
    net.set_params(theta)
    loss, g = net.grads(_cuda(x), _cuda(t), _cuda(m))
    rl, rg = mo.loss_and_grad(theta, x, t, m)
    scale = mo.grad_scale(theta, x, t, m)
    g = g.astype(np.float64)
    assert abs(loss - rl) <= 1e-5 * max(1.0, rl)
    o = 0
    for name, shape in mo.SIZES:
        k = int(np.prod(shape))
        share, worst = _elementwise(g[o:o + k], rg[o:o + k], scale[o:o + k], f"n={n} {name}")
        assert share <= FLIP_SHARE, name
        assert worst <= FLIP, name
        o += k


def _grad_unrounded_dz3(theta, x, t, m):
    """The oracle's gradient with one rounding point moved: dz3 enters the
    W3 products unrounded (a planted mistake, on the CPU)."""
    y, c = mo.forward(theta, x)
    P, r = c["P"], c["r"]
    dy = 2.0 * (y - t) * m / m.sum()
    dz3 = np.outer(dy, r(P["w4"])) * mo.gelu_grad(c["z3"])
    dW3 = dz3.T @ r(c["h2"])
    dh2 = dz3 @ r(P["W3"])
    dz2 = dh2 * mo.gelu_grad(c["z2"])
    dW2 = r(dz2).T @ r(c["h1"])
    return dW3.reshape(-1), dW2.reshape(-1)


def test_elementwise_bound_catches_a_moved_rounding_point(pcpd):
    """The element-wise bound is tight enough to see a rounding point placed
    differently: against an oracle that skips the bfloat16 rounding of dz3,
    the GPU's weight gradients break it."""
    n = 200
    theta = _theta(2)
    x, t, m = _data(n, 10 + n)
    x = x.astype(np.float32).astype(np.float64)
    t = t.astype(np.float32).astype(np.float64)
    net = pcpd.Surrogate(seed=0)
    net.set_params(theta)
    _, g = net.grads(_cuda(x), _cuda(t), _cuda(m))
    g = g.astype(np.float64)
    scale = mo.grad_scale(theta, x, t, m)
    offs = {}
    o = 0
    for name, shape in mo.SIZES:
        offs[name] = (o, o + int(np.prod(shape)))
        o = offs[name][1]
    dW3, dW2 = _grad_unrounded_dz3(theta, x, t, m)
    for name, planted in (("W3", dW3), ("W2", dW2)):
        a, b = offs[name]
        share, _ = _elementwise(g[a:b], planted, scale[a:b], f"planted {name}")
        assert share > FLIP_SHARE, name


def test_mask_all_zero_gives_zero_gradient(pcpd):
    theta = _theta(3)
    x, t, _ = _data(130, 3)
    net = pcpd.Surrogate(seed=0)
    net.set_params(theta)
    loss, g = net.grads(_cuda(x), _cuda(t), _cuda(np.zeros(130)))
    assert loss == 0.0 and not np.any(g)


def test_adam_steps_match_oracle(pcpd):
    """Three Adam steps on both sides from the same start, compared element by
    element. An Adam step moves a parameter by lr * mhat / (sqrt(vhat) + eps);
    where the two gradients agree to EXACT of their scale the steps agree to a
    small fraction of lr. Only parameters whose gradient is itself within a few
    EXACT of zero (relative to its scale) may step differently, by at most
    2 lr per step."""
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
    tiny = np.zeros(mo.N_PARAMS, dtype=bool)   # gradient ~0 at this or an earlier step
    for step in range(3):
        loss = net.train_step(xs, ts, ms, lr=lr, want_loss=True)
        rl, rg = mo.loss_and_grad(th, x, t, m)
        scale = mo.grad_scale(th, x, t, m)
        assert abs(loss - rl) <= 1e-5 * max(1.0, rl), step
        th = opt.step(th, rg)
        gpu = net.params().astype(np.float64)
        diff = np.abs(gpu - th)
        # float32 master copy: a few float32 ulps of the parameter (one rounding per
        # step) plus the step's own error
        ok = diff <= 1e-3 * lr + 2.0 ** -21 * np.abs(th)
        tiny |= np.abs(rg) <= 100 * EXACT * scale
        print(f"[mlp adam] step {step}: {ok.mean():.6f} of parameters within 1e-3 lr; "
              f"outside: {int((~ok).sum())}, of which gradient ~0: {int((~ok & tiny).sum())}; "
              f"max diff {diff.max() / lr:.2e} lr", flush=True)
        assert (ok | tiny).all(), step
        assert diff.max() <= 2.0 * lr * (step + 1)


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
