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


# Element-wise bounds. Gradients are compared relative to mlp_oracle.grad_scale,
# the magnitudes of all the terms an element is computed from, propagated
# through the backward chain: float32 evaluation of a dot product is off by a
# small multiple of the unit roundoff u = 2^-24 times the sum of the magnitudes
# of its terms, and an upstream sum that cancels passes that absolute error on.
# With rounding errors of random sign the multiple grows like the square root
# of the number of terms summed (here up to max(n, 128)), so an element must
# agree within exact_bound(n) = 8 sqrt(max(n, 128)) u of its scale. Where one
# side rounds an operand to the other neighbouring bfloat16 value (a tie
# decided by the last float32 bit), the elements that operand enters move by
# at most FLIP of their scale. One such activation of one row enters a whole
# row or column of a weight gradient (1/128 of its elements), so a handful of
# them moves a few percent of the elements: at most FLIP_SHARE of the elements
# (about six flipped activations) may lie beyond the exact bound. Forward
# outputs use forward_scale and EXACT.
EXACT = 2e-5
FLIP = 2.0 ** -6
FLIP_SHARE = 0.05


def exact_bound(n):
    return 8.0 * np.sqrt(max(n, mo.H)) * 2.0 ** -24


def _elementwise(a, b, scale, tag, bound=EXACT):
    """(share of elements beyond `bound`, largest relative error) of a vs b."""
    rel = np.abs(a - b) / (scale + 1e-30)
    share = float((rel > bound).mean())
    print(f"[mlp elem] {tag}: max rel {rel.max():.2e}, 99.9% {np.quantile(rel, 0.999):.2e}, "
          f"share beyond {bound:.2g}: {share:.2e}", flush=True)
    return share, float(rel.max())


@pytest.mark.parametrize("n", [128, 200, 777, 4096, 40000])
def test_gradient_matches_oracle_elementwise(pcpd, n):
    """n = 40000 is 625 tiles of 64 rows on the backward pass's 512
    workgroups: some workgroups sum two tiles into their partial."""
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
        share, worst = _elementwise(g[o:o + k], rg[o:o + k], scale[o:o + k], f"n={n} {name}",
                                    exact_bound(n))
        assert share <= FLIP_SHARE, name
        assert worst <= FLIP, name
        o += k


def _planted_grads(theta, x, t, m):
    """The oracle's weight gradients with one rounding point moved per layer
    (planted mistakes, on the CPU): dz3 enters the W3 product unrounded, dz2
    the W2 product, x the W1 sums."""
    y, c = mo.forward(theta, x)
    P, r = c["P"], c["r"]
    dy = 2.0 * (y - t) * m / m.sum()
    dz3 = np.outer(dy, r(P["w4"])) * mo.gelu_grad(c["z3"])
    dW3 = dz3.T @ r(c["h2"])
    dz2 = (r(dz3) @ r(P["W3"])) * mo.gelu_grad(c["z2"])
    dW2 = dz2.T @ r(c["h1"])
    dz1 = (r(dz2) @ r(P["W2"])) * mo.gelu_grad(c["z1"])
    dW1 = dz1.T @ np.asarray(x, dtype=np.float64)
    return {"W3": dW3.reshape(-1), "W2": dW2.reshape(-1), "W1": dW1.reshape(-1)}


def test_elementwise_bound_catches_a_moved_rounding_point(pcpd):
    """The element-wise bound is tight enough to see a rounding point placed
    differently in any layer: against an oracle that skips one bfloat16
    rounding (of dz3, of dz2 or of x), the GPU's gradient of that layer's
    weights breaks it."""
    n = 128
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
    for name, planted in _planted_grads(theta, x, t, m).items():
        a, b = offs[name]
        share, _ = _elementwise(g[a:b], planted, scale[a:b], f"planted {name}", exact_bound(n))
        assert share > FLIP_SHARE, name


def test_mask_all_zero_gives_zero_gradient(pcpd):
    theta = _theta(3)
    x, t, _ = _data(130, 3)
    net = pcpd.Surrogate(seed=0)
    net.set_params(theta)
    loss, g = net.grads(_cuda(x), _cuda(t), _cuda(np.zeros(130)))
    assert loss == 0.0 and not np.any(g)


def test_adam_steps_match_oracle(pcpd):
    """Three Adam steps, each checked element by element against the oracle's
    Adam applied to the same gradient: the GPU's own gradient at the GPU's
    current parameters (pcpd_mlp_grads runs the kernels of the training step
    on the same rows, so it is that step's gradient). This isolates the
    optimiser from the gradient, whose parity is tested above; what remains
    is float32 against float64 arithmetic in the update (a few float32 ulps of
    lr) and the rounding of the float32 master copy (half an ulp of the
    parameter). The loss of each step is also compared with the oracle's."""
    theta = _theta(4)
    x, t, m = _data(512, 4)
    x = x.astype(np.float32).astype(np.float64)
    t = t.astype(np.float32).astype(np.float64)
    lr = 1e-3
    net = pcpd.Surrogate(seed=0)
    net.set_params(theta)
    opt = mo.Adam(mo.N_PARAMS, lr=lr)
    xs, ts, ms = _cuda(x), _cuda(t), _cuda(m)
    before = net.params().astype(np.float64)
    for step in range(3):
        _, g = net.grads(xs, ts, ms)
        loss = net.train_step(xs, ts, ms, lr=lr, want_loss=True)
        rl, _ = mo.loss_and_grad(before, x, t, m)
        assert abs(loss - rl) <= 1e-5 * max(1.0, rl), step
        want = opt.step(before, g.astype(np.float64))
        after = net.params().astype(np.float64)
        diff = np.abs(after - want)
        bound = 1e-5 * lr + 2.0 ** -24 * np.abs(want)
        print(f"[mlp adam] step {step}: max |diff| {diff.max() / lr:.2e} lr, "
              f"max diff/bound {(diff / bound).max():.3f}", flush=True)
        assert (diff <= bound).all(), step
        before = after


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


def test_loss_call_and_row_limits(pcpd):
    """pcpd_mlp_loss (forward only) returns the loss of pcpd_mlp_grads and the
    oracle's, on more rows than a gradient call takes; a gradient call beyond
    PCPD_MLP_MAX_TRAIN_ROWS is refused before any device work."""
    theta = _theta(3)
    n = 70000
    x, t, m = _data(n, 77)
    x = x.astype(np.float32).astype(np.float64)
    t = t.astype(np.float32).astype(np.float64)
    net = pcpd.Surrogate(seed=0)
    try:
        net.set_params(theta)
        X, T, M = _cuda(x), _cuda(t), _cuda(m)
        lf = net.loss(X, T, M)
        lg, _ = net.grads(X, T, M)
        rl, _ = mo.loss_and_grad(theta, x, t, m)
        assert lf == lg
        assert abs(lf - rl) <= 1e-5 * max(1.0, rl)
        big = pcpd.MLP_MAX_TRAIN_ROWS + 1
        xb = torch.zeros((big, 3), dtype=torch.float32, device="cuda")
        tb = torch.zeros(big, dtype=torch.float32, device="cuda")
        assert net.loss(xb, tb) >= 0.0          # forward-only calls take it
        with pytest.raises(pcpd.PcpdError):
            net.grads(xb, tb)
    finally:
        net.close()
