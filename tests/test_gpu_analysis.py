"""delta_eff(rho) of particles and pairs from GPU runs near the paper's
critical point (Sec. 5.3, d = 0.25, p_c = 0.125141): the densities are the
GPU's recorded counts (bit-exact against the oracle elsewhere); here the
effective exponents must behave as at a critical point at this small scale:
finite, between the saturating (0) and the diffusive (1/2) limits."""
import numpy as np
import pytest
import torch

from paper_1301_6082_amd import analysis as an

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def curves():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return an.run_near_pc(0.125141, 0.25, L=1 << 14, runs=16, planes=1, steps=20000)


def test_particle_and_pair_exponents_near_pc(curves):
    assert np.all(curves.rho_pair <= curves.rho)
    assert curves.times[0] == 1 and 0.5 < curves.rho[0] < 1.0   # first record after one step
    for name, (t, r, d) in (("particles", curves.particle(4)), ("pairs", curves.pair(4))):
        late = t > 2000
        print(f"[delta_eff] {name}: late median {np.median(d[late]):.3f}, "
              f"rho {r[late][0]:.3g}..{r[late][-1]:.3g}", flush=True)
        assert late.sum() >= 10
        assert np.all(np.isfinite(d))
        assert 0.05 < np.median(d[late]) < 0.45, name
    delta, _ = an.extrapolate(*curves.particle(4)[1:], rho_max=0.2)
    assert np.isfinite(delta)


def test_mask_bit_comparison_runs_and_is_exact_at_quarter_rates():
    """At rates in quarters m = 2 and m = 4 fire on the same bits (pinned in
    the oracle), so the two curves coincide; elsewhere they are two valid
    realizations with finite deviations."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    curves, dev = an.compare_mask_bits(0.25, 0.5, (2, 4), L=1 << 12, runs=4, steps=500)
    np.testing.assert_array_equal(curves[2].rho, curves[4].rho)
    assert dev[2] == 0.0
    curves, dev = an.compare_mask_bits(0.13, 0.3, (2, 4), L=1 << 12, runs=4, steps=500)
    assert not np.array_equal(curves[2].rho, curves[4].rho)
    assert np.isfinite(dev[2]) and dev[4] == 0.0
