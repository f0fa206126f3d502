"""Pins of the float64 model reference and of the plan features (CPU)."""
import math

import numpy as np

from oracle import mlp


def test_reference_gradient_is_the_derivative():
    """The chain-rule gradient equals central finite differences of the
    loss, for every parameter."""
    rng = np.random.default_rng(0)
    n_in, h = 6, 9
    npar = n_in * h + h + h * h + h + h + 1
    p = rng.normal(size=npar) * 0.5
    x = rng.normal(size=(17, n_in))
    t = rng.normal(size=17)
    g = mlp.grad(p, x, t, n_in, h)
    ng = mlp.numeric_grad(p, x, t, n_in, h, np.arange(npar))
    assert np.allclose(g, ng, rtol=1e-6, atol=1e-8)


def test_reference_adam_first_step():
    """At step 1 the bias-corrected moments are g and g^2, so each parameter
    moves by lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p, m, v = mlp.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.1)
    assert np.allclose(p, -0.1 * g / (np.abs(g) + 1e-8))


def test_plan_features_by_hand():
    from paper_2408_06213_amd import brr

    # one shuffle of 256 u32 under shuffle_6: 42 batches of 6 dice + 1 of 3
    f = brr.brr_plan_features(np.array([0, 256], np.uint64), 4, None, 512)
    want = [math.log2(257) / 32, 1 / 16, 0.5, 0, 1, 0, 0, 0, 8 / 32, 0, 43 / 255, 252 / 255, 0,
            6 / 8, math.log2(512) / 10, 1]
    assert np.allclose(f, want, atol=1e-6)
    # k = 1 schedule, two sizes in different bands, u64
    off = np.array([0, 100, 100 + 40000], np.uint64)
    f = brr.brr_plan_features(off, 8, brr.brr_schedule_paper(1), 64)
    steps = 99 + 39999
    assert f[2] == 1.0 and math.isclose(f[10], 1.0)  # one word per step
    assert math.isclose(f[12], 1.0) and f[11] == 0  # every die in batches of one
    assert math.isclose(f[4], 100 / 40100, rel_tol=1e-6) and math.isclose(f[6], 40000 / 40100, rel_tol=1e-6)
    assert f[15] == 0 and steps == 40098
