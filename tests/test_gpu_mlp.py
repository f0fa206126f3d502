"""The model's HIP forward/backward/Adam kernels against the float64
reference, and what the trained model gains over the paper's rule."""
import math

import numpy as np
import pytest

from conftest import say, to_dev, to_host
from oracle import mlp

pytestmark = pytest.mark.gpu


def make_net(gpu, n_in=16, h=32, seed=3):
    return gpu.MLP(n_in, h, seed)


def test_forward_and_gradients_match_reference(gpu):
    import torch

    rng = np.random.default_rng(1)
    n_in, h, B = 16, 32, 300
    net = make_net(gpu, n_in, h)
    x = rng.normal(size=(B, n_in)).astype(np.float32)
    t = rng.normal(size=B).astype(np.float32)
    d_x, d_t = to_dev(x), to_dev(t)
    d_y = torch.empty(B, dtype=torch.float32, device="cuda")
    say("mlp forward")
    net.forward(d_x, B, d_y)
    p = net.params().astype(np.float64)
    y_ref = mlp.forward(p, x.astype(np.float64), n_in, h)
    # fp32 dot products of length <= 32: relative error well under 1e-5
    assert np.allclose(to_host(d_y), y_ref, rtol=1e-4, atol=1e-5)
    say("mlp backward")
    d_loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.backward(d_x, d_t, B, d_loss)
    torch.cuda.synchronize()
    g = net.grads().astype(np.float64)
    g_ref = mlp.grad(p, x.astype(np.float64), t.astype(np.float64), n_in, h)
    # fp32 sums over a batch of 300: tolerance relative to the gradient scale
    scale = np.abs(g_ref).max()
    assert np.allclose(g, g_ref, rtol=1e-3, atol=1e-4 * scale)
    assert math.isclose(float(d_loss.item()), mlp.loss(p, x, t, n_in, h), rel_tol=1e-4)
    say("mlp adam")
    net.adam_step(0.01)
    torch.cuda.synchronize()
    p1, _, _ = mlp.adam(p, g_ref, np.zeros_like(p), np.zeros_like(p), 1, 0.01)
    assert np.allclose(net.params(), p1, rtol=1e-4, atol=1e-5)
    net.close()


def test_adam_moments_over_many_steps(gpu):
    """Eight successive backward + Adam steps on the device against the
    float64 reference carrying its own first and second moments and step
    count: at every step the device gradient matches the reference gradient
    at the device's current parameters, and the device parameters match the
    reference's Adam trajectory fed those gradients (bias corrections for
    steps 1..8, moments accumulated across steps)."""
    import torch

    rng = np.random.default_rng(5)
    n_in, h, B, lr = 16, 32, 200, 0.02
    net = make_net(gpu, n_in, h, seed=9)
    x = rng.normal(size=(B, n_in)).astype(np.float32)
    t = rng.normal(size=B).astype(np.float32)
    d_x, d_t = to_dev(x), to_dev(t)
    p_ref = net.params().astype(np.float64)
    m = np.zeros_like(p_ref)
    v = np.zeros_like(p_ref)
    for step in range(1, 9):
        say("mlp adam step", step)
        p_dev = net.params().astype(np.float64)
        net.backward(d_x, d_t, B)
        torch.cuda.synchronize()
        g = net.grads().astype(np.float64)
        g_ref = mlp.grad(p_dev, x.astype(np.float64), t.astype(np.float64), n_in, h)
        assert np.allclose(g, g_ref, rtol=1e-3, atol=1e-4 * np.abs(g_ref).max()), step
        net.adam_step(lr)
        torch.cuda.synchronize()
        p_ref, m, v = mlp.adam(p_ref, g, m, v, step, lr)
        # each update moves a parameter by at most ~lr; fp32 rounding of the
        # moments and of the parameters themselves stays far below 1e-5
        assert np.allclose(net.params(), p_ref, rtol=1e-4, atol=1e-5), step
    net.close()


def test_training_fits_a_smooth_target(gpu):
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, size=(512, 16)).astype(np.float32)
    y = (np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2]).astype(np.float32)
    net = make_net(gpu, 16, 32, seed=4)
    say("mlp train")
    start = mlp.loss(net.params().astype(np.float64), X.astype(np.float64), y, 16, 32)
    final = net.train(to_dev(X), to_dev(y), 512, 2000, 3e-3)
    assert final < 0.05 * start
    net.close()


@pytest.mark.slow
def test_learned_model_held_out(gpu, orc):
    """What the trained network gains, measured on batches it never saw.
    Trained on measured times of random batches (each batch's candidates
    relative to their mean), the model ranks every candidate configuration
    (schedule x wavefront limit) of 8 fresh random batches; each
    candidate's time is the median of 7 single runs. Checked: the learned
    tuner, which times the shuffle_6 default and the model's top 3 (4
    configurations), picks a configuration within 10% on average (15% at
    worst) of the exhaustive tuner's pick (29 timed): the network buys an
    eighth of the tuning runs at that cost; and its pick is never slower
    than the default beyond twice the measured spread. Reported, not
    asserted: the model's Spearman rank correlation with the measured times
    (weak, about 0.3: most candidates lie within the run-to-run spread of
    each other) and the gain over the default (within the spread on most
    batches: the analytic default is close to the best). Outputs under the
    learned choice stay bit-exact with the oracle."""
    from paper_2408_06213_amd import learned, workloads

    rng = np.random.default_rng(7)
    say("learned: collect")
    X, y, _ = learned.collect(gpu, to_dev, rng, nbatch=16, ncand=40)
    net, loss = learned.train(gpu, to_dev, X, y, steps=4000, lr=3e-3, hidden=64)
    print("train mse", loss, "target variance", float(np.var(y)))
    assert loss < np.var(y)  # better than predicting the mean
    say("learned: held-out evaluation")
    rows = learned.evaluate(gpu, to_dev, net, rng, nbatch=8, reps=7)
    for r in rows:
        print("held-out", {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()})
    rho = np.array([r["spearman"] for r in rows])
    quality = np.array([r["learned_vs_exhaustive"] for r in rows])
    gain = np.array([r["gain_learned_vs_default"] for r in rows])
    spread = np.array([max(r["learned_spread"], r["default_spread"]) for r in rows])
    print("mean spearman", rho.mean(), "learned/exhaustive", quality, "gain", gain,
          "spread", spread, "significant gains", int(np.sum(gain > 1 + 2 * spread)))
    # near the exhaustive tuner's pick at an eighth of its tuning runs
    assert quality.mean() >= 0.9 and quality.min() >= 0.85, quality
    assert all(4 * r["learned_timed"] <= r["exhaustive_timed"] for r in rows)
    # never measurably slower than the shuffle_6 default
    assert np.all(gain >= 1 / (1 + 2 * spread)), (gain, spread)
    # outputs under a learned choice stay bit-exact
    sizes = learned.random_batch(rng)
    off = workloads.csr_offsets(sizes)
    data = workloads.iota_segments(sizes)
    d, d_off = to_dev(data), to_dev(off)
    plan = gpu.Plan(off, 4)
    gpu.brr_plan_autotune_learned(plan, net, 3, d, d_off, seed=2, inst_base=0)
    gpu.check(gpu.brr_shuffle_batched(d, d_off, sizes.size, 4, plan, 2, 0))
    sched = plan.schedule()
    want = data.copy()
    osched = orc.Schedule.from_segments(sched.steps(), tail=bool(sched.tail), u_tail=sched.u_tail)
    assert orc.shuffle_batched(want, off, osched, 2, 0) == 0
    assert np.array_equal(to_host(d), want)
    plan.close()
    net.close()
