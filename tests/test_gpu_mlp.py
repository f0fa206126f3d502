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
def test_learned_tuner_gain(gpu, orc):
    """Trained on measured times of random batches, the model ranks held-out
    configurations; the learned tuner times 3 of ~100 candidates and its
    choice is compared with the paper's rule (shuffle_6, default mapping) and
    with exhaustive search. Outputs stay bit-exact with the oracle."""
    from paper_2408_06213_amd import learned, workloads

    rng = np.random.default_rng(7)
    say("learned: collect")
    X, y, _ = learned.collect(gpu, to_dev, rng, nbatch=12, ncand=30)
    net, loss = learned.train(gpu, to_dev, X, y, steps=3000, lr=3e-3, hidden=64)
    assert loss < np.var(y)  # better than predicting the mean
    gains, found = [], []
    for b in range(3):
        sizes = learned.random_batch(rng)
        off = workloads.csr_offsets(sizes)
        data = workloads.iota_segments(sizes)
        d, d_off = to_dev(data), to_dev(off)
        say("learned: held-out batch", b, sizes.size)
        plan = gpu.Plan(off, 4)
        rep = gpu.brr_plan_autotune_learned(plan, net, 3, d, d_off, seed=2, inst_base=0)
        assert rep.candidates == 4 and rep.ms_best <= rep.ms_default
        gains.append(rep.ms_default / rep.ms_best)
        ex = gpu.Plan(off, 4)
        full = ex.autotune(d, d_off, seed=2, inst_base=0)
        found.append(full.ms_best / rep.ms_best)
        ex.close()
        gpu.check(gpu.brr_shuffle_batched(d, d_off, sizes.size, 4, plan, 2, 0))
        sched = plan.schedule()
        want = data.copy()
        osched = orc.Schedule.from_segments(sched.steps(), tail=bool(sched.tail), u_tail=sched.u_tail)
        assert orc.shuffle_batched(want, off, osched, 2, 0) == 0
        assert np.array_equal(to_host(d), want)
        plan.close()
    print("learned tuner: gain over shuffle_6", gains, "best-found ratio", found)
    assert min(gains) >= 1.0
