"""GPU checks of the work predictor: the HIP forward, gradient and Adam
kernels against the float64 CPU reference (oracle/mlp_ref.py), bit-for-bit
reproducibility, training on runs of the method, and what the trained
network gains when it orders work (shortest predicted job first) over the
method without it (arrival order)."""
import sys

import numpy as np
import pytest

from oracle import mlp_ref

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bz():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_2603_29942_amd import bz as _bz
    _bz.lib()
    return _bz


def _setup(n, seed):
    import torch
    rng = np.random.default_rng([31, seed])
    theta = rng.normal(0, 0.25, mlp_ref.NPARAM).astype(np.float32)
    x = rng.normal(0, 1, (n, 4)).astype(np.float32)
    t = rng.normal(0, 1, n).astype(np.float32)
    d = torch.device("cuda:0")
    return theta, x, t, torch.from_numpy(theta).to(d), torch.from_numpy(x).to(d), torch.from_numpy(t).to(d)


@pytest.mark.parametrize("n", [1, 37, 256, 1000])
def test_forward_and_gradient_match_reference(bz, n):
    import torch
    say(f"case mlp n={n}")
    theta, x, t, P, X, T = _setup(n, n)
    cache = torch.empty((n, 128), dtype=torch.float32, device="cuda")
    dz = torch.empty((n, 129), dtype=torch.float32, device="cuda")
    grad = torch.empty(mlp_ref.NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    y = bz.bz_mlp_forward(P, X, cache)
    bz.bz_mlp_backward(P, X, T, y, cache, dz, grad, loss)
    y_ref, (z1, h1, z2, h2) = mlp_ref.forward(theta.astype(np.float64), x)
    # FP32 sums of at most 65 terms against float64: relative 1e-5 of the terms' scale
    assert np.allclose(y.cpu().numpy(), y_ref, rtol=1e-4, atol=1e-4)
    assert np.allclose(cache.cpu().numpy()[:, 64:], h2, rtol=1e-4, atol=1e-4)
    g_ref = mlp_ref.grad(theta.astype(np.float64), x, t)
    g = grad.cpu().numpy()
    scale = np.abs(g_ref).max()
    assert np.abs(g - g_ref).max() <= 1e-4 * scale + 1e-6, np.abs(g - g_ref).max() / scale
    assert abs(loss.item() - mlp_ref.loss(theta.astype(np.float64), x, t)) <= 1e-4 * max(1.0, loss.item())


def test_adam_step_matches_reference(bz):
    """One Adam step from given parameters, gradient and moments (an
    elementwise map) against the reference."""
    import torch
    rng = np.random.default_rng(41)
    th = rng.normal(0, 1, mlp_ref.NPARAM).astype(np.float32)
    g = rng.normal(0, 0.1, mlp_ref.NPARAM).astype(np.float32)
    m = rng.normal(0, 0.05, mlp_ref.NPARAM).astype(np.float32)
    v = rng.uniform(0, 0.01, mlp_ref.NPARAM).astype(np.float32)
    d = torch.device("cuda:0")
    P, G, M, V = (torch.from_numpy(a.copy()).to(d) for a in (th, g, m, v))
    bz.bz_mlp_adam(P, G, M, V, 7, 3e-3)
    th_r, m_r, v_r = mlp_ref.adam(th.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                                  v.astype(np.float64), 7, 3e-3)
    assert np.allclose(M.cpu().numpy(), m_r, rtol=1e-5, atol=1e-7)
    assert np.allclose(V.cpu().numpy(), v_r, rtol=1e-5, atol=1e-9)
    assert np.allclose(P.cpu().numpy(), th_r, rtol=1e-5, atol=1e-6)


def test_training_is_reproducible(bz):
    """Fixed summation order everywhere: two training runs agree bit for bit."""
    import torch
    theta, x, t, P, X, T = _setup(300, 5)
    n = x.shape[0]

    def run():
        p = P.clone()
        m = torch.zeros_like(p)
        v = torch.zeros_like(p)
        cache = torch.empty((n, 128), dtype=torch.float32, device="cuda")
        dz = torch.empty((n, 129), dtype=torch.float32, device="cuda")
        grad = torch.empty_like(p)
        for step in range(1, 21):
            y = bz.bz_mlp_forward(p, X, cache)
            bz.bz_mlp_backward(p, X, T, y, cache, dz, grad)
            bz.bz_mlp_adam(p, grad, m, v, step, 1e-2)
        return p.cpu().numpy()

    assert np.array_equal(run(), run())


def queue_mean_latency(arrivals, service, order_key):
    """Non-preemptive single server: when it frees, it serves the waiting job
    with the smallest key (ties by arrival).  Returns the mean time from
    arrival to completion."""
    idx = np.argsort(arrivals, kind="stable")
    t, i, done, waiting = 0.0, 0, [], []
    import heapq
    while i < len(idx) or waiting:
        if not waiting and t < arrivals[idx[i]]:
            t = arrivals[idx[i]]
        while i < len(idx) and arrivals[idx[i]] <= t:
            j = idx[i]
            heapq.heappush(waiting, (order_key[j], arrivals[j], j))
            i += 1
        _, _, j = heapq.heappop(waiting)
        t += service[j]
        done.append(t - arrivals[j])
    return float(np.mean(done))


def test_trained_predictor_gains_over_arrival_order(bz):
    """Train on 2400 runs of the method, then on 600 held-out codes: the
    predictions rank the work well, and serving shortest-predicted-first beats
    arrival order on mean latency at 70% load (service time = the code's
    combinations at a fixed rate)."""
    from paper_2603_29942_amd import predictor
    X, Y = predictor.collect(3000, seed=7, log=say)
    split = int(0.8 * len(Y))
    net = predictor.Net(seed=1)
    hist = net.fit(X[:split], Y[:split], steps=1500, lr=3e-3)
    say(f"  mse {hist[0]:.3f} -> {hist[-1]:.3f}")
    assert hist[-1] < 0.2 * hist[0]
    pred = net.predict(X[split:])
    y = Y[split:]
    rho = np.corrcoef(np.argsort(np.argsort(pred)), np.argsort(np.argsort(y)))[0, 1]
    say(f"  held-out spearman {rho:.3f}, mae {np.mean(np.abs(pred - y)):.3f} decades")
    assert rho > 0.8
    work = 10.0 ** y
    service = work / work.mean()  # mean service time 1
    rng = np.random.default_rng(11)
    arrivals = np.cumsum(rng.exponential(1.0 / 0.7, len(work)))  # load 0.7
    fifo = queue_mean_latency(arrivals, service, arrivals)
    sjf = queue_mean_latency(arrivals, service, pred)
    ideal = queue_mean_latency(arrivals, service, y)
    say(f"  mean latency: arrival order {fifo:.3f}, predicted-shortest-first {sjf:.3f}, true shortest-first {ideal:.3f}")
    assert sjf < 0.8 * fifo
