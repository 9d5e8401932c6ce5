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


def serve_latencies(bz, reqs, policy, params, slots):
    """Submits every request at once (a burst at t = 0, the same trace for
    every policy) to a continuous-batching server and returns each request's
    time to its result, as the polling loop sees it."""
    import time
    srv = bz.Server(policy=policy, mlp_params=params, slots=slots, max_n=80, wait_timeout_s=30)
    lat = {}
    try:
        t0 = time.perf_counter()
        for tag, (p, G) in enumerate(reqs):
            srv.submit(p, G, tag)
        while len(lat) < len(reqs):
            for tag, r in srv.poll():
                lat[tag] = time.perf_counter() - t0
                assert r["status"] in (0, bz.ERR_RANK), r["status"]
            assert time.perf_counter() - t0 < 120, "server stalled"
    finally:
        srv.stop()
    return np.array([lat[i] for i in range(len(reqs))])


def test_trained_predictor_gains_on_the_server(bz):
    """Train the network on 2400 runs of the method, check how it ranks 600
    held-out codes, then serve 400 other codes on the real continuous-batching
    server (128 slots, all submitted at once) in arrival order and with the
    trained network ordering the work: shortest predicted work first finishes
    the requests much sooner on average."""
    from paper_2603_29942_amd import predictor, synth
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
    reqs = [(p, G) for _, p, G in synth.serving_requests(8, 400, rate_per_s=1.0)]
    fifo = serve_latencies(bz, reqs, "fifo", None, 128)
    spf = serve_latencies(bz, reqs, "predicted", net.theta(), 128)
    say(f"  served 400 requests: mean latency arrival order {fifo.mean() * 1e3:.1f} ms, "
        f"shortest predicted first {spf.mean() * 1e3:.1f} ms (p50 {np.median(fifo) * 1e3:.1f} / "
        f"{np.median(spf) * 1e3:.1f} ms)")
    assert spf.mean() < 0.7 * fifo.mean()
