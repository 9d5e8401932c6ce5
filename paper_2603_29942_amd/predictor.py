"""Learned work predictor for admission and packing.

    python -m paper_2603_29942_amd.predictor [--count 10000] [--seed 0] [--out PATH]

Features of a code (after its information-set decomposition): the field p,
the length n, the dimension k and the rank deficit k - k_m of the last
information set (the rank profile decides how fast the lower bound grows).
Target: log10 of the combinations the method evaluates.  The network is a
4 -> 64 -> 64 -> 1 FP32 multilayer perceptron trained with the library's own
HIP kernels (forward, gradient, Adam) on runs of the method itself (the
batched path on codes of the serving distribution).  Its output only orders
and admits work; d always comes from the stage-by-stage L >= U test.
"""
import argparse
import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "mlp_weights.json")
NPARAM = 4545
FEATURES = ("p", "n", "k", "k - k_m")


def features(p, n, k, km):
    """Normalised inputs of the network."""
    return np.array([(p - 5.0) / 2.0, (n - 60.0) / 30.0, (k - 25.0) / 15.0, (k - km) / 8.0], dtype=np.float32)


def features_of(p, G, result):
    k, n = G.shape
    km = result["ranks"][-1] if result["m"] > 0 else k
    return features(p, n, k, km)


def target_of(result):
    return float(np.log10(max(1, result["codewords_total"])))


def init_params(seed=0):
    """He-style initialisation: weights N(0, 2 / fan_in), biases 0."""
    rng = np.random.default_rng([9, seed])
    W1 = rng.normal(0, np.sqrt(2 / 4), (64, 4))
    W2 = rng.normal(0, np.sqrt(2 / 64), (64, 64))
    w3 = rng.normal(0, np.sqrt(1 / 64), 64)
    theta = np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), w3, [0.0]])
    return theta.astype(np.float32)


def collect(count=10000, seed=0, chunk=1024, log=print):
    """Runs the method (batched path) on `count` codes of the serving
    distribution; returns features X (count, 4), targets Y and the codes' work."""
    import torch
    from . import bz, synth
    dev = torch.device("cuda:0")
    reqs = synth.serving_requests(seed, count, rate_per_s=1.0)
    X, Y = [], []
    t0 = time.perf_counter()
    for lo in range(0, count, chunk):
        codes = [(p, G) for _, p, G in reqs[lo:lo + chunk]]
        res = bz.min_distance_batch(codes, device=dev)
        for (p, G), r in zip(codes, res):
            if r["status"] != bz.OK:
                continue
            X.append(features_of(p, G, r))
            Y.append(target_of(r))
        log(f"  collected {min(lo + chunk, count)}/{count} runs in {time.perf_counter() - t0:.1f} s")
    return np.stack(X), np.array(Y, dtype=np.float32)


class Net:
    """Parameters and Adam state on the GPU; every step is the library's kernels."""

    def __init__(self, theta=None, seed=0):
        import torch
        self.dev = torch.device("cuda:0")
        th = init_params(seed) if theta is None else np.asarray(theta, dtype=np.float32)
        self.params = torch.from_numpy(th.copy()).to(self.dev)
        self.m = torch.zeros(NPARAM, dtype=torch.float32, device=self.dev)
        self.v = torch.zeros(NPARAM, dtype=torch.float32, device=self.dev)
        self.step = 0

    def predict(self, X):
        import torch
        from . import bz
        x = torch.as_tensor(np.asarray(X, dtype=np.float32), device=self.dev).contiguous()
        return bz.bz_mlp_forward(self.params, x).cpu().numpy()

    def fit(self, X, Y, steps=3000, lr=3e-3, log=None):
        """Full-batch Adam on mean squared error; returns the loss history."""
        import torch
        from . import bz
        x = torch.as_tensor(np.asarray(X, dtype=np.float32), device=self.dev).contiguous()
        t = torch.as_tensor(np.asarray(Y, dtype=np.float32), device=self.dev).contiguous()
        n = x.shape[0]
        cache = torch.empty((n, 128), dtype=torch.float32, device=self.dev)
        dz = torch.empty((n, 129), dtype=torch.float32, device=self.dev)
        grad = torch.empty(NPARAM, dtype=torch.float32, device=self.dev)
        loss = torch.empty(1, dtype=torch.float32, device=self.dev)
        hist = []
        for it in range(steps):
            y = bz.bz_mlp_forward(self.params, x, cache)
            bz.bz_mlp_backward(self.params, x, t, y, cache, dz, grad, loss)
            self.step += 1
            bz.bz_mlp_adam(self.params, grad, self.m, self.v, self.step, lr)
            if it % 100 == 0 or it == steps - 1:
                hist.append(float(loss.item()))
                if log:
                    log(f"  step {it}: mse {hist[-1]:.4f}")
        return hist

    def theta(self):
        return self.params.cpu().numpy()


def save(path, theta, meta):
    with open(path, "w") as f:
        json.dump({"params": [float(v) for v in theta], "features": FEATURES, **meta}, f)


def load(path=WEIGHTS):
    with open(path) as f:
        d = json.load(f)
    return np.array(d["params"], dtype=np.float32), d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=10000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()
    X, Y = collect(args.count, args.seed)
    n = len(Y)
    split = int(0.8 * n)
    net = Net(seed=args.seed)
    t0 = time.perf_counter()
    hist = net.fit(X[:split], Y[:split], steps=args.steps, log=print)
    train_s = time.perf_counter() - t0
    pred = net.predict(X[split:])
    err = pred - Y[split:]
    rank_corr = float(np.corrcoef(np.argsort(np.argsort(pred)), np.argsort(np.argsort(Y[split:])))[0, 1])
    meta = {"runs": n, "train": split, "held_out": n - split, "steps": args.steps,
            "train_mse": hist[-1], "held_out_mse": float(np.mean(err ** 2)),
            "held_out_mae_log10": float(np.mean(np.abs(err))), "held_out_spearman": rank_corr,
            "train_seconds": round(train_s, 2),
            "command": f"python -m paper_2603_29942_amd.predictor --count {args.count} --seed {args.seed}"}
    save(args.out, net.theta(), meta)
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
