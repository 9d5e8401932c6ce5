"""Seeded synthetic inputs: random generator matrices over F_3 and F_7.

This module only draws random numbers; it holds none of the minimum-distance
arithmetic, so the GPU library and the CPU oracle can both be fed from it.

The paper evaluates on randomly generated codes (Sec. 5.2.1 and 5.3: random
matrices over F_7 with k <= 25, n <= 58 and over F_3 with k <= 50, n <= 74);
those datasets are not published, so these seeded draws of the same kind
stand in for them.

Recipe: ``rng = numpy.random.default_rng([stream, seed])``; every entry of the
k x n generator is drawn i.i.d. uniform in {0, ..., p-1}.  A draw is not
checked for rank here: a k x n uniform matrix with n >= 2k is rank deficient
with probability below p^-(n-k), and both the library and the oracle report
such an input as a rank error instead of computing on it.
"""
import numpy as np

# the three single-code workloads: (p, n, k)
CONFIGS = {
    1: (3, 40, 10),   # F_3 [40,10]: small enough for brute force over 3^10 messages
    2: (3, 72, 36),   # F_3 [72,36], rate 1/2
    3: (7, 48, 24),   # F_7 [48,24], rate 1/2
}


def random_generator(p, n, k, seed, stream=0):
    """k x n uint8 matrix with i.i.d. uniform entries in [0, p)."""
    rng = np.random.default_rng([int(stream), int(seed)])
    return rng.integers(0, p, size=(k, n), dtype=np.uint8)


def config_code(cfg, seed):
    """(p, G) for single-code workload ``cfg`` (1, 2 or 3) and ``seed``."""
    p, n, k = CONFIGS[cfg]
    return p, random_generator(p, n, k, seed, stream=cfg)


def batch_codes(seed, count=512, f7_caps=(56, 63)):
    """Mixed batch: half F_3, half F_7 (shuffled), n uniform in [30, 90],
    rate 1/2 or 1/3 at random (k = n // 2 or n // 3).

    F_7 codes above ``f7_caps`` = (max n at rate 1/2, max n at rate 1/3) are
    redrawn: larger random F_7 codes need more than ~1e11 combinations and
    would not finish.  Returns a list of (p, G)."""
    rng = np.random.default_rng([4, int(seed)])
    ps = np.array([3] * (count // 2) + [7] * (count - count // 2))
    rng.shuffle(ps)
    out = []
    for p in ps:
        while True:
            n = int(rng.integers(30, 91))
            half = bool(rng.integers(0, 2))
            if p == 7 and n > (f7_caps[0] if half else f7_caps[1]):
                continue
            break
        k = n // 2 if half else n // 3
        G = rng.integers(0, int(p), size=(k, n), dtype=np.uint8)
        out.append((int(p), G))
    return out


def serving_requests(seed, count, rate_per_s, f7_kmax=28):
    """Poisson arrivals: list of (arrival_time_s, p, G) with p uniform in
    {3, 7}, k uniform in [10, 40] (F_7 capped at ``f7_kmax``) and n = 2k."""
    rng = np.random.default_rng([5, int(seed)])
    t = 0.0
    out = []
    for _ in range(count):
        t += float(rng.exponential(1.0 / rate_per_s))
        p = 3 if rng.integers(0, 2) == 0 else 7
        while True:
            k = int(rng.integers(10, 41))
            if p == 7 and k > f7_kmax:
                continue
            break
        G = rng.integers(0, p, size=(k, 2 * k), dtype=np.uint8)
        out.append((t, p, G))
    return out
