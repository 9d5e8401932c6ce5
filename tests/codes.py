"""Generator matrices of classical codes whose parameters mathematics fixes.

Test helpers only (plain numpy, mod-p integers); shared by the oracle pins and
the GPU parity tests as *inputs*, never as expected values of either side.
"""
import itertools
import json
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def poly_mod(a, b, p):
    """Remainder of a(x) / b(x) over F_p, coefficient lists low to high."""
    a = [x % p for x in a]
    inv = pow(b[-1], p - 2, p)
    while len(a) >= len(b) and any(a):
        if a[-1] == 0:
            a.pop()
            continue
        f = a[-1] * inv % p
        shift = len(a) - len(b)
        for i, c in enumerate(b):
            a[shift + i] = (a[shift + i] - f * c) % p
        a.pop()
    while a and a[-1] == 0:
        a.pop()
    return a


def cyclic_generator(gpoly, n, p):
    """Rows x^i g(x), i = 0..n-deg(g)-1."""
    k = n - (len(gpoly) - 1)
    G = np.zeros((k, n), dtype=np.uint8)
    for i in range(k):
        G[i, i:i + len(gpoly)] = gpoly
    return G


def ternary_golay():
    spec = golden("classical_codes.json")["ternary_golay_11_6_5"]
    return cyclic_generator(spec["generator_poly_low_to_high"], 11, 3)


def extended_golay():
    G = ternary_golay().astype(np.int64)
    par = (-G.sum(axis=1)) % 3
    return np.concatenate([G, par[:, None]], axis=1).astype(np.uint8)


def reed_solomon(p, n, k):
    """Evaluation code: rows x^i, i < k, at n distinct points of F_p.

    n = p uses all of F_p, n = p - 1 the nonzero elements; MDS, d = n - k + 1."""
    pts = list(range(p)) if n == p else list(range(1, p))[:n]
    return np.array([[pow(x, i, p) for x in pts] for i in range(k)], dtype=np.uint8)


def mds_weight_distribution(n, k, q):
    """A_w of an [n,k,n-k+1] MDS code over F_q (closed form)."""
    d = n - k + 1
    A = [0] * (n + 1)
    A[0] = 1
    for w in range(d, n + 1):
        s = sum((-1) ** j * math.comb(w, j) * (q ** (w - d + 1 - j) - 1) for j in range(w - d + 1))
        A[w] = math.comb(n, w) * s
    return A


def projective_points(r, p):
    """One representative (first nonzero entry 1) of every 1-dim subspace of F_p^r."""
    pts = []
    for v in itertools.product(range(p), repeat=r):
        nz = [x for x in v if x]
        if nz and nz[0] == 1:
            pts.append(v)
    return pts


def simplex(r, p):
    """[ (p^r-1)/(p-1), r, p^(r-1) ] simplex code: every nonzero word has weight p^(r-1)."""
    return np.array(projective_points(r, p), dtype=np.uint8).T.copy()


def hamming(r, p):
    """Hamming code of redundancy r: dual of the simplex code, d = 3.

    H = [A | I_r] with the columns of A the projective points that are not unit
    vectors; G = [I | -A^T]."""
    pts = projective_points(r, p)
    units = {tuple(1 if i == j else 0 for i in range(r)) for j in range(r)}
    A = np.array([v for v in pts if v not in units], dtype=np.int64).T  # r x (n-r)
    nk = A.shape[1]
    G = np.concatenate([np.eye(nk, dtype=np.int64), (-A.T) % p], axis=1)
    return G.astype(np.uint8)


def repetition(n, p):
    return np.ones((1, n), dtype=np.uint8)


def zero_sum(n, p):
    """[n, n-1, 2]: G = [I | -1]."""
    G = np.zeros((n - 1, n), dtype=np.uint8)
    G[:, :n - 1] = np.eye(n - 1, dtype=np.uint8)
    G[:, n - 1] = p - 1
    return G


def full_space(n, p):
    return np.eye(n, dtype=np.uint8)


def direct_sum(A, B):
    k1, n1 = A.shape
    k2, n2 = B.shape
    G = np.zeros((k1 + k2, n1 + n2), dtype=np.uint8)
    G[:k1, :n1] = A
    G[k1:, n1:] = B
    return G


def random_invertible(k, p, rng):
    """Unit lower-triangular times upper-triangular with a nonzero diagonal."""
    Lo = np.tril(rng.integers(0, p, size=(k, k)), -1) + np.eye(k, dtype=np.int64)
    Up = np.triu(rng.integers(0, p, size=(k, k)), 1) + np.diag(rng.integers(1, p, size=k))
    return (Lo @ Up) % p


def matmul_mod(A, B, p):
    return ((np.asarray(A, dtype=np.int64) @ np.asarray(B, dtype=np.int64)) % p).astype(np.uint8)


def rank_mod_p(A, p):
    """Rank over F_p by plain elimination (test-side, independent of the oracle)."""
    A = np.array(A, dtype=np.int64) % p
    rows, cols = A.shape
    r = 0
    for c in range(cols):
        piv = next((i for i in range(r, rows) if A[i, c]), None)
        if piv is None:
            continue
        A[[r, piv]] = A[[piv, r]]
        A[r] = A[r] * pow(int(A[r, c]), p - 2, p) % p
        for i in range(rows):
            if i != r and A[i, c]:
                A[i] = (A[i] - A[i, c] * A[r]) % p
        r += 1
        if r == rows:
            break
    return r
