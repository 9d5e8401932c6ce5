"""Reference element encoding and F_p addition via F_2 (test infrastructure).

Pure Python on single symbols and short vectors; used only by the tests.

Paper: Hernando & Quintana-Orti, arXiv 2603.29942, Sec. 2.
  - natural binary expansion A = sum_i a_i 2^i with r = floor(log2 p) + 1
    bits, least significant bit first (Sec. 2);
  - sliced-bit storage: bit i of every symbol of a vector goes to plane i
    (Sec. 2, with the worked example (2,0,1) in F_3);
  - addition for p = 2^r - 1 (Sec. 2.1, Algorithm 1): xor gives the sum
    without carries, and gives the carries; carries move one position up,
    the top one wrapping around to bit 0 (2^r = 1 mod p); repeat until no
    carry is left, then map the all-ones pattern (which is p) to zero.
"""


def nbits(p):
    """r = floor(log2 p) + 1."""
    return p.bit_length()


def expand(A, p):
    """Binary expansion of the symbol A, least significant bit first."""
    return tuple((A >> i) & 1 for i in range(nbits(p)))


def value(bits):
    return sum(b << i for i, b in enumerate(bits))


def slice_vector(U, p):
    """Sliced-bit storage: list of r planes, plane i = bit i of every symbol."""
    return [tuple(expand(u, p)[i] for u in U) for i in range(nbits(p))]


def unslice(planes):
    n = len(planes[0])
    return [value([pl[t] for pl in planes]) for t in range(n)]


def _rotate_up(bits):
    """phi: circular shift moving bit i to position i+1 and the top bit to 0."""
    return (bits[-1],) + tuple(bits[:-1])


def alg1_add(V, W, p):
    """V + W in F_p for p = 2^r - 1 by the carry loop of Algorithm 1.

    Returns (result_symbol, number_of_loop_iterations)."""
    r = nbits(p)
    if p != (1 << r) - 1:
        raise ValueError("Algorithm 1 needs p = 2^r - 1")
    v, w = expand(V, p), expand(W, p)
    d = tuple(a ^ b for a, b in zip(v, w))
    e = tuple(a & b for a, b in zip(v, w))
    iters = 0
    while any(e):
        v, w = d, _rotate_up(e)
        d = tuple(a ^ b for a, b in zip(v, w))
        e = tuple(a & b for a, b in zip(v, w))
        iters += 1
    t = int(all(d))
    c = tuple(b ^ t for b in d)
    return value(c), iters


def times_two_by_rotation(W, p):
    """2*W in F_p (p = 2^r - 1) as a circular shift of the expansion (Sec. 4.2)."""
    return value(_rotate_up(expand(W, p)))
