"""ctypes binding of the oracle library ``libbzref.so`` (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use this module.  It computes the minimum distance of a linear
code over F_3 / F_7 in plain mod-p integer arithmetic, following Algorithm 6
(Sec. 3.1) of Hernando & Quintana-Orti, arXiv 2603.29942, with the readings
documented in ``bzref.c``.
"""
import ctypes
import os

import numpy as np

from . import build as _build

MAX_N, MAX_K, MAX_M, MAX_STAGES = 128, 64, 128, 256
OK, ERR_ARG, ERR_VALUE, ERR_RANK, ERR_LIMIT = 0, -1, -2, -3, -6
CHECK_ROUND, NO_TERMINATION = 1, 2


class _Stage(ctypes.Structure):
    _fields_ = [("g", ctypes.c_int32), ("j", ctypes.c_int32), ("codewords", ctypes.c_uint64),
                ("stage_min", ctypes.c_int32), ("upper_after", ctypes.c_int32),
                ("lower_after", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("m", ctypes.c_int32), ("ranks", ctypes.c_int32 * MAX_M),
                ("n_stages", ctypes.c_int32), ("terminated_by", ctypes.c_int32),
                ("codewords_total", ctypes.c_uint64), ("stages", _Stage * MAX_STAGES)]


def load(path):
    """Bind the functions of an oracle library built at ``path``."""
    L = ctypes.CDLL(path)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    L.bzref_rank.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p]
    L.bzref_decompose.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p, u8p, i32p, i32p]
    L.bzref_min_distance.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_uint64, u64p, ctypes.POINTER(_Result)]
    L.bzref_stage_enum.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int, u64p, u64p]
    L.bzref_brute_force.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p, u64p]
    L.bzref_threads.argtypes = [ctypes.c_int]
    return L


_lib = None


def lib():
    """The oracle library, built first only if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = load(_build.LIB)
    return _lib


def _u8(G):
    G = np.ascontiguousarray(G, dtype=np.uint8)
    return G, G.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def threads(nthreads=0, _L=None):
    return (_L or lib()).bzref_threads(int(nthreads))


def rank(p, G, _L=None):
    G, ptr = _u8(G)
    k, n = G.shape
    return (_L or lib()).bzref_rank(p, n, k, ptr)


def decompose(p, G, _L=None):
    """Return (status_or_m, gammas[m,k,n], ranks[m], pivots[m,k])."""
    G, ptr = _u8(G)
    k, n = G.shape
    gam = np.zeros((MAX_M, k, n), dtype=np.uint8)
    ranks = np.zeros(MAX_M, dtype=np.int32)
    piv = np.zeros((MAX_M, k), dtype=np.int32)
    m = (_L or lib()).bzref_decompose(p, n, k, ptr, gam.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                              ranks.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              piv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if m < 0:
        return m, None, None, None
    return m, gam[:m].copy(), ranks[:m].copy(), piv[:m].copy()


def min_distance(p, G, *, check="stage", no_termination=False, nthreads=0, max_codewords=0,
                 histograms=False, _L=None):
    """Oracle Brouwer-Zimmermann run.

    Returns a dict: status, d, m, ranks, stages (list of (g, j, codewords,
    stage_min, upper_after, lower_after)), terminated_by, codewords_total and,
    with ``histograms``, hist[n_stages, n+1].
    """
    G, ptr = _u8(G)
    k, n = G.shape
    flags = (CHECK_ROUND if check == "round" else 0) | (NO_TERMINATION if no_termination else 0)
    res = _Result()
    hist = np.zeros((MAX_STAGES, n + 1), dtype=np.uint64) if histograms else None
    hptr = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)) if histograms else None
    st = (_L or lib()).bzref_min_distance(p, n, k, ptr, flags, int(nthreads), int(max_codewords), hptr,
                                  ctypes.byref(res))
    return _result_dict(st, res, hist)


def _result_dict(st, res, hist):
    out = {"status": st, "d": res.d, "m": res.m, "ranks": [res.ranks[i] for i in range(res.m)],
           "terminated_by": res.terminated_by, "codewords_total": res.codewords_total,
           "stages": [(s.g, s.j, s.codewords, s.stage_min, s.upper_after, s.lower_after)
                      for s in res.stages[:res.n_stages]]}
    if hist is not None:
        out["hist"] = hist[:res.n_stages].copy()
    return out


def stage_enum(p, gamma, g, *, nthreads=0, first_row_lo=0, first_row_hi=0, _L=None):
    """All g-row combinations of ``gamma`` (lowest coefficient 1).

    Returns (min_weight, count, hist[n+1])."""
    gamma, ptr = _u8(gamma)
    k, n = gamma.shape
    cnt = np.zeros(1, dtype=np.uint64)
    hist = np.zeros(n + 1, dtype=np.uint64)
    mn = (_L or lib()).bzref_stage_enum(p, n, k, ptr, g, int(nthreads), int(first_row_lo), int(first_row_hi),
                                cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                hist.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return mn, int(cnt[0]), hist


def brute_force(p, G, _L=None):
    """Weight distribution A_w over all p^k messages; returns (d, A)."""
    G, ptr = _u8(G)
    k, n = G.shape
    hist = np.zeros(n + 1, dtype=np.uint64)
    d = (_L or lib()).bzref_brute_force(p, n, k, ptr, hist.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return d, hist
