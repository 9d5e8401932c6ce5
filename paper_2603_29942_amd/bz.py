"""Python binding of the C ABI in ``include/bz.h`` (``libbz.so``, HIP for gfx950).

Argument marshalling only: every step of the minimum-distance path runs in the
library's GPU kernels.  The functions keep the C names; ``min_distance`` is a
convenience wrapper returning a dict.  There is no CPU fallback: if the built
library is missing, loading fails with an error.

PyTorch is used only for device memory and streams: pass ``G`` as a CUDA
(ROCm) uint8 tensor to hand the library a device pointer, and its current
stream is used.
"""
import atexit
import ctypes
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbz.so")

MAX_N, MAX_K, MAX_M, MAX_STAGES = 128, 64, 128, 256
OK, ERR_ARG, ERR_VALUE, ERR_RANK, ERR_DEVICE, ERR_NOMEM, ERR_LIMIT = 0, -1, -2, -3, -4, -5, -6
CHECK_STAGE, CHECK_ROUND = 0, 1
OP_ADD, OP_SUB, OP_DOUBLE, OP_ISO_ADD, OP_ISO_SUB, OP_KAT_ADD = range(6)
ENC_NATURAL, ENC_KAT = 0, 1

INFO_AHEAD = 1
INFO_PAIRS = 2
NOALLOC_SCRATCH_BYTES = 640 * 1024

EXPORTS = ("bz_default_options", "bz_min_distance", "bz_min_distance_ex", "bz_status_str",
           "bz_min_distance_noalloc", "bz_release",
           "bz_default_batch_options", "bz_min_distance_batch",
           "bz_mlp_forward", "bz_mlp_backward", "bz_mlp_adam",
           "bz_default_server_options", "bz_server_start", "bz_server_submit", "bz_server_poll", "bz_server_stats", "bz_server_stop",
           "bz_sliced_pack", "bz_sliced_unpack", "bz_sliced_op", "bz_valu_rate")


class bz_stage(ctypes.Structure):
    _fields_ = [("g", ctypes.c_int32), ("j", ctypes.c_int32), ("codewords", ctypes.c_uint64),
                ("stage_min", ctypes.c_int32), ("upper_after", ctypes.c_int32),
                ("lower_after", ctypes.c_int32)]


class bz_result(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("m", ctypes.c_int32), ("ranks", ctypes.c_int32 * MAX_M),
                ("n_stages", ctypes.c_int32), ("terminated_by", ctypes.c_int32),
                ("codewords_total", ctypes.c_uint64), ("stages", bz_stage * MAX_STAGES),
                ("decompose_ms", ctypes.c_float), ("enum_ms", ctypes.c_float), ("info", ctypes.c_int32)]


class bz_options(ctypes.Structure):
    _fields_ = [("check", ctypes.c_int32), ("no_termination", ctypes.c_int32),
                ("identity_skip", ctypes.c_int32), ("histograms", ctypes.c_int32),
                ("hist_out", ctypes.POINTER(ctypes.c_uint64)), ("max_codewords", ctypes.c_uint64),
                ("hip_stream", ctypes.c_void_p), ("device", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("wait_timeout_s", ctypes.c_int32), ("trace_out", ctypes.POINTER(ctypes.c_uint64)),
                ("cooperative", ctypes.c_int32), ("no_ahead", ctypes.c_int32), ("pair_tables", ctypes.c_int32)]


class bz_code(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("n", ctypes.c_int32), ("k", ctypes.c_int32),
                ("sweep_ops", ctypes.c_int32), ("g_offset", ctypes.c_uint64)]


class bz_batch_options(ctypes.Structure):
    _fields_ = [("check", ctypes.c_int32), ("no_termination", ctypes.c_int32),
                ("identity_skip", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("max_codewords", ctypes.c_uint64), ("hip_stream", ctypes.c_void_p),
                ("device", ctypes.c_int32), ("wait_timeout_s", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("decompose_ms", ctypes.c_float), ("enum_ms", ctypes.c_float), ("cooperative", ctypes.c_int32),
                ("code_ms_out", ctypes.POINTER(ctypes.c_float))]


class bz_server_options(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("policy", ctypes.c_int32), ("mlp_params", ctypes.c_void_p),
                ("check", ctypes.c_int32), ("identity_skip", ctypes.c_int32), ("max_codewords", ctypes.c_uint64),
                ("blocks_per_cu", ctypes.c_int32), ("device", ctypes.c_int32), ("wait_timeout_s", ctypes.c_int32),
                ("max_n", ctypes.c_int32), ("cooperative", ctypes.c_int32), ("admit_budget", ctypes.c_double)]


SERVE_FIFO, SERVE_PREDICTED = 0, 1

_lib = None
_devices_used = set()
_live_servers = weakref.WeakSet()


class LibraryMissing(RuntimeError):
    pass


def _release_at_exit():
    """Stop the servers still running and release the library's per-device
    state (streams, events, device and host buffers) while the HIP runtime is
    still up."""
    if _lib is None:
        return
    for srv in list(_live_servers):
        try:
            srv.stop()
        except Exception:
            pass
    for dev in sorted(_devices_used):
        _lib.bz_release(int(dev))


def lib():
    """Load ``libbz.so`` (build it with ``python -m paper_2603_29942_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} is not built; run python -m paper_2603_29942_amd.build")
        _lib = load(LIB_PATH)
        atexit.register(_release_at_exit)
    return _lib


def load(path):
    """Bind the C ABI of the library built at ``path`` (argument and result types)."""
    L = ctypes.CDLL(path)
    u8p, u32p = ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_uint32)
    vp = ctypes.c_void_p
    L.bz_default_options.argtypes = [ctypes.POINTER(bz_options)]
    L.bz_default_options.restype = None
    L.bz_min_distance.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(bz_result)]
    L.bz_min_distance_ex.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int,
                                     ctypes.POINTER(bz_options), ctypes.POINTER(bz_result)]
    L.bz_min_distance_noalloc.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                          ctypes.POINTER(bz_options), ctypes.POINTER(bz_result)]
    L.bz_release.argtypes = [ctypes.c_int]
    L.bz_status_str.argtypes = [ctypes.c_int]
    L.bz_status_str.restype = ctypes.c_char_p
    L.bz_sliced_pack.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    L.bz_sliced_unpack.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    L.bz_sliced_op.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp,
                               ctypes.c_int, vp]
    L.bz_valu_rate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(ctypes.c_float),
                               ctypes.POINTER(ctypes.c_double), vp]
    del u8p, u32p
    L.bz_default_batch_options.argtypes = [ctypes.POINTER(bz_batch_options)]
    L.bz_default_batch_options.restype = None
    L.bz_min_distance_batch.argtypes = [ctypes.c_int, ctypes.POINTER(bz_code), vp, ctypes.c_uint64,
                                        ctypes.c_int, ctypes.POINTER(bz_batch_options),
                                        ctypes.POINTER(bz_result), ctypes.POINTER(ctypes.c_int32)]
    fp = ctypes.c_void_p
    L.bz_mlp_forward.argtypes = [fp, fp, ctypes.c_int, fp, fp, vp]
    L.bz_mlp_backward.argtypes = [fp, fp, fp, ctypes.c_int, fp, fp, fp, fp, fp, vp]
    L.bz_mlp_adam.argtypes = [fp, fp, fp, fp, ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, vp]
    L.bz_default_server_options.argtypes = [ctypes.POINTER(bz_server_options)]
    L.bz_default_server_options.restype = None
    L.bz_server_start.argtypes = [ctypes.POINTER(bz_server_options), ctypes.POINTER(ctypes.c_void_p)]
    L.bz_server_submit.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.c_uint64]
    L.bz_server_poll.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(bz_result),
                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(ctypes.c_int)]
    L.bz_server_stop.argtypes = [vp]
    L.bz_server_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
    return L


def bz_default_options():
    o = bz_options()
    lib().bz_default_options(ctypes.byref(o))
    return o


def bz_status_str(status):
    return lib().bz_status_str(int(status)).decode()


def _stream_of(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def bz_min_distance_ex(p, G, options=None, out=None):
    """Run the library on G (numpy uint8 on the host, or a torch uint8 CUDA
    tensor on the device).  Returns (status, bz_result)."""
    out = out if out is not None else bz_result()
    o = options if options is not None else bz_default_options()
    if hasattr(G, "is_cuda") and G.is_cuda:
        k, n = G.shape
        if not G.is_contiguous():
            raise ValueError("G must be contiguous")
        if o.hip_stream is None:
            o.hip_stream = _stream_of(G)
        o.device = G.device.index or 0
        _devices_used.add(o.device)
        st = lib().bz_min_distance_ex(p, n, k, ctypes.c_void_p(G.data_ptr()), 1, ctypes.byref(o),
                                      ctypes.byref(out))
    else:
        G = np.ascontiguousarray(G, dtype=np.uint8)
        k, n = G.shape
        _devices_used.add(o.device)
        st = lib().bz_min_distance_ex(p, n, k, G.ctypes.data_as(ctypes.c_void_p), 0, ctypes.byref(o),
                                      ctypes.byref(out))
    return st, out


def bz_min_distance_noalloc(p, G, options=None, out=None):
    """The entry point that allocates nothing: G must be a contiguous torch
    uint8 CUDA tensor (device memory); runs on the tensor's current stream.
    Returns (status, bz_result)."""
    out = out if out is not None else bz_result()
    o = options if options is not None else bz_default_options()
    if not (hasattr(G, "is_cuda") and G.is_cuda and G.is_contiguous()):
        raise ValueError("G must be a contiguous device tensor")
    k, n = G.shape
    if o.hip_stream is None:
        o.hip_stream = _stream_of(G)
    o.device = G.device.index or 0
    st = lib().bz_min_distance_noalloc(p, n, k, ctypes.c_void_p(G.data_ptr()), ctypes.byref(o), ctypes.byref(out))
    return st, out


def bz_release(device=0):
    return lib().bz_release(int(device))


def bz_min_distance(p, G):
    G = np.ascontiguousarray(G, dtype=np.uint8)
    k, n = G.shape
    out = bz_result()
    st = lib().bz_min_distance(p, n, k, G.ctypes.data_as(ctypes.c_void_p), ctypes.byref(out))
    return st, out


def result_dict(st, r, hist=None):
    d = {"status": st, "d": r.d, "m": r.m, "ranks": [r.ranks[i] for i in range(r.m)],
         "terminated_by": r.terminated_by, "codewords_total": r.codewords_total,
         "stages": [(s.g, s.j, s.codewords, s.stage_min, s.upper_after, s.lower_after)
                    for s in r.stages[:r.n_stages]], "info": r.info}
    if hist is not None:
        d["hist"] = hist[:r.n_stages].copy()
    return d


def min_distance(p, G, *, check="stage", no_termination=False, identity_skip=True, max_codewords=0,
                 histograms=False, blocks_per_cu=0, trace=False, ahead=True,
                 wait_timeout_s=0, stream=None, pair_tables=0):
    """Convenience wrapper: same keys as the oracle's result dict (plus
    ``info`` and, when asked for, ``trace``, the device timeline in ns).
    stream: a torch stream to run on (G on the device), else the current one.
    pair_tables: 0 the library's choice, 1 always, -1 never (bz_options)."""
    o = bz_default_options()
    o.no_ahead = int(not ahead)
    o.pair_tables = int(pair_tables)
    o.wait_timeout_s = int(wait_timeout_s)
    if stream is not None:
        o.hip_stream = ctypes.c_void_p(stream.cuda_stream)
    tr = None
    if trace:
        tr = np.zeros((MAX_STAGES + 2, 4), dtype=np.uint64)
        o.trace_out = tr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    o.check = CHECK_ROUND if check == "round" else CHECK_STAGE
    o.no_termination = int(bool(no_termination))
    o.identity_skip = int(bool(identity_skip))
    o.max_codewords = int(max_codewords)
    o.blocks_per_cu = int(blocks_per_cu)
    n = G.shape[1]
    hist = None
    if histograms:
        hist = np.zeros((MAX_STAGES, n + 1), dtype=np.uint64)
        o.histograms = 1
        o.hist_out = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    st, r = bz_min_distance_ex(p, G, o)
    out = result_dict(st, r, hist)
    if trace:
        out["trace"] = tr[:2 + r.n_stages].copy()
    return out


# ---------------------------------------------------------------- batches
def bz_default_batch_options():
    o = bz_batch_options()
    lib().bz_default_batch_options(ctypes.byref(o))
    return o


def pack_batch(codes, device=None, align=16):
    """codes: list of (p, G), G (k, n) uint8.  Returns (buffer, descriptors):
    one contiguous uint8 buffer holding every generator at a 16-byte aligned
    offset (a torch CUDA tensor when device is given, else numpy) and the
    bz_code array (sweep_ops 0)."""
    offs, total = [], 0
    for _, G in codes:
        offs.append(total)
        total += -(-int(np.prod(G.shape)) // align) * align
    host = np.zeros(max(total, align), dtype=np.uint8)
    descs = (bz_code * len(codes))()
    for i, ((p, G), off) in enumerate(zip(codes, offs)):
        Gh = G.cpu().numpy() if hasattr(G, "cpu") else np.asarray(G, dtype=np.uint8)
        k, n = Gh.shape
        host[off:off + k * n] = Gh.reshape(-1)
        descs[i].p, descs[i].n, descs[i].k, descs[i].sweep_ops, descs[i].g_offset = int(p), n, k, 0, off
    if device is None:
        return host, descs
    import torch
    return torch.from_numpy(host).to(device), descs


def bz_min_distance_batch(buf, descs, options=None):
    """Run a packed batch (see pack_batch).  Returns (status, [(status_i, bz_result_i)], options)."""
    o = options if options is not None else bz_default_batch_options()
    nc = len(descs)
    out = (bz_result * max(nc, 1))()
    sts = (ctypes.c_int32 * max(nc, 1))()
    _devices_used.add(o.device)
    if hasattr(buf, "is_cuda") and buf.is_cuda:
        if o.hip_stream is None:
            o.hip_stream = _stream_of(buf)
        o.device = buf.device.index or 0
        _devices_used.add(o.device)
        st = lib().bz_min_distance_batch(nc, descs, ctypes.c_void_p(buf.data_ptr()), buf.numel(), 1,
                                         ctypes.byref(o), out, sts)
    else:
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        st = lib().bz_min_distance_batch(nc, descs, buf.ctypes.data_as(ctypes.c_void_p), buf.size, 0,
                                         ctypes.byref(o), out, sts)
    return st, [(int(sts[i]), out[i]) for i in range(nc)], o


def min_distance_batch(codes, *, check="stage", no_termination=False, identity_skip=True, max_codewords=0,
                       blocks_per_cu=0, sweep_ops=None, device=None, timing=False, wait_timeout_s=0):
    """Convenience wrapper: one result dict per code (same keys as
    min_distance).  sweep_ops: None, an int for every code, or a function
    (p, W) -> int (e.g. the autotuner's table).  timing: also return the two
    launches' times and every code's time to d within the batch (ms)."""
    buf, descs = pack_batch(codes, device=device)
    for i in range(len(codes)):
        if sweep_ops is None:
            continue
        if callable(sweep_ops):
            W = (descs[i].n - descs[i].k + 31) // 32 if identity_skip else (descs[i].n + 31) // 32
            descs[i].sweep_ops = int(sweep_ops(descs[i].p, max(W, 1)))
        else:
            descs[i].sweep_ops = int(sweep_ops)
    o = bz_default_batch_options()
    o.check = CHECK_ROUND if check == "round" else CHECK_STAGE
    o.no_termination = int(bool(no_termination))
    o.identity_skip = int(bool(identity_skip))
    o.max_codewords = int(max_codewords)
    o.blocks_per_cu = int(blocks_per_cu)
    o.timing = int(bool(timing))
    o.wait_timeout_s = int(wait_timeout_s)
    code_ms = np.zeros(max(len(codes), 1), dtype=np.float32)
    if timing:
        o.code_ms_out = code_ms.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    st, res, o = bz_min_distance_batch(buf, descs, o)
    if st != OK:
        raise RuntimeError(f"bz_min_distance_batch: {bz_status_str(st)}")
    out = [result_dict(s_i, r_i) for s_i, r_i in res]
    if timing:
        return out, {"decompose_ms": o.decompose_ms, "enum_ms": o.enum_ms, "code_ms": code_ms[:len(codes)].copy()}
    return out


# ---------------------------------------------------------------- serving
class Server:
    """Continuous-batching server (see bz_server_* in include/bz.h).

    submit(p, G, tag) queues a code (host numpy uint8 (k, n)); poll() advances
    the server and returns [(tag, result dict)] of the codes that finished."""

    def __init__(self, policy="fifo", mlp_params=None, slots=1024, max_n=0, check="stage", identity_skip=True,
                 max_codewords=0, blocks_per_cu=0, wait_timeout_s=0, max_out=1024, admit_budget=0.0):
        o = bz_server_options()
        lib().bz_default_server_options(ctypes.byref(o))
        o.slots = int(slots)
        o.policy = SERVE_PREDICTED if policy == "predicted" else SERVE_FIFO
        self._mlp = None
        if mlp_params is not None:
            self._mlp = np.ascontiguousarray(mlp_params, dtype=np.float32)
            o.mlp_params = self._mlp.ctypes.data_as(ctypes.c_void_p)
        o.check = CHECK_ROUND if check == "round" else CHECK_STAGE
        o.identity_skip = int(bool(identity_skip))
        o.max_codewords = int(max_codewords)
        o.blocks_per_cu = int(blocks_per_cu)
        o.wait_timeout_s = int(wait_timeout_s)
        o.max_n = int(max_n)
        o.admit_budget = float(admit_budget)
        h = ctypes.c_void_p()
        _check(lib().bz_server_start(ctypes.byref(o), ctypes.byref(h)), "bz_server_start")
        self._h = h
        _devices_used.add(o.device)
        _live_servers.add(self)
        self._max = int(max_out)
        self._tags = (ctypes.c_uint64 * self._max)()
        self._res = (bz_result * self._max)()
        self._sts = (ctypes.c_int32 * self._max)()

    def submit(self, p, G, tag):
        G = np.ascontiguousarray(G, dtype=np.uint8)
        k, n = G.shape
        _check(lib().bz_server_submit(self._h, int(p), n, k, G.ctypes.data_as(ctypes.c_void_p), int(tag)),
               "bz_server_submit")

    def poll(self):
        n_out, in_flight = ctypes.c_int(), ctypes.c_int()
        _check(lib().bz_server_poll(self._h, self._max, self._tags, self._res, self._sts, ctypes.byref(n_out),
                                    ctypes.byref(in_flight)), "bz_server_poll")
        self.in_flight = in_flight.value
        return [(int(self._tags[i]), result_dict(int(self._sts[i]), self._res[i])) for i in range(n_out.value)]

    def stats(self):
        r, y = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().bz_server_stats(self._h, ctypes.byref(r), ctypes.byref(y)), "bz_server_stats")
        return {"rounds": r.value, "yields": y.value}

    def stop(self):
        if self._h:
            lib().bz_server_stop(self._h)
            self._h = None

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


# ---------------------------------------------------------------- work predictor network
MLP_PARAMS = 4545


def _check(st, name):
    if st != OK:
        raise RuntimeError(f"{name}: {bz_status_str(st)}")


def bz_mlp_forward(params, x, cache=None):
    """params: float32 CUDA tensor (4545,); x: (n, 4) float32 CUDA tensor.
    Returns y (n,); fills cache (n, 128) when given."""
    import torch
    n = x.shape[0]
    y = torch.empty(n, dtype=torch.float32, device=x.device)
    _check(lib().bz_mlp_forward(_ptr(params), _ptr(x), n, _ptr(y), _ptr(cache), _stream_of(x)), "bz_mlp_forward")
    return y


def bz_mlp_backward(params, x, t, y, cache, dz, grad, loss=None):
    _check(lib().bz_mlp_backward(_ptr(params), _ptr(x), _ptr(t), x.shape[0], _ptr(y), _ptr(cache), _ptr(dz),
                                 _ptr(grad), _ptr(loss), _stream_of(x)), "bz_mlp_backward")


def bz_mlp_adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().bz_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr), float(beta1),
                             float(beta2), float(eps), _stream_of(params)), "bz_mlp_adam")


# ---------------------------------------------------------------- sliced vectors
def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def bz_sliced_pack(p, sym, encoding=ENC_NATURAL):
    """sym: torch uint8 CUDA tensor (nvec, nsym) -> int32 tensor (nvec, r, words)."""
    import torch
    nvec, nsym = sym.shape
    r = 2 if p == 3 else 3
    planes = torch.empty((nvec, r, (nsym + 31) // 32), dtype=torch.int32, device=sym.device)
    st = lib().bz_sliced_pack(p, encoding, nvec, nsym, _ptr(sym), _ptr(planes), _stream_of(sym))
    if st != OK:
        raise RuntimeError(bz_status_str(st))
    return planes


def bz_sliced_unpack(p, planes, nsym, encoding=ENC_NATURAL):
    import torch
    nvec = planes.shape[0]
    sym = torch.empty((nvec, nsym), dtype=torch.uint8, device=planes.device)
    st = lib().bz_sliced_unpack(p, encoding, nvec, nsym, _ptr(planes), _ptr(sym), _stream_of(planes))
    if st != OK:
        raise RuntimeError(bz_status_str(st))
    return sym


def bz_sliced_op(p, op, a, b, nsym, reps=1, out=None):
    import torch
    out = torch.empty_like(a) if out is None else out
    st = lib().bz_sliced_op(p, op, a.shape[0], nsym, _ptr(a), _ptr(b), _ptr(out), reps, _stream_of(a))
    if st != OK:
        raise RuntimeError(bz_status_str(st))
    return out


# ---------------------------------------------------------------- VALU issue rates
VALU_PROBE_OPS = ("v_xor_b32", "v_add_u32", "v_bitop3_b32", "v_bcnt_u32_b32", "v_min_u32", "v_fma_f32")


def valu_rate(op, iters=4096, blocks_per_cu=8):
    """Issue rate of one VALU instruction (see bz_valu_rate): lane-ops per second."""
    import torch
    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(dev)
    out = torch.empty(props.multi_processor_count * blocks_per_cu * 256, dtype=torch.int32, device=dev)
    ms, ops = ctypes.c_float(), ctypes.c_double()
    _check(lib().bz_valu_rate(int(op), int(iters), int(blocks_per_cu), _ptr(out), ctypes.byref(ms), ctypes.byref(ops),
                              _stream_of(out)), "bz_valu_rate")
    return ops.value / (ms.value * 1e-3)
