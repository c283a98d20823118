"""ctypes binding of ``libdc.so`` (include/dc.h), argument marshalling only.

Every step of the method runs in the HIP library.  Inputs may be numpy arrays
(host memory) or torch tensors on the GPU (device memory, passed by pointer);
the library enqueues its work on torch's current stream.  The binding fails
loudly when the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdc.so")

OK = 0
PENDING = 1
MODE_DELTA, MODE_ALL, MODE_STATIC, MODE_LEARNED = 0, 1, 2, 3
MLP_INPUTS, MLP_HIDDEN, MLP_PARAMS = 8, 64, 4801
DEL_GAIN, DEL_CONSERVATIVE = 0, 1
ALGO_LOUVAIN, ALGO_SLM = 0, 1
STATUS = {
    0: "OK", -1: "ARG", -2: "RANGE", -3: "SELF_LOOP", -4: "WEIGHT", -5: "NO_EDGE",
    -6: "DUP", -7: "OVERFLOW", -8: "OOM", -9: "DEVICE", -10: "STATE",
}


class Options(ct.Structure):
    _fields_ = [
        ("mode", ct.c_int32), ("max_levels", ct.c_int32), ("max_sweeps", ct.c_int32),
        ("singleton_guard", ct.c_int32), ("del_rule", ct.c_int32), ("timing", ct.c_int32),
        ("tau_den", ct.c_int64), ("stream", ct.c_void_p), ("collect", ct.c_int32),
        ("full_coarsen", ct.c_int32), ("cascade_num", ct.c_int64), ("cascade_den", ct.c_int64),
        ("algorithm", ct.c_int32), ("reserved", ct.c_int32),
    ]


class Edges(ct.Structure):
    _fields_ = [
        ("count", ct.c_int64), ("u", ct.c_void_p), ("v", ct.c_void_p), ("w", ct.c_void_p),
        ("on_device", ct.c_int32), ("pad", ct.c_int32),
    ]


class SweepRec(ct.Structure):
    _fields_ = [
        ("level", ct.c_int32), ("sweep", ct.c_int32), ("n_level", ct.c_int32),
        ("n_active", ct.c_int32), ("nnz_level", ct.c_int64), ("moves", ct.c_int64),
        ("dN", ct.c_int64), ("kept", ct.c_int32), ("phase", ct.c_int32),
    ]


class StepStats(ct.Structure):
    _fields_ = [
        ("changes", ct.c_int64), ("R_size", ct.c_int64), ("ds_sources", ct.c_int64),
        ("ds_accepted", ct.c_int64), ("del_sources", ct.c_int64), ("del_accepted", ct.c_int64),
        ("levels", ct.c_int32), ("sweeps", ct.c_int32), ("moves", ct.c_int64),
        ("vertex_evals", ct.c_int64), ("N", ct.c_int64), ("two_m", ct.c_int64), ("q", ct.c_double),
        ("ms_total", ct.c_double), ("ms_sweep_kernel", ct.c_double),
        ("sweep_launches", ct.c_int64), ("sweep_bytes", ct.c_int64),
        ("level0_sweeps", ct.c_int64), ("level0_active", ct.c_int64),
        ("level0_volume", ct.c_int64), ("touched", ct.c_int64), ("screened", ct.c_int64),
        ("cascade_candidates", ct.c_int64), ("cascade_expanded", ct.c_int64),
        ("ms_phase", ct.c_double * 4), ("bytes_phase", ct.c_int64 * 4),
        ("screen_volume", ct.c_int64), ("screen_vertices", ct.c_int64),
        ("accepted_volume", ct.c_int64),
    ]

    def as_dict(self):
        out = {}
        for f, _ in self._fields_:
            x = getattr(self, f)
            out[f] = list(x) if isinstance(x, ct.Array) else x
        return out


EXPORTS = [
    "dc_default_options", "dc_init", "dc_apply_batch", "dc_modularity", "dc_communities",
    "dc_last_R", "dc_last_trace", "dc_last_stats", "dc_num_entries", "dc_export_csr",
    "dc_destroy", "dc_trim_device_cache", "dc_strerror", "dc_last_error", "dc_screener_set", "dc_last_samples",
    "dc_mlp_create", "dc_mlp_set_weights", "dc_mlp_get_weights", "dc_mlp_forward", "dc_mlp_grad",
    "dc_mlp_grad_noalloc", "dc_mlp_train_step", "dc_mlp_destroy", "dc_export_state", "dc_init_from_state",
    "dc_server_create", "dc_server_add_graph", "dc_server_submit", "dc_server_poll",
    "dc_server_stats_get", "dc_server_destroy",
]


class ServerStats(ct.Structure):
    _fields_ = [
        ("graphs", ct.c_int64), ("batches", ct.c_int64), ("rounds", ct.c_int64),
        ("merged_rounds", ct.c_int64), ("merged_graphs", ct.c_int64), ("evictions", ct.c_int64),
        ("restores", ct.c_int64), ("deferred", ct.c_int64), ("resident_bytes", ct.c_int64),
        ("peak_resident_bytes", ct.c_int64), ("reserved", ct.c_int64 * 6),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}

_lib = None


def load(path: str = LIB_PATH):
    """Load libdc.so and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1904_08553_amd/build.py "
                           "(there is no CPU fallback)")
    # torch first: its HIP runtime (soname libamdhip64.so.7) then satisfies
    # libdc.so's dependency, so one runtime serves both and torch's stream
    # handles are valid in the library.
    import torch  # noqa: F401
    L = ct.CDLL(path)
    P, i32, i64 = ct.c_void_p, ct.c_int32, ct.c_int64
    L.dc_default_options.argtypes = [P]
    L.dc_default_options.restype = None
    L.dc_init.argtypes = [P, i32, P, P]
    L.dc_init.restype = i32
    L.dc_apply_batch.argtypes = [P, P, P, P, i32, P]
    L.dc_apply_batch.restype = i32
    L.dc_modularity.argtypes = [P, P, P, P]
    L.dc_modularity.restype = i32
    L.dc_communities.argtypes = [P, P, i32]
    L.dc_communities.restype = i32
    L.dc_last_R.argtypes = [P, P, i32]
    L.dc_last_R.restype = i32
    L.dc_last_trace.argtypes = [P, P, i32, P]
    L.dc_last_trace.restype = i32
    L.dc_last_stats.argtypes = [P, P]
    L.dc_last_stats.restype = i32
    L.dc_num_entries.argtypes = [P, P]
    L.dc_num_entries.restype = i32
    L.dc_export_csr.argtypes = [P, P, P, P]
    L.dc_export_csr.restype = i32
    L.dc_destroy.argtypes = [P]
    L.dc_destroy.restype = None
    L.dc_trim_device_cache.argtypes = []
    L.dc_trim_device_cache.restype = None
    L.dc_strerror.argtypes = [i32]
    L.dc_strerror.restype = ct.c_char_p
    L.dc_last_error.argtypes = []
    L.dc_last_error.restype = ct.c_char_p
    f32, f64p = ct.c_float, ct.c_void_p
    L.dc_screener_set.argtypes = [P, P, f32]
    L.dc_screener_set.restype = i32
    L.dc_last_samples.argtypes = [P, P, P, P, P, P, i32]
    L.dc_last_samples.restype = i32
    L.dc_mlp_create.argtypes = [P, P, P]
    L.dc_mlp_create.restype = i32
    L.dc_mlp_set_weights.argtypes = [P, P]
    L.dc_mlp_set_weights.restype = i32
    L.dc_mlp_get_weights.argtypes = [P, P]
    L.dc_mlp_get_weights.restype = i32
    L.dc_mlp_forward.argtypes = [P, P, i64, P]
    L.dc_mlp_forward.restype = i32
    L.dc_mlp_grad.argtypes = [P, P, P, i64, f32, P, f64p]
    L.dc_mlp_grad.restype = i32
    L.dc_mlp_grad_noalloc.argtypes = [P, P, P, i64, f32, P, f64p]
    L.dc_mlp_grad_noalloc.restype = i32
    L.dc_mlp_train_step.argtypes = [P, P, P, i64, f32, f32, f64p]
    L.dc_mlp_train_step.restype = i32
    L.dc_mlp_destroy.argtypes = [P]
    L.dc_mlp_destroy.restype = None
    L.dc_export_state.argtypes = [P, P, P, P, P]
    L.dc_export_state.restype = i32
    L.dc_init_from_state.argtypes = [P, i32, P, P, P, P, P]
    L.dc_init_from_state.restype = i32
    L.dc_server_create.argtypes = [P, P, i64, i32]
    L.dc_server_create.restype = i32
    L.dc_server_add_graph.argtypes = [P, i32, P, P]
    L.dc_server_add_graph.restype = i32
    L.dc_server_submit.argtypes = [P, i32, P, P, i64, P]
    L.dc_server_submit.restype = i32
    L.dc_server_poll.argtypes = [P, i64, i32, P, P, P]
    L.dc_server_poll.restype = i32
    L.dc_server_stats_get.argtypes = [P, P]
    L.dc_server_stats_get.restype = i32
    L.dc_server_destroy.argtypes = [P]
    L.dc_server_destroy.restype = None
    _lib = L
    return L


class DCError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = load().dc_strerror(status).decode()
        detail = load().dc_last_error().decode() if status in (-8, -9) else ""
        super().__init__(f"{where}: {STATUS.get(status, status)} ({msg}) {detail}".rstrip())
        self.status = status


def _check(status, where):
    if status != OK:
        raise DCError(status, where)


def _is_torch(x):
    return type(x).__module__.startswith("torch")


class _Arr:
    """Pointer to an int32 array, host (numpy) or device (torch tensor)."""

    def __init__(self, x):
        if x is None:
            self.ptr, self.n, self.dev, self.keep = None, 0, 0, None
        elif _is_torch(x):
            import torch
            if x.dtype != torch.int32 or not x.is_contiguous():
                x = x.to(torch.int32).contiguous()
            self.ptr, self.n, self.dev, self.keep = x.data_ptr(), x.numel(), int(x.is_cuda), x
            if not x.is_cuda:
                self.keep = x.numpy()
                self.ptr = self.keep.ctypes.data
        else:
            a = np.ascontiguousarray(np.asarray(x, dtype=np.int32))
            self.ptr, self.n, self.dev, self.keep = a.ctypes.data, a.size, 0, a


def _edges(u, v, w=None):
    au, av, aw = _Arr(u), _Arr(v), _Arr(w)
    if au.n != av.n or (w is not None and aw.n != au.n):
        raise ValueError("edge arrays differ in length")
    if au.dev != av.dev or (w is not None and aw.dev != au.dev):
        raise ValueError("edge arrays must all be on the host or all on the device")
    e = Edges(au.n, au.ptr, av.ptr, aw.ptr, au.dev, 0)
    return e, (au, av, aw)


def current_stream():
    """torch's current HIP stream handle (0 when torch or a GPU is absent)."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


def options(mode=MODE_DELTA, max_levels=32, max_sweeps=100, singleton_guard=1,
            del_rule=DEL_GAIN, timing=0, tau_den=1_000_000, stream="current", collect=0,
            full_coarsen=0, cascade=None, algorithm=None):
    """cascade: None (off) or (num, den) for the cascade-aware screening
    threshold theta = num/den.  algorithm: ALGO_LOUVAIN (default) or
    ALGO_SLM, the host method of the levels."""
    o = Options()
    load().dc_default_options(ct.byref(o))
    if algorithm is not None:
        o.algorithm = algorithm
    o.mode, o.max_levels, o.max_sweeps = mode, max_levels, max_sweeps
    o.singleton_guard, o.del_rule, o.timing, o.tau_den = singleton_guard, del_rule, timing, tau_den
    o.collect = collect
    o.full_coarsen = full_coarsen
    if cascade is not None:
        o.cascade_num, o.cascade_den = int(cascade[0]), int(cascade[1])
    o.stream = current_stream() if stream == "current" else stream
    return o


class DynamicCommunities:
    """A dynamic graph with its communities, held on the GPU by libdc.so."""

    def __init__(self, n, u, v, w, **opt):
        self.n = int(n)
        self._opt = options(**opt)
        e, keep = _edges(u, v, w)
        h = ct.c_void_p()
        _check(load().dc_init(ct.byref(h), self.n, ct.byref(e), ct.byref(self._opt)), "dc_init")
        self._h = h
        del keep

    @classmethod
    def from_state(cls, n, off, col, w, C, **opt):
        """Resume from a checkpoint (see export_state); runs no levels."""
        self = cls.__new__(cls)
        self.n = int(n)
        self._opt = options(**opt)
        off = np.ascontiguousarray(off, np.int64)
        col = np.ascontiguousarray(col, np.int32)
        w = np.ascontiguousarray(w, np.int32)
        C = np.ascontiguousarray(C, np.int32)
        h = ct.c_void_p()
        _check(load().dc_init_from_state(ct.byref(h), self.n, off.ctypes.data, col.ctypes.data,
                                         w.ctypes.data, C.ctypes.data, ct.byref(self._opt)),
               "dc_init_from_state")
        self._h = h
        return self

    def export_state(self):
        """Checkpoint: (off, col, w, C) in host memory."""
        nnz = ct.c_int64()
        _check(load().dc_num_entries(self._h, ct.byref(nnz)), "dc_num_entries")
        off = np.empty(self.n + 1, np.int64)
        col = np.empty(max(nnz.value, 1), np.int32)
        w = np.empty(max(nnz.value, 1), np.int32)
        C = np.empty(self.n, np.int32)
        _check(load().dc_export_state(self._h, off.ctypes.data, col.ctypes.data, w.ctypes.data,
                                      C.ctypes.data), "dc_export_state")
        return off, col[: nnz.value], w[: nnz.value], C

    def apply_batch(self, add_u=None, add_v=None, add_w=None, del_u=None, del_v=None, out=None):
        """Apply one batch; returns C_t as a numpy array (or fills ``out``,
        a device tensor, without a host copy)."""
        add, ka = _edges(add_u if add_u is not None else [], add_v if add_v is not None else [],
                         add_w if add_w is not None else [])
        dele, kd = _edges(del_u if del_u is not None else [], del_v if del_v is not None else [])
        st = StepStats()
        if out is not None:
            o = _Arr(out)
            _check(load().dc_apply_batch(self._h, ct.byref(add), ct.byref(dele), o.ptr, o.dev,
                                         ct.byref(st)), "dc_apply_batch")
            self.stats = st
            return out
        C = np.empty(self.n, np.int32)
        _check(load().dc_apply_batch(self._h, ct.byref(add), ct.byref(dele), C.ctypes.data, 0,
                                     ct.byref(st)), "dc_apply_batch")
        self.stats = st
        del ka, kd
        return C

    def modularity(self):
        q, N, tm = ct.c_double(), ct.c_int64(), ct.c_int64()
        _check(load().dc_modularity(self._h, ct.byref(q), ct.byref(N), ct.byref(tm)),
               "dc_modularity")
        return q.value, N.value, tm.value

    def communities(self):
        C = np.empty(self.n, np.int32)
        _check(load().dc_communities(self._h, C.ctypes.data, 0), "dc_communities")
        return C

    def last_R(self):
        R = np.empty(self.n, np.uint8)
        _check(load().dc_last_R(self._h, R.ctypes.data, 0), "dc_last_R")
        return R

    def last_trace(self):
        cnt = ct.c_int32()
        _check(load().dc_last_trace(self._h, None, 0, ct.byref(cnt)), "dc_last_trace")
        recs = (SweepRec * max(cnt.value, 1))()
        _check(load().dc_last_trace(self._h, recs, cnt.value, ct.byref(cnt)), "dc_last_trace")
        # SLM refinement sweeps carry their phase as a ninth field
        return [(r.level, r.sweep, r.n_level, r.n_active, r.nnz_level, r.moves, r.dN, r.kept)
                + ((r.phase,) if r.phase else ()) for r in recs[: cnt.value]]

    def last_stats(self):
        st = StepStats()
        _check(load().dc_last_stats(self._h, ct.byref(st)), "dc_last_stats")
        return st

    def set_screener(self, w, theta):
        """Screener parameters (MLP_PARAMS floats, or None to clear) and the
        logit threshold of LEARNED mode."""
        if w is None:
            _check(load().dc_screener_set(self._h, None, 0.0), "dc_screener_set")
            return
        a = np.ascontiguousarray(np.asarray(w, dtype=np.float32))
        if a.size != MLP_PARAMS:
            raise ValueError(f"expected {MLP_PARAMS} parameters")
        _check(load().dc_screener_set(self._h, a.ctypes.data, float(theta)), "dc_screener_set")

    def samples(self, device=False, labels=True, logits=False):
        """Screener samples of the last batch: dict of ids (int32), X (uint16
        bfloat16 bits, [count, 8]), y (uint8) and logits (float32), as numpy
        arrays or (device=True) torch tensors on the GPU."""
        L = load()
        cnt = ct.c_int64()
        _check(L.dc_last_samples(self._h, ct.byref(cnt), None, None, None, None, 0),
               "dc_last_samples")
        c = cnt.value
        if device:
            import torch
            dev = torch.device("cuda")
            ids = torch.empty(max(c, 1), dtype=torch.int32, device=dev)
            X = torch.empty((max(c, 1), MLP_INPUTS), dtype=torch.int16, device=dev)
            y = torch.empty(max(c, 1), dtype=torch.uint8, device=dev) if labels else None
            z = torch.empty(max(c, 1), dtype=torch.float32, device=dev) if logits else None
            ptr = lambda t: None if t is None else t.data_ptr()
        else:
            ids = np.empty(max(c, 1), np.int32)
            X = np.empty((max(c, 1), MLP_INPUTS), np.uint16)
            y = np.empty(max(c, 1), np.uint8) if labels else None
            z = np.empty(max(c, 1), np.float32) if logits else None
            ptr = lambda a: None if a is None else a.ctypes.data
        if c > 0:
            _check(L.dc_last_samples(self._h, ct.byref(cnt), ptr(ids), ptr(X), ptr(y), ptr(z),
                                     int(device)), "dc_last_samples")
        out = dict(ids=ids[:c], X=X[:c])
        if labels:
            out["y"] = y[:c]
        if logits:
            out["logits"] = z[:c]
        return out

    def csr(self):
        nnz = ct.c_int64()
        _check(load().dc_num_entries(self._h, ct.byref(nnz)), "dc_num_entries")
        off = np.empty(self.n + 1, np.int64)
        col = np.empty(max(nnz.value, 1), np.int32)
        w = np.empty(max(nnz.value, 1), np.int32)
        _check(load().dc_export_csr(self._h, off.ctypes.data, col.ctypes.data, w.ctypes.data),
               "dc_export_csr")
        return off, col[: nnz.value], w[: nnz.value]

    def close(self):
        if getattr(self, "_h", None):
            load().dc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Durable checkpoint files: G_t (CSR) and C_t, as exported by export_state.

CKPT_VERSION = 1


class CheckpointError(RuntimeError):
    """A checkpoint file that is not a complete, intact checkpoint."""


def trim_device_cache():
    """Frees the device blocks that destroyed contexts left in the library's
    block cache (dc_trim_device_cache); live contexts keep their memory."""
    load().dc_trim_device_cache()


def _ckpt_digest(n, off, col, w, C):
    import hashlib
    h = hashlib.sha256()
    h.update(np.int64(n).tobytes())
    for a in (off, col, w, C):
        h.update(np.ascontiguousarray(a).tobytes())
    return np.frombuffer(h.digest(), np.uint8)


def write_checkpoint(path, n, off, col, w, C):
    """Write a checkpoint of (n, off, col, w, C) to ``path``: the arrays go
    to a temporary file in the same directory, which is flushed to disk and
    then renamed over ``path`` (so a crash leaves the old file or the new
    one, never a torn one); a SHA-256 digest of the arrays is stored with
    them.  Plain arrays only (numpy .npz, nothing pickled)."""
    off = np.ascontiguousarray(off, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    w = np.ascontiguousarray(w, np.int32)
    C = np.ascontiguousarray(C, np.int32)
    path = os.fspath(path)
    d = os.path.dirname(os.path.abspath(path))
    tmp = os.path.join(d, f".{os.path.basename(path)}.{os.getpid()}.tmp")
    try:
        with open(tmp, "wb") as f:
            np.savez(f, version=np.array([CKPT_VERSION], np.int64), n=np.array([n], np.int64),
                     off=off, col=col, w=w, C=C, digest=_ckpt_digest(n, off, col, w, C))
            f.flush()
            os.fsync(f.fileno())
        os.replace(tmp, path)
    finally:
        if os.path.exists(tmp):
            os.unlink(tmp)
    try:
        fd = os.open(d, os.O_RDONLY)
    except OSError:
        return
    try:
        os.fsync(fd)
    finally:
        os.close(fd)


def read_checkpoint(path):
    """(n, off, col, w, C) of a checkpoint file; CheckpointError when the
    file is not a complete checkpoint of this version or its digest fails."""
    try:
        with np.load(os.fspath(path), allow_pickle=False) as z:
            need = ("version", "n", "off", "col", "w", "C", "digest")
            if any(k not in z.files for k in need):
                raise CheckpointError(f"{path}: missing arrays")
            if int(z["version"][0]) != CKPT_VERSION:
                raise CheckpointError(f"{path}: version {int(z['version'][0])}")
            n = int(z["n"][0])
            off, col, w, C = z["off"], z["col"], z["w"], z["C"]
            digest = z["digest"]
    except CheckpointError:
        raise
    except Exception as e:  # unreadable zip, truncated file, bad array
        raise CheckpointError(f"{path}: {e}") from e
    if off.shape != (n + 1,) or C.shape != (n,) or col.shape != w.shape:
        raise CheckpointError(f"{path}: array shapes do not match n = {n}")
    if not np.array_equal(digest, _ckpt_digest(n, off, col, w, C)):
        raise CheckpointError(f"{path}: digest mismatch")
    return n, off, col, w, C


def save_checkpoint(g, path):
    """Durable checkpoint file of a DynamicCommunities (see write_checkpoint)."""
    write_checkpoint(path, g.n, *g.export_state())


def load_checkpoint(path, **opt):
    """A DynamicCommunities resumed from a checkpoint file (options as for
    DynamicCommunities; the state itself is validated again by the library)."""
    n, off, col, w, C = read_checkpoint(path)
    return DynamicCommunities.from_state(n, off, col, w, C, **opt)


class MLP:
    """The screener network on the GPU (libdc.so's dc_mlp): forward, loss
    gradient and Adam steps over device tensors of bfloat16 feature bits."""

    def __init__(self, w):
        a = np.ascontiguousarray(np.asarray(w, dtype=np.float32))
        if a.size != MLP_PARAMS:
            raise ValueError(f"expected {MLP_PARAMS} parameters")
        h = ct.c_void_p()
        _check(load().dc_mlp_create(ct.byref(h), a.ctypes.data, current_stream()),
               "dc_mlp_create")
        self._h = h

    @staticmethod
    def _dev(t, dtype_name):
        if not (_is_torch(t) and t.is_cuda and t.is_contiguous()):
            raise ValueError(f"{dtype_name} must be a contiguous CUDA tensor")
        return t.data_ptr()

    def set_weights(self, w):
        a = np.ascontiguousarray(np.asarray(w, dtype=np.float32))
        _check(load().dc_mlp_set_weights(self._h, a.ctypes.data), "dc_mlp_set_weights")

    def weights(self):
        w = np.empty(MLP_PARAMS, np.float32)
        _check(load().dc_mlp_get_weights(self._h, w.ctypes.data), "dc_mlp_get_weights")
        return w

    def forward(self, X):
        import torch
        n = X.shape[0]
        z = torch.empty(max(n, 1), dtype=torch.float32, device=X.device)
        _check(load().dc_mlp_forward(self._h, self._dev(X, "X"), n, z.data_ptr()),
               "dc_mlp_forward")
        return z[:n]

    def grad(self, X, y, pos_weight):
        g = np.empty(MLP_PARAMS, np.float32)
        loss = ct.c_double()
        _check(load().dc_mlp_grad(self._h, self._dev(X, "X"), self._dev(y, "y"), X.shape[0],
                                  float(pos_weight), g.ctypes.data, ct.byref(loss)),
               "dc_mlp_grad")
        return loss.value, g

    def grad_noalloc(self, X, y, pos_weight):
        """grad() through dc_mlp_grad_noalloc: the library's fixed device
        scratch instead of allocated buffers (same result)."""
        g = np.empty(MLP_PARAMS, np.float32)
        loss = ct.c_double()
        _check(load().dc_mlp_grad_noalloc(self._h, self._dev(X, "X"), self._dev(y, "y"),
                                          X.shape[0], float(pos_weight), g.ctypes.data,
                                          ct.byref(loss)),
               "dc_mlp_grad_noalloc")
        return loss.value, g

    def train_step(self, X, y, pos_weight, lr, want_loss=False):
        loss = ct.c_double()
        _check(load().dc_mlp_train_step(self._h, self._dev(X, "X"), self._dev(y, "y"), X.shape[0],
                                        float(pos_weight), float(lr),
                                        ct.byref(loss) if want_loss else None),
               "dc_mlp_train_step")
        return loss.value if want_loss else None

    def close(self):
        if getattr(self, "_h", None):
            load().dc_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Many dynamic graphs served from one GPU by libdc.so (dc_server_*):
    continuous batching with merged level-0 sweeps and admission of graphs
    by device-memory footprint (budget_bytes <= 0: unlimited)."""

    def __init__(self, budget_bytes=0, max_inflight=8, **opt):
        self._opt = options(stream=None, **opt)
        h = ct.c_void_p()
        _check(load().dc_server_create(ct.byref(h), ct.byref(self._opt), int(budget_bytes),
                                       int(max_inflight)), "dc_server_create")
        self._h = h
        self.n = {}

    def add_graph(self, n, u, v, w):
        e, keep = _edges(u, v, w)
        gid = ct.c_int32()
        _check(load().dc_server_add_graph(self._h, int(n), ct.byref(e), ct.byref(gid)),
               "dc_server_add_graph")
        self.n[gid.value] = int(n)
        return gid.value

    def submit(self, gid, add_u=(), add_v=(), add_w=(), del_u=(), del_v=(), arrival_ns=None):
        import time
        add, ka = _edges(add_u, add_v, add_w)
        dele, kd = _edges(del_u, del_v)
        t = ct.c_int64()
        arr = time.monotonic_ns() if arrival_ns is None else int(arrival_ns)
        _check(load().dc_server_submit(self._h, int(gid), ct.byref(add), ct.byref(dele), arr,
                                       ct.byref(t)), "dc_server_submit")
        return t.value

    def poll(self, ticket, gid, wait=True):
        """None while pending (wait=False); else (C, stats, (arrival, start,
        done) ns).  Raises DCError for a failed batch."""
        C = np.empty(self.n[gid], np.int32)
        st = StepStats()
        times = (ct.c_int64 * 3)()
        s = load().dc_server_poll(self._h, int(ticket), int(bool(wait)), C.ctypes.data,
                                  ct.byref(st), times)
        if s == PENDING:
            return None
        _check(s, "dc_server_poll")
        return C, st, tuple(times)

    def stats(self):
        st = ServerStats()
        _check(load().dc_server_stats_get(self._h, ct.byref(st)), "dc_server_stats_get")
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            load().dc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
