"""ctypes wrapper of the plain CPU oracle (``dc_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Imported by the test suite, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py``; the product package never imports
this module.  See ``dc_oracle.c`` for the passages of arXiv 1904.08553 each
function follows.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dc_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

MODE_DELTA, MODE_ALL, MODE_STATIC, MODE_LEARNED = 0, 1, 2, 3
ALGO_LOUVAIN, ALGO_SLM = 0, 1
FEATURES = 8
NO_GAIN = -(1 << 63)
DEL_GAIN, DEL_CONSERVATIVE = 0, 1

STATUS_NAMES = {
    0: "OK", -1: "ARG", -2: "RANGE", -3: "SELF_LOOP", -4: "WEIGHT",
    -5: "NO_EDGE", -6: "DUP", -7: "OVERFLOW", -8: "OOM",
}


def build(force: bool = True) -> str:
    """Compile the oracle with plain gcc (single thread, no SIMD pragmas)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
             "-o", tmp, SRC],
            check=True,
        )
        os.replace(tmp, LIB)
    return LIB


class Options(ct.Structure):
    _fields_ = [
        ("mode", ct.c_int32), ("max_levels", ct.c_int32),
        ("max_sweeps", ct.c_int32), ("singleton_guard", ct.c_int32),
        ("del_rule", ct.c_int32), ("collect", ct.c_int32), ("tau_den", ct.c_int64),
        ("cascade_num", ct.c_int64), ("cascade_den", ct.c_int64),
        ("algorithm", ct.c_int32), ("pad", ct.c_int32),
    ]


class SweepRec(ct.Structure):
    _fields_ = [
        ("level", ct.c_int32), ("sweep", ct.c_int32), ("n_level", ct.c_int32),
        ("n_active", ct.c_int32), ("nnz_level", ct.c_int64),
        ("moves", ct.c_int64), ("dN", ct.c_int64), ("kept", ct.c_int32),
        ("phase", ct.c_int32),
    ]


class StepInfo(ct.Structure):
    _fields_ = [
        ("R_size", ct.c_int64), ("ds_sources", ct.c_int64),
        ("ds_accepted", ct.c_int64), ("del_sources", ct.c_int64),
        ("del_accepted", ct.c_int64), ("cascade_candidates", ct.c_int64),
        ("cascade_expanded", ct.c_int64), ("levels", ct.c_int32),
        ("n_sweeps", ct.c_int32), ("N", ct.c_int64), ("two_m", ct.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("DC_ORACLE_LIB", LIB)  # tests may load a planted-mistake build
        if path == LIB and not os.path.exists(LIB):
            build(force=True)
        L = ct.CDLL(path)
        P = ct.c_void_p
        i32, i64 = ct.c_int32, ct.c_int64
        L.orc_default_options.argtypes = [P]
        L.orc_init.argtypes = [P, i32, i64, P, P, P, P, P, P, i32, P]
        L.orc_init.restype = i32
        L.orc_apply_batch.argtypes = [P, i64, P, P, P, i64, P, P, P, P, P, i32, P]
        L.orc_apply_batch.restype = i32
        L.orc_stage_batch.argtypes = [P, i64, P, P, P, i64, P, P]
        L.orc_stage_batch.restype = i32
        L.orc_finish_batch.argtypes = [P, P, P, P, P, i32, P]
        L.orc_finish_batch.restype = i32
        L.orc_last_samples.argtypes = [P, P, P, P, P, P]
        L.orc_last_samples.restype = i32
        L.orc_modularity.argtypes = [P, P, P, P]
        L.orc_modularity.restype = i32
        L.orc_communities.argtypes = [P, P]
        L.orc_communities.restype = i32
        L.orc_num_entries.argtypes = [P]
        L.orc_num_entries.restype = i64
        L.orc_export_csr.argtypes = [P, P, P, P]
        L.orc_export_csr.restype = i32
        L.orc_destroy.argtypes = [P]
        L.orc_csr_modularity.argtypes = [i32, P, P, P, P, P, P]
        L.orc_csr_modularity.restype = i32
        L.orc_csr_gain.argtypes = [i32, P, P, P, P, i32, i32]
        L.orc_csr_gain.restype = i64
        L.orc_csr_decide.argtypes = [i32, P, P, P, P, i32, i32, P]
        L.orc_csr_decide.restype = i32
        L.orc_csr_run_levels.argtypes = [i32, P, P, P, P, P, P, P, i32, P, P]
        L.orc_csr_run_levels.restype = i32
        L.orc_csr_coarsen.argtypes = [i32, P, P, P, P, P, P, P, P, P, P]
        L.orc_csr_coarsen.restype = i32
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def options(mode=MODE_DELTA, max_levels=32, max_sweeps=100, singleton_guard=1,
            del_rule=DEL_GAIN, tau_den=1000000, collect=0, cascade=None,
            algorithm=ALGO_LOUVAIN) -> Options:
    """cascade: None (off) or (num, den), theta = num/den (cascade-aware
    screening, an extension; see screen_cascade in dc_oracle.c).
    algorithm: ALGO_LOUVAIN or ALGO_SLM (the host method, Sec. 3.4)."""
    o = Options()
    o.algorithm = algorithm
    o.mode, o.max_levels, o.max_sweeps = mode, max_levels, max_sweeps
    o.singleton_guard, o.del_rule, o.tau_den = singleton_guard, del_rule, tau_den
    o.collect = collect
    if cascade is not None:
        o.cascade_num, o.cascade_den = int(cascade[0]), int(cascade[1])
    return o


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status} ({STATUS_NAMES.get(status, '?')})")
        self.status = status


def _i32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32))


def _i64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int64))


class Oracle:
    """One dynamic graph driven through the oracle."""

    TRACE_CAP = 1 << 16

    def __init__(self, n, u, v, w, **opt):
        self.n = int(n)
        self.opt = options(**opt)
        u, v, w = _i32(u), _i32(v), _i32(w)
        self._h = ct.c_void_p()
        C = np.empty(self.n, np.int32)
        recs = (SweepRec * self.TRACE_CAP)()
        info = StepInfo()
        st = lib().orc_init(ct.byref(self._h), self.n, len(u), _p(u), _p(v), _p(w),
                            ct.byref(self.opt), _p(C), recs, self.TRACE_CAP,
                            ct.byref(info))
        if st != 0:
            raise OracleError(st)
        self.C = C
        self.info = info
        self.trace = _trace(recs, info.n_sweeps, self.TRACE_CAP)
        self.R = np.ones(self.n, np.uint8)

    def apply_batch(self, add_u=(), add_v=(), add_w=(), del_u=(), del_v=()):
        au, av, aw = _i32(add_u), _i32(add_v), _i32(add_w)
        du, dv = _i32(del_u), _i32(del_v)
        C = np.empty(self.n, np.int32)
        R = np.empty(self.n, np.uint8)
        recs = (SweepRec * self.TRACE_CAP)()
        info = StepInfo()
        st = lib().orc_apply_batch(self._h, len(au), _p(au), _p(av), _p(aw),
                                   len(du), _p(du), _p(dv), _p(C), _p(R), recs,
                                   self.TRACE_CAP, ct.byref(info))
        if st != 0:
            raise OracleError(st)
        self.C, self.R, self.info = C, R, info
        self.trace = _trace(recs, info.n_sweeps, self.TRACE_CAP)
        return C

    def stage_batch(self, add_u=(), add_v=(), add_w=(), del_u=(), del_v=()):
        """First half of a step: validate, update G_t, screen, collect samples."""
        au, av, aw = _i32(add_u), _i32(add_v), _i32(add_w)
        du, dv = _i32(del_u), _i32(del_v)
        st = lib().orc_stage_batch(self._h, len(au), _p(au), _p(av), _p(aw),
                                   len(du), _p(du), _p(dv))
        if st != 0:
            raise OracleError(st)

    def finish_batch(self, R=None):
        """Second half: levels over R (0/1 per vertex) or the staged set."""
        Ro = None if R is None else np.ascontiguousarray(R, np.uint8)
        C = np.empty(self.n, np.int32)
        Rout = np.empty(self.n, np.uint8)
        recs = (SweepRec * self.TRACE_CAP)()
        info = StepInfo()
        st = lib().orc_finish_batch(self._h, _p(Ro), _p(C), _p(Rout), recs, self.TRACE_CAP,
                                    ct.byref(info))
        if st != 0:
            raise OracleError(st)
        self.C, self.R, self.info = C, Rout, info
        self.trace = _trace(recs, info.n_sweeps, self.TRACE_CAP)
        return C

    def samples(self):
        """Screener samples of the last staged batch: ids (int32, ascending),
        X (fp64 [count, 8]), raw (int64 [count, 8]), y (uint8)."""
        cnt = ct.c_int64()
        lib().orc_last_samples(self._h, ct.byref(cnt), None, None, None, None)
        c = cnt.value
        ids = np.empty(max(c, 1), np.int32)
        X = np.empty((max(c, 1), FEATURES), np.float64)
        raw = np.empty((max(c, 1), FEATURES), np.int64)
        y = np.empty(max(c, 1), np.uint8)
        lib().orc_last_samples(self._h, ct.byref(cnt), _p(ids), _p(X), _p(raw), _p(y))
        return dict(ids=ids[:c], X=X[:c], raw=raw[:c], y=y[:c])

    def modularity(self):
        N, tm, q = ct.c_int64(), ct.c_int64(), ct.c_double()
        st = lib().orc_modularity(self._h, ct.byref(N), ct.byref(tm), ct.byref(q))
        if st != 0:
            raise OracleError(st)
        return q.value, N.value, tm.value

    def communities(self):
        out = np.empty(self.n, np.int32)
        lib().orc_communities(self._h, _p(out))
        return out

    def csr(self):
        nnz = lib().orc_num_entries(self._h)
        off = np.empty(self.n + 1, np.int64)
        col = np.empty(max(nnz, 1), np.int32)
        w = np.empty(max(nnz, 1), np.int32)
        lib().orc_export_csr(self._h, _p(off), _p(col), _p(w))
        return off, col[:nnz], w[:nnz]

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _trace(recs, count, cap):
    out = []
    for r in range(min(count, cap)):
        x = recs[r]
        rec = (x.level, x.sweep, x.n_level, x.n_active, x.nnz_level, x.moves, x.dN, x.kept)
        # SLM refinement sweeps carry their phase as a ninth field
        out.append(rec + (x.phase,) if x.phase else rec)
    return out


# ---- stateless helpers over a CSR (diagonal entries allowed) ----

def csr_modularity(off, col, w, C):
    off, col, w, C = _i64(off), _i32(col), _i64(w), _i32(C)
    N, tm = ct.c_int64(), ct.c_int64()
    st = lib().orc_csr_modularity(len(off) - 1, _p(off), _p(col), _p(w), _p(C),
                                  ct.byref(N), ct.byref(tm))
    if st != 0:
        raise OracleError(st)
    return N.value, tm.value


def csr_gain(off, col, w, C, i, D):
    off, col, w, C = _i64(off), _i32(col), _i64(w), _i32(C)
    return lib().orc_csr_gain(len(off) - 1, _p(off), _p(col), _p(w), _p(C), int(i), int(D))


def csr_decide(off, col, w, C, i, guard=1):
    off, col, w, C = _i64(off), _i32(col), _i64(w), _i32(C)
    bg = ct.c_int64()
    d = lib().orc_csr_decide(len(off) - 1, _p(off), _p(col), _p(w), _p(C), int(i),
                             int(guard), ct.byref(bg))
    return d, bg.value


def csr_run_levels(off, col, w, C, active=None, **opt):
    off, col, w = _i64(off), _i32(col), _i64(w)
    n = len(off) - 1
    C = _i32(C).copy()
    act = np.ones(n, np.uint8) if active is None else np.ascontiguousarray(active, np.uint8)
    o = options(**opt)
    cap = 1 << 14
    recs = (SweepRec * cap)()
    ns, lv = ct.c_int32(), ct.c_int32()
    st = lib().orc_csr_run_levels(n, _p(off), _p(col), _p(w), _p(C), _p(act),
                                  ct.byref(o), recs, cap, ct.byref(ns), ct.byref(lv))
    if st != 0:
        raise OracleError(st)
    return C, _trace(recs, ns.value, cap), lv.value


def csr_coarsen(off, col, w, C):
    off, col, w, C = _i64(off), _i32(col), _i64(w), _i32(C)
    n = len(off) - 1
    rank = np.empty(n, np.int32)
    nout, nnz = ct.c_int32(), ct.c_int64()
    offo = np.empty(n + 1, np.int64)
    colo = np.empty(max(len(col), 1), np.int32)
    wo = np.empty(max(len(col), 1), np.int64)
    st = lib().orc_csr_coarsen(n, _p(off), _p(col), _p(w), _p(C), _p(rank),
                               ct.byref(nout), _p(offo), _p(colo), _p(wo), ct.byref(nnz))
    if st != 0:
        raise OracleError(st)
    k = nout.value
    return rank, offo[: k + 1], colo[: nnz.value], wo[: nnz.value]
