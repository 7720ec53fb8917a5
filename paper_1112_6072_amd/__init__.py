"""Python binding of libhperm: exact permanents of sparse non-negative integer matrices on MI355X.

Argument marshalling only: every step of the computation runs in the C++/HIP library
(``_build/libhperm.so``, built by ``paper_1112_6072_amd.build``). PyTorch supplies the HIP
stream (``torch.cuda.current_stream()``) and, optionally, the device arena the library
sub-allocates from. Importing this package fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libhperm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1112_6072_amd/build.py`")

# torch first: its HIP runtime is then the one the library binds to, whichever of the two is
# used first in the process (loading the library first left two runtimes, and contexts created
# afterwards saw no device)
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

OK, NOT_READY = 0, 1
ORDER_ESTIMATE, ORDER_NATURAL, ORDER_RANDOM, ORDER_EXACT_COST = 0, 1, 2, 3
ARITH_AUTO, ARITH_W64, ARITH_W128, ARITH_RES = 0, 1, 2, 3
ORDERS = {"estimate": 0, "natural": 1, "random": 2, "exact_cost": 3}
ARITHS = {"auto": 0, "w64": 1, "w128": 2, "res": 3}


class HpermError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_lib.hperm_status_string(status).decode()} ({status}): {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("m_cut", ctypes.c_int32), ("m_cap", ctypes.c_int32), ("s_leaf", ctypes.c_int32),
                ("arith", ctypes.c_int32), ("order", ctypes.c_int32), ("trials", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("chunk_log2", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("host_threads", ctypes.c_int32),
                ("max_table_mib", ctypes.c_int32), ("time_jobs", ctypes.c_int32),
                ("split_order", ctypes.c_int32), ("device_expand", ctypes.c_int32),
                ("device_expand_mib", ctypes.c_int32), ("use_graphs", ctypes.c_int32),
                ("serve_limit_ms", ctypes.c_int32)]


class Coeff(ctypes.Structure):
    _fields_ = [("limb", ctypes.c_uint64 * 8), ("nlimb", ctypes.c_int32), ("negative", ctypes.c_int32)]

    @property
    def value(self) -> int:
        v = sum(int(self.limb[k]) << (64 * k) for k in range(self.nlimb))
        return -v if self.negative else v


class Result(ctypes.Structure):
    _fields_ = [("limb", ctypes.c_uint64 * 8), ("nlimb", ctypes.c_int32), ("n_jobs", ctypes.c_int32),
                ("max_m", ctypes.c_int32), ("arith_mask", ctypes.c_int32),
                ("subset_terms", ctypes.c_uint64), ("t_expand_s", ctypes.c_double),
                ("t_estimate_s", ctypes.c_double), ("t_rnw_s", ctypes.c_double),
                ("t_total_s", ctypes.c_double)]

    @property
    def value(self) -> int:
        return sum(int(self.limb[k]) << (64 * k) for k in range(self.nlimb))

    def stats(self) -> dict:
        return {"n_jobs": self.n_jobs, "max_m": self.max_m, "arith_mask": self.arith_mask,
                "subset_terms": int(self.subset_terms), "t_expand_s": self.t_expand_s,
                "t_estimate_s": self.t_estimate_s, "t_rnw_s": self.t_rnw_s, "t_total_s": self.t_total_s}


class LaunchStat(ctypes.Structure):
    _fields_ = [("ring", ctypes.c_int32), ("bucket", ctypes.c_int32), ("n_jobs", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("variant", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("items", ctypes.c_uint64), ("terms", ctypes.c_uint64),
                ("row_updates", ctypes.c_uint64), ("alg_slots", ctypes.c_double), ("ms", ctypes.c_double),
                ("leaves", ctypes.c_uint64), ("leaf_terms", ctypes.c_uint64), ("splits", ctypes.c_uint64),
                ("split_stops", ctypes.c_uint64), ("deferred", ctypes.c_uint64),
                ("deferred_bound", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class TuneEntry(ctypes.Structure):
    _fields_ = [("ring", ctypes.c_int32), ("bucket", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("chunk_delta", ctypes.c_int32), ("grid_pct", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("ms_default", ctypes.c_double), ("ms_tuned", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_P = ctypes.c_void_p
_I32, _U64, _SZ = ctypes.c_int32, ctypes.c_uint64, ctypes.c_size_t
_SIGS = {
    "hperm_version": [ctypes.POINTER(_I32), ctypes.POINTER(_I32)],
    "hperm_default_opts": [ctypes.POINTER(Opts)],
    "hperm_ctx_create": [ctypes.POINTER(Opts), _P, ctypes.POINTER(_P)],
    "hperm_ctx_create_host": [ctypes.POINTER(Opts), ctypes.POINTER(_P)],
    "hperm_ctx_set_opts": [_P, ctypes.POINTER(Opts)],
    "hperm_ctx_get_opts": [_P, ctypes.POINTER(Opts)],
    "hperm_ctx_set_arena": [_P, _P, _SZ],
    "hperm_permanent_csr": [_P, _I32, _P, _P, _P, ctypes.POINTER(Result)],
    "hperm_permanent_dense": [_P, _I32, _P, ctypes.POINTER(Result)],
    "hperm_permanent_dense_noalloc": [_P, _I32, _P, ctypes.POINTER(Result)],
    "hperm_permanent_batch_csr": [_P, _I32, _P, _P, _P, _P, _P, _P, _P],
    "hperm_permanent_mod_batch_csr": [_P, _I32, _P, _P, _P, _P, _P, _P, ctypes.c_uint32, _P],
    "hperm_polynomial_from_residues": [_I32, _I32, _P, _P, _I32, _P],
    "hperm_expand_batch_csr": [_P, _I32, _P, _P, _P, _P, _P, _P, ctypes.POINTER(_P)],
    "hperm_jobs_from_dense": [_P, _I32, _P, _P, _P, ctypes.POINTER(_P)],
    "hperm_jobs_info": [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32)],
    "hperm_jobs_describe": [_P, _P, _P, _P, _P],
    "hperm_estimate": [_P, _P, _I32, _U64, _P],
    "hperm_run_jobs": [_P, _P, _I32, _I32, _P, _P],
    "hperm_serve_start": [_P, _I32, _SZ],
    "hperm_serve_stop": [_P],
    "hperm_submit": [_P, _I32, _P, _P, _P, ctypes.POINTER(_U64)],
    "hperm_poll": [_P, _U64, ctypes.POINTER(Result)],
    "hperm_wait": [_P, _U64, ctypes.c_double, ctypes.POINTER(Result)],
    "hperm_cancel": [_P, _U64],
    "hperm_last_launches": [_P, ctypes.POINTER(LaunchStat), _I32, ctypes.POINTER(_I32)],
    "hperm_jobs_cycles": [_P, _P],
    "hperm_jobs_matrix": [_P, _I32, _P],
    "hperm_device_expand_sample": [_P, _I32, _P, _P, _P, _I32, _I32, _P, _P, ctypes.POINTER(_I32),
                                   ctypes.POINTER(Result)],
    "hperm_permanental_polynomial": [_P, _I32, _P, _P, _P, _P],
    "hperm_polynomial_interpolate": [_I32, _P, _I32, _P],
    "hperm_list_schedule": [_I32, _P, _P, _I32, ctypes.POINTER(_U64), _P],
    "hperm_tree_estimate": [ctypes.POINTER(Opts), _I32, _P, _P, _P, _I32, _U64, _P, _P],
    "hperm_autotune": [_P, _P, ctypes.c_char_p, _I32, ctypes.POINTER(TuneEntry), _I32, ctypes.POINTER(_I32)],
    "hperm_tune_clear": [_P],
    "hperm_matrix_invariants": [_I32, _P, _P],
    "hperm_ols": [_I32, _I32, _P, _P, _P, ctypes.POINTER(ctypes.c_double)],
    "hperm_stepwise": [_I32, _I32, _P, _P, ctypes.c_double, ctypes.c_double, _P, ctypes.POINTER(_I32)],
    "hperm_kendall_tau": [_I32, _P, _P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(ctypes.c_double)],
}
for _name, _args in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = ctypes.c_int
_lib.hperm_ctx_destroy.argtypes = [_P]
_lib.hperm_ctx_destroy.restype = None
_lib.hperm_jobs_free.argtypes = [_P]
_lib.hperm_jobs_free.restype = None
_lib.hperm_status_string.argtypes = [ctypes.c_int]
_lib.hperm_status_string.restype = ctypes.c_char_p
_lib.hperm_last_error.argtypes = [_P]
_lib.hperm_last_error.restype = ctypes.c_char_p
_lib.hperm_ctx_arena_required.argtypes = [_P]
_lib.hperm_ctx_arena_required.restype = _SZ

EXPORTED = sorted(list(_SIGS) + ["hperm_ctx_destroy", "hperm_jobs_free", "hperm_status_string",
                                 "hperm_last_error", "hperm_ctx_arena_required"])


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_P)


def _csr(A) -> tuple[int, np.ndarray, np.ndarray, np.ndarray]:
    A = np.asarray(A)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("square matrix expected")
    if A.size and (A.min() < 0):
        raise ValueError("entries must be non-negative")
    n = A.shape[0]
    rows, cols = np.nonzero(A)
    rp = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    return n, rp, cols.astype(np.int32), A[rows, cols].astype(np.uint32)


def _batch_csr(mats):
    parts = [_csr(A) for A in mats]
    n = np.array([p[0] for p in parts], dtype=np.int32)
    rp_off = np.zeros(len(parts), dtype=np.int64)
    nz_off = np.zeros(len(parts), dtype=np.int64)
    o1 = o2 = 0
    for k, p in enumerate(parts):
        rp_off[k], nz_off[k] = o1, o2
        o1 += p[1].size
        o2 += p[2].size
    cat = lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(1, dt)  # noqa: E731
    rp = cat([p[1] for p in parts], np.int32)
    ci = cat([p[2] for p in parts] + [np.zeros(1, np.int32)], np.int32)
    va = cat([p[3] for p in parts] + [np.zeros(1, np.uint32)], np.uint32)
    return n, rp_off, nz_off, rp, ci, va


def default_opts() -> dict:
    o = Opts()
    _lib.hperm_default_opts(ctypes.byref(o))
    return {f: getattr(o, f) for f, _ in Opts._fields_}


def _opts(d: dict | None) -> Opts:
    o = Opts()
    _lib.hperm_default_opts(ctypes.byref(o))
    for k, v in (d or {}).items():
        if k == "order" and isinstance(v, str):
            v = ORDERS[v]
        if k == "arith" and isinstance(v, str):
            v = ARITHS[v]
        setattr(o, k, v)
    return o


class Jobs:
    """A job table owned by the library (sub-matrices produced by the expansion)."""

    def __init__(self, ctx: "Context", handle):
        self._ctx = ctx
        self.handle = handle

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.hperm_jobs_free(self.handle)
        self.handle = None

    def info(self) -> tuple[int, int]:
        nj, npb = _I32(), _I32()
        _lib.hperm_jobs_info(self.handle, ctypes.byref(nj), ctypes.byref(npb))
        return nj.value, npb.value

    def describe(self) -> dict:
        nj, _ = self.info()
        m = np.zeros(max(nj, 1), np.int32)
        prob = np.zeros(max(nj, 1), np.int32)
        ar = np.zeros(max(nj, 1), np.int32)
        terms = np.zeros(max(nj, 1), np.uint64)
        _lib.hperm_jobs_describe(self.handle, _ptr(m), _ptr(prob), _ptr(ar), _ptr(terms))
        return {"m": m[:nj], "problem": prob[:nj], "arith": ar[:nj], "terms": terms[:nj]}

    def matrix(self, k: int) -> np.ndarray:
        """Job k's sub-matrix as the kernels hold it (rows in job order, Gray columns, then the
        fixed column)."""
        d = self.describe()["m"]
        m = int(d[k]) if 0 <= k < len(d) else 0
        out = np.zeros(max(m * m, 1), np.uint32)
        st = _lib.hperm_jobs_matrix(self.handle, int(k), _ptr(out))
        if st != OK:
            raise HpermError(st, "job index out of range")
        return out[:m * m].reshape(m, m)

    def cycles(self) -> np.ndarray:
        """Per-job work cycles of the last timed persistent run (opts time_jobs=1)."""
        nj, _ = self.info()
        out = np.zeros(max(nj, 1), np.uint64)
        st = _lib.hperm_jobs_cycles(self.handle, _ptr(out))
        if st != OK:
            raise HpermError(st, "no timed run on these jobs (set time_jobs=1 and run persistent)")
        return out[:nj]


class Context:
    """A library context on the current HIP device, running on torch's current stream.

    ``host_only=True`` makes a context without a device (host stages only)."""

    def __init__(self, opts: dict | None = None, stream=None, arena_bytes: int = 0,
                 host_only: bool = False):
        self._opts = _opts(opts)
        h = _P()
        if host_only:
            st = _lib.hperm_ctx_create_host(ctypes.byref(self._opts), ctypes.byref(h))
        else:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("no HIP device visible")
            if stream is None:
                stream = torch.cuda.current_stream().cuda_stream
            st = _lib.hperm_ctx_create(ctypes.byref(self._opts), _P(stream), ctypes.byref(h))
        if st != OK:
            raise HpermError(st, "hperm_ctx_create")
        self.handle = h
        self._arena = None
        if arena_bytes:
            self.set_arena(arena_bytes)

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.hperm_ctx_destroy(self.handle)
        self.handle = None
        self._arena = None

    __del__ = close

    def _check(self, st: int, what: str):
        if st not in (OK,):
            raise HpermError(st, f"{what}: {_lib.hperm_last_error(self.handle).decode()}")

    def set_opts(self, **kw):
        o = _opts(None)
        ctypes.memmove(ctypes.byref(o), ctypes.byref(self._opts), ctypes.sizeof(Opts))
        for k, v in kw.items():
            if k == "order" and isinstance(v, str):
                v = ORDERS[v]
            if k == "arith" and isinstance(v, str):
                v = ARITHS[v]
            setattr(o, k, v)
        self._check(_lib.hperm_ctx_set_opts(self.handle, ctypes.byref(o)), "set_opts")
        self._opts = o

    def set_arena(self, nbytes: int):
        """Give the library a torch-allocated device arena of nbytes (0 returns to its own memory)."""
        import torch
        if nbytes:
            self._arena = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
            ptr, size = self._arena.data_ptr(), self._arena.numel()
        else:
            self._arena, ptr, size = None, None, 0
        self._check(_lib.hperm_ctx_set_arena(self.handle, _P(ptr) if ptr else None, size), "set_arena")

    def last_launches(self) -> list[dict]:
        """R-NW launches of the last run: ring, bucket, jobs, items, terms, alg_slots, ms."""
        buf = (LaunchStat * 64)()
        n = _I32()
        self._check(_lib.hperm_last_launches(self.handle, buf, 64, ctypes.byref(n)), "last_launches")
        return [buf[k].as_dict() for k in range(min(n.value, 64))]

    def arena_required(self) -> int:
        return int(_lib.hperm_ctx_arena_required(self.handle))

    # ---------------------------------------------------------------- blocking calls
    def permanent(self, A) -> int:
        return self.permanent_batch([A])[0]

    def permanent_batch(self, mats, with_stats: bool = False):
        n, rp_off, nz_off, rp, ci, va = _batch_csr(mats)
        out = (Result * max(len(mats), 1))()
        st = _lib.hperm_permanent_batch_csr(self.handle, len(mats), _ptr(n), _ptr(rp_off), _ptr(nz_off),
                                            _ptr(rp), _ptr(ci), _ptr(va), out)
        self._check(st, "permanent_batch")
        vals = [out[k].value for k in range(len(mats))]
        if with_stats:
            return vals, [out[k].stats() for k in range(len(mats))]
        return vals

    def permanent_mod_batch(self, mats, prime: int) -> list[int]:
        """per(A) mod prime for each matrix (odd prime below 2^18, orders above the device
        expansion's order up to 64), on the device path in modular arithmetic."""
        n, rp_off, nz_off, rp, ci, va = _batch_csr(mats)
        out = np.zeros(max(len(mats), 1), np.uint64)
        st = _lib.hperm_permanent_mod_batch_csr(self.handle, len(mats), _ptr(n), _ptr(rp_off), _ptr(nz_off),
                                                _ptr(rp), _ptr(ci), _ptr(va), int(prime), _ptr(out))
        self._check(st, "permanent_mod_batch")
        return [int(out[k]) for k in range(len(mats))]

    def permanent_dense(self, A) -> int:
        """per(A) through hperm_permanent_dense (expansion as the options say)."""
        a = np.ascontiguousarray(np.asarray(A, dtype=np.uint32))
        r = Result()
        self._check(_lib.hperm_permanent_dense(self.handle, int(a.shape[0]), _ptr(a) if a.size else None,
                                               ctypes.byref(r)), "permanent_dense")
        return r.value

    def permanent_dense_noalloc(self, A) -> int:
        """per(A) of a dense matrix of order <= 40 as one job, with no allocation in the call
        (the library's fixed scratch array per GPU; overlapping calls on one GPU race)."""
        a = np.ascontiguousarray(np.asarray(A, dtype=np.uint32))
        if a.ndim != 2 or a.shape[0] != a.shape[1]:
            raise ValueError("square matrix expected")
        r = Result()
        self._check(_lib.hperm_permanent_dense_noalloc(self.handle, int(a.shape[0]), _ptr(a) if a.size else None,
                                                       ctypes.byref(r)), "permanent_dense_noalloc")
        return r.value

    def permanental_polynomial(self, A) -> list[int]:
        """Exact coefficients c_0..c_n of per(xI - A) = sum_k c_k x^k (c_k of x^k)."""
        n, rp, ci, va = _csr(A)
        ci = ci if ci.size else np.zeros(1, np.int32)
        va = va if va.size else np.zeros(1, np.uint32)
        out = (Coeff * (n + 1))()
        self._check(_lib.hperm_permanental_polynomial(self.handle, n, _ptr(rp), _ptr(ci), _ptr(va), out),
                    "permanental_polynomial")
        return [out[k].value for k in range(n + 1)]

    def permanent_csr(self, n, row_ptr, col_idx, val) -> int:
        rp = np.ascontiguousarray(row_ptr, np.int32)
        ci = np.ascontiguousarray(col_idx, np.int32)
        va = np.ascontiguousarray(val, np.uint32)
        r = Result()
        st = _lib.hperm_permanent_csr(self.handle, int(n), _ptr(rp), _ptr(ci) if ci.size else None,
                                      _ptr(va) if va.size else None, ctypes.byref(r))
        self._check(st, "permanent_csr")
        return r.value

    def device_expand_sample(self, A, max_jobs: int, stop_early: bool = False):
        """The device expansion (options device_expand = T, split_order = t) of one matrix,
        keeping its first max_jobs jobs of order T in tree order: returns (total or None when
        stopped early, list of T x T job matrices, their exact values, stats of the total)."""
        n, rp, ci, va = _csr(A)
        T = int(self._opts.device_expand)
        k = max(int(max_jobs), 0)
        mats = np.zeros(max(k * T * T, 1), np.uint32)
        vals = (Result * max(k, 1))()
        got = _I32()
        tot = Result()
        st = _lib.hperm_device_expand_sample(self.handle, n, _ptr(rp), _ptr(ci) if ci.size else None,
                                             _ptr(va) if va.size else None, k, 1 if stop_early else 0,
                                             _ptr(mats), vals, ctypes.byref(got), ctypes.byref(tot))
        self._check(st, "device_expand_sample")
        g = got.value
        jobs = [mats[q * T * T:(q + 1) * T * T].reshape(T, T).copy() for q in range(g)]
        total = tot.value if tot.max_m else None
        return total, jobs, [vals[q].value for q in range(g)], tot.stats()

    # ---------------------------------------------------------------- stages
    def expand(self, mats) -> Jobs:
        n, rp_off, nz_off, rp, ci, va = _batch_csr(mats)
        h = _P()
        st = _lib.hperm_expand_batch_csr(self.handle, len(mats), _ptr(n), _ptr(rp_off), _ptr(nz_off),
                                         _ptr(rp), _ptr(ci), _ptr(va), ctypes.byref(h))
        self._check(st, "expand")
        return Jobs(self, h)

    def jobs_from_dense(self, mats) -> Jobs:
        mats = [np.ascontiguousarray(np.asarray(A, dtype=np.uint32)) for A in mats]
        m = np.array([A.shape[0] for A in mats], np.int32)
        sizes = np.array([A.size for A in mats], np.int64)
        off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        a = np.concatenate([A.ravel() for A in mats] + [np.zeros(1, np.uint32)])
        h = _P()
        st = _lib.hperm_jobs_from_dense(self.handle, len(mats), _ptr(m), _ptr(off), _ptr(a), ctypes.byref(h))
        self._check(st, "jobs_from_dense")
        return Jobs(self, h)

    def estimate(self, jobs: Jobs, trials: int = 32, seed: int = 1) -> np.ndarray:
        nj, _ = jobs.info()
        keys = np.zeros(max(nj, 1), np.float32)
        self._check(_lib.hperm_estimate(self.handle, jobs.handle, int(trials), int(seed), _ptr(keys)),
                    "estimate")
        return keys[:nj]

    def run(self, jobs: Jobs, order="estimate", persistent: bool = True, per_job: bool = False):
        """Evaluate all jobs; returns (totals, per_job values or None, total Result list)."""
        nj, npb = jobs.info()
        order = ORDERS[order] if isinstance(order, str) else int(order)
        pj = (Result * max(nj, 1))() if per_job else None
        tot = (Result * max(npb, 1))()
        st = _lib.hperm_run_jobs(self.handle, jobs.handle, order, 1 if persistent else 0, pj, tot)
        self._check(st, "run_jobs")
        totals = [tot[k].value for k in range(npb)]
        pjv = [pj[k].value for k in range(nj)] if per_job else None
        return totals, pjv, [tot[k] for k in range(npb)]

    def autotune(self, jobs: "Jobs | None" = None, cache_path: str | None = None, force: bool = False) -> list[dict]:
        """Tune the persistent R-NW launches on a job table's launch groups (or only load a
        cache); returns the context's tuning table."""
        buf = (TuneEntry * 64)()
        n = _I32()
        self._check(_lib.hperm_autotune(self.handle, jobs.handle if jobs is not None else None,
                                        cache_path.encode() if cache_path else None, 1 if force else 0,
                                        buf, 64, ctypes.byref(n)), "autotune")
        return [buf[k].as_dict() for k in range(min(n.value, 64))]

    def tune_clear(self):
        self._check(_lib.hperm_tune_clear(self.handle), "tune_clear")

    # ---------------------------------------------------------------- serving
    def serve_start(self, max_requests: int = 1024, arena_bytes: int = 1 << 30):
        """Start continuous batching: requests share device queues, admitted by arena_bytes."""
        self._check(_lib.hperm_serve_start(self.handle, int(max_requests), int(arena_bytes)), "serve_start")

    def serve_stop(self):
        self._check(_lib.hperm_serve_stop(self.handle), "serve_stop")

    def submit(self, A) -> int | None:
        """Submit per(A); returns a ticket, or None when every request slot is taken."""
        n, rp, ci, va = _csr(A)
        t = _U64()
        st = _lib.hperm_submit(self.handle, n, _ptr(rp), _ptr(ci) if ci.size else None,
                               _ptr(va) if va.size else None, ctypes.byref(t))
        if st == -5:   # HPERM_E_BUSY
            return None
        self._check(st, "submit")
        return int(t.value)

    def poll(self, ticket: int):
        """(value, stats) when done, None while running."""
        r = Result()
        st = _lib.hperm_poll(self.handle, int(ticket), ctypes.byref(r))
        if st == NOT_READY:
            return None
        self._check(st, "poll")
        return r.value, r.stats()

    def wait(self, ticket: int, timeout_s: float = -1.0):
        """Block until the request is done (timeout_s < 0: no limit); returns (value, stats)."""
        r = Result()
        self._check(_lib.hperm_wait(self.handle, int(ticket), float(timeout_s), ctypes.byref(r)), "wait")
        return r.value, r.stats()

    def cancel(self, ticket: int):
        self._check(_lib.hperm_cancel(self.handle, int(ticket)), "cancel")


def version() -> tuple[int, int]:
    a, b = _I32(), _I32()
    _lib.hperm_version(ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


_default_ctx = None


def permanent(A, **opts) -> int:
    """per(A) of a square non-negative integer matrix (numpy array or nested lists), exact."""
    global _default_ctx
    if opts:
        ctx = Context(opts)
        try:
            return ctx.permanent(A)
        finally:
            ctx.close()
    if _default_ctx is None:
        _default_ctx = Context()
    return _default_ctx.permanent(A)


def tree_estimate(A, samples: int = 2000, seed: int = 1, **opts) -> tuple[np.ndarray, np.ndarray]:
    """Knuth's estimate of per(A)'s expansion tree under the default path's rule (options as
    for Context): (nodes per order, leaves per order), arrays of length n + 1."""
    n, rp, ci, va = _csr(A)
    o = _opts(opts)
    nodes = np.zeros(n + 1, np.float64)
    leaves = np.zeros(n + 1, np.float64)
    st = _lib.hperm_tree_estimate(ctypes.byref(o), n, _ptr(rp), _ptr(ci) if ci.size else None,
                                  _ptr(va) if va.size else None, int(samples), int(seed), _ptr(nodes), _ptr(leaves))
    if st != OK:
        raise HpermError(st, "tree_estimate")
    return nodes, leaves


def list_schedule(times, order, machines: int) -> tuple[int, np.ndarray]:
    """List scheduling (Step 3 of Algorithm PH): (makespan, per-machine loads) of the jobs with
    the given integer times assigned in `order` to the least-loaded of `machines` machines."""
    t = np.ascontiguousarray(times, dtype=np.uint64)
    o = np.ascontiguousarray(order, dtype=np.int32)
    if t.ndim != 1 or o.shape != t.shape:
        raise ValueError("times and order must be 1-D of equal length")
    loads = np.zeros(max(int(machines), 1), np.uint64)
    ms = _U64()
    st = _lib.hperm_list_schedule(int(t.size), _ptr(t), _ptr(o), int(machines), ctypes.byref(ms), _ptr(loads))
    if st != OK:
        raise HpermError(st, "list_schedule")
    return int(ms.value), loads


def kendall_tau(x, y) -> tuple[float, float, float]:
    """Kendall's tau with tie correction (tau_b), its normal score under independence and the
    two-sided p-value."""
    a = np.ascontiguousarray(x, dtype=np.float64)
    b = np.ascontiguousarray(y, dtype=np.float64)
    if a.ndim != 1 or a.shape != b.shape:
        raise ValueError("x and y must be 1-D of equal length")
    tau, z, p = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    st = _lib.hperm_kendall_tau(int(a.size), _ptr(a), _ptr(b), ctypes.byref(tau), ctypes.byref(z), ctypes.byref(p))
    if st != OK:
        raise HpermError(st, "kendall_tau")
    return tau.value, z.value, p.value


def matrix_invariants(A) -> tuple[float, int, float, float]:
    """(|D|, S, V1, V2) of a dense non-negative integer matrix: |det| (a float), the nonzero
    count and the population variances of the row and column sums (Section 3.1)."""
    a = np.ascontiguousarray(A, dtype=np.uint32)
    if a.ndim != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("A must be square")
    out = np.zeros(4, np.float64)
    st = _lib.hperm_matrix_invariants(int(a.shape[0]), _ptr(a), _ptr(out))
    if st != OK:
        raise HpermError(st, "matrix_invariants")
    return float(out[0]), int(out[1]), float(out[2]), float(out[3])


def ols(X, y) -> tuple[np.ndarray, float]:
    """Least squares of y on the columns of X with an intercept: (a0..ak, R^2 as the paper
    defines it)."""
    yy = np.ascontiguousarray(y, dtype=np.float64)
    Xa = np.ascontiguousarray(np.asarray(X, dtype=np.float64).reshape(yy.size, -1))
    coef = np.zeros(Xa.shape[1] + 1, np.float64)
    r2 = ctypes.c_double()
    st = _lib.hperm_ols(int(yy.size), int(Xa.shape[1]), _ptr(Xa), _ptr(yy), _ptr(coef), ctypes.byref(r2))
    if st != OK:
        raise HpermError(st, "ols")
    return coef, r2.value


def stepwise(X, y, f_enter: float = 4.0, f_remove: float = 3.9) -> list[int]:
    """Efroymson's stepwise selection: the chosen columns of X in entry order."""
    yy = np.ascontiguousarray(y, dtype=np.float64)
    Xa = np.ascontiguousarray(np.asarray(X, dtype=np.float64).reshape(yy.size, -1))
    chosen = np.zeros(Xa.shape[1], np.int32)
    nc = _I32()
    st = _lib.hperm_stepwise(int(yy.size), int(Xa.shape[1]), _ptr(Xa), _ptr(yy), float(f_enter), float(f_remove),
                             _ptr(chosen), ctypes.byref(nc))
    if st != OK:
        raise HpermError(st, "stepwise")
    return [int(c) for c in chosen[:nc.value]]


def polynomial_interpolate(values, alternate: bool = False) -> list[int]:
    """Integer coefficients (low to high) of the degree-n polynomial through (x, values[x]),
    x = 0..n, for non-negative integer values below 2^512 (the host step of the permanental
    polynomial; with alternate, coefficient k is negated when n - k is odd)."""
    n = len(values) - 1
    if n < 0:
        raise ValueError("at least one value")
    limbs = np.zeros((n + 1) * 8, dtype=np.uint64)
    for x, v in enumerate(values):
        v = int(v)
        if v < 0 or v >> 512:
            raise ValueError("values must be non-negative and below 2^512")
        for k in range(8):
            limbs[8 * x + k] = (v >> (64 * k)) & ((1 << 64) - 1)
    out = (Coeff * (n + 1))()
    st = _lib.hperm_polynomial_interpolate(n, _ptr(limbs), 1 if alternate else 0, out)
    if st != OK:
        raise HpermError(st, "polynomial_interpolate")
    return [out[k].value for k in range(n + 1)]


def polynomial_from_residues(primes, residues, alternate: bool = False) -> list[int]:
    """Coefficients (low to high) of the polynomial with non-negative coefficients below the
    product of primes[:-1] whose values at x = 0..n are residues[j][x] modulo primes[j]: per-prime
    interpolation and the Chinese remainder theorem, checked against the last prime."""
    pr = np.ascontiguousarray(primes, dtype=np.uint32)
    res = np.ascontiguousarray(residues, dtype=np.uint64)
    if res.ndim != 2 or res.shape[0] != pr.size:
        raise ValueError("one row of residues per prime")
    n = res.shape[1] - 1
    out = (Coeff * max(n + 1, 1))()
    st = _lib.hperm_polynomial_from_residues(n, int(pr.size), _ptr(pr), _ptr(res), 1 if alternate else 0, out)
    if st != OK:
        raise HpermError(st, "polynomial_from_residues")
    return [out[k].value for k in range(n + 1)]
