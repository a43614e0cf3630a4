"""ctypes binding of libgrest (include/grest.h).

Argument marshalling only: every step of the update runs in the HIP library.
Host arrays are NumPy arrays; device arrays are torch tensors on the state's
device (their data pointers are passed through).  The library must have been
built (``python -m paper_2603_19439_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrest.so")

OK, EINVAL, ENOMEM, EDEVICE, ENUMERIC, ENODEV, EAGAIN = range(7)
OP = {"adj": 0, "lap": 1, "nlap": 2}
VARIANT = {"g2": 2, "g3": 3, "rsvd": 4}
PRECISION = {"fp64": 0, "fp32": 1, "mixed": 2}
HOST, DEVICE = 0, 1
F64, F32 = 0, 1


class GrestError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__(f"{where}: status {status} ({_strerror(status)}) {detail}".strip())


class Config(C.Structure):
    _fields_ = [("k", C.c_int32), ("variant", C.c_int32), ("L", C.c_int32), ("P", C.c_int32),
                ("op", C.c_int32), ("precision", C.c_int32), ("max_new", C.c_int32),
                ("proj", C.c_int32), ("rank_tol", C.c_double)]


_lib = None

BATCH_MAX = 64


class BatchItem(C.Structure):
    """grest_batch_item of include/grest.h."""
    _fields_ = [("state", C.c_void_p), ("n_new", C.c_int64), ("n_changes", C.c_int64), ("ei", C.c_void_p),
                ("ej", C.c_void_p), ("sign", C.c_void_p), ("omega", C.c_void_p), ("where", C.c_int32),
                ("status", C.c_int32)]

# (name, restype, argtypes) of every entry point of include/grest.h
_SIGS = [
    ("grest_abi_version", C.c_int32, []),
    ("grest_strerror", C.c_char_p, [C.c_int]),
    ("grest_last_error", C.c_char_p, []),
    ("grest_validate_changes", C.c_int, [C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("grest_create", C.c_int, [C.POINTER(Config), C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                               C.c_int64, C.POINTER(C.c_void_p)]),
    ("grest_set_pairs", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    ("grest_init_pairs", C.c_int, [C.c_void_p, C.c_int32, C.c_uint64]),
    ("grest_init_pairs_tol", C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_uint64, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_double)]),
    ("grest_init_stats", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    ("grest_update", C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_int32]),
    ("grest_update_noalloc", C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_int32]),
    ("grest_update_batch", C.c_int, [C.c_void_p, C.c_int32]),
    ("grest_sync", C.c_int, [C.c_void_p]),
    ("grest_get", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32]),
    ("grest_shape", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                              C.POINTER(C.c_int32)]),
    ("grest_get_graph", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("grest_profile", C.c_int, [C.c_void_p, C.c_int32]),
    ("grest_stage_times", C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_double),
                                    C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    ("grest_destroy", None, [C.c_void_p]),
    ("grest_set_stream", C.c_int, [C.c_void_p, C.c_void_p]),
    ("grest_set_overlap", C.c_int, [C.c_void_p, C.c_int32]),
    ("grest_memory", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("grest_release_graph", C.c_int, [C.c_void_p]),
    ("grest_save", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t)]),
    ("grest_load", C.c_int, [C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    ("grest_view", C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                             C.POINTER(C.c_int32)]),
    ("grest_drift", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("grest_set_restart", C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_uint64]),
    ("grest_restart_stats", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]),
    ("grest_now_ns", C.c_int64, []),
    ("grest_server_create", C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.POINTER(C.c_void_p)]),
    ("grest_server_create_batched", C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_void_p)]),
    ("grest_server_attach", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]),
    ("grest_submit", C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_uint64]),
    ("grest_poll", C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("grest_server_detach", C.c_int, [C.c_void_p, C.c_int32]),
    ("grest_server_memory", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    ("grest_server_drain", C.c_int, [C.c_void_p]),
    ("grest_server_destroy", None, [C.c_void_p]),
    # measurement aid (grest_calib.h)
    ("grest_calib_gather", C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_int64,
                                     C.c_uint64, C.c_void_p]),
]


def lib():
    """Load libgrest.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_19439_amd.build`")
        # Load torch's HIP runtime first: libgrest then binds to the same libamdhip64.so.7,
        # so device memory and streams handed over by torch belong to one runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _strerror(status: int) -> str:
    try:
        return lib().grest_strerror(status).decode()
    except Exception:  # library not loadable
        return "?"


def _check(status: int, where: str):
    if status != OK:
        detail = lib().grest_last_error().decode()
        raise GrestError(status, where, detail)


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _ptr(a, dtype):
    """(keepalive, pointer, where) for a NumPy array (host) or a torch tensor (device)."""
    if a is None:
        return None, None, HOST
    mod = type(a).__module__
    if mod.startswith("torch"):
        if not a.is_contiguous():
            raise ValueError("device arrays must be contiguous")
        return a, C.c_void_p(a.data_ptr()), (DEVICE if a.is_cuda else HOST)
    arr, p = _host(a, dtype)
    return arr, p, HOST


def validate_changes(n: int, n_new: int, i, j, sign) -> bool:
    i, pi = _host(i, np.int32)
    j, pj = _host(j, np.int32)
    s, ps = _host(sign, np.int8)
    return lib().grest_validate_changes(int(n), int(n_new), int(i.size), pi, pj, ps) == OK


def calib_gather(rp, Z, w: int, Y, seed: int = 1, stream=None):
    """Random-gather ceiling (grest_calib_gather): rp a device int64 tensor of n + 1 row
    pointers, Z and Y device FP32 tensors of n rows whose strides meet the call's rules;
    the call only enqueues on `stream` (a torch stream, default the current one)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(Z.device)
    n = int(rp.numel()) - 1
    if rp.dtype != torch.int64 or not rp.is_cuda or not rp.is_contiguous() or Z.shape[0] != n or Y.shape[0] != n:
        raise GrestError(1, "calib_gather: rp must be a contiguous device int64 tensor of n + 1 entries, Z and Y n rows")
    _check(lib().grest_calib_gather(n, C.c_void_p(rp.data_ptr()), C.c_void_p(Z.data_ptr()), int(Z.stride(0)), int(w),
                                    C.c_void_p(Y.data_ptr()), int(Y.stride(0)), int(seed),
                                    C.c_void_p(stream.cuda_stream)), "grest_calib_gather")


def update_batch(updates):
    """Updates of several states at once (grest_update_batch): updates is a list of
    (state, n_new, i, j, sign, omega) with distinct states; returns the per-member statuses
    and raises on the first failure."""
    items = (BatchItem * len(updates))()
    keep = []
    for it, (st, n_new, i, j, sign, omega) in zip(items, updates):
        ai, pi, w1 = _ptr(i, np.int32)
        aj, pj, _ = _ptr(j, np.int32)
        asg, ps, _ = _ptr(sign, np.int8)
        ao, po, w4 = _ptr(omega, np.float64)
        if omega is not None and w4 != w1:
            raise ValueError("omega must live where the change arrays live")
        nc = int(ai.numel() if hasattr(ai, "numel") else np.asarray(ai).size)
        it.state = st._h.value
        it.n_new = int(n_new)
        it.n_changes = nc
        it.ei, it.ej, it.sign, it.omega = (None if p is None else p.value for p in (pi, pj, ps, po))
        it.where = w1
        keep.append((ai, aj, asg, ao))
    rc = lib().grest_update_batch(items, len(updates))
    for (st, *_), k in zip(updates, keep):
        st._keep = k
    _check(rc, "grest_update_batch")
    return [it.status for it in items]


class State:
    """A G-REST state on the current HIP device (see grest.h)."""

    def __init__(self, rowptr, col, k: int, variant: str = "g3", op: str = "adj", precision: str = "fp64",
                 L: int = 0, P: int = 0, max_new: int = 0, rank_tol: float = 0.0, stream=None,
                 node_capacity: int = 0, nnz_capacity: int = 0, proj: str = "exact"):
        self._h = C.c_void_p()
        cfg = Config(k=k, variant=VARIANT[variant], L=L, P=P, op=OP[op], precision=PRECISION[precision],
                     max_new=max_new, proj={"exact": 0, "lowrank": 1}[proj], rank_tol=rank_tol)
        rp, prp = _host(rowptr, np.int64)
        cl, pcl = _host(col, np.int32)
        n0 = rp.size - 1
        sp = C.c_void_p(stream) if stream else None
        _check(lib().grest_create(C.byref(cfg), sp, n0, prp, pcl, int(node_capacity), int(nnz_capacity),
                                  C.byref(self._h)), "grest_create")
        self.k = k
        self.op = op
        self.precision = precision
        self._lib = lib()  # kept for the destructor, which may run during interpreter exit

    def save(self) -> bytes:
        """Checkpoint of the state (graph, capacities, pairs, kept product) as bytes."""
        size = C.c_size_t(0)
        _check(lib().grest_save(self._h, None, C.byref(size)), "grest_save")
        buf = C.create_string_buffer(size.value)
        _check(lib().grest_save(self._h, buf, C.byref(size)), "grest_save")
        return buf.raw[:size.value]

    @classmethod
    def load(cls, blob: bytes, stream=None) -> "State":
        """A new state resumed from a checkpoint made by save()."""
        import struct
        self = cls.__new__(cls)
        self._h = C.c_void_p()
        buf = C.create_string_buffer(blob, len(blob))
        sp = C.c_void_p(stream) if stream else None
        _check(lib().grest_load(buf, len(blob), sp, C.byref(self._h)), "grest_load")
        # header: magic, abi, element size, then the config's k, variant, L, P, op, precision
        k, _, _, _, op, prec = struct.unpack_from("<6i", blob, 16)
        self.k = k
        self.op = {v: n for n, v in OP.items()}[op]
        self.precision = {v: n for n, v in PRECISION.items()}[prec]
        self._lib = lib()
        return self

    def view(self) -> Tuple[int, int, int, int]:
        """(device address, rows, leading dimension, dtype code) of the basis buffer whose
        first k columns are the tracked block (borrowed: valid until the state changes)."""
        x, n, ld, dt = C.c_void_p(), C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib().grest_view(self._h, C.byref(x), C.byref(n), C.byref(ld), C.byref(dt)), "grest_view")
        return int(x.value or 0), n.value, ld.value, dt.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.grest_destroy(self._h)
            self._h = C.c_void_p()

    __del__ = close

    def set_pairs(self, values, X):
        v, pv, wv = _ptr(values, np.float64)
        x, px, wx = _ptr(X, np.float64)
        if wv != wx:
            raise ValueError("values and X must both be host or both be device arrays")
        _check(lib().grest_set_pairs(self._h, pv, px, wx), "grest_set_pairs")

    def init_pairs(self, iterations: int = 30, seed: int = 0, tol: Optional[float] = None):
        """Initial pairs on the device (at most ``iterations`` products with the operator);
        with ``tol`` the residual target of grest_init_pairs_tol, else the precision's
        default.  Returns (products used, final residual)."""
        if tol is None:
            _check(lib().grest_init_pairs(self._h, int(iterations), int(seed)), "grest_init_pairs")
            return self.init_stats()
        p, r = C.c_int32(), C.c_double()
        _check(lib().grest_init_pairs_tol(self._h, int(iterations), float(tol), int(seed), C.byref(p), C.byref(r)),
               "grest_init_pairs_tol")
        return p.value, r.value

    def init_stats(self) -> Tuple[int, float]:
        """(products, final residual) of the last initial eigensolve."""
        p, r = C.c_int32(), C.c_double()
        _check(lib().grest_init_stats(self._h, C.byref(p), C.byref(r)), "grest_init_stats")
        return p.value, r.value

    def update(self, n_new: int, i, j, sign, omega=None, noalloc: bool = False):
        """One update (grest_update); noalloc=True calls grest_update_noalloc, which
        allocates nothing and needs the state's capacities to suffice."""
        ai, pi, w1 = _ptr(i, np.int32)
        aj, pj, w2 = _ptr(j, np.int32)
        asg, ps, w3 = _ptr(sign, np.int8)
        ao, po, w4 = _ptr(omega, np.float64)
        nc = int(ai.numel() if hasattr(ai, "numel") else np.asarray(ai).size)
        where = w1
        if omega is not None and w4 != where:
            raise ValueError("omega must live where the change arrays live")
        name = "grest_update_noalloc" if noalloc else "grest_update"
        _check(getattr(lib(), name)(self._h, int(n_new), nc, pi, pj, ps, po, where), name)
        self._keep = (ai, aj, asg, ao)

    def update_delta(self, d, omega=None, noalloc: bool = False):
        return self.update(d.n_new, d.i, d.j, d.sign, omega, noalloc=noalloc)

    def sync(self):
        _check(lib().grest_sync(self._h), "grest_sync")

    def shape(self) -> Tuple[int, int, int, int]:
        n, m = C.c_int64(), C.c_int64()
        k, w = C.c_int32(), C.c_int32()
        _check(lib().grest_shape(self._h, C.byref(n), C.byref(m), C.byref(k), C.byref(w)), "grest_shape")
        return n.value, m.value, k.value, w.value

    def get(self, dtype=np.float64, out=None):
        """(values, X): values FP64 host, X n x k host array (or ``out``, a device tensor)."""
        n, _, k, _ = self.shape()
        vals = np.empty(k, dtype=np.float64)
        xd = F64 if np.dtype(dtype) == np.float64 else F32
        if out is None:
            X = np.empty((n, k), dtype=dtype)
            _check(lib().grest_get(self._h, vals.ctypes.data_as(C.c_void_p), X.ctypes.data_as(C.c_void_p), xd, HOST),
                   "grest_get")
            return vals, X
        _check(lib().grest_get(self._h, vals.ctypes.data_as(C.c_void_p), C.c_void_p(out.data_ptr()), xd, DEVICE),
               "grest_get")
        return vals, out

    def values(self):
        n, _, k, _ = self.shape()
        vals = np.empty(k, dtype=np.float64)
        _check(lib().grest_get(self._h, vals.ctypes.data_as(C.c_void_p), None, F64, HOST), "grest_get")
        return vals

    STAGES = ["graph_update", "delta_x", "augment", "project_orth", "spmm", "projected_matrix", "small_eig",
              "back_projection"]

    def memory(self) -> int:
        """Device bytes held by the state."""
        b = C.c_int64()
        _check(lib().grest_memory(self._h, C.byref(b)), "grest_memory")
        return int(b.value)

    def release_graph(self):
        """Low-rank states: free the stored graph; updates then keep Delta alone."""
        _check(lib().grest_release_graph(self._h), "grest_release_graph")

    def drift(self) -> Tuple[float, float]:
        """(max |U^T U - I|, max_j ||M u_j - lambda_j u_j|| / scale), measured on the device now."""
        o, r = C.c_double(), C.c_double()
        _check(lib().grest_drift(self._h, C.byref(o), C.byref(r)), "grest_drift")
        return o.value, r.value

    def set_restart(self, tol_resid: float, tol_orth: float, check_every: int = 1, min_gap: int = 5,
                    iterations: int = 30, seed: int = 0):
        """Recompute the pairs from scratch when their drift passes a threshold (check_every = 0: off)."""
        _check(lib().grest_set_restart(self._h, float(tol_resid), float(tol_orth), int(check_every), int(min_gap),
                                       int(iterations), int(seed)), "grest_set_restart")

    def restart_stats(self) -> Tuple[int, float, float]:
        """(restarts so far, last orth, last resid measured by the restart policy)."""
        c, o, r = C.c_int64(), C.c_double(), C.c_double()
        _check(lib().grest_restart_stats(self._h, C.byref(c), C.byref(o), C.byref(r)), "grest_restart_stats")
        return c.value, o.value, r.value

    def set_stream(self, stream: Optional[int]):
        _check(lib().grest_set_stream(self._h, C.c_void_p(stream) if stream else None), "grest_set_stream")

    def set_overlap(self, enable: bool = True):
        """Run each update's graph stage on a second stream, overlapping the previous update."""
        _check(lib().grest_set_overlap(self._h, int(bool(enable))), "grest_set_overlap")

    def profile(self, enable=True):
        """True/1: every stage's events; 2: only those around the sparse product; False/0: off."""
        _check(lib().grest_profile(self._h, int(enable)), "grest_profile")

    def stage_times(self):
        """({stage: total ms}, total ms of the sparse-product kernel alone, updates timed,
        summed width of those sparse products)."""
        ms = np.zeros(len(self.STAGES), dtype=np.float64)
        spmm = C.c_double()
        cnt = C.c_int64()
        cols = C.c_int64()
        _check(lib().grest_stage_times(self._h, ms.ctypes.data_as(C.c_void_p), len(self.STAGES), C.byref(spmm),
                                       C.byref(cnt), C.byref(cols)), "grest_stage_times")
        return dict(zip(self.STAGES, ms.tolist())), spmm.value, cnt.value, cols.value

    def graph(self):
        n, m, _, _ = self.shape()
        if m < 0:  # no stored graph: the library refuses
            _check(lib().grest_get_graph(self._h, None, None), "grest_get_graph")
        rp = np.empty(n + 1, dtype=np.int64)
        col = np.empty(m, dtype=np.int32)
        _check(lib().grest_get_graph(self._h, rp.ctypes.data_as(C.c_void_p), col.ctypes.data_as(C.c_void_p)),
               "grest_get_graph")
        return rp, col


def now_ns() -> int:
    """The monotonic clock of the server's time stamps, in nanoseconds."""
    return int(lib().grest_now_ns())


class Server:
    """Batched execution of many graphs on the current device (grest_server_* in grest.h)."""

    def __init__(self, lanes: int = 4, max_queue: int = 1 << 16, hbm_budget_bytes: int = 0, batch: int = 1):
        """batch > 1: each lane runs up to `batch` requests of distinct graphs as one
        grest_update_batch (grest_server_create_batched)."""
        self._lib = lib()
        self._h = C.c_void_p()
        _check(self._lib.grest_server_create_batched(int(hbm_budget_bytes), int(lanes), int(max_queue), int(batch),
                                                     C.byref(self._h)), "grest_server_create_batched")
        self._states = []

    def attach(self, state: "State") -> int:
        gid = C.c_int32()
        _check(self._lib.grest_server_attach(self._h, state._h, C.byref(gid)), "grest_server_attach")
        self._states.append(state)
        return int(gid.value)

    def submit(self, graph_id: int, n_new: int, i, j, sign, omega=None, tag: int = 0) -> int:
        """Queues one update (host arrays); returns the status (OK, EAGAIN or EINVAL)."""
        i, pi = _host(i, np.int32)
        j, pj = _host(j, np.int32)
        sg, ps = _host(sign, np.int8)
        om, po = (None, None) if omega is None else _host(omega, np.float64)
        return int(self._lib.grest_submit(self._h, int(graph_id), int(n_new), int(i.size), pi, pj, ps, po,
                                          C.c_uint64(int(tag))))

    def poll(self, max_items: int = 4096):
        """Finished requests: arrays (tag, status, t_submit_ns, t_done_ns)."""
        tags = np.empty(max_items, np.uint64)
        st = np.empty(max_items, np.int32)
        ts = np.empty(max_items, np.int64)
        td = np.empty(max_items, np.int64)
        c = int(self._lib.grest_poll(self._h, int(max_items), tags.ctypes.data_as(C.c_void_p),
                                     st.ctypes.data_as(C.c_void_p), ts.ctypes.data_as(C.c_void_p),
                                     td.ctypes.data_as(C.c_void_p)))
        return tags[:c], st[:c], ts[:c], td[:c]

    def detach(self, graph_id: int) -> int:
        """Detaches an idle graph; returns the status (OK, EAGAIN while it is busy)."""
        return int(self._lib.grest_server_detach(self._h, int(graph_id)))

    def memory(self) -> Tuple[int, int]:
        """(reserved device bytes, budget)."""
        r, b = C.c_int64(), C.c_int64()
        _check(self._lib.grest_server_memory(self._h, C.byref(r), C.byref(b)), "grest_server_memory")
        return r.value, b.value

    def drain(self):
        _check(self._lib.grest_server_drain(self._h), "grest_server_drain")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.grest_server_destroy(self._h)
            self._h = C.c_void_p()

    __del__ = close
