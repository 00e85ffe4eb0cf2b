"""Python binding of libgp.so, the gfx950 two-way task-DAG partitioner.

Argument marshalling only: every step of the partition runs in the HIP
kernels of ``libgp.so``.  PyTorch supplies device memory and the current HIP
stream.  The library must be built first (``python
paper_1502_07451_amd/build.py`` or ``__graft_entry__.build()``); importing the
binding without it raises ImportError.

Names follow the C ABI in ``include/gp.h``: ``create`` wraps ``gp_create``,
``Graph.partition`` wraps ``gp_partition`` / ``gp_partition_trace``,
``ratio_from_times`` wraps ``gp_ratio_from_times`` (Eq. (1)-(2)).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgp.so")

OK, EINVAL, EASYM, EDUP, ESELF, ERANGE, EOVERFLOW, ENOMEM, EDEVICE, EMODEL = range(10)
HOST_PTRS, LEARNED, TRACE, TIME_BALANCE, VOLUME = 1, 2, 4, 8, 16


class GPError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: status {status} ({strerror(status)})")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("ratio", ctypes.c_int64 * 2), ("eps_ppm", ctypes.c_int32),
                ("balance_on", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("coarsen_to", ctypes.c_int32), ("match_rounds", ctypes.c_int32),
                ("refine_passes", ctypes.c_int32), ("init_trials", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("model", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("cut", ctypes.c_int64), ("load", ctypes.c_int64 * 2),
                ("time", ctypes.c_int64 * 2), ("feasible", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("used_learned", ctypes.c_int32),
                ("status", ctypes.c_int32), ("volume", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return dict(cut=self.cut, load=(self.load[0], self.load[1]),
                    time=(self.time[0], self.time[1]), feasible=self.feasible,
                    levels=self.levels, used_learned=self.used_learned, status=self.status,
                    volume=self.volume)


class KwayResult(ctypes.Structure):
    _fields_ = [("cut", ctypes.c_int64), ("feasible", ctypes.c_int32),
                ("bisections", ctypes.c_int32)]


class SimResult(ctypes.Structure):
    _fields_ = [("makespan", ctypes.c_int64), ("transfers", ctypes.c_int64),
                ("bytes", ctypes.c_int64), ("busy", ctypes.c_int64 * 2),
                ("tasks", ctypes.c_int64 * 2)]


SIM_EAGER, SIM_DMDA, SIM_GP = 0, 1, 2


def simulate(g, policy: int, part=None, ncpu: int = 3, ngpu: int = 1, latency: int = 0,
             bw: int = 1):
    """gp_simulate on host arrays of a graph (dagen.Graph-like).  Returns
    (SimResult, task node int8[n], task finish int64[n])."""
    n = int(g.n)
    xadj = np.ascontiguousarray(g.xadj, np.int32)
    adj = np.ascontiguousarray(g.adjncy if len(g.adjncy) else np.zeros(1), np.int32)
    w = np.ascontiguousarray(g.adjwgt if len(g.adjwgt) else np.zeros(1), np.int64)
    vw = np.ascontiguousarray(g.vwgt, np.int64).reshape(-1)
    pt = None if part is None else np.ascontiguousarray(part, np.int8)
    node = np.zeros(max(n, 1), np.int8)
    fin = np.zeros(max(n, 1), np.int64)
    res = SimResult()
    st = _lib.gp_simulate(n, _ptr(xadj), _ptr(adj), _ptr(w), _ptr(vw), _ptr(pt), int(policy),
                          int(ncpu), int(ngpu), int(latency), int(bw), ctypes.byref(res),
                          _ptr(node), _ptr(fin))
    if st != OK:
        raise GPError(st, "gp_simulate")
    return res, node[:n], fin[:n]


class ProfRow(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int64),
                ("executed", ctypes.c_int64), ("ms", ctypes.c_double), ("bytes", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python paper_1502_07451_amd/build.py`")
    # torch first: its HIP runtime then satisfies libgp.so's, so device
    # pointers and streams from torch are valid in the library (loading
    # libgp.so first would pull in a second copy of the runtime)
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.gp_options_default.argtypes = [ctypes.POINTER(Options)]
    lib.gp_options_default.restype = None
    lib.gp_ratio_from_times.argtypes = [i64, i64, vp]
    lib.gp_ratio_from_times.restype = ctypes.c_int
    lib.gp_create.argtypes = [ctypes.POINTER(vp), i32, vp, vp, vp, vp, i32, vp]
    lib.gp_create.restype = ctypes.c_int
    lib.gp_set_stream.argtypes = [vp, vp]
    lib.gp_set_stream.restype = ctypes.c_int
    lib.gp_partition.argtypes = [vp, ctypes.POINTER(Options), vp, ctypes.POINTER(Result)]
    lib.gp_partition.restype = ctypes.c_int
    lib.gp_partition_trace.argtypes = [vp, ctypes.POINTER(Options), vp, ctypes.POINTER(Result),
                                       vp, i32]
    lib.gp_partition_trace.restype = ctypes.c_int
    lib.gp_destroy.argtypes = [vp]
    lib.gp_destroy.restype = None
    lib.gp_set_workspace_limit.argtypes = [vp, i64]
    lib.gp_set_workspace_limit.restype = ctypes.c_int
    lib.gp_workspace_bytes.argtypes = [vp]
    lib.gp_workspace_bytes.restype = i64
    lib.gp_profile_enable.argtypes = [vp, i32]
    lib.gp_profile_enable.restype = ctypes.c_int
    lib.gp_profile_read.argtypes = [vp, ctypes.POINTER(ProfRow), i32, i32]
    lib.gp_profile_read.restype = i32
    lib.gp_batch_create.argtypes = [ctypes.POINTER(vp), vp]
    lib.gp_batch_create.restype = ctypes.c_int
    lib.gp_batch_team_width.argtypes = [vp, i32]
    lib.gp_batch_team_width.restype = ctypes.c_int
    lib.gp_batch_timeline.argtypes = [vp, i32, vp, ctypes.POINTER(i64)]
    lib.gp_batch_timeline.restype = ctypes.c_int
    lib.gp_batch_config.argtypes = [vp, i32, i32, i32]
    lib.gp_batch_config.restype = ctypes.c_int
    lib.gp_partition_batch.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Options),
                                       vp, ctypes.POINTER(Result)]
    lib.gp_partition_batch.restype = ctypes.c_int
    lib.gp_batch_destroy.argtypes = [vp]
    lib.gp_batch_destroy.restype = None
    lib.gp_partition_kway.argtypes = [vp, i32, vp, ctypes.POINTER(Options), vp, vp,
                                      ctypes.POINTER(KwayResult)]
    lib.gp_simulate.argtypes = [i32, vp, vp, vp, vp, vp, i32, i32, i32, i64, i64,
                                ctypes.POINTER(SimResult), vp, vp]
    lib.gp_simulate.restype = ctypes.c_int
    lib.gp_partition_kway.restype = ctypes.c_int
    lib.gp_partition_batch_noalloc.argtypes = [i32, vp, vp, vp, vp, vp, vp,
                                               ctypes.POINTER(Options), i32, i32, i64, i64, vp,
                                               vp, vp]
    lib.gp_partition_batch_noalloc.restype = ctypes.c_int
    lib.gp_model_create.argtypes = [vp, i32, ctypes.POINTER(vp)]
    lib.gp_model_create.restype = ctypes.c_int
    lib.gp_model_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
    lib.gp_model_load.restype = i32
    lib.gp_model_free.argtypes = [vp]
    lib.gp_model_free.restype = None
    lib.gp_model_scores.argtypes = [vp, vp, vp]
    lib.gp_model_scores.restype = ctypes.c_int
    lib.gp_level_read.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i64), vp, vp, vp,
                                  vp, vp, vp]
    lib.gp_level_read.restype = ctypes.c_int
    lib.gp_batch_autotune.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Options),
                                      vp, vp, i32, vp, ctypes.POINTER(ctypes.c_double)]
    lib.gp_batch_autotune.restype = ctypes.c_int
    lib.gp_batch_export.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp, i64]
    lib.gp_batch_export.restype = ctypes.c_int
    lib.gp_train_create.argtypes = [ctypes.POINTER(vp), vp, i32, vp]
    lib.gp_train_create.restype = ctypes.c_int
    lib.gp_train_set_data.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, i32]
    lib.gp_train_set_data.restype = ctypes.c_int
    lib.gp_train_step.argtypes = [vp, i32, i32, ctypes.c_float, ctypes.POINTER(ctypes.c_float)]
    lib.gp_train_step.restype = ctypes.c_int
    lib.gp_train_grad.argtypes = [vp, i32, i32, vp, ctypes.POINTER(ctypes.c_float)]
    lib.gp_train_grad.restype = ctypes.c_int
    lib.gp_train_params.argtypes = [vp, vp, vp]
    lib.gp_train_params.restype = ctypes.c_int
    lib.gp_train_destroy.argtypes = [vp]
    lib.gp_train_destroy.restype = None
    lib.gp_strerror.argtypes = [ctypes.c_int]
    lib.gp_strerror.restype = ctypes.c_char_p
    return lib


_lib = _load()

EXPORTED = ["gp_options_default", "gp_ratio_from_times", "gp_create", "gp_set_stream",
            "gp_partition", "gp_partition_trace", "gp_destroy", "gp_strerror",
            "gp_profile_enable", "gp_profile_read", "gp_batch_create", "gp_batch_config",
            "gp_partition_batch", "gp_batch_destroy", "gp_model_create", "gp_model_free",
            "gp_model_scores", "gp_level_read", "gp_batch_export", "gp_batch_autotune", "gp_train_create", "gp_train_set_data",
            "gp_train_step", "gp_train_grad", "gp_train_params", "gp_train_destroy"]


def strerror(status: int) -> str:
    return _lib.gp_strerror(status).decode()


def options(ratio=(1, 4), eps_ppm=30000, balance_on=0, seed=0, coarsen_to=2048, match_rounds=8,
            refine_passes=8, init_trials=16, flags=0, model=None) -> Options:
    o = Options()
    _lib.gp_options_default(ctypes.byref(o))
    o.ratio[0], o.ratio[1] = int(ratio[0]), int(ratio[1])
    o.eps_ppm, o.balance_on = int(eps_ppm), int(balance_on)
    o.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    o.coarsen_to, o.match_rounds = int(coarsen_to), int(match_rounds)
    o.refine_passes, o.init_trials = int(refine_passes), int(init_trials)
    o.flags = int(flags)
    o.model = model
    return o


def ratio_from_times(t_cpu: int, t_gpu: int):
    out = (ctypes.c_int64 * 2)()
    st = _lib.gp_ratio_from_times(int(t_cpu), int(t_gpu), out)
    return st, (out[0], out[1])


def _current_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(a):
    """Device pointer of a torch tensor, host pointer of a numpy array; the
    pointer object holds a reference to a, so a temporary argument stays
    alive until the call returns."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)
    p = ctypes.c_void_p(a.data_ptr())
    p._keep = a
    return p


class Graph:
    """A library-owned copy of one graph (gp_create); reuse it for many partitions."""

    def __init__(self, n, xadj, adjncy, adjwgt, vwgt, stream=None):
        import torch
        self.n = int(n)
        self.host = isinstance(xadj, np.ndarray)
        arrays = (xadj, adjncy, adjwgt, vwgt)
        want = (np.int32, np.int32, np.int64, np.int64)
        tw = (torch.int32, torch.int32, torch.int64, torch.int64)
        for a, dn, dt in zip(arrays, want, tw):
            if self.host:
                if a.dtype != dn or not a.flags["C_CONTIGUOUS"]:
                    raise TypeError("host arrays must be contiguous int32/int32/int64/int64")
            elif a.dtype != dt or not a.is_contiguous() or not a.is_cuda:
                raise TypeError("device tensors must be contiguous cuda int32/int32/int64/int64")
        self.device = None if self.host else xadj.device
        self.stream = stream if stream is not None else (None if self.host else _current_stream())
        h = ctypes.c_void_p()
        st = _lib.gp_create(ctypes.byref(h), self.n, *(_ptr(a) for a in arrays),
                            HOST_PTRS if self.host else 0, self.stream)
        if st != OK:
            raise GPError(st, "gp_create")
        self._h = h

    def set_stream(self, stream):
        self.stream = stream
        st = _lib.gp_set_stream(self._h, stream)
        if st != OK:
            raise GPError(st, "gp_set_stream")

    def set_workspace_limit(self, nbytes: int):
        """Most device bytes the handle's buffers may grow to (-1: no limit)."""
        st = _lib.gp_set_workspace_limit(self._h, int(nbytes))
        if st != OK:
            raise GPError(st, "gp_set_workspace_limit")

    def workspace_bytes(self) -> int:
        return int(_lib.gp_workspace_bytes(self._h))

    def partition(self, opts: Options | None = None, part=None, trace_cap: int = 0):
        """Returns (part, Result[, trace]) - part is int8[n]: 0 = CPU, 1 = GPU."""
        import torch
        opts = opts or options()
        if part is None:
            if self.host:
                part = np.zeros(max(self.n, 1), np.int8)
            else:
                part = torch.empty(max(self.n, 1), dtype=torch.int8, device=self.device)
        res = Result()
        if trace_cap > 0:
            tr = np.zeros(8 * trace_cap, np.int64)
            st = _lib.gp_partition_trace(self._h, ctypes.byref(opts), _ptr(part),
                                         ctypes.byref(res), _ptr(tr), trace_cap)
        else:
            st = _lib.gp_partition(self._h, ctypes.byref(opts), _ptr(part), ctypes.byref(res))
        if st != OK:
            raise GPError(st, "gp_partition")
        part = part[:self.n]
        if trace_cap > 0:
            return part, res, tr.reshape(trace_cap, 8)[:res.levels + 1].copy()
        return part, res

    def partition_kway(self, k: int, ratio, opts: Options | None = None, part=None):
        """gp_partition_kway: returns (part int32[n] with parts 0..k-1, KwayResult,
        list of the k part loads)."""
        import torch
        opts = opts or options()
        if part is None:
            if self.host:
                part = np.zeros(max(self.n, 1), np.int32)
            else:
                part = torch.empty(max(self.n, 1), dtype=torch.int32, device=self.device)
        r = np.ascontiguousarray(ratio, dtype=np.int64)
        if r.size != k:
            raise ValueError(f"ratio needs {k} shares")
        load = np.zeros(max(k, 1), np.int64)
        res = KwayResult()
        st = _lib.gp_partition_kway(self._h, int(k), _ptr(r), ctypes.byref(opts), _ptr(part),
                                    _ptr(load), ctypes.byref(res))
        if st != OK:
            raise GPError(st, "gp_partition_kway")
        return part[:self.n], res, [int(x) for x in load[:k]]

    def level(self, level: int) -> dict:
        """Level `level` of the last partition (host numpy arrays): n, xadj,
        adjncy, adjwgt, vwgt (n x 2), match (None at the coarsest) and part."""
        n, nnz = ctypes.c_int32(0), ctypes.c_int64(0)
        st = _lib.gp_level_read(self._h, int(level), ctypes.byref(n), ctypes.byref(nnz),
                                None, None, None, None, None, None)
        if st != OK:
            raise GPError(st, "gp_level_read")
        nv, ne = n.value, nnz.value
        out = dict(n=nv, xadj=np.zeros(nv + 1, np.int32), adjncy=np.zeros(max(ne, 1), np.int32),
                   adjwgt=np.zeros(max(ne, 1), np.int64), vwgt=np.zeros((max(nv, 1), 2), np.int64),
                   match=np.full(max(nv, 1), -3, np.int32), part=np.zeros(max(nv, 1), np.int8))
        st = _lib.gp_level_read(self._h, int(level), None, None, _ptr(out["xadj"]),
                                _ptr(out["adjncy"]), _ptr(out["adjwgt"]), _ptr(out["vwgt"]),
                                _ptr(out["match"]), _ptr(out["part"]))
        if st != OK:
            raise GPError(st, "gp_level_read")
        for k in ("adjncy", "adjwgt"):
            out[k] = out[k][:ne]
        for k in ("vwgt", "match", "part"):
            out[k] = out[k][:nv]
        if nv and out["match"][0] == -3:
            out["match"] = None
        return out

    def scores(self, model: "Model"):
        """The learned network's score of every vertex (float32[n])."""
        import torch
        if self.host:
            out = np.zeros(max(self.n, 1), np.float32)
        else:
            out = torch.empty(max(self.n, 1), dtype=torch.float32, device=self.device)
        st = _lib.gp_model_scores(model.handle, self._h, _ptr(out))
        if st != OK:
            raise GPError(st, "gp_model_scores")
        return out[:self.n]

    def profile(self, on: bool = True):
        """Start (or stop) per-launch event timing on this handle."""
        _lib.gp_profile_enable(self._h, 1 if on else 0)

    def profile_read(self, reset: bool = True) -> list:
        """Per-kernel rows: name, launches, executed, ms, bytes."""
        n = _lib.gp_profile_read(self._h, None, 0, 0)
        rows = (ProfRow * max(n, 1))()
        n = _lib.gp_profile_read(self._h, rows, n, 1 if reset else 0)
        return [dict(name=r.name.decode(), launches=r.launches, executed=r.executed, ms=r.ms,
                     bytes=r.bytes) for r in rows[:n]]

    def close(self):
        if getattr(self, "_h", None):
            _lib.gp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def create_status(n, xadj, adjncy, adjwgt, vwgt, host: bool) -> int:
    """gp_create's status for the given arrays (the handle is destroyed again)."""
    h = ctypes.c_void_p()
    st = _lib.gp_create(ctypes.byref(h), int(n), _ptr(xadj), _ptr(adjncy), _ptr(adjwgt),
                        _ptr(vwgt), HOST_PTRS if host else 0,
                        None if host else _current_stream())
    if st == OK:
        _lib.gp_destroy(h)
    return st


def to_device(g, device="cuda"):
    """Copies a graph given as numpy arrays (n, xadj, adjncy, adjwgt, vwgt) to device tensors."""
    import torch
    vw = np.ascontiguousarray(g.vwgt, dtype=np.int64).reshape(-1)
    return (g.n, torch.from_numpy(np.ascontiguousarray(g.xadj, np.int32)).to(device),
            torch.from_numpy(np.ascontiguousarray(g.adjncy, np.int32)).to(device),
            torch.from_numpy(np.ascontiguousarray(g.adjwgt, np.int64)).to(device),
            torch.from_numpy(vw).to(device))


def create(g, device="cuda", stream=None) -> Graph:
    """gp_create from an object with n, xadj, adjncy, adjwgt, vwgt (numpy) on a device."""
    return Graph(*to_device(g, device), stream=stream)


class Batch:
    """A batch context (gp_batch_create) for partitioning many graphs per call."""

    def __init__(self, stream=None):
        self.stream = stream if stream is not None else _current_stream()
        h = ctypes.c_void_p()
        st = _lib.gp_batch_create(ctypes.byref(h), self.stream)
        if st != OK:
            raise GPError(st, "gp_batch_create")
        self._h = h

    def export(self, rec=None, xadj=None, vwgt=None, part=None, adjncy=None, adjwgt=None):
        """Export every graph's coarsest level during later calls (device tensors);
        rec=None turns it off."""
        if rec is None:
            st = _lib.gp_batch_export(self._h, None, None, None, None, 0, None, None, 0)
        else:
            st = _lib.gp_batch_export(self._h, _ptr(rec), _ptr(xadj), _ptr(vwgt), _ptr(part),
                                      int(xadj.numel()), _ptr(adjncy), _ptr(adjwgt),
                                      int(adjncy.numel()))
        if st != OK:
            raise GPError(st, "gp_batch_export")

    def team_width(self, shift: int):
        st = _lib.gp_batch_team_width(self._h, int(shift))
        if st != OK:
            raise GPError(st, "gp_batch_team_width")

    def timeline(self, G: int):
        """(ticks int64[G, 2]: start / end of each graph of the last call, clock rate in Hz)."""
        t = np.zeros((max(int(G), 1), 2), np.int64)
        hz = ctypes.c_int64()
        st = _lib.gp_batch_timeline(self._h, int(G), t.ctypes.data, ctypes.byref(hz))
        if st != OK:
            raise GPError(st, "gp_batch_timeline")
        return t[:G], int(hz.value)

    def config(self, workgroups: int = 0, chunk: int = 1, order_mode: int = 0):
        st = _lib.gp_batch_config(self._h, workgroups, chunk, order_mode)
        if st != OK:
            raise GPError(st, "gp_batch_config")

    def partition(self, G, voff, eoff, xadj, adjncy, adjwgt, vwgt, opts=None, part=None):
        """Device tensors in the concatenated layout of include/gp.h.
        Returns (part, list of Result)."""
        import torch
        opts = opts or options()
        if part is None:
            part = torch.empty(max(int(vwgt.numel()) // 2, 1), dtype=torch.int8,
                               device=xadj.device)
        res = (Result * max(G, 1))()
        st = _lib.gp_partition_batch(self._h, int(G), _ptr(voff), _ptr(eoff), _ptr(xadj),
                                     _ptr(adjncy), _ptr(adjwgt), _ptr(vwgt), ctypes.byref(opts),
                                     _ptr(part), res)
        if st != OK:
            raise GPError(st, "gp_partition_batch")
        return part, list(res[:G])

    def autotune(self, G, voff, eoff, xadj, adjncy, adjwgt, vwgt, opts=None, part=None,
                 reps: int = 3):
        """gp_batch_autotune: returns (part, results, (workgroups, chunk, order_mode,
        team width shift), ms)."""
        import torch
        opts = opts or options()
        if part is None:
            part = torch.empty(max(int(vwgt.numel()) // 2, 1), dtype=torch.int8,
                               device=xadj.device)
        res = (Result * max(G, 1))()
        chosen = (ctypes.c_int32 * 4)()
        ms = ctypes.c_double(0)
        st = _lib.gp_batch_autotune(self._h, int(G), _ptr(voff), _ptr(eoff), _ptr(xadj),
                                    _ptr(adjncy), _ptr(adjwgt), _ptr(vwgt), ctypes.byref(opts),
                                    _ptr(part), res, int(reps), chosen, ctypes.byref(ms))
        if st != OK:
            raise GPError(st, "gp_batch_autotune")
        return part, list(res[:G]), (chosen[0], chosen[1], chosen[2], chosen[3]), ms.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.gp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def partition_batch_noalloc(G, voff, eoff, xadj, adjncy, adjwgt, vwgt, opts=None, part=None,
                            res=None, nmax=None, nnzmax=None, ntot=None, nnztot=None,
                            stream=None):
    """gp_partition_batch_noalloc: the batched partition with the library's
    fixed device scratch, queued on `stream` without waiting.  Device
    tensors as in Batch.partition; res is a device uint8 tensor of
    G * sizeof(Result) bytes.  The size bounds default to the exact ones
    (read from voff / eoff).  Returns (part, res); results_from_device turns
    res into Result records once the stream has finished."""
    import torch
    opts = opts or options()
    if part is None:
        part = torch.empty(max(int(vwgt.numel()) // 2, 1), dtype=torch.int8, device=xadj.device)
    if res is None:
        res = torch.empty(max(G, 1) * ctypes.sizeof(Result), dtype=torch.uint8,
                          device=xadj.device)
    if None in (nmax, nnzmax, ntot, nnztot):
        hv, he = voff.cpu().numpy(), eoff.cpu().numpy()
        nmax = (int(np.diff(hv).max()) if G else 0) if nmax is None else nmax
        nnzmax = (int(np.diff(he).max()) if G else 0) if nnzmax is None else nnzmax
        ntot = int(hv[-1]) if ntot is None else ntot
        nnztot = int(he[-1]) if nnztot is None else nnztot
    st = _lib.gp_partition_batch_noalloc(int(G), _ptr(voff), _ptr(eoff), _ptr(xadj),
                                         _ptr(adjncy), _ptr(adjwgt), _ptr(vwgt),
                                         ctypes.byref(opts), int(nmax), int(nnzmax), int(ntot),
                                         int(nnztot), _ptr(part), _ptr(res),
                                         stream if stream is not None else _current_stream())
    if st != OK:
        raise GPError(st, "gp_partition_batch_noalloc")
    return part, res


def results_from_device(res, G):
    """Result records from a device tensor filled by partition_batch_noalloc."""
    raw = res.cpu().numpy().tobytes()
    arr = (Result * max(G, 1)).from_buffer_copy(raw[:ctypes.sizeof(Result) * max(G, 1)])
    return list(arr[:G])


def batch_to_device(b, device="cuda"):
    """Device tensors (G, voff, eoff, xadj, adjncy, adjwgt, vwgt) of a concatenated batch."""
    import torch
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)
    return (b.G, t(b.voff, np.int64), t(b.eoff, np.int64), t(b.xadj, np.int32),
            t(b.adjncy, np.int32), t(b.adjwgt, np.int64),
            t(np.ascontiguousarray(b.vwgt).reshape(-1), np.int64))


NPARAM = 25153


class Model:
    """Device copy of the learned proposal's BF16 parameters (gp_model_create)."""

    def __init__(self, params_bf16_bits: np.ndarray):
        p = np.ascontiguousarray(params_bf16_bits, dtype=np.uint16)
        if p.size != NPARAM:
            raise ValueError(f"expected {NPARAM} parameters, got {p.size}")
        h = ctypes.c_void_p()
        st = _lib.gp_model_create(_ptr(p), NPARAM, ctypes.byref(h))
        if st != OK:
            raise GPError(st, "gp_model_create")
        self.handle = h

    @classmethod
    def load(cls, path: str) -> "Model":
        """gp_model_load: the parameter blob read by the library from a file."""
        h = ctypes.c_void_p()
        st = _lib.gp_model_load(os.fsencode(path), ctypes.byref(h))
        if st != OK:
            raise GPError(st, "gp_model_load")
        m = cls.__new__(cls)
        m.handle = h
        return m

    def close(self):
        if getattr(self, "handle", None):
            _lib.gp_model_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Trainer:
    """GPU trainer of the learned proposal (gp_train_*)."""

    def __init__(self, init_params_f32: np.ndarray, stream=None):
        p = np.ascontiguousarray(init_params_f32, dtype=np.float32)
        self.stream = stream if stream is not None else _current_stream()
        h = ctypes.c_void_p()
        st = _lib.gp_train_create(ctypes.byref(h), _ptr(p), p.size, self.stream)
        if st != OK:
            raise GPError(st, "gp_train_create")
        self._h = h

    def set_data(self, G, voff, eoff, xadj, adjncy, adjwgt, vwgt, labels, balance_on=0):
        self._keep = (voff, eoff, xadj, adjncy, adjwgt, vwgt, labels)
        st = _lib.gp_train_set_data(self._h, int(G), _ptr(voff), _ptr(eoff), _ptr(xadj),
                                    _ptr(adjncy), _ptr(adjwgt), _ptr(vwgt), _ptr(labels),
                                    int(balance_on))
        if st != OK:
            raise GPError(st, "gp_train_set_data")

    def step(self, g0: int, g1: int, lr: float) -> float:
        loss = ctypes.c_float(0)
        st = _lib.gp_train_step(self._h, int(g0), int(g1), float(lr), ctypes.byref(loss))
        if st != OK:
            raise GPError(st, "gp_train_step")
        return loss.value

    def grad(self, g0: int, g1: int):
        g = np.zeros(NPARAM, np.float32)
        loss = ctypes.c_float(0)
        st = _lib.gp_train_grad(self._h, int(g0), int(g1), _ptr(g), ctypes.byref(loss))
        if st != OK:
            raise GPError(st, "gp_train_grad")
        return loss.value, g

    def params(self):
        f = np.zeros(NPARAM, np.float32)
        b = np.zeros(NPARAM, np.uint16)
        st = _lib.gp_train_params(self._h, _ptr(f), _ptr(b))
        if st != OK:
            raise GPError(st, "gp_train_params")
        return f, b

    def close(self):
        if getattr(self, "_h", None):
            _lib.gp_train_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
