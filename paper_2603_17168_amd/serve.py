"""Python driver of the serving loop (cskv_serve_trace): builds a request trace on the device,
runs it through the native loop, and reports latency percentiles.  Every request's work runs in
the HIP library; this module marshals arguments and computes statistics."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import cskv

REQ_FIND, REQ_INSERT_AND_EVICT = 0, 1
P = ctypes.c_void_p


class Request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("n", ctypes.c_uint64),
                ("d_keys", P), ("d_values", P), ("d_scores", P),
                ("d_values_out", P), ("d_flags", P), ("d_ev_keys", P), ("d_ev_values", P), ("d_ev_scores", P),
                ("d_n_evicted", P),
                ("arrival_s", ctypes.c_double), ("admit_s", ctypes.c_double), ("launch_s", ctypes.c_double),
                ("complete_s", ctypes.c_double), ("seq", ctypes.c_uint64), ("group", ctypes.c_uint32)]


class Config(ctypes.Structure):
    _fields_ = [("arena_budget_bytes", ctypes.c_uint64), ("max_inflight_groups", ctypes.c_uint32),
                ("max_merge", ctypes.c_uint32), ("realtime", ctypes.c_int), ("reader_streams", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("groups", ctypes.c_uint64), ("reader_launches", ctypes.c_uint64),
                ("inserter_launches", ctypes.c_uint64), ("deferred_for_memory", ctypes.c_uint64),
                ("peak_inflight_bytes", ctypes.c_uint64), ("wall_s", ctypes.c_double)]


def _lib():
    L = cskv.lib()
    if not getattr(L, "_serve_sig", False):
        L.cskv_serve_workspace_bytes.restype = ctypes.c_size_t
        L.cskv_serve_workspace_bytes.argtypes = [P, ctypes.c_uint64, ctypes.c_uint64]
        L.cskv_serve_trace.restype = ctypes.c_int
        L.cskv_serve_trace.argtypes = [P, ctypes.POINTER(Request), ctypes.c_uint64, ctypes.POINTER(Config), P,
                                       ctypes.c_size_t, P, ctypes.POINTER(Stats)]
        L._serve_sig = True
    return L


class Trace:
    """Requests over concatenated device buffers.

    ops: int array (REQ_*), sizes: int array, keys: int64 device tensor of sum(sizes) keys,
    values: float32 [sum(insert sizes), dim] device tensor for the inserts (in request order),
    arrivals: float seconds.  with_results allocates per-request result buffers (for checks);
    otherwise outputs live in the server's recycled arena.  shared_values: `values` holds the rows
    of the largest insert only, and every insert reads its rows from its start (timing runs)."""

    def __init__(self, table: cskv.Table, ops, sizes, keys, values, arrivals, with_results=False,
                 shared_values=False):
        self.table = table
        self.ops = np.asarray(ops, dtype=np.int64)
        self.sizes = np.asarray(sizes, dtype=np.int64)
        self.keys = keys.contiguous()
        self.values = values.contiguous() if values is not None else None
        self.arrivals = np.asarray(arrivals, dtype=np.float64)
        self.with_results = with_results
        dim, dev = table.dim, table.device
        self.key_off = np.concatenate([[0], np.cumsum(self.sizes)])
        ins = self.ops == REQ_INSERT_AND_EVICT
        self.val_off = np.concatenate([[0], np.cumsum(np.where(ins, self.sizes, 0))])
        if shared_values:  # every insert reads its rows from the start of `values` (timing runs)
            if with_results:
                raise ValueError("shared_values is for timing runs: its inserts share result offsets")
            self.val_off = np.zeros_like(self.val_off)
        nf = int(self.sizes[~ins].sum())
        ni = int(self.sizes[ins].sum())
        if with_results:
            self.find_out = torch.zeros((max(nf, 1), dim), dtype=torch.float32, device=dev)
            self.find_flag = torch.zeros(max(nf, 1), dtype=torch.uint8, device=dev)
            self.ins_status = torch.zeros(max(ni, 1), dtype=torch.uint8, device=dev)
            self.ev_keys = torch.zeros(max(ni, 1), dtype=torch.int64, device=dev)
            self.ev_vals = torch.zeros((max(ni, 1), dim), dtype=torch.float32, device=dev)
            self.ev_scores = torch.zeros(max(ni, 1), dtype=torch.int64, device=dev)
            self.ev_count = torch.zeros(max(len(self.ops), 1), dtype=torch.int64, device=dev)
        self.find_off = np.concatenate([[0], np.cumsum(np.where(~ins, self.sizes, 0))])

    def requests(self):
        n = len(self.ops)
        arr = (Request * max(n, 1))()
        kp = self.keys.data_ptr()
        vp = self.values.data_ptr() if self.values is not None else 0
        row = self.table.dim * 4
        for i in range(n):
            r = arr[i]
            r.op = int(self.ops[i])
            r.n = int(self.sizes[i])
            r.d_keys = kp + int(self.key_off[i]) * 8
            r.arrival_s = float(self.arrivals[i])
            if r.op == REQ_INSERT_AND_EVICT:
                r.d_values = vp + int(self.val_off[i]) * row
            if self.with_results:
                if r.op == REQ_FIND:
                    o = int(self.find_off[i])
                    r.d_values_out = self.find_out.data_ptr() + o * row
                    r.d_flags = self.find_flag.data_ptr() + o
                else:
                    o = int(self.val_off[i])
                    r.d_flags = self.ins_status.data_ptr() + o
                    r.d_ev_keys = self.ev_keys.data_ptr() + o * 8
                    r.d_ev_values = self.ev_vals.data_ptr() + o * row
                    r.d_ev_scores = self.ev_scores.data_ptr() + o * 8
                    r.d_n_evicted = self.ev_count.data_ptr() + i * 8
        return arr


def serve(table: cskv.Table, trace: Trace, budget_bytes=4 << 30, max_inflight_groups=2, max_merge=64,
          realtime=True, stream=None, reader_streams=0):
    """Run the trace; returns (stats dict, per-request arrays: latency_s, admit_s, launch_s, complete_s, seq, group)."""
    L = _lib()
    reqs = trace.requests()
    n = len(trace.ops)
    max_n = int(trace.sizes.max()) if n else 1
    need = int(L.cskv_serve_workspace_bytes(table._h, max_n, budget_bytes))
    ws = torch.empty(need, dtype=torch.uint8, device=table.device)
    cfg = Config(budget_bytes, max_inflight_groups, max_merge, 1 if realtime else 0, reader_streams)
    st = Stats()
    s = stream if stream is not None else torch.cuda.current_stream(table.device)
    torch.cuda.synchronize(table.device)
    with torch.cuda.device(table.device):
        rc = L.cskv_serve_trace(table._h, reqs, n, ctypes.byref(cfg), ctypes.c_void_p(ws.data_ptr()), need,
                                ctypes.c_void_p(s.cuda_stream), ctypes.byref(st))
    torch.cuda.synchronize(table.device)
    if rc != 0:
        raise cskv.CskvError(f"cskv_serve_trace: {L.cskv_strerror(rc).decode()} ({rc})")
    get = lambda f: np.array([getattr(reqs[i], f) for i in range(n)])
    out = {f: get(f) for f in ("admit_s", "launch_s", "complete_s", "seq", "group")}
    out["latency_s"] = out["complete_s"] - trace.arrivals
    stats = {f: getattr(st, f) for f, _ in Stats._fields_}
    return stats, out


def percentiles_ms(lat_s):
    return {"p50": float(np.percentile(lat_s, 50) * 1e3), "p99": float(np.percentile(lat_s, 99) * 1e3),
            "mean": float(np.mean(lat_s) * 1e3)}
