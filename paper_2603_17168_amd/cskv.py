"""Python binding of the cskv C-ABI (include/cskv.h): argument marshalling over torch tensors.

Every step of every call runs in the HIP library ``libcskv.so``; this module only allocates
device tensors (table storage, workspaces, outputs) with torch, passes their pointers and the
current HIP stream, and turns return codes into exceptions.  If the library is missing the
import of :class:`Table` fails loudly: there is no fallback.

Keys and scores are 64-bit words carried in torch.int64 (or torch.uint64) tensors; values are
float32 [n, dim] tensors.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcskv.so")

MODE = {"single": 1, "dual": 2}
POLICY = {"custom": 0, "lru": 1, "lfu": 2}
OP_FIND, OP_INSERT_OR_ASSIGN, OP_INSERT_AND_EVICT, OP_ERASE, OP_ASSIGN, OP_FIND_OR_INSERT = 0, 1, 2, 3, 4, 5
TUNE = {"find_group": 1, "route_group": 2, "find_prefetch_b2": 3, "find_blocks_per_cu": 4, "find_pairs": 5, "find_digest": 6}
ST_UPDATED, ST_INSERTED, ST_INSERTED_EVICT, ST_REJECTED, ST_INVALID_KEY = 1, 2, 3, 4, 5
LOCK = {"none": 0, "triple_group": 1, "reader_writer": 2}
NOALLOC_MAX_KEYS = 65536  # CSKV_NOALLOC_MAX_KEYS
MT_OP = {"find": 0, "assign": 1, "insert_erase": 2}

_lib = None


class CskvError(RuntimeError):
    pass


def lib():
    """The loaded libcskv.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise CskvError(f"{LIB_PATH} is missing: build it with paper_2603_17168_amd/build.py "
                        "(or __graft_entry__.build()); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    P, U64, U32, I, SZ = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_size_t
    sig = {
        "cskv_table_bytes": (SZ, [U64, U32, U32]),
        "cskv_create": (I, [ctypes.POINTER(P), U64, U32, U32, I, I, P, SZ, P]),
        "cskv_destroy": (I, [P]),
        "cskv_clear": (I, [P, P]),
        "cskv_workspace_bytes": (SZ, [P, I, U64]),
        "cskv_find": (I, [P, U64, P, P, P, P, P]),
        "cskv_insert_or_assign": (I, [P, U64, P, P, P, P, P, SZ, P]),
        "cskv_insert_or_assign_noalloc": (I, [P, U64, P, P, P, P, P]),
        "cskv_noalloc_scratch_bytes": (SZ, []),
        "cskv_insert_and_evict": (I, [P, U64, P, P, P, P, P, P, P, P, P, SZ, P]),
        "cskv_erase": (I, [P, U64, P, P, P, SZ, P]),
        "cskv_size": (I, [P, P, P]),
        "cskv_export": (I, [P, U64, U64, P, P, P, P, P, P]),
        "cskv_export_if": (I, [P, U64, U64, U64, P, P, P, P, P, P]),
        "cskv_contains": (I, [P, U64, P, P, P]),
        "cskv_find_ptr": (I, [P, U64, P, P, P, P, P]),
        "cskv_assign": (I, [P, U64, P, P, P, P, P, SZ, P]),
        "cskv_assign_scores": (I, [P, U64, P, P, P, P, SZ, P]),
        "cskv_find_or_insert": (I, [P, U64, P, P, P, P, P, P, SZ, P]),
        "cskv_program_create": (I, [ctypes.POINTER(P), P]),
        "cskv_program_destroy": (I, [P]),
        "cskv_program_add_find": (I, [P, U64, P, P, P, P]),
        "cskv_program_add_insert_or_assign": (I, [P, U64, P, P, P, P]),
        "cskv_program_add_insert_and_evict": (I, [P, U64, P, P, P, P, P, P, P, P]),
        "cskv_program_add_erase": (I, [P, U64, P, P]),
        "cskv_program_workspace_bytes": (SZ, [P]),
        "cskv_program_set_overlap": (I, [P, I]),
        "cskv_program_set_workspace": (I, [P, P, SZ]),
        "cskv_program_segments": (U32, [P]),
        "cskv_program_phases": (U32, [P]),
        "cskv_program_launch": (I, [P, P]),
        "cskv_program_capture": (I, [P, P]),
        "cskv_program_replay": (I, [P, P]),
        "cskv_set_tuning": (I, [P, I, I]),
        "cskv_get_tuning": (I, [P, I]),
        "cskv_clock": (U64, [P]),
        "cskv_set_clock": (I, [P, U64]),
        "cskv_num_buckets": (U64, [P]),
        "cskv_dim": (U32, [P]),
        "cskv_mode": (I, [P]),
        "cskv_policy": (I, [P]),
        "cskv_strerror": (ctypes.c_char_p, [I]),
        "cskv_set_lock_mode": (I, [P, I]),
        "cskv_set_route_subrounds": (I, [P, U32]),
        "cskv_get_route_subrounds": (U32, [P]),
        "cskv_table_bytes_tiered": (SZ, [U64, U32, U32, U64]),
        "cskv_host_value_bytes": (SZ, [U64, U32, U64]),
        "cskv_create_tiered": (I, [ctypes.POINTER(P), U64, U32, U32, I, I, P, SZ, U64, P, SZ, P]),
        "cskv_hbm_value_rows": (U64, [P]),
        "cskv_row_address": (U64, [P, U64]),
        "cskv_get_lock_mode": (I, [P]),
        "cskv_mt_run": (I, [P, I, P, ctypes.POINTER(ctypes.c_double)]),
        "cskv_probe_copy": (I, [P, P, SZ, P]),
        "cskv_probe_gather": (I, [P, SZ, U32, U64, U64, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != 0:
        raise CskvError(f"{what}: {lib().cskv_strerror(rc).decode()} ({rc})")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _as_i64(t: torch.Tensor, device) -> torch.Tensor:
    if t.dtype == torch.uint64:
        t = t.view(torch.int64)
    if t.dtype != torch.int64:
        raise TypeError("keys/scores must be int64 or uint64 tensors (64-bit words)")
    if t.device != device:
        raise ValueError(f"tensor on {t.device}, table on {device}")
    return t.contiguous()


def probe_copy(src: torch.Tensor, dst: torch.Tensor):
    """cskv_probe_copy: the 16-byte-per-lane reference copy of src's bytes into dst (same size)."""
    if src.numel() * src.element_size() != dst.numel() * dst.element_size() or src.device != dst.device:
        raise ValueError("probe_copy needs two equal-sized buffers on one device")
    with torch.cuda.device(src.device):
        _check(lib().cskv_probe_copy(_ptr(src), _ptr(dst), src.numel() * src.element_size(), _stream(src.device)),
               "cskv_probe_copy")


def probe_gather(src: torch.Tensor, width: int, n: int, salt: int, out: torch.Tensor):
    """cskv_probe_gather: n random `width`-byte reads from src (power-of-two bytes) into out."""
    if out.numel() * out.element_size() < n * width or src.device != out.device:
        raise ValueError("probe_gather: out must hold n * width bytes on src's device")
    with torch.cuda.device(src.device):
        _check(lib().cskv_probe_gather(_ptr(src), src.numel() * src.element_size(), width, n, salt, _ptr(out),
                                       _stream(src.device)), "cskv_probe_gather")


class Table:
    """A cache-semantic hash table in device memory (one caller-visible storage tensor).

    hbm_value_rows (default: all) keeps only that many value rows in HBM; the rest live in a
    pinned host tensor (``host_values``) that the kernels reach through its device alias."""

    def __init__(self, capacity: int, dim: int, mode: str = "dual", policy: str = "lru",
                 device="cuda", bucket_size: int = 128, hbm_value_rows: int | None = None):
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the table lives in GPU memory")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        L = lib()
        hbm_rows = int(capacity if hbm_value_rows is None else hbm_value_rows)
        nbytes = int(L.cskv_table_bytes_tiered(capacity, bucket_size, dim, hbm_rows))
        if nbytes == 0:
            raise CskvError(f"invalid table geometry capacity={capacity} bucket_size={bucket_size} dim={dim} "
                            f"hbm_value_rows={hbm_rows}")
        self.hbm_value_rows = hbm_rows
        self.host_values = None
        host_bytes = int(L.cskv_host_value_bytes(capacity, dim, hbm_rows))
        if host_bytes:
            self.host_values = torch.empty(host_bytes, dtype=torch.uint8, pin_memory=True)
        self.capacity, self.dim, self.bucket_size = int(capacity), int(dim), int(bucket_size)
        self.mode, self.policy = mode, policy
        self.n_buckets = self.capacity // self.bucket_size
        self.storage = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.cskv_create_tiered(ctypes.byref(h), capacity, bucket_size, dim, MODE[mode], POLICY[policy],
                                        _ptr(self.storage), nbytes, hbm_rows, _ptr(self.host_values), host_bytes,
                                        _stream(self.device)), "cskv_create_tiered")
        self._h = h
        self._ws = threading.local()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.cskv_destroy(h)
            self._h = None

    # ------------------------------------------------------------------ helpers
    def workspace(self, op: int, n: int) -> torch.Tensor:
        """Scratch for one call, kept per host thread (calls from different threads may overlap
        on the GPU under a role lock, so they must not share it)."""
        need = int(lib().cskv_workspace_bytes(self._h, op, n))
        ws = getattr(self._ws, "t", None)
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
            self._ws.t = ws
        return ws

    def _vals(self, v: torch.Tensor, n: int) -> torch.Tensor:
        if v.dtype != torch.float32 or v.device != self.device:
            raise TypeError("values must be float32 on the table's device")
        v = v.contiguous()
        if v.numel() != n * self.dim:
            raise ValueError(f"values must hold n*dim = {n * self.dim} floats")
        return v

    # ------------------------------------------------------------------ API
    @property
    def clock(self) -> int:
        return int(lib().cskv_clock(self._h))

    @clock.setter
    def clock(self, c: int):
        _check(lib().cskv_set_clock(self._h, c), "cskv_set_clock")

    def set_tuning(self, **kw):
        """Launch-shape knobs (find_group, route_group, find_prefetch_b2, find_blocks_per_cu); results
        never change."""
        for k, v in kw.items():
            _check(lib().cskv_set_tuning(self._h, TUNE[k], int(v)), f"cskv_set_tuning({k}={v})")

    def get_tuning(self) -> dict:
        return {k: int(lib().cskv_get_tuning(self._h, v)) for k, v in TUNE.items()}

    def set_route_subrounds(self, rounds: int):
        """Route sub-rounds per upsert call (1..64): the call's distinct keys, ordered by last
        occurrence, are routed and applied in that many chunks, each against the table the
        chunks before it left.  Results depend on it (unlike the tuning knobs)."""
        _check(lib().cskv_set_route_subrounds(self._h, int(rounds)), f"cskv_set_route_subrounds({rounds})")

    @property
    def route_subrounds(self) -> int:
        return int(lib().cskv_get_route_subrounds(self._h))

    def row_address(self, slot: int) -> int:
        """Device address of the value row of slot e = bucket * 128 + slot (a device alias of host
        memory for rows past hbm_value_rows)."""
        return int(lib().cskv_row_address(self._h, int(slot)))

    def set_lock_mode(self, mode: str):
        """"none" (the caller orders calls), "triple_group" or "reader_writer" (calls from several
        threads / streams are ordered by role; change only while no call is in flight)."""
        _check(lib().cskv_set_lock_mode(self._h, LOCK[mode]), f"cskv_set_lock_mode({mode})")

    @property
    def lock_mode(self) -> str:
        m = int(lib().cskv_get_lock_mode(self._h))
        return {v: k for k, v in LOCK.items()}[m]

    def clear(self):
        with torch.cuda.device(self.device):
            _check(lib().cskv_clear(self._h, _stream(self.device)), "cskv_clear")

    def find(self, keys: torch.Tensor, values_out=None, found_out=None, scores_out=None, want_scores=True):
        keys = _as_i64(keys, self.device)
        n = keys.numel()
        if values_out is None:
            values_out = torch.zeros((n, self.dim), dtype=torch.float32, device=self.device)
        if found_out is None:
            found_out = torch.empty(n, dtype=torch.uint8, device=self.device)
        if scores_out is None and want_scores:
            scores_out = torch.zeros(n, dtype=torch.int64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().cskv_find(self._h, n, _ptr(keys), _ptr(values_out), _ptr(found_out), _ptr(scores_out),
                                   _stream(self.device)), "cskv_find")
        return values_out, found_out, scores_out

    def insert_or_assign(self, keys, values, scores=None, status_out=None, want_status=True):
        keys = _as_i64(keys, self.device)
        n = keys.numel()
        values = self._vals(values, n)
        if scores is not None:
            scores = _as_i64(scores, self.device)
        if status_out is None and want_status:
            status_out = torch.empty(n, dtype=torch.uint8, device=self.device)
        ws = self.workspace(OP_INSERT_OR_ASSIGN, n)
        with torch.cuda.device(self.device):
            _check(lib().cskv_insert_or_assign(self._h, n, _ptr(keys), _ptr(values), _ptr(scores), _ptr(status_out),
                                               _ptr(ws), ws.numel(), _stream(self.device)), "cskv_insert_or_assign")
        return status_out

    def insert_or_assign_noalloc(self, keys, values, scores=None, status_out=None, want_status=True):
        """cskv_insert_or_assign_noalloc: insert_or_assign with the library's fixed workspace
        (at most NOALLOC_MAX_KEYS keys; no workspace tensor is allocated)."""
        keys = _as_i64(keys, self.device)
        n = keys.numel()
        values = self._vals(values, n)
        if scores is not None:
            scores = _as_i64(scores, self.device)
        if status_out is None and want_status:
            status_out = torch.empty(n, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().cskv_insert_or_assign_noalloc(self._h, n, _ptr(keys), _ptr(values), _ptr(scores),
                                                       _ptr(status_out), _stream(self.device)),
                   "cskv_insert_or_assign_noalloc")
        return status_out

    def insert_and_evict(self, keys, values, scores=None, out=None):
        """Returns (status, ev_keys, ev_values, ev_scores, n_evicted_device_tensor); the first
        n_evicted rows of the ev_* tensors are valid."""
        keys = _as_i64(keys, self.device)
        n = keys.numel()
        values = self._vals(values, n)
        if scores is not None:
            scores = _as_i64(scores, self.device)
        if out is None:
            out = (torch.empty(n, dtype=torch.uint8, device=self.device),
                   torch.empty(max(n, 1), dtype=torch.int64, device=self.device),
                   torch.empty((max(n, 1), self.dim), dtype=torch.float32, device=self.device),
                   torch.empty(max(n, 1), dtype=torch.int64, device=self.device),
                   torch.zeros(1, dtype=torch.int64, device=self.device))
        status, ek, evv, es, cnt = out
        ws = self.workspace(OP_INSERT_AND_EVICT, n)
        with torch.cuda.device(self.device):
            _check(lib().cskv_insert_and_evict(self._h, n, _ptr(keys), _ptr(values), _ptr(scores), _ptr(status),
                                               _ptr(ek), _ptr(evv), _ptr(es), _ptr(cnt), _ptr(ws), ws.numel(),
                                               _stream(self.device)), "cskv_insert_and_evict")
        return status, ek, evv, es, cnt

    def erase(self, keys, erased_out=None, want_erased=True):
        keys = _as_i64(keys, self.device)
        n = keys.numel()
        if erased_out is None and want_erased:
            erased_out = torch.empty(n, dtype=torch.uint8, device=self.device)
        ws = self.workspace(OP_ERASE, n)
        with torch.cuda.device(self.device):
            _check(lib().cskv_erase(self._h, n, _ptr(keys), _ptr(erased_out), _ptr(ws), ws.numel(),
                                    _stream(self.device)), "cskv_erase")
        return erased_out

    def contains(self, keys, found_out=None):
        keys = _as_i64(keys, self.device)
        n = keys.numel()
        if found_out is None:
            found_out = torch.empty(n, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().cskv_contains(self._h, n, _ptr(keys), _ptr(found_out), _stream(self.device)), "cskv_contains")
        return found_out

    def find_ptr(self, keys, ptrs_out=None, found_out=None, scores_out=None):
        """(device addresses of the resident rows as int64, 0 when absent; found; scores or None)."""
        keys = _as_i64(keys, self.device)
        n = keys.numel()
        if ptrs_out is None:
            ptrs_out = torch.empty(n, dtype=torch.int64, device=self.device)
        if found_out is None:
            found_out = torch.empty(n, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().cskv_find_ptr(self._h, n, _ptr(keys), _ptr(ptrs_out), _ptr(found_out), _ptr(scores_out),
                                       _stream(self.device)), "cskv_find_ptr")
        return ptrs_out, found_out, scores_out

    def assign(self, keys, values, scores=None, found_out=None):
        keys = _as_i64(keys, self.device)
        n = keys.numel()
        values = self._vals(values, n)
        if scores is not None:
            scores = _as_i64(scores, self.device)
        if found_out is None:
            found_out = torch.empty(n, dtype=torch.uint8, device=self.device)
        ws = self.workspace(OP_ASSIGN, n)
        with torch.cuda.device(self.device):
            _check(lib().cskv_assign(self._h, n, _ptr(keys), _ptr(values), _ptr(scores), _ptr(found_out), _ptr(ws),
                                     ws.numel(), _stream(self.device)), "cskv_assign")
        return found_out

    def assign_scores(self, keys, scores=None, found_out=None):
        keys = _as_i64(keys, self.device)
        n = keys.numel()
        if scores is not None:
            scores = _as_i64(scores, self.device)
        if found_out is None:
            found_out = torch.empty(n, dtype=torch.uint8, device=self.device)
        ws = self.workspace(OP_ASSIGN, n)
        with torch.cuda.device(self.device):
            _check(lib().cskv_assign_scores(self._h, n, _ptr(keys), _ptr(scores), _ptr(found_out), _ptr(ws),
                                            ws.numel(), _stream(self.device)), "cskv_assign_scores")
        return found_out

    def find_or_insert(self, keys, init_values, scores=None, values_out=None, status_out=None):
        """Returns (values_out [n, dim], status)."""
        keys = _as_i64(keys, self.device)
        n = keys.numel()
        init_values = self._vals(init_values, n)
        if scores is not None:
            scores = _as_i64(scores, self.device)
        if values_out is None:
            values_out = torch.zeros((n, self.dim), dtype=torch.float32, device=self.device)
        if status_out is None:
            status_out = torch.empty(n, dtype=torch.uint8, device=self.device)
        ws = self.workspace(OP_FIND_OR_INSERT, n)
        with torch.cuda.device(self.device):
            _check(lib().cskv_find_or_insert(self._h, n, _ptr(keys), _ptr(init_values), _ptr(scores),
                                             _ptr(values_out), _ptr(status_out), _ptr(ws), ws.numel(),
                                             _stream(self.device)), "cskv_find_or_insert")
        return values_out, status_out

    def size_tensor(self, out=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(1, dtype=torch.int64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().cskv_size(self._h, _ptr(out), _stream(self.device)), "cskv_size")
        return out

    def size(self) -> int:
        return int(self.size_tensor().item())

    def export(self, bucket_begin: int = 0, bucket_end: int | None = None, with_values: bool = True,
               min_score: int = 0):
        """(keys, values, scores, slots) of every entry in the bucket range (order unspecified);
        with min_score > 0 only the entries whose score is at least min_score (export_if)."""
        b1 = self.n_buckets if bucket_end is None else bucket_end
        cap = max(1, (b1 - bucket_begin) * self.bucket_size)
        k = torch.empty(cap, dtype=torch.int64, device=self.device)
        v = torch.empty((cap, self.dim), dtype=torch.float32, device=self.device) if with_values else None
        s = torch.empty(cap, dtype=torch.int64, device=self.device)
        sl = torch.empty(cap, dtype=torch.int64, device=self.device)
        c = torch.zeros(1, dtype=torch.int64, device=self.device)
        with torch.cuda.device(self.device):
            if min_score:
                _check(lib().cskv_export_if(self._h, bucket_begin, b1, int(min_score), _ptr(k), _ptr(v), _ptr(s),
                                            _ptr(sl), _ptr(c), _stream(self.device)), "cskv_export_if")
            else:
                _check(lib().cskv_export(self._h, bucket_begin, b1, _ptr(k), _ptr(v), _ptr(s), _ptr(sl), _ptr(c),
                                         _stream(self.device)), "cskv_export")
        n = int(c.item())
        return k[:n], (v[:n] if v is not None else None), s[:n], sl[:n]


class Program:
    """A batched program over one table (cskv_program_*): consecutive finds merge into one reader
    run; upserts and erases are serialization points; the whole program can be captured once as a
    hipGraph and replayed.  Tensors passed to add_* are kept alive by the program."""

    def __init__(self, table: Table, overlap=False):
        """overlap: False / 0 (one stream), True / 1 (phase graph on several streams) or 2 (only
        each upsert's scratch preparation runs ahead on a side stream)."""
        self.table = table
        h = ctypes.c_void_p()
        _check(lib().cskv_program_create(ctypes.byref(h), table._h), "cskv_program_create")
        self._h = h
        _check(lib().cskv_program_set_overlap(h, int(overlap)), "cskv_program_set_overlap")
        self._keep = []
        self._ws = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.cskv_program_destroy(h)
            self._h = None

    def _k(self, t):
        t = _as_i64(t, self.table.device)
        self._keep.append(t)
        return t

    def _o(self, t):
        if t is not None:
            if not t.is_contiguous():
                raise ValueError("program outputs must be contiguous")
            self._keep.append(t)
        return t

    def add_find(self, keys, values_out, found_out, scores_out=None):
        keys = self._k(keys)
        _check(lib().cskv_program_add_find(self._h, keys.numel(), _ptr(keys), _ptr(self._o(values_out)),
                                           _ptr(self._o(found_out)), _ptr(self._o(scores_out))),
               "cskv_program_add_find")

    def add_insert_or_assign(self, keys, values, scores=None, status_out=None):
        keys = self._k(keys)
        values = self._o(self.table._vals(values, keys.numel()))
        scores = self._k(scores) if scores is not None else None
        _check(lib().cskv_program_add_insert_or_assign(self._h, keys.numel(), _ptr(keys), _ptr(values), _ptr(scores),
                                                       _ptr(self._o(status_out))),
               "cskv_program_add_insert_or_assign")

    def add_insert_and_evict(self, keys, values, scores, status, ev_keys, ev_values, ev_scores, n_evicted):
        keys = self._k(keys)
        values = self._o(self.table._vals(values, keys.numel()))
        scores = self._k(scores) if scores is not None else None
        _check(lib().cskv_program_add_insert_and_evict(
            self._h, keys.numel(), _ptr(keys), _ptr(values), _ptr(scores), _ptr(self._o(status)),
            _ptr(self._o(ev_keys)), _ptr(self._o(ev_values)), _ptr(self._o(ev_scores)), _ptr(self._o(n_evicted))),
            "cskv_program_add_insert_and_evict")

    def add_erase(self, keys, erased_out=None):
        keys = self._k(keys)
        _check(lib().cskv_program_add_erase(self._h, keys.numel(), _ptr(keys), _ptr(self._o(erased_out))),
               "cskv_program_add_erase")

    def finalize(self):
        need = int(lib().cskv_program_workspace_bytes(self._h))
        self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.table.device)
        _check(lib().cskv_program_set_workspace(self._h, _ptr(self._ws), self._ws.numel()),
               "cskv_program_set_workspace")
        return self

    @property
    def segments(self) -> int:
        return int(lib().cskv_program_segments(self._h))

    @property
    def phases(self) -> int:
        return int(lib().cskv_program_phases(self._h))

    def _s(self, stream):
        s = stream if stream is not None else torch.cuda.current_stream(self.table.device)
        return ctypes.c_void_p(s.cuda_stream)

    def launch(self, stream=None):
        with torch.cuda.device(self.table.device):
            _check(lib().cskv_program_launch(self._h, self._s(stream)), "cskv_program_launch")

    def capture(self, stream):
        """Record the program on `stream` (a non-default torch.cuda.Stream) into a hipGraph."""
        with torch.cuda.device(self.table.device):
            _check(lib().cskv_program_capture(self._h, self._s(stream)), "cskv_program_capture")

    def replay(self, stream=None):
        with torch.cuda.device(self.table.device):
            _check(lib().cskv_program_replay(self._h, self._s(stream)), "cskv_program_replay")


class MtThread(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("n", ctypes.c_uint64), ("calls", ctypes.c_uint64),
                ("d_keys", ctypes.c_void_p), ("d_values", ctypes.c_void_p), ("d_scores", ctypes.c_void_p),
                ("d_values_out", ctypes.c_void_p), ("d_flags", ctypes.c_void_p), ("d_ws", ctypes.c_void_p),
                ("ws_bytes", ctypes.c_size_t), ("status", ctypes.c_int), ("hip_error", ctypes.c_int),
                ("failed_call", ctypes.c_uint64)]


def run_threads(table: Table, specs) -> float:
    """Runs the concurrent-caller driver (include/cskv_mt.h): one host thread and stream per spec,
    all started together.  A spec is a dict: op ("find" / "assign" / "insert_erase"), calls, keys
    (int64 [n]), and per op values (float32 [n, dim]), scores (int64 [n] or None), values_out
    (float32 [n, dim], find) and flags (uint8 [n]).  Workspaces are allocated here, one per
    thread.  Returns the wall time in ms."""
    arr = (MtThread * len(specs))()
    keep = []
    for i, sp in enumerate(specs):
        keys = _as_i64(sp["keys"], table.device)
        n = keys.numel()
        op = MT_OP[sp["op"]]
        ws = None
        if op == MT_OP["assign"]:
            need = int(lib().cskv_workspace_bytes(table._h, OP_ASSIGN, n))
        elif op == MT_OP["insert_erase"]:
            need = max(int(lib().cskv_workspace_bytes(table._h, OP_INSERT_OR_ASSIGN, n)),
                       int(lib().cskv_workspace_bytes(table._h, OP_ERASE, n)))
        else:
            need = 0
        if need:
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device=table.device)
        vals = sp.get("values")
        if vals is not None:
            vals = table._vals(vals, n)
        sc = sp.get("scores")
        if sc is not None:
            sc = _as_i64(sc, table.device)
        keep += [keys, ws, vals, sc, sp.get("values_out"), sp["flags"]]
        arr[i] = MtThread(op, n, int(sp["calls"]), keys.data_ptr(), None if vals is None else vals.data_ptr(),
                          None if sc is None else sc.data_ptr(),
                          None if sp.get("values_out") is None else sp["values_out"].data_ptr(),
                          sp["flags"].data_ptr(), None if ws is None else ws.data_ptr(), 0 if ws is None else ws.numel())
    torch.cuda.synchronize(table.device)
    ms = ctypes.c_double(0.0)
    rc = lib().cskv_mt_run(table._h, len(specs), ctypes.cast(arr, ctypes.c_void_p), ctypes.byref(ms))
    del keep
    if rc != 0:
        bad = [(i, arr[i].status, arr[i].hip_error, arr[i].failed_call) for i in range(len(specs)) if arr[i].status]
        raise CskvError(f"cskv_mt_run: {lib().cskv_strerror(rc).decode()} ({rc}); "
                        f"failing threads (index, status, hip error, call): {bad}")
    return ms.value
