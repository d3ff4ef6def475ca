"""Binding of the native serving loop (``pir_server_*`` in include/qpir.h).

Argument marshalling only: batching, admission, graph replay and latency
accounting all run in the library's threads.  Queries and answers live in
host memory (numpy uint32 arrays); this object keeps references to them
until the server is drained, since the library reads and writes them
asynchronously.
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import ServerConfig, ServerStats, _P, _U32, _U64, check, lib

UINT64_MAX = (1 << 64) - 1


def _host_words(a: np.ndarray, n: int, name: str) -> np.ndarray:
    if not isinstance(a, np.ndarray) or a.dtype not in (np.uint32, np.int32):
        raise TypeError(f"{name}: expected a uint32 numpy array")
    if a.size != n or not a.flags.c_contiguous:
        raise ValueError(f"{name}: expected {n} contiguous words")
    return a


class Server:
    """Continuous-batching PIR server over open :class:`Database` objects.

    ``max_inflight`` caps the batches with kernels pending over all
    databases; one that only copies its answers out no longer counts (0: only
    ``slots_per_db`` bounds them).  Under load the cap keeps
    requests queued while the device is busy, so they leave in larger
    batches; the database with the longest-waiting request goes first.
    """

    def __init__(self, dbs, max_batch: int = 64, slots_per_db: int = 2,
                 mem_budget_bytes: int = 2 << 30, max_queue: int = 0, use_graphs: bool = True,
                 max_inflight: int = 4):
        self.dbs = list(dbs)
        cfg = ServerConfig(max_batch=max_batch, slots_per_db=slots_per_db,
                           mem_budget_bytes=mem_budget_bytes, max_queue=max_queue,
                           use_graphs=1 if use_graphs else 0, max_inflight=max_inflight)
        h = _P()
        import torch
        self.device = self.dbs[0].device
        with torch.cuda.device(self.device):
            check(lib().pir_server_create(ctypes.byref(cfg), ctypes.byref(h)), "pir_server_create")
            self._h = h
            for db in self.dbs:
                idx = _U32()
                check(lib().pir_server_add_db(h, db.handle, ctypes.byref(idx)), "pir_server_add_db")
            check(lib().pir_server_start(h), "pir_server_start")
        self._keep = []

    @staticmethod
    def now_ns() -> int:
        return int(lib().pir_server_now_ns())

    def submit(self, db_index: int, q: np.ndarray, out: np.ndarray = None,
               t_arrival_ns: int = 0) -> int:
        db = self.dbs[db_index]
        _host_words(q, db.cols, "q")
        if out is not None:
            _host_words(out, db.rows, "out")
        t = _U64()
        check(lib().pir_server_submit(self._h, db_index, q.ctypes.data,
                                      None if out is None else out.ctypes.data,
                                      t_arrival_ns, ctypes.byref(t)), "pir_server_submit")
        self._keep.append((q, out))
        return int(t.value)

    def wait(self, ticket: int, timeout_s: float = None) -> None:
        tmo = UINT64_MAX if timeout_s is None else int(timeout_s * 1e9)
        check(lib().pir_server_wait(self._h, ticket, tmo), "pir_server_wait")

    def drain(self) -> None:
        check(lib().pir_server_drain(self._h), "pir_server_drain")
        self._keep.clear()

    def pause(self, db_index: int) -> None:
        check(lib().pir_server_pause_db(self._h, db_index), "pir_server_pause_db")

    def resume(self, db_index: int) -> None:
        check(lib().pir_server_resume_db(self._h, db_index), "pir_server_resume_db")

    def stats(self) -> dict:
        st = ServerStats()
        check(lib().pir_server_stats_get(self._h, ctypes.byref(st)), "pir_server_stats_get")
        return {name: int(getattr(st, name)) for name, _ in ServerStats._fields_}

    def latencies(self, first: int, count: int) -> np.ndarray:
        out = np.zeros(count, dtype=np.uint64)
        check(lib().pir_server_latencies(self._h, first, count, out.ctypes.data),
              "pir_server_latencies")
        return out

    def replay(self, offsets_ns: np.ndarray, db_index: np.ndarray, queries, answers=None) -> int:
        """Open-loop arrivals (see ``pir_server_replay``); returns the first ticket."""
        n = len(offsets_ns)
        off = np.ascontiguousarray(offsets_ns, dtype=np.uint64)
        dbi = np.ascontiguousarray(db_index, dtype=np.uint32)
        for i in range(n):
            _host_words(queries[i], self.dbs[int(dbi[i])].cols, "q")
        qp = (ctypes.c_void_p * n)(*[q.ctypes.data for q in queries])
        ap = None
        if answers is not None:
            ap = (ctypes.c_void_p * n)(*[a.ctypes.data if a is not None else None for a in answers])
        first = _U64()
        self._keep.append((off, dbi, qp, ap, queries, answers))
        check(lib().pir_server_replay(self._h, n, off.ctypes.data, dbi.ctypes.data, qp, ap,
                                      ctypes.byref(first)), "pir_server_replay")
        return int(first.value)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            st = lib().pir_server_destroy(self._h)
            self._h = None
            self._keep.clear()
            check(st, "pir_server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
