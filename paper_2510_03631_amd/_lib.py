"""ctypes binding of ``libqpir.so`` (argument marshalling only).

Every computation runs in the HIP library.  If the library is missing or
cannot be loaded, :func:`lib` raises: there is no fallback of any kind.
Tensors are torch tensors on the GPU; 32-bit words may be ``torch.int32`` or
``torch.uint32`` (the bits are what count).  Each call enqueues on the
current torch stream of the tensor's device unless a stream is given.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqpir.so")

PIR_OK = 0
STATUS_NAMES = {
    0: "PIR_OK", 1: "PIR_ERR_INVALID_ARG", 2: "PIR_ERR_SHAPE", 3: "PIR_ERR_NO_MEMORY",
    4: "PIR_ERR_DEVICE", 5: "PIR_ERR_UNSUPPORTED", 6: "PIR_ERR_WORKSPACE",
    7: "PIR_ERR_BUSY", 8: "PIR_ERR_TIMEOUT",
}

_lib = None
_lock = threading.Lock()

_P = ctypes.c_void_p
_U64 = ctypes.c_uint64
_U32 = ctypes.c_uint32
_SZ = ctypes.c_size_t
_ST = ctypes.c_int


class ServerConfig(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_uint32), ("slots_per_db", ctypes.c_uint32),
                ("mem_budget_bytes", ctypes.c_uint64), ("max_queue", ctypes.c_uint32),
                ("use_graphs", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "submitted", "completed", "failed", "rejected", "batches", "batched_queries",
        "budget_bytes", "peak_inflight_bytes", "p50_ns", "p99_ns", "max_ns", "device_bytes")]


# name -> (restype, argtypes); mirrors include/qpir.h
SIGNATURES = {
    "pir_status_string": (ctypes.c_char_p, [_ST]),
    "pir_version": (_U32, []),
    "pir_db_open": (_ST, [_P, _U64, _U64, _U64, _P, ctypes.POINTER(_P)]),
    "pir_db_close": (_ST, [_P]),
    "pir_db_shape": (_ST, [_P, ctypes.POINTER(_U64), ctypes.POINTER(_U64)]),
    "pir_workspace_bytes": (_SZ, [_P, _U32]),
    "pir_answer": (_ST, [_P, _P, _P, _P, _SZ, _P]),
    "pir_answer_batch": (_ST, [_P, _P, _U32, _P, _P, _SZ, _P]),
    "pir_setup_hint": (_ST, [_P, _P, _U32, _P, _P, _SZ, _P]),
    "pir_update_rows": (_ST, [_P, _P, _U32, _P, _P]),
    "pir_hint_update_rows": (_ST, [_P, _P, _U32, _P, _U32, _P, _P, _SZ, _P]),
    "pir_answer_batch_qmajor": (_ST, [_P, _P, _U32, _P, _P, _SZ, _P]),
    "pir_answer_batch_modp": (_ST, [_P, _P, _U32, _U32, _P, _P, _SZ, _P]),
    "pir_answer_batch_noalloc": (_ST, [_P, _P, _U32, _P, _P]),
    "pir_hint_planes_bytes": (_SZ, [_P, _U32]),
    "pir_hint_planes": (_ST, [_P, _P, _U32, _P, _SZ, _P]),
    "pir_hint_update_rows_planes": (_ST, [_P, _P, _U32, _P, _SZ, _U32, _P, _P, _SZ, _P]),
    "pir_variant_count": (_U32, [_U32]),
    "pir_variant_name": (ctypes.c_char_p, [_U32, _U32]),
    "pir_db_set_variant": (_ST, [_P, _U32, _U32]),
    "pir_db_get_variant": (_U32, [_P, _U32]),
    "pir_server_create": (_ST, [ctypes.POINTER(ServerConfig), ctypes.POINTER(_P)]),
    "pir_server_add_db": (_ST, [_P, _P, ctypes.POINTER(_U32)]),
    "pir_server_start": (_ST, [_P]),
    "pir_server_submit": (_ST, [_P, _U32, _P, _P, _U64, ctypes.POINTER(_U64)]),
    "pir_server_now_ns": (_U64, []),
    "pir_server_wait": (_ST, [_P, _U64, _U64]),
    "pir_server_drain": (_ST, [_P]),
    "pir_server_pause_db": (_ST, [_P, _U32]),
    "pir_server_resume_db": (_ST, [_P, _U32]),
    "pir_server_stats_get": (_ST, [_P, ctypes.POINTER(ServerStats)]),
    "pir_server_latencies": (_ST, [_P, _U64, _U64, _P]),
    "pir_server_replay": (_ST, [_P, _U64, _P, _P, _P, _P, ctypes.POINTER(_U64)]),
    "pir_server_destroy": (_ST, [_P]),
    "pir_client_query": (_ST, [_P, _U32, _U32, _P, _P, _P, _U32, _P, _P]),
    "pir_client_decode": (_ST, [_P, _U32, _U32, _P, _P, _U32, _P, _P]),
    "pir_client_mat_open": (_ST, [_P, _U32, _U32, _P, ctypes.POINTER(_P)]),
    "pir_client_mat_close": (_ST, [_P]),
    "pir_client_mat_workspace_bytes": (_SZ, [_P, _U32]),
    "pir_client_mat_set_variant": (_ST, [_P, _U32, _U32]),
    "pir_client_query_mat": (_ST, [_P, _P, _P, _P, _U32, _P, _P, _SZ, _P]),
    "pir_client_decode_mat": (_ST, [_P, _P, _P, _U32, _P, _P, _SZ, _P]),
    "pir_chor_answer": (_ST, [_P, _U32, _U32, _U64, _P, _U32, _P, _P]),
    "pir_prg_expand": (_ST, [_P, _U32, _U32, _P, _P]),
    "pir_oop_workspace_bytes": (_SZ, [_U32, _U32, _U32]),
    "pir_oop_offline": (_ST, [_P, _U32, _U32, _U32, _U64, _P, _U32, _P, _P, _SZ, _P]),
    "pir_oop_answer": (_ST, [_P, _U32, _U32, _U64, _P, _U32, _P, _P, _P]),
}


class PirError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{what}: {name} ({_status_string(status)})")


def lib() -> ctypes.CDLL:
    """Load ``libqpir.so``; raise if it is not built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is not built; run `python -m paper_2510_03631_amd.build`")
            h = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(h, name)
                fn.restype = res
                fn.argtypes = args
            _lib = h
    return _lib


def _status_string(status: int) -> str:
    try:
        return lib().pir_status_string(status).decode()
    except Exception:
        return "?"


def check(status: int, what: str) -> None:
    if status != PIR_OK:
        raise PirError(status, what)


def _stream_ptr(stream, device) -> int:
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return stream.cuda_stream


_WORD = (torch.int32, torch.uint32)


def _ptr_words(t: torch.Tensor, name: str, shape, device) -> int:
    if t.dtype not in _WORD:
        raise TypeError(f"{name}: expected a 32-bit word tensor, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    if t.device != device or not t.is_contiguous():
        raise ValueError(f"{name}: must be a contiguous tensor on {device}")
    return t.data_ptr()


def _ptr_bytes(t: torch.Tensor, name: str, shape, device) -> int:
    if t.dtype != torch.uint8:
        raise TypeError(f"{name}: expected uint8, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    if t.device != device or not t.is_contiguous():
        raise ValueError(f"{name}: must be a contiguous tensor on {device}")
    return t.data_ptr()


class Database:
    """A database resident in GPU memory, opened through ``pir_db_open``.

    ``D`` is an ``R x C`` uint8 CUDA tensor whose rows may be padded (a 2-D
    view with ``stride(1) == 1``).  The handle borrows its memory; this
    object keeps a reference so it stays alive until :meth:`close`.
    """

    def __init__(self, D: torch.Tensor, stream=None):
        if D.dtype != torch.uint8 or D.dim() != 2 or D.stride(1) != 1 or not D.is_cuda:
            raise ValueError("D must be a 2-D uint8 CUDA tensor with unit column stride")
        self.D = D
        self.device = D.device
        self.rows, self.cols = int(D.shape[0]), int(D.shape[1])
        self.pitch = int(D.stride(0)) if self.rows > 1 else self.cols
        self._ws = {}
        h = _P()
        with torch.cuda.device(self.device):
            check(lib().pir_db_open(D.data_ptr(), self.rows, self.cols, self.pitch,
                                    _stream_ptr(stream, self.device), ctypes.byref(h)),
                  "pir_db_open")
        self._h = h

    # -- lifecycle
    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            with torch.cuda.device(self.device):
                check(lib().pir_db_close(self._h), "pir_db_close")
            self._h = None
        self._ws.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        if self._h is None:
            raise PirError(1, "database is closed")
        return self._h

    # -- workspace
    def workspace_bytes(self, batch: int = 0) -> int:
        return int(lib().pir_workspace_bytes(self.handle, batch))

    def workspace(self, batch: int = 0):
        """A cached device buffer of ``workspace_bytes(batch)`` bytes (or None)."""
        nbytes = self.workspace_bytes(batch)
        if nbytes == 0:
            return None
        buf = self._ws.get(batch)
        if buf is None or buf.numel() < nbytes:
            buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self._ws[batch] = buf
        return buf

    @staticmethod
    def _ws_args(ws):
        if ws is None:
            return None, 0
        return ws.data_ptr(), ws.numel() * ws.element_size()

    # -- entry points
    def answer(self, q: torch.Tensor, out: torch.Tensor = None, stream=None, ws=None):
        """``a = D q mod 2^32`` (``pir_answer``)."""
        qp = _ptr_words(q, "q", (self.cols,), self.device)
        if out is None:
            out = torch.empty(self.rows, dtype=torch.int32, device=self.device)
        op = _ptr_words(out, "out", (self.rows,), self.device)
        if ws is None:
            ws = self.workspace(0)
        wp, wn = self._ws_args(ws)
        check(lib().pir_answer(self.handle, qp, op, wp, wn, _stream_ptr(stream, self.device)),
              "pir_answer")
        return out

    def answer_batch(self, Q: torch.Tensor, out: torch.Tensor = None, stream=None, ws=None):
        """``Out = D Q mod 2^32`` for ``Q`` of shape C x B (``pir_answer_batch``)."""
        if Q.dim() != 2:
            raise ValueError("Q must be C x B")
        B = int(Q.shape[1])
        qp = _ptr_words(Q, "Q", (self.cols, B), self.device)
        if out is None:
            out = torch.empty((self.rows, B), dtype=torch.int32, device=self.device)
        op = _ptr_words(out, "out", (self.rows, B), self.device)
        if ws is None:
            ws = self.workspace(B)
        wp, wn = self._ws_args(ws)
        check(lib().pir_answer_batch(self.handle, qp, B, op, wp, wn,
                                     _stream_ptr(stream, self.device)), "pir_answer_batch")
        return out

    def answer_batch_noalloc(self, Q: torch.Tensor, out: torch.Tensor, stream=None):
        """``pir_answer_batch`` without a workspace or any allocation
        (``pir_answer_batch_noalloc``): the caller passes ``out`` (R x B)."""
        if Q.dim() != 2:
            raise ValueError("Q must be C x B")
        B = int(Q.shape[1])
        qp = _ptr_words(Q, "Q", (self.cols, B), self.device)
        op = _ptr_words(out, "out", (self.rows, B), self.device)
        check(lib().pir_answer_batch_noalloc(self.handle, qp, B, op,
                                             _stream_ptr(stream, self.device)),
              "pir_answer_batch_noalloc")
        return out

    def answer_batch_qmajor(self, Qt: torch.Tensor, out: torch.Tensor = None, stream=None,
                            ws=None):
        """``out[b] = D Qt[b] mod 2^32`` for ``Qt`` of shape B x C
        (``pir_answer_batch_qmajor``); ``out`` is B x R."""
        if Qt.dim() != 2:
            raise ValueError("Qt must be B x C")
        B = int(Qt.shape[0])
        qp = _ptr_words(Qt, "Qt", (B, self.cols), self.device)
        if out is None:
            out = torch.empty((B, self.rows), dtype=torch.int32, device=self.device)
        op = _ptr_words(out, "out", (B, self.rows), self.device)
        if ws is None:
            ws = self.workspace(B)
        wp, wn = self._ws_args(ws)
        check(lib().pir_answer_batch_qmajor(self.handle, qp, B, op, wp, wn,
                                            _stream_ptr(stream, self.device)),
              "pir_answer_batch_qmajor")
        return out

    def answer_batch_modp(self, Q: torch.Tensor, p: int, out: torch.Tensor = None, stream=None,
                          ws=None):
        """``Out = D Q mod p`` for ``Q`` of shape C x B, ``2 <= p < 2^32``
        (``pir_answer_batch_modp``, the Goldberg share product)."""
        if Q.dim() != 2:
            raise ValueError("Q must be C x B")
        p = int(p)
        if not 2 <= p < 1 << 32:
            raise ValueError("p must be in [2, 2^32)")
        B = int(Q.shape[1])
        qp = _ptr_words(Q, "Q", (self.cols, B), self.device)
        if out is None:
            out = torch.empty((self.rows, B), dtype=torch.int32, device=self.device)
        op = _ptr_words(out, "out", (self.rows, B), self.device)
        if ws is None:
            ws = self.workspace(B)
        wp, wn = self._ws_args(ws)
        check(lib().pir_answer_batch_modp(self.handle, qp, B, p, op, wp, wn,
                                          _stream_ptr(stream, self.device)),
              "pir_answer_batch_modp")
        return out

    def set_variant(self, batch: int, variant, rows: bool = False) -> None:
        """Pin a kernel variant (index or name) for ``batch``'s bucket; with
        ``rows``, for the row-gathered products (``hint_update_rows``)."""
        if isinstance(variant, str):
            variant = variant_names(batch).index(variant)
        key = batch | (VARIANT_ROWS if rows else 0)
        check(lib().pir_db_set_variant(self.handle, key, int(variant)), "pir_db_set_variant")

    def get_variant(self, batch: int, rows: bool = False) -> int:
        key = batch | (VARIANT_ROWS if rows else 0)
        return int(lib().pir_db_get_variant(self.handle, key))

    def setup_hint(self, A: torch.Tensor, out: torch.Tensor = None, stream=None, ws=None):
        """``H = D A mod 2^32`` for ``A`` of shape C x n (``pir_setup_hint``)."""
        n = int(A.shape[1])
        ap = _ptr_words(A, "A", (self.cols, n), self.device)
        if out is None:
            out = torch.empty((self.rows, n), dtype=torch.int32, device=self.device)
        op = _ptr_words(out, "H", (self.rows, n), self.device)
        if ws is None:
            ws = self.workspace(n)
        wp, wn = self._ws_args(ws)
        check(lib().pir_setup_hint(self.handle, ap, n, op, wp, wn,
                                   _stream_ptr(stream, self.device)), "pir_setup_hint")
        return out

    def update_rows(self, rows: torch.Tensor, new: torch.Tensor, stream=None):
        """``D[rows[i]] = new[i]`` and refresh the handle's metadata."""
        m = int(rows.numel())
        rp = _ptr_words(rows, "rows", (m,), self.device)
        np_ = _ptr_bytes(new, "new", (m, self.cols), self.device)
        check(lib().pir_update_rows(self.handle, rp, m, np_, _stream_ptr(stream, self.device)),
              "pir_update_rows")

    def hint_update_rows(self, rows: torch.Tensor, A: torch.Tensor, H: torch.Tensor,
                         stream=None, ws=None):
        """``H[rows[i]] = D[rows[i]] A mod 2^32``; other rows of H are kept."""
        m = int(rows.numel())
        n = int(A.shape[1])
        rp = _ptr_words(rows, "rows", (m,), self.device)
        ap = _ptr_words(A, "A", (self.cols, n), self.device)
        hp = _ptr_words(H, "H", (self.rows, n), self.device)
        if ws is None:
            ws = self.workspace(n)
        wp, wn = self._ws_args(ws)
        check(lib().pir_hint_update_rows(self.handle, rp, m, ap, n, hp, wp, wn,
                                         _stream_ptr(stream, self.device)),
              "pir_hint_update_rows")
        return H

    def hint_planes(self, A: torch.Tensor, out: torch.Tensor = None, stream=None):
        """A's limb planes for the incremental hint (``pir_hint_planes``):
        a uint8 device tensor, opaque, valid for databases with this column
        count until A changes."""
        n = int(A.shape[1])
        ap = _ptr_words(A, "A", (self.cols, n), self.device)
        nb = int(lib().pir_hint_planes_bytes(self.handle, n))
        if out is None:
            out = torch.empty(nb, dtype=torch.uint8, device=self.device)
        if out.dtype != torch.uint8 or out.numel() < nb or not out.is_contiguous():
            raise ValueError(f"planes: expected a contiguous uint8 tensor of {nb} bytes")
        check(lib().pir_hint_planes(self.handle, ap, n, out.data_ptr(), out.numel(),
                                    _stream_ptr(stream, self.device)), "pir_hint_planes")
        return out

    def hint_update_rows_planes(self, rows: torch.Tensor, planes: torch.Tensor, n: int,
                                H: torch.Tensor, stream=None, ws=None):
        """``hint_update_rows`` with A given by :meth:`hint_planes`
        (``pir_hint_update_rows_planes``)."""
        m = int(rows.numel())
        rp = _ptr_words(rows, "rows", (m,), self.device)
        hp = _ptr_words(H, "H", (self.rows, n), self.device)
        if planes.dtype != torch.uint8 or not planes.is_contiguous() or planes.device != self.device:
            raise ValueError("planes: expected a contiguous uint8 tensor on the database's device")
        if ws is None:
            ws = self.workspace(n)
        wp, wn = self._ws_args(ws)
        check(lib().pir_hint_update_rows_planes(self.handle, rp, m, planes.data_ptr(),
                                                planes.numel(), n, hp, wp, wn,
                                                _stream_ptr(stream, self.device)),
              "pir_hint_update_rows_planes")
        return H


# Flag of pir_db_set_variant's batch argument: the row-gathered table.
VARIANT_ROWS = 0x80000000


def variant_names(batch: int) -> list:
    """Names of the kernel variants for a batch size (0: single query)."""
    h = lib()
    return [h.pir_variant_name(batch, i).decode() for i in range(h.pir_variant_count(batch))]


def client_query(A: torch.Tensor, S: torch.Tensor, E: torch.Tensor, cols: torch.Tensor,
                 out: torch.Tensor = None, stream=None) -> torch.Tensor:
    """LWE queries ``Qt[b] = A S[b] + E[b] + 2^24 u_{cols[b]}`` (B x C words)."""
    C, n = int(A.shape[0]), int(A.shape[1])
    B = int(S.shape[0])
    dev = A.device
    ap = _ptr_words(A, "A", (C, n), dev)
    sp = _ptr_words(S, "S", (B, n), dev)
    ep = _ptr_words(E, "E", (B, C), dev)
    cp = _ptr_words(cols, "cols", (B,), dev)
    if out is None:
        out = torch.empty((B, C), dtype=torch.int32, device=dev)
    op = _ptr_words(out, "out", (B, C), dev)
    with torch.cuda.device(dev):
        check(lib().pir_client_query(ap, C, n, sp, ep, cp, B, op, _stream_ptr(stream, dev)),
              "pir_client_query")
    return out


def client_decode(H: torch.Tensor, S: torch.Tensor, answers: torch.Tensor,
                  out: torch.Tensor = None, stream=None) -> torch.Tensor:
    """Recovered bytes ``((answers[b] - H S[b] + 2^23) mod 2^32) >> 24`` (B x R)."""
    R, n = int(H.shape[0]), int(H.shape[1])
    B = int(S.shape[0])
    dev = H.device
    hp = _ptr_words(H, "H", (R, n), dev)
    sp = _ptr_words(S, "S", (B, n), dev)
    ap = _ptr_words(answers, "answers", (B, R), dev)
    if out is None:
        out = torch.empty((B, R), dtype=torch.uint8, device=dev)
    op = _ptr_bytes(out, "out", (B, R), dev)
    with torch.cuda.device(dev):
        check(lib().pir_client_decode(hp, R, n, sp, ap, B, op, _stream_ptr(stream, dev)),
              "pir_client_decode")
    return out


class ClientMatrix:
    """A word matrix prepared for the matrix-core client steps
    (``pir_client_mat_*``): the public matrix A for :meth:`query`, the hint H
    for :meth:`decode`.  Holds rows x 4n bytes of device memory until
    :meth:`close`."""

    def __init__(self, M: torch.Tensor, stream=None):
        if M.dim() != 2:
            raise ValueError("M must be rows x n")
        self.rows, self.n = int(M.shape[0]), int(M.shape[1])
        self.device = M.device
        mp = _ptr_words(M, "M", (self.rows, self.n), self.device)
        h = _P()
        with torch.cuda.device(self.device):
            check(lib().pir_client_mat_open(mp, self.rows, self.n,
                                            _stream_ptr(stream, self.device), ctypes.byref(h)),
                  "pir_client_mat_open")
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            h, self._h = self._h, None
            check(lib().pir_client_mat_close(h), "pir_client_mat_close")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_variant(self, batch: int, variant) -> None:
        """Kernel variant of the product for ``batch``'s bucket (index or name)."""
        if isinstance(variant, str):
            variant = variant_names(batch).index(variant)
        check(lib().pir_client_mat_set_variant(self._h, batch, variant),
              "pir_client_mat_set_variant")

    def workspace(self, B: int) -> torch.Tensor:
        nb = int(lib().pir_client_mat_workspace_bytes(self._h, B))
        return torch.empty(max(nb, 1), dtype=torch.uint8, device=self.device)

    def query(self, S: torch.Tensor, E: torch.Tensor, cols: torch.Tensor,
              out: torch.Tensor = None, ws: torch.Tensor = None, stream=None) -> torch.Tensor:
        """``Qt[b] = A S[b] + E[b] + 2^24 u_{cols[b]}`` (B x C words)."""
        B = int(S.shape[0])
        sp = _ptr_words(S, "S", (B, self.n), self.device)
        ep = _ptr_words(E, "E", (B, self.rows), self.device)
        cp = _ptr_words(cols, "cols", (B,), self.device)
        if out is None:
            out = torch.empty((B, self.rows), dtype=torch.int32, device=self.device)
        op = _ptr_words(out, "out", (B, self.rows), self.device)
        if ws is None:
            ws = self.workspace(B)
        with torch.cuda.device(self.device):
            check(lib().pir_client_query_mat(self._h, sp, ep, cp, B, op, ws.data_ptr(),
                                             ws.numel(), _stream_ptr(stream, self.device)),
                  "pir_client_query_mat")
        return out

    def decode(self, S: torch.Tensor, answers: torch.Tensor, out: torch.Tensor = None,
               ws: torch.Tensor = None, stream=None) -> torch.Tensor:
        """``((answers[b] - H S[b] + 2^23) mod 2^32) >> 24`` (B x R bytes)."""
        B = int(S.shape[0])
        sp = _ptr_words(S, "S", (B, self.n), self.device)
        ap = _ptr_words(answers, "answers", (B, self.rows), self.device)
        if out is None:
            out = torch.empty((B, self.rows), dtype=torch.uint8, device=self.device)
        op = _ptr_bytes(out, "out", (B, self.rows), self.device)
        if ws is None:
            ws = self.workspace(B)
        with torch.cuda.device(self.device):
            check(lib().pir_client_decode_mat(self._h, sp, ap, B, op, ws.data_ptr(), ws.numel(),
                                              _stream_ptr(stream, self.device)),
                  "pir_client_decode_mat")
        return out


def chor_answer(DB: torch.Tensor, Q: torch.Tensor, out: torch.Tensor = None,
                stream=None) -> torch.Tensor:
    """Chor XOR-PIR responses: ``DB`` is rows x W words (row stride may be
    padded), ``Q`` is B x ceil(rows/32) packed selector words; returns B x W."""
    if DB.dim() != 2 or DB.stride(1) != 1 or DB.dtype not in _WORD:
        raise ValueError("DB must be a 2-D 32-bit word tensor with unit column stride")
    rows, W = int(DB.shape[0]), int(DB.shape[1])
    dev = DB.device
    if not DB.is_cuda:
        raise ValueError("DB must be on the GPU")
    B = int(Q.shape[0])
    qp_ = _ptr_words(Q, "Q", (B, (rows + 31) // 32), dev)
    if out is None:
        out = torch.empty((B, W), dtype=torch.int32, device=dev)
    op = _ptr_words(out, "out", (B, W), dev)
    pitch = int(DB.stride(0)) if rows > 1 else W
    with torch.cuda.device(dev):
        check(lib().pir_chor_answer(DB.data_ptr(), rows, W, pitch, qp_, B, op,
                                    _stream_ptr(stream, dev)), "pir_chor_answer")
    return out


def _word_matrix(DB: torch.Tensor, name: str):
    if DB.dim() != 2 or DB.stride(1) != 1 or DB.dtype not in _WORD:
        raise ValueError(f"{name} must be a 2-D 32-bit word tensor with unit column stride")
    if not DB.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    rows, W = int(DB.shape[0]), int(DB.shape[1])
    return rows, W, (int(DB.stride(0)) if rows > 1 else W)


def prg_expand(seeds: torch.Tensor, bits: int, out: torch.Tensor = None,
               stream=None) -> torch.Tensor:
    """ChaCha20 expansion of ``count`` 8-word seeds into ``bits`` bits each
    (``pir_prg_expand``); returns count x ceil(bits/32) words."""
    count = int(seeds.shape[0])
    dev = seeds.device
    sp = _ptr_words(seeds, "seeds", (count, 8), dev)
    nw = (int(bits) + 31) // 32
    if out is None:
        out = torch.empty((count, nw), dtype=torch.int32, device=dev)
    op = _ptr_words(out, "out", (count, nw), dev)
    with torch.cuda.device(dev):
        check(lib().pir_prg_expand(sp, count, int(bits), op, _stream_ptr(stream, dev)),
              "pir_prg_expand")
    return out


def oop_offline(local: torch.Tensor, k: int, t: int, seeds: torch.Tensor,
                out: torch.Tensor = None, ws: torch.Tensor = None, stream=None) -> torch.Tensor:
    """Offline values A (count x W) of a server's local database (t*k x W
    words, flip chunk first) for ``count`` seeds (``pir_oop_offline``)."""
    rows, W, pitch = _word_matrix(local, "local")
    if rows != int(k) * int(t):
        raise ValueError("local must hold t * k rows")
    count = int(seeds.shape[0])
    dev = local.device
    sp = _ptr_words(seeds, "seeds", (count, 8), dev)
    if out is None:
        out = torch.empty((count, W), dtype=torch.int32, device=dev)
    op = _ptr_words(out, "out", (count, W), dev)
    nbytes = int(lib().pir_oop_workspace_bytes(int(k), int(t), count))
    if ws is None and nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    wp = ws.data_ptr() if ws is not None else None
    wn = ws.numel() * ws.element_size() if ws is not None else 0
    with torch.cuda.device(dev):
        check(lib().pir_oop_offline(local.data_ptr(), int(k), int(t), W, pitch, sp, count, op,
                                    wp, wn, _stream_ptr(stream, dev)), "pir_oop_offline")
    return out


def oop_answer(local: torch.Tensor, k: int, Q: torch.Tensor, A: torch.Tensor,
               out: torch.Tensor = None, stream=None) -> torch.Tensor:
    """Online responses (B x W): ``A[b]`` xor the flip-chunk rows (the first
    ``k`` rows of ``local``) selected by query ``Q[b]`` (``pir_oop_answer``)."""
    rows, W, pitch = _word_matrix(local, "local")
    if rows < int(k):
        raise ValueError("local must hold at least k rows")
    B = int(Q.shape[0])
    dev = local.device
    qp_ = _ptr_words(Q, "Q", (B, (int(k) + 31) // 32), dev)
    ap = _ptr_words(A, "A", (B, W), dev)
    if out is None:
        out = torch.empty((B, W), dtype=torch.int32, device=dev)
    op = _ptr_words(out, "out", (B, W), dev)
    with torch.cuda.device(dev):
        check(lib().pir_oop_answer(local.data_ptr(), int(k), W, pitch, qp_, B, ap, op,
                                   _stream_ptr(stream, dev)), "pir_oop_answer")
    return out
