"""ctypes binding of libwc (include/wc.h): argument marshalling only.

Every step of counting, merging and ranking runs in the HIP kernels of libwc.so; PyTorch
supplies device memory (the caller-owned workspace) and the stream. There is no CPU path:
when the library or a GPU is missing these functions raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libwc.so")

WC_OK, WC_EINVAL, WC_ENOMEM, WC_ETABLEFULL, WC_EOVERFLOW, WC_EDEVICE, WC_EAGAIN = \
    0, -1, -2, -3, -4, -5, -6
WC_GLOBAL, WC_PER_DOC = 0, 1
WC_FLUSH_ALL, WC_FLUSH_BYPASS = 0, 1
WC_DEBUG_TIME, WC_DEBUG_NO_LDS, WC_DEBUG_DIRECT, WC_DEBUG_SPILL = 1, 2, 4, 8


class WcError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib().wc_strerror(status).decode()
        if status == WC_EDEVICE:
            msg += f" (hipError {lib().wc_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{status}]")


class Tuning(ctypes.Structure):
    _fields_ = [("stage_bytes", ctypes.c_uint32), ("lds_entries", ctypes.c_uint32),
                ("flush_policy", ctypes.c_uint32), ("grid_blocks", ctypes.c_uint32),
                ("lds_load_pct", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class Opts(ctypes.Structure):
    _fields_ = [("count_bytes", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("table_slots", ctypes.c_uint64), ("tuning", ctypes.POINTER(Tuning)),
                ("debug_flags", ctypes.c_uint32), ("debug_hash_bits", ctypes.c_uint32),
                ("word_bytes_cap", ctypes.c_uint64)]


class Plan(ctypes.Structure):
    _fields_ = [("table_slots", ctypes.c_uint64), ("workspace_bytes", ctypes.c_uint64),
                ("max_entries", ctypes.c_uint64), ("word_bytes_cap", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("n_entries", ctypes.c_uint64), ("total_tokens", ctypes.c_uint64),
                ("word_bytes", ctypes.c_uint64), ("n_docs", ctypes.c_uint64),
                ("table_slots", ctypes.c_uint64), ("count_bytes", ctypes.c_uint32),
                ("mode", ctypes.c_uint32), ("d_word_offsets", ctypes.c_void_p),
                ("d_words", ctypes.c_void_p), ("d_counts", ctypes.c_void_p),
                ("d_doc_ptr", ctypes.c_void_p), ("d_docs", ctypes.c_void_p),
                ("kernel_ms", ctypes.c_float), ("total_ms", ctypes.c_float)]


class TopKStruct(ctypes.Structure):
    _fields_ = [("n_corpora", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("vocab_size", ctypes.c_uint64), ("d_word_offsets", ctypes.c_void_p),
                ("d_words", ctypes.c_void_p), ("d_n_c", ctypes.c_void_p),
                ("d_n_rest", ctypes.c_void_p), ("d_score", ctypes.c_void_p),
                ("n_rows", ctypes.c_uint64 * 64), ("word_bytes", ctypes.c_uint64)]


_lib = None


def lib():
    """Load libwc.so (building it first when it has never been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(_LIB_PATH)
        vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
        L.wc_strerror.restype = ctypes.c_char_p
        L.wc_strerror.argtypes = [ctypes.c_int32]
        L.wc_last_hip_error.restype = ctypes.c_int32
        L.wc_count_plan.argtypes = [u64, u64, ctypes.POINTER(Opts), ctypes.POINTER(Plan)]
        L.wc_count.argtypes = [vp, u64, vp, u64, ctypes.POINTER(Opts), vp, u64,
                               ctypes.POINTER(Result), vp]
        L.wc_merge_plan.argtypes = [ctypes.POINTER(ctypes.POINTER(Result)), u32,
                                    ctypes.POINTER(Opts), ctypes.POINTER(Plan)]
        L.wc_merge.argtypes = [ctypes.POINTER(ctypes.POINTER(Result)), u32, ctypes.POINTER(Opts),
                               vp, u64, ctypes.POINTER(Result), vp]
        L.wc_topk_ratio_plan.argtypes = [ctypes.POINTER(ctypes.POINTER(Result)), u32, u32,
                                         ctypes.POINTER(u64)]
        L.wc_topk_ratio.argtypes = [ctypes.POINTER(ctypes.POINTER(Result)), u32, u32, u64, vp,
                                    u64, ctypes.POINTER(TopKStruct), vp]
        L.wc_hash_words.argtypes = [vp, vp, u64, vp, vp]
        for f in ("wc_count_plan", "wc_count", "wc_merge_plan", "wc_merge", "wc_topk_ratio_plan",
                  "wc_topk_ratio", "wc_hash_words"):
            getattr(L, f).restype = ctypes.c_int32
        _lib = L
    return _lib


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _require_cuda(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")


def _alloc(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class Table:
    """A word table in device memory (result of count or merge); owns its workspace."""

    def __init__(self, res: Result, workspace: torch.Tensor, keep: tuple = ()):
        self.res = res
        self.workspace = workspace
        self._keep = keep  # inputs that long-word references may point into

    # --- device views -------------------------------------------------------------------
    def _view(self, ptr: int, nbytes: int, dtype) -> torch.Tensor:
        base = self.workspace.data_ptr()
        off = int(ptr) - base
        if nbytes == 0:
            return torch.empty(0, dtype=dtype, device=self.workspace.device)
        assert 0 <= off and off + nbytes <= self.workspace.numel()
        return self.workspace[off:off + nbytes].view(dtype)

    @property
    def n_entries(self) -> int:
        return int(self.res.n_entries)

    @property
    def total_tokens(self) -> int:
        return int(self.res.total_tokens)

    def word_offsets(self) -> torch.Tensor:
        return self._view(self.res.d_word_offsets, 8 * (self.n_entries + 1), torch.int64)

    def words(self) -> torch.Tensor:
        return self._view(self.res.d_words, int(self.res.word_bytes), torch.uint8)

    def counts(self) -> torch.Tensor:
        dt = torch.int32 if self.res.count_bytes == 4 else torch.int64
        return self._view(self.res.d_counts, self.res.count_bytes * self.n_entries, dt)

    def doc_ptr(self) -> Optional[torch.Tensor]:
        if not self.res.d_doc_ptr:
            return None
        return self._view(self.res.d_doc_ptr, 8 * (int(self.res.n_docs) + 1), torch.int64)

    def docs(self) -> Optional[torch.Tensor]:
        if not self.res.d_docs:
            return None
        return self._view(self.res.d_docs, 8 * self.n_entries, torch.int64)

    # --- host copies --------------------------------------------------------------------
    def to_host(self):
        """(words uint8, word_offsets int64[n+1], counts int64[n], docs int64[n] or None)."""
        w = self.words().cpu().numpy()
        o = self.word_offsets().cpu().numpy()
        c = self.counts().cpu().numpy().astype(np.int64)
        d = self.docs()
        return w, o, c, (d.cpu().numpy() if d is not None else None)

    def as_dict(self) -> dict:
        """{word: count}, or {(doc, word): count} for a per-document table."""
        w, o, c, d = self.to_host()
        wb = w.tobytes()
        if d is None:
            return {wb[o[e]:o[e + 1]]: int(c[e]) for e in range(len(c))}
        return {(int(d[e]), wb[o[e]:o[e + 1]]): int(c[e]) for e in range(len(c))}


def _opts(count_bytes, per_doc, table_slots, tuning, debug_flags, debug_hash_bits,
          word_bytes_cap):
    o = Opts()
    o.count_bytes = count_bytes
    o.mode = WC_PER_DOC if per_doc else WC_GLOBAL
    o.table_slots = table_slots
    o.tuning = ctypes.pointer(tuning) if tuning is not None else None
    o.debug_flags = debug_flags
    o.debug_hash_bits = debug_hash_bits
    o.word_bytes_cap = word_bytes_cap
    return o


def make_tuning(stage_bytes=0, lds_entries=0, flush_policy=WC_FLUSH_ALL, grid_blocks=0,
                lds_load_pct=0) -> Tuning:
    return Tuning(stage_bytes, lds_entries, flush_policy, grid_blocks, lds_load_pct, 0)


def count_plan(corpus_len: int, n_docs: int, *, count_bytes=8, per_doc=False, table_slots=0,
               tuning=None, word_bytes_cap=0) -> Plan:
    o = _opts(count_bytes, per_doc, table_slots, tuning, 0, 0, word_bytes_cap)
    p = Plan()
    st = lib().wc_count_plan(corpus_len, n_docs, ctypes.byref(o), ctypes.byref(p))
    if st != WC_OK:
        raise WcError(st, "wc_count_plan")
    return p


def count(corpus: torch.Tensor, offsets: Optional[torch.Tensor] = None, *, count_bytes: int = 8,
          per_doc: bool = False, table_slots: int = 0, tuning: Optional[Tuning] = None,
          debug_flags: int = 0, debug_hash_bits: int = 0, word_bytes_cap: int = 0,
          stream=None, regrow: bool = True, workspace: Optional[torch.Tensor] = None) -> Table:
    """Count the words of a device corpus (uint8) split into documents by offsets (int64).

    On a full table the call is repeated with twice the slots (regrow=True), and on an
    exported-word overflow with the reported byte count; other errors raise WcError.
    """
    _require_cuda(corpus, "corpus")
    if corpus.dtype != torch.uint8 or corpus.dim() != 1 or not corpus.is_contiguous():
        raise ValueError("corpus must be a contiguous 1-D uint8 tensor")
    n = corpus.numel()
    if offsets is None:
        offsets = torch.tensor([0, n], dtype=torch.int64, device=corpus.device)
    _require_cuda(offsets, "offsets")
    if offsets.dtype not in (torch.int64, torch.uint64) or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous int64 tensor")
    n_docs = offsets.numel() - 1
    if n_docs < 0:
        raise ValueError("offsets must hold at least one value")
    while True:
        o = _opts(count_bytes, per_doc, table_slots, tuning, debug_flags, debug_hash_bits,
                  word_bytes_cap)
        p = Plan()
        st = lib().wc_count_plan(n, n_docs, ctypes.byref(o), ctypes.byref(p))
        if st != WC_OK:
            raise WcError(st, "wc_count_plan")
        ws = workspace if (workspace is not None and workspace.numel() >= p.workspace_bytes) \
            else _alloc(p.workspace_bytes, corpus.device)
        res = Result()
        st = lib().wc_count(ctypes.c_void_p(corpus.data_ptr()), n,
                            ctypes.c_void_p(offsets.data_ptr()), n_docs, ctypes.byref(o),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(res),
                            _stream_handle(stream))
        if st == WC_ETABLEFULL and regrow:
            table_slots = 2 * int(p.table_slots)
            continue
        if st == WC_ENOMEM and regrow and res.word_bytes > p.word_bytes_cap:
            word_bytes_cap = int(res.word_bytes)
            continue
        if st != WC_OK:
            raise WcError(st, "wc_count")
        return Table(res, ws)


def _result_array(tables: Sequence[Table]):
    arr = (ctypes.POINTER(Result) * len(tables))(*[ctypes.pointer(t.res) for t in tables])
    return arr


def merge(tables: Sequence[Table], *, count_bytes: int = 8, table_slots: int = 0, stream=None,
          debug_flags: int = 0) -> Table:
    """Pointwise sum of word tables over the union of their words (one global table)."""
    if not tables:
        raise ValueError("merge needs at least one table")
    dev = tables[0].workspace.device
    while True:
        o = _opts(count_bytes, False, table_slots, None, debug_flags, 0, 0)
        arr = _result_array(tables)
        p = Plan()
        st = lib().wc_merge_plan(arr, len(tables), ctypes.byref(o), ctypes.byref(p))
        if st != WC_OK:
            raise WcError(st, "wc_merge_plan")
        ws = _alloc(p.workspace_bytes, dev)
        res = Result()
        st = lib().wc_merge(arr, len(tables), ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()),
                            ws.numel(), ctypes.byref(res), _stream_handle(stream))
        if st == WC_ETABLEFULL:
            table_slots = 2 * int(p.table_slots)
            continue
        if st != WC_OK:
            raise WcError(st, "wc_merge")
        return Table(res, ws)


@dataclass
class TopK:
    words: list       # per corpus: list of bytes
    n_c: list         # per corpus: int64 arrays
    n_rest: list
    score: list       # per corpus: float64 arrays
    vocab_size: int


def topk_ratio(tables: Sequence[Table], k: int, min_count: int = 1, stream=None) -> TopK:
    """Per-corpus top-k distinctive words (see wc_topk in include/wc.h)."""
    C = len(tables)
    dev = tables[0].workspace.device
    arr = _result_array(tables)
    need = ctypes.c_uint64()
    st = lib().wc_topk_ratio_plan(arr, C, k, ctypes.byref(need))
    if st != WC_OK:
        raise WcError(st, "wc_topk_ratio_plan")
    ws = _alloc(need.value, dev)
    out = TopKStruct()
    st = lib().wc_topk_ratio(arr, C, k, min_count, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                             ctypes.byref(out), _stream_handle(stream))
    if st != WC_OK:
        raise WcError(st, "wc_topk_ratio")
    base = ws.data_ptr()

    def view(ptr, nbytes, dtype):
        off = int(ptr) - base
        return ws[off:off + nbytes].view(dtype) if nbytes else torch.empty(0, dtype=dtype)

    rows = C * k
    woff = view(out.d_word_offsets, 8 * (rows + 1), torch.int64).cpu().numpy()
    wbytes = view(out.d_words, int(out.word_bytes), torch.uint8).cpu().numpy().tobytes()
    nc = view(out.d_n_c, 8 * rows, torch.int64).cpu().numpy()
    nr = view(out.d_n_rest, 8 * rows, torch.int64).cpu().numpy()
    sc = view(out.d_score, 8 * rows, torch.float64).cpu().numpy()
    words, ncs, nrs, scs = [], [], [], []
    for c in range(C):
        r = int(out.n_rows[c])
        b = c * k
        words.append([wbytes[woff[b + j]:woff[b + j + 1]] for j in range(r)])
        ncs.append(nc[b:b + r].copy())
        nrs.append(nr[b:b + r].copy())
        scs.append(sc[b:b + r].copy())
    return TopK(words, ncs, nrs, scs, int(out.vocab_size))


def hash_words(words: Sequence[bytes], device="cuda") -> list:
    """FNV-1a 64 of each (folded) byte string, computed by the library's device function."""
    blob = b"".join(words)
    off = np.zeros(len(words) + 1, dtype=np.int64)
    np.cumsum([len(w) for w in words], out=off[1:])
    d_b = torch.tensor(list(blob) or [0], dtype=torch.uint8, device=device)
    d_o = torch.from_numpy(off).to(device)
    d_out = torch.zeros(max(len(words), 1), dtype=torch.int64, device=device)
    st = lib().wc_hash_words(ctypes.c_void_p(d_b.data_ptr()), ctypes.c_void_p(d_o.data_ptr()),
                             len(words), ctypes.c_void_p(d_out.data_ptr()),
                             _stream_handle(None))
    if st != WC_OK:
        raise WcError(st, "wc_hash_words")
    return [int(x) & 0xFFFFFFFFFFFFFFFF for x in d_out[:len(words)].cpu().tolist()]
